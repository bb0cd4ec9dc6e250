// Root-core norms (FP64) for the norm-growth check of the step calls, the
// isometry test behind the canonical-center check, the reduced density of a
// wavefunction state, and a zero fill.
#include "checks.h"

#include <algorithm>

namespace tenso {

__global__ void __launch_bounds__(256) k_norms(const NormOp* __restrict__ ops, double* __restrict__ out) {
  const NormOp op = ops[blockIdx.x];
  double s = 0;
  for (long i = threadIdx.x; i < op.n; i += 256) s += op.p[i] * op.p[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

hipError_t launch_norms(const NormOp* ops, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_norms, dim3(n), dim3(256), 0, s, ops, out);
  return hipGetLastError();
}

// Each thread forms Gram entries (a, b) = sum_{x,y} conj(C[x,a,y]) C[x,b,y]
// for pairs q = a*d + b strided by the workgroup size, and keeps the largest
// deviation from the identity; a tree reduction takes the maximum.
__global__ void __launch_bounds__(256) k_isometry(const IsoOp* __restrict__ ops, double* __restrict__ out) {
  const IsoOp op = ops[blockIdx.x];
  const long d = op.d;
  double worst = 0;
  for (long q = threadIdx.x; q < d * d; q += 256) {
    const long a = q / d, b = q % d;
    double re = 0, im = 0;
    for (long x = 0; x < op.p0; ++x)
      for (long y = 0; y < op.p1; ++y) {
        const double* u = op.C + 2 * ((x * d + a) * op.p1 + y);
        const double* v = op.C + 2 * ((x * d + b) * op.p1 + y);
        re += u[0] * v[0] + u[1] * v[1];
        im += u[0] * v[1] - u[1] * v[0];
      }
    if (a == b) re -= 1.0;
    worst = fmax(worst, sqrt(re * re + im * im));
  }
  __shared__ double red[256];
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t launch_isometry(const IsoOp* ops, int n, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_isometry, dim3(n), dim3(256), 0, s, ops, out);
  return hipGetLastError();
}

// Reduced density of a wavefunction held by a root core viewed as [d, p1]
// (its first end is the system, every other index is traced):
// out[a, b] = sum_y C[a, y] conj(C[b, y]), one workgroup per entry (a, b).
__global__ void __launch_bounds__(256) k_rho_pure(const double* __restrict__ C, int d, long p1,
                                                  double* __restrict__ out) {
  const long a = blockIdx.x / d, b = blockIdx.x % d;
  double re = 0, im = 0;
  for (long y = threadIdx.x; y < p1; y += 256) {
    const double* u = C + 2 * (a * p1 + y);
    const double* v = C + 2 * (b * p1 + y);
    re += u[0] * v[0] + u[1] * v[1];
    im += u[1] * v[0] - u[0] * v[1];
  }
  __shared__ double rr[256], ri[256];
  rr[threadIdx.x] = re;
  ri[threadIdx.x] = im;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rr[threadIdx.x] += rr[threadIdx.x + w];
      ri[threadIdx.x] += ri[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = rr[0];
    out[2 * blockIdx.x + 1] = ri[0];
  }
}

hipError_t launch_rho_pure(const double* C, int d, long p1, double* out, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho_pure, dim3(d * d), dim3(256), 0, s, C, d, p1, out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_zero(uint4* __restrict__ p, size_t n16, unsigned char* tail,
                                              size_t n_tail) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
  if (blockIdx.x == 0 && threadIdx.x < n_tail) tail[threadIdx.x] = 0;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t blocks = std::min<size_t>(2048, std::max<size_t>(1, (n16 + 255) / 256));
  hipLaunchKernelGGL(k_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)p, n16,
                     (unsigned char*)p + n16 * 16, bytes - n16 * 16);
  return hipGetLastError();
}

}  // namespace tenso
