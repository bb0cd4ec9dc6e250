// Kernels of direct (vmf) integration, FP64 (see vmf.h).
#include "vmf.h"

namespace tenso {

namespace {

struct zc {
  double r, i;
};
__device__ inline zc zmul(zc a, zc b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline zc zdiv(zc a, zc b) {
  const double d = b.r * b.r + b.i * b.i;
  return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}

// In-place Gauss-Jordan inversion of A + reg I (r <= kVmfMaxRank), one
// workgroup per op.  Step k: scale pivot row k by 1 / A[k][k] (with the
// pivot entry itself replaced by 1 first), then remove column k from every
// other row; after r steps the array holds the inverse.
__global__ void __launch_bounds__(256) k_reginv(const RegInvOp* __restrict__ ops) {
  const RegInvOp op = ops[blockIdx.x];
  __shared__ zc A[kVmfMaxRank * kVmfMaxRank];
  __shared__ zc col[kVmfMaxRank];
  const int r = op.r, rr = r * r;
  for (int e = threadIdx.x; e < rr; e += blockDim.x) {
    zc v{op.rho[2 * e], op.rho[2 * e + 1]};
    if (e / r == e % r) v.r += op.reg;
    A[e] = v;
  }
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    const zc piv = A[k * r + k];
    // column k of the other rows, before the pivot row changes
    for (int i = threadIdx.x; i < r; i += blockDim.x) col[i] = A[i * r + k];
    __syncthreads();
    for (int j = threadIdx.x; j < r; j += blockDim.x) {
      const zc v = j == k ? zc{1.0, 0.0} : A[k * r + j];
      A[k * r + j] = zdiv(v, piv);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rr; e += blockDim.x) {
      const int i = e / r, j = e % r;
      if (i == k) continue;
      const zc f = col[i];
      const zc base = j == k ? zc{0.0, 0.0} : A[e];
      const zc p = zmul(f, A[k * r + j]);
      A[e] = {base.r - p.r, base.i - p.i};
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < rr; e += blockDim.x) {
    op.M[2 * e] = A[e].r;
    op.M[2 * e + 1] = A[e].i;
  }
}

// Y[a, b] -= sum_a' S[a', a] U[a', b]; grid (chunks, ops), lanes over the
// flattened (a, b) entries of a chunk.
__global__ void __launch_bounds__(256) k_vproj(const VProjOp* __restrict__ ops) {
  const VProjOp op = ops[blockIdx.y];
  const long n = (long)op.r * op.post;
  const long e0 = (long)blockIdx.x * kVmfChunk;
  if (e0 >= n) return;
  const long e1 = e0 + kVmfChunk < n ? e0 + kVmfChunk : n;
  for (long e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    const int a = (int)(e / op.post);
    const long b = e - (long)a * op.post;
    double sr = 0, si = 0;
    for (int ap = 0; ap < op.r; ++ap) {
      const zc s{op.S[2 * (ap * op.r + a)], op.S[2 * (ap * op.r + a) + 1]};
      const zc u{op.U[2 * (ap * op.post + b)], op.U[2 * (ap * op.post + b) + 1]};
      const zc p = zmul(s, u);
      sr += p.r;
      si += p.i;
    }
    op.Y[2 * e] -= sr;
    op.Y[2 * e + 1] -= si;
  }
}

// grid (chunks, segments)
__global__ void __launch_bounds__(256) k_lincomb(const LinCombOp op) {
  const VecSeg sg = op.segs[blockIdx.y];
  const long e0 = (long)blockIdx.x * kVmfChunk;
  if (e0 >= sg.n) return;
  const long e1 = e0 + kVmfChunk < sg.n ? e0 + kVmfChunk : sg.n;
  for (long e = sg.off + e0 + threadIdx.x; e < sg.off + e1; e += blockDim.x) {
    double vr = op.base ? op.base[2 * e] : 0.0, vi = op.base ? op.base[2 * e + 1] : 0.0;
    for (int j = 0; j < op.n_src; ++j) {
      vr += op.c[j] * op.src[j][2 * e];
      vi += op.c[j] * op.src[j][2 * e + 1];
    }
    op.out[2 * e] = vr;
    op.out[2 * e + 1] = vi;
  }
}

__global__ void __launch_bounds__(256) k_errnorm(const ErrNormOp op) {
  const VecSeg sg = op.segs[blockIdx.y];
  const long e0 = (long)blockIdx.x * kVmfChunk;
  double acc = 0.0;
  if (e0 < sg.n) {
    const long e1 = e0 + kVmfChunk < sg.n ? e0 + kVmfChunk : sg.n;
    for (long e = sg.off + e0 + threadIdx.x; e < sg.off + e1; e += blockDim.x) {
      double er = 0.0, ei = 0.0;
      for (int j = 0; j < op.n_src; ++j) {
        er += op.c[j] * op.src[j][2 * e];
        ei += op.c[j] * op.src[j][2 * e + 1];
      }
      const double a0 = sqrt(op.y0[2 * e] * op.y0[2 * e] + op.y0[2 * e + 1] * op.y0[2 * e + 1]);
      const double a1 = sqrt(op.y1[2 * e] * op.y1[2 * e] + op.y1[2 * e + 1] * op.y1[2 * e + 1]);
      const double sc = op.atol + op.rtol * (a0 > a1 ? a0 : a1);
      acc += (er * er + ei * ei) / (sc * sc);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) op.part[(long)blockIdx.y * op.chunks + blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(const double* __restrict__ part, int n,
                                                      double* __restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) acc += part[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

}  // namespace

hipError_t launch_reginv(const RegInvOp* ops, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reginv, dim3(n), dim3(256), 0, s, ops);
  return hipGetLastError();
}

hipError_t launch_vproj(const VProjOp* ops, int n, long max_elems, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const long chunks = (max_elems + kVmfChunk - 1) / kVmfChunk;
  hipLaunchKernelGGL(k_vproj, dim3((unsigned)chunks, n), dim3(256), 0, s, ops);
  return hipGetLastError();
}

hipError_t launch_lincomb(const LinCombOp& op, int chunks, hipStream_t s) {
  if (op.n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_lincomb, dim3(chunks, op.n_seg), dim3(256), 0, s, op);
  return hipGetLastError();
}

hipError_t launch_errnorm(const ErrNormOp& op, hipStream_t s) {
  if (op.n_seg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_errnorm, dim3(op.chunks, op.n_seg), dim3(256), 0, s, op);
  return hipGetLastError();
}

hipError_t launch_sum_partials(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, n, out);
  return hipGetLastError();
}

}  // namespace tenso
