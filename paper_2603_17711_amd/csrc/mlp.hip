// Surrogate network kernels (project addition, not part of the paper's
// method): BF16 MFMA GEMMs with FP32 accumulation and the elementwise pieces
// of a SiLU MLP's forward / backward pass and an Adam update.  Buffers are
// FP32; GEMM operands are rounded to BF16 (nearest even) when loaded.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace tenso {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline short to_bf16(float x) {
  union {
    float f;
    uint32_t u;
  } v;
  v.f = x;
  if ((v.u & 0x7f800000u) == 0x7f800000u) return (short)(v.u >> 16);  // inf / nan
  const uint32_t rounding = 0x7fffu + ((v.u >> 16) & 1u);
  return (short)((v.u + rounding) >> 16);
}

__device__ inline float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// C[m, n] = beta * C[m, n] + sum_k A(m, k) B(k, n), A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn]; optional bias[n] and SiLU epilogue writing the
// post-activation to H.  One workgroup = 32 x 32 output tile, one wavefront per
// 16 x 16 sub-tile, K in steps of 16 (v_mfma_f32_16x16x16_bf16).
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const float* __restrict__ A,
                                                   long sam, long sak, const float* __restrict__ B,
                                                   long sbk, long sbn, float* __restrict__ C, long ldc,
                                                   float beta, const float* __restrict__ bias, int act,
                                                   float* __restrict__ H) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int m0 = blockIdx.y * 32 + 16 * (wave >> 1), n0 = blockIdx.x * 32 + 16 * (wave & 1);
  v4f acc = {0, 0, 0, 0};
  const int row = m0 + c, col = n0 + c;
  for (int k0 = 0; k0 < K; k0 += 16) {
    v4s a, b;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = k0 + 4 * g + q;
      const float av = (row < M && kk < K) ? A[(long)row * sam + (long)kk * sak] : 0.0f;
      const float bv = (col < N && kk < K) ? B[(long)kk * sbk + (long)col * sbn] : 0.0f;
      a[q] = to_bf16(av);
      b[q] = to_bf16(bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int rr = m0 + 4 * g + r, cc = n0 + c;
    if (rr < M && cc < N) {
      float v = acc[r] + (beta != 0.0f ? beta * C[(long)rr * ldc + cc] : 0.0f);
      if (bias) v += bias[cc];
      C[(long)rr * ldc + cc] = v;
      if (H) H[(long)rr * ldc + cc] = act ? silu(v) : v;
    }
  }
}

__global__ void k_silu_bwd(const float* __restrict__ dH, const float* __restrict__ Z,
                           float* __restrict__ dZ, long n) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += 256L * gridDim.x)
    dZ[e] = dH[e] * silu_grad(Z[e]);
}

__global__ void k_col_sum(const float* __restrict__ X, int rows, int cols, float* __restrict__ out) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= cols) return;
  float s = 0;
  for (int r = 0; r < rows; ++r) s += X[(long)r * cols + col];
  out[col] = s;
}

// dY = 2 (Y - T) / n; loss[0] += sum (Y - T)^2 / n
__global__ void k_mse(const float* __restrict__ Y, const float* __restrict__ T, long n,
                      float* __restrict__ dY, float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += 256L * gridDim.x) {
    const float d = Y[e] - T[e];
    dY[e] = 2.0f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0] / (float)n);
}

// Adam (Kingma & Ba) on FP32 master parameters.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += 256L * gridDim.x) {
    const float ge = g[e];
    const float me = b1 * m[e] + (1.0f - b1) * ge;
    const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
    m[e] = me;
    v[e] = ve;
    p[e] -= lr * (me / c1) / (sqrtf(ve / c2) + eps);
  }
}

}  // namespace tenso

using namespace tenso;

extern "C" {

int tenso_mlp_gemm(int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk,
                   long sbn, float* C, long ldc, float beta, const float* bias, int act, float* H,
                   hipStream_t s) {
  if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return -1;
  if (M == 0 || N == 0) return 0;
  dim3 grid((N + 31) / 32, (M + 31) / 32);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, ldc,
                     beta, bias, act, H);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int tenso_mlp_silu_bwd(const float* dH, const float* Z, float* dZ, long n, hipStream_t s) {
  if (n <= 0) return 0;
  int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_silu_bwd, dim3(blocks), dim3(256), 0, s, dH, Z, dZ, n);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int tenso_mlp_col_sum(const float* X, int rows, int cols, float* out, hipStream_t s) {
  if (cols <= 0) return 0;
  hipLaunchKernelGGL(k_col_sum, dim3((cols + 255) / 256), dim3(256), 0, s, X, rows, cols, out);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int tenso_mlp_mse(const float* Y, const float* T, long n, float* dY, float* loss, hipStream_t s) {
  if (n <= 0) return 0;
  int blocks = (int)((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024);
  hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, s, Y, T, n, dY, loss);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

int tenso_mlp_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1,
                   float b2, float eps, int t, hipStream_t s) {
  if (n <= 0) return 0;
  const float c1 = 1.0f - powf(b1, (float)t), c2 = 1.0f - powf(b2, (float)t);
  int blocks = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(k_adam, dim3(blocks), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // extern "C"
