// Root-core norms (FP64) for the norm-growth check of the step calls.
#include "checks.h"

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

}  // namespace tenso
