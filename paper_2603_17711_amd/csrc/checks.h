// Norms of root cores for the norm-growth check of the step calls.  A state
// kept canonical toward the root carries its whole Frobenius norm in the root
// core (every other core is an isometry toward its parent).
#pragma once
#include <hip/hip_runtime.h>

namespace tenso {

// A state grown by more than this factor over one step call is reported as
// a numerical failure (ENUMERIC).
constexpr double kNormGrowthLimit = 1e6;

struct NormOp {
  const double* p;  // root core, interleaved complex: 2 * elements doubles
  long n;           // number of doubles
};

// out[i] = sqrt(sum_k p_i[k]^2), one workgroup per op.
hipError_t launch_norms(const NormOp* ops, int n, double* out, hipStream_t s);

}  // namespace tenso
