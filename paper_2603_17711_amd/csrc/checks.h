// Small FP64 checks on states: root-core norms for the norm-growth check of
// the step calls, the isometry test of the canonical-center rule, and a
// zero fill for caller-visible scratch memory.
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

// A core viewed as [p0, d, p1] (complex FP64, row-major) whose middle leg
// points toward the canonical center.
struct IsoOp {
  const double* C;
  long p0, p1;
  int d;
  int pad;
};

// out[i] = max_{a,b} | sum_{x,y} conj(C[x,a,y]) C[x,b,y] - delta(a,b) |: zero
// when the core's rows along the middle leg are orthonormal.  One workgroup
// per op.
hipError_t launch_isometry(const IsoOp* ops, int n, double* out, hipStream_t s);

// out (d x d complex, row-major) = C C^H for a root core C viewed as [d, p1]
// (complex FP64): the reduced density of a wavefunction whose system end is
// the core's first index, when the core holds the state's norm (canonical
// toward the root).  One workgroup per entry.
hipError_t launch_rho_pure(const double* C, int d, long p1, double* out, hipStream_t s);

// Zero `bytes` bytes at p (a kernel, so that it may sit in captured graphs).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace tenso
