// Device operations of direct (vmf) integration: the regularised inverse of
// the bond densities, the tangent-space projection of the non-root cores, and
// the dopri5 stage combinations and error norm over a whole state.  All FP64
// complex (interleaved re, im), row-major.
#pragma once
#include <hip/hip_runtime.h>

namespace tenso {

// Largest bond the inverse handles (one workgroup, the matrix in LDS).
constexpr int kVmfMaxRank = 64;

// M = (rho + reg I)^-1 for an r x r complex rho (Gauss-Jordan in place,
// pivots on the diagonal: the shifted density is Hermitian positive definite).
struct RegInvOp {
  const double* rho;
  double* M;
  double reg;
  int r, pad_;
};

// Y[a, b] -= sum_a' S[a', a] U[a', b] for a core U viewed as r x post:
// Y minus its projection onto the span of U's rows, given S = U^H Y.
struct VProjOp {
  double* Y;
  const double* U;
  const double* S;
  long post;
  int r, pad_;
};

// Segments of a state buffer that hold core entries (offsets and lengths in
// complex elements); every state-shaped buffer of a plan shares them.
struct VecSeg {
  long off, n;
};

constexpr int kLinCombMax = 7;

// out = base + sum_j c[j] src[j] over the segments (base nullable: zero).
struct LinCombOp {
  double* out;
  const double* base;
  const double* src[kLinCombMax];
  double c[kLinCombMax];
  int n_src;
  int n_seg;
  const VecSeg* segs;
};

// Per-workgroup partial sums of |e|^2 / (atol + rtol max(|y0|, |y1|))^2 over
// the complex entries of the segments, with e = sum_j c[j] src[j].  Partial
// k of segment g sits at part[g * chunks + k]; launch_sum_partials adds the
// n partials in a fixed order into out[0].
struct ErrNormOp {
  const double* y0;
  const double* y1;
  const double* src[kLinCombMax];
  double c[kLinCombMax];
  double rtol, atol;
  int n_src;
  int n_seg;
  const VecSeg* segs;
  double* part;
  int chunks;
  int pad_;
};

// Elements (complex) of one workgroup chunk of the segment kernels: one per
// thread, so that a workgroup's loads are in flight together.
constexpr int kVmfChunk = 256;

hipError_t launch_reginv(const RegInvOp* ops, int n, hipStream_t s);
hipError_t launch_vproj(const VProjOp* ops, int n, long max_elems, hipStream_t s);
hipError_t launch_lincomb(const LinCombOp& op, int chunks, hipStream_t s);
hipError_t launch_errnorm(const ErrNormOp& op, hipStream_t s);
hipError_t launch_sum_partials(const double* part, int n, double* out, hipStream_t s);

}  // namespace tenso
