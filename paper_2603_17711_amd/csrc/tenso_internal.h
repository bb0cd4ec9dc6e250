// Internal descriptors shared by the host plan compiler and the HIP kernels.
// Every device-side operation of a propagation step is described by one of the
// plain structs below; a launch hands a kernel an array of them.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tenso {

// One SOP term as seen by a contraction: Y += coef(t) * A x_{l1} B x_{l2} X.
// A (d1 x d1) or B (d2 x d2) is null for an identity factor.  Matrices are
// row-major complex in the plan's compute precision.
struct TermRef {
  double cre, cim;     // base coefficient
  int slot;            // drive slot (-1: time independent)
  int pad;
  const void* A;
  const void* B;
};

// One pair group of one contraction: X viewed as [P0, d1, P1, d2, P2]; the
// free index f = (p0, p1, p2) runs over F = P0*P1*P2 matrices X_f (d1 x d2).
// Y (same view) receives sum_terms coef * A X_f B^T.
struct ApplyGroup {
  const void* X;       // input: FP64 master (in_fp64 1 or 2) or compute precision (0)
  void* Y;             // output, compute precision
  const TermRef* terms;
  const double* drive; // drive table of the instance (nullable)
  int in_fp64;         // 2: an RK4 stage input formed while staging (xp below)
  int n_terms;
  int d1, d2, P1, P2;
  int F;
  int drive_ld;        // row length of the drive table
  int rel;             // stage time index relative to the step (0..4)
  int accumulate;      // 1: Y += result, 0: Y = result
  int per_term_out;    // 1: term m writes its own result to Y + m * F*d1*d2 (no sum)
  int xp_half;         // in_fp64 2: xp_s is sign * h (0) or sign * h / 2 (1) before binding
  // in_fp64 2: the input is (compute precision)(X + xp_s * k), X the FP64
  // master and k the sum, in order, of the previous stage's xp_np partial
  // outputs (compute precision, xp_n elements apart): the stage update of an
  // RK4 sub-flow, formed while the input is staged instead of by a launch
  const void* xp;
  long xp_n;
  int xp_np;
  int pad2_;
  double xp_s;
};

// Wavefronts of an apply workgroup, accumulator tiles per wavefront, and the
// most units of one tile (kApplyWaves * (kApplyAccTiles / nib) for nib 16-row
// blocks of leg 1: every wavefront's units fit its accumulators).
constexpr int kApplyWaves = 4;
constexpr int kApplyAccTiles = 4;
constexpr int kApplyMaxUnits = 16;
static_assert(kApplyMaxUnits <= kApplyWaves * kApplyAccTiles, "tile units");

// A tile of the apply kernel: a range of units of one group.  A unit is one
// (free index f, 16-column block jb of leg 2) pair, u = f * njb + jb; wavefront
// w of the workgroup takes units u0 + w, u0 + w + kApplyWaves, ...
// Dynamic LDS available to one apply tile: the 160 KB of a CU less 1 KB
// kept for the kernel's static LDS.
constexpr int kApplyLdsBudget = 159 * 1024;
// FP32 tiles are shrunk (fewer units) until their LDS fits this share, when
// they can: two workgroups then share a CU (the register budget allows two),
// so one wavefront's LDS and barrier waits overlap the other's MFMAs.  A
// launch takes the largest LDS of its tiles.
constexpr int kApplyLdsShare = 78 * 1024;

struct ApplyTile {
  int group;           // index into the launch's group array
  int u0, nu;
  int pad;
};

// Weighted sum of matrices: out = sum_i coef_i(t) * M_i (single-leg terms).
// Finiteness check of one FP64 state: *flag is set to 1 if any of its n
// doubles is NaN or infinite (the caller clears the flags first).
struct FiniteOp {
  const double* p;
  long n;
  int* flag;
  int pad_[2];
};

// Largest number of terms one presum sums (its descriptors are staged in LDS).
constexpr int PRESUM_MAX_TERMS = 512;

struct PresumOp {
  void* out;           // compute precision, dim x dim
  const TermRef* terms;  // uses cre/cim/slot and A
  const double* drive;
  int n_terms, dim, drive_ld, rel;
};

// RK4 stage update after an apply: k = sum of n_parts partial outputs.
struct CombineOp {
  double* y0;          // FP64 master (updated at stage 4)
  void* xin;           // compute-precision stage input for the next apply
  double* acc;         // FP64 RK4 accumulator
  const void* parts;   // n_parts consecutive slabs of n elements
  long n;
  int n_parts;
  int stage;           // 1..4; 0: y0 = sum of parts; 5: xin = sum of parts;
                       // 6: y0 += h/6 (k1 + 2 k2 + 2 k3 + k4), k_s the sum of
                       // stage s's parts, stage_stride elements after stage s-1's
  double h;            // sign * tau
  long stage_stride;
};

// Householder QR (LAPACK geqr2/ung2r convention) of a core matricised as
// (other legs, row-major) x (leg of dim n); Q replaces the core in place.
// The m x n matrix element (row = pre*Ppost + post, col) sits at
// pre*n*Ppost + col*Ppost + post.
// Tallest QR whose columns are worked on in registers (taller ones take a
// form with every row loop in global memory).  Every form works on the
// scratch V, apart from C.
constexpr int kQrBlockedMaxM = 1024;

// Residual columns at or below tol * ||A||_F count as exact zeros (identity
// reflector): kQrRankTol for gauge moves; 0 (plain Householder) inside the
// ps2 SVD, whose range finder needs no fixed completion.
constexpr double kQrRankTol = 1e-10;

struct QrOp {
  double* C;           // FP64 complex core
  double* R;           // out: n x n (or its transpose when transposeR)
  double* V;           // scratch m x n complex, apart from C
  double* tau;         // scratch n complex
  int m, n, Ppost, transposeR;
  double tol;          // relative rank threshold
};

// Forms of a QR launch, chosen from its ops: the whole matrix in LDS (every
// op m <= kQrLdsMaxM and m n <= kQrLdsElems), column by column on the scratch
// copy (every op m <= kQrLdsMaxM), or blocked (any taller op).
constexpr int kQrLdsMaxM = 512;
constexpr int kQrLdsElems = 8192;
enum { kQrFormColumns = 0, kQrFormLds = 1, kQrFormBlocked = 2 };
inline int qr_form(const QrOp& q) {
  if (q.m > kQrLdsMaxM) return kQrFormBlocked;
  return q.m * q.n <= kQrLdsElems ? kQrFormLds : kQrFormColumns;
}
// the form that serves every op of a launch
inline int qr_form_join(int a, int b) {
  if (a == kQrFormBlocked || b == kQrFormBlocked) return kQrFormBlocked;
  return (a == kQrFormLds && b == kQrFormLds) ? kQrFormLds : kQrFormColumns;
}

// In-place mode product of an FP64 core with an n x n FP64 matrix on one leg:
// C[pre, a, post] <- sum_a' Mx[a, a'] C[pre, a', post], Mx = M or M^T.
// A launch's dynamic LDS: the n x n operator plus its tiles' fibers (at most
// 2048 elements per tile, or n when n is larger), 16 bytes per element.
constexpr int kAbsorbMaxN = 64;
constexpr size_t kAbsorbLdsMax = (size_t)(kAbsorbMaxN * kAbsorbMaxN + 2048) * 16;
inline size_t absorb_lds(int n, int per) { return ((size_t)n * n + (size_t)per * n) * 16; }
struct AbsorbOp {
  double* C;
  const double* M;
  int n, Ppost, Ppre, transposeM;
};

// Environment finalisation: E[a', a] = sum_{rest} conj(C[.., a', ..]) T[.., a, ..]
// over every leg but the open one (dim r): C is the FP64 master core, T the
// operator-applied copy (compute precision), E compute precision r x r.
struct GramOp {
  const double* C;
  const void* T;
  void* E;
  int r, Ppost, Ppre;
};

// Bottom-up vacuum contraction for rho_S.
struct RhoNode {
  const double* C;     // FP64 core
  int n_legs;
  int dims[8];
  int kind[8];         // 0 parent, 1 end (index 0), 2 system end (kept), 3 child bond
  int child_slot[8];   // for kind 3: index into the vector scratch
  int out_slot;        // vector scratch index of this node (-1 for the root)
};

struct RhoProg {
  const RhoNode* nodes;  // reverse preorder (root last)
  int n_nodes;
  double* vecs;          // scratch: n_nodes vectors of up to max_rank complex
  int vec_ld;
  double* rho_out;       // M*M complex
};

// ps2 edge operations (FP64).  Theta is the merged two-site tensor stored as a
// rows x cols row-major matrix: rows = the s-side legs in order (the legs of
// core s except its leg toward c), cols = the c-side legs (core c except its
// parent leg).
struct MergeOp {           // Theta[row, col] = sum_a Cs[pre, a, post] Cc[a, col]
  const double* Cs;
  const double* Cc;
  double* Theta;
  int rows, cols, r, Ppost;  // row = pre * Ppost + post
};

// ps2 SVD of Theta (see svd.hip).  Test-matrix width, the most power steps
// the caller adds while the leading singular values still move, and the
// sweep cap of the small Jacobi SVD.
constexpr int kSvdP = 64;
constexpr int kSvdMaxPower = 3;
constexpr int kSvdMaxSweeps = 40;

// out (M x p, column-major) = Theta * B (mode 0, M = rows, summed over cols) or
// Theta^H * B (mode 1, M = cols, summed over rows).  B: column-major K x p, or
// null for the hashed test matrix of `seed`.  nsplit > 1: summed-index ranges
// of kchunk write partial slabs into `part` (nsplit x M x p), summed by the
// reduce kernel.  Mode 0 with norm_part: per-workgroup partial sums of
// |Theta|^2 (grid order).
struct SvdGemmOp {
  const double* Theta;
  const double* B;
  double* out;
  double* part;
  double* norm_part;
  int rows, cols, p, mode;
  int nsplit, kchunk;
  uint32_t seed;
  int pad_;
};

// One-sided Jacobi SVD of R^H (R: p x p row-major): sigma descending, Up and
// Wp (p x p column-major) its left and right singular vectors.
struct SvdJacobiOp {
  const double* R;
  double* Up;
  double* Wp;
  double* sigma;
  int p, max_sweeps;
};

// Singular vectors of the isometry side (iso 0: Q Up, rows x p; iso 1: W Wp,
// cols x p; row-major into `out`) and the truncation decision (FP64).
struct SvdFinishOp {
  const double* Q;         // rows x p column-major
  const double* W;         // cols x p column-major
  const double* Up;
  const double* Wp;
  const double* sigma;
  const double* norm_part;
  double* out;
  int* rec_i;              // r', k, r_eps
  double* rec_d;           // ||Theta||_F^2, energy outside the captured subspace
  double eps;
  int n_norm_part, rows, cols, p, iso, max_rank, cap_r, pad_;
  // ratio > 0: keep ceil(ratio * r_atol) directions instead of r_eps + 1,
  // r_atol = the number of singular values above atol (at least 1)
  double atol, ratio;
};

// Split Theta into an isometry W (m_iso x r': the first k columns are the
// leading singular vectors of the isometry side, E (m_iso x ld_e, row-major),
// the rest completed by projecting unit vectors) and the projected other
// core.  iso 0: W on the rows (new C_s), C_c = W^H Theta; iso 1: W on the
// cols (new C_c = W^H as r' x cols), C_s = Theta W.
struct SplitOp {
  const double* Theta;
  const double* E;
  int rows, cols, iso, k, rp, ld_e;
  double* W;               // scratch m_iso x rp complex
  double* Cs;              // new core s: (rows x rp) scattered with leg i in place
  double* Cc;              // new core c: rp x cols
  int Ppost_s;             // product of s's legs after leg i (for the scatter)
  int pad_;
};

}  // namespace tenso
