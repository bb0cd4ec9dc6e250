// FP64 SVD of the ps2 two-site tensor Theta (rows x cols) and the truncation
// decision, computed from Theta itself (no Gram matrix, so singular values
// keep their accuracy relative to sigma_1 down to rounding):
//
//   range finder  Y = Theta Omega (Omega: p hashed test columns), Q = qr(Y)
//   [power step   Z = Theta^H Q, W = qr(Z), Y = Theta W, Q = qr(Y)]
//   projection    Z = Theta^H Q = W R2   (so Q^H Theta = R2^H W^H)
//   small SVD     R2^H = U' S W'^H by one-sided Jacobi (p <= 64, in LDS)
//   vectors       U = Q U', V = W W';  Theta ~= U S V^H
//
// The QR steps are the gauge-move Householder kernel (k_qr) without its rank
// rule.  With p = min(64, rows, cols) the factorisation is exact when p
// equals the smaller side; otherwise it captures the leading p-dimensional
// singular subspace up to a factor (s_{p+1} / s_j)^(2q+1) on direction j
// after q power steps; the caller adds power steps while s_{p-1} exceeds
// 1e-13 s_1 (the numerical rank may exceed p) and the leading singular values
// still move.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tenso_internal.h"

namespace tenso {

namespace {

struct c2 {
  double r, i;
};

__device__ inline c2 cmul(c2 a, c2 b) { return c2{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }

// Entry (k, j) of the test matrix: real and imaginary parts uniform in
// [-1, 1), from the SplitMix64 finaliser of a counter (Steele, Lea & Flood,
// OOPSLA 2014) keyed by the seed.
__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ inline c2 test_entry(uint32_t seed, long k, int j) {
  const uint64_t c = ((uint64_t)seed << 40) ^ ((uint64_t)k << 8) ^ (uint64_t)j;
  const uint64_t a = splitmix64(2 * c), b = splitmix64(2 * c + 1);
  const double s = 1.0 / 9007199254740992.0;  // 2^-53
  return c2{(double)(a >> 11) * s * 2.0 - 1.0, (double)(b >> 11) * s * 2.0 - 1.0};
}

constexpr int kTM = 64;   // output rows per workgroup
constexpr int kKC = 16;   // summed index per LDS stage

}  // namespace

// out (M x p, column-major) = op(Theta) * B over the summed index range of
// blockIdx.y; with nsplit > 1 each range writes its own partial slab.  Mode 0
// also accumulates sum |Theta|^2 over the elements it loads (each element is
// loaded by exactly one workgroup).
__global__ void __launch_bounds__(256) k_svd_gemm(const SvdGemmOp* __restrict__ ops) {
  const SvdGemmOp op = ops[0];
  const c2* __restrict__ Th = reinterpret_cast<const c2*>(op.Theta);
  const c2* __restrict__ B = reinterpret_cast<const c2*>(op.B);
  const int M = op.mode == 0 ? op.rows : op.cols;
  const int K = op.mode == 0 ? op.cols : op.rows;
  const int m0 = blockIdx.x * kTM;
  const int kb = blockIdx.y * op.kchunk, ke = min(K, kb + op.kchunk);
  __shared__ c2 As[kKC][kTM + 1];
  __shared__ c2 Bs[kKC][64 + 1];
  __shared__ double red[4];
  const int tid = threadIdx.x, ti = tid >> 4, tj = tid & 15;
  c2 acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = c2{0.0, 0.0};
  double nrm = 0.0;
  for (int k0 = kb; k0 < ke; k0 += kKC) {
    for (int e = tid; e < kTM * kKC; e += 256) {
      int i, kk;
      c2 v{0.0, 0.0};
      if (op.mode == 0) {  // Theta[m0 + i, k0 + kk], contiguous in kk
        i = e / kKC;
        kk = e % kKC;
        if (m0 + i < M && k0 + kk < ke) v = Th[(long)(m0 + i) * op.cols + k0 + kk];
        nrm += v.r * v.r + v.i * v.i;
      } else {  // conj(Theta[k0 + kk, m0 + i]), contiguous in i
        kk = e / kTM;
        i = e % kTM;
        if (m0 + i < M && k0 + kk < ke) {
          const c2 t = Th[(long)(k0 + kk) * op.cols + m0 + i];
          v = c2{t.r, -t.i};
        }
      }
      As[kk][i] = v;
    }
    for (int e = tid; e < kKC * 64; e += 256) {
      const int kk = e % kKC, j = e / kKC;  // contiguous in k for a column of B
      c2 v{0.0, 0.0};
      if (j < op.p && k0 + kk < ke) v = B ? B[(long)j * K + k0 + kk] : test_entry(op.seed, k0 + kk, j);
      Bs[kk][j] = v;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kKC; ++kk) {
      c2 a[4], b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[kk][ti * 4 + u];
#pragma unroll
      for (int v = 0; v < 4; ++v) b[v] = Bs[kk][tj * 4 + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc[u][v].r = fma(a[u].r, b[v].r, fma(-a[u].i, b[v].i, acc[u][v].r));
          acc[u][v].i = fma(a[u].r, b[v].i, fma(a[u].i, b[v].r, acc[u][v].i));
        }
    }
    __syncthreads();
  }
  c2* __restrict__ out = reinterpret_cast<c2*>(op.nsplit > 1 ? op.part + 2L * blockIdx.y * M * op.p
                                                               : op.out);
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = m0 + ti * 4 + u, j = tj * 4 + v;
      if (i < M && j < op.p) out[(long)j * M + i] = acc[u][v];
    }
  if (op.mode == 0 && op.norm_part) {
    for (int off = 32; off > 0; off >>= 1) nrm += __shfl_xor(nrm, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = nrm;
    __syncthreads();
    if (tid == 0) op.norm_part[blockIdx.y * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
  }
}

// out = sum of the nsplit partial slabs (fixed order: deterministic).
__global__ void __launch_bounds__(256) k_svd_reduce(const SvdGemmOp* __restrict__ ops) {
  const SvdGemmOp op = ops[0];
  const int M = op.mode == 0 ? op.rows : op.cols;
  const long n = 2L * M * op.p;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += 256L * gridDim.x) {
    double s = 0.0;
    for (int z = 0; z < op.nsplit; ++z) s += op.part[z * n + e];
    op.out[e] = s;
  }
}

// One-sided Jacobi SVD of Mx = R^H (R: p x p row-major, p <= 64): columns of
// Mx are rotated pairwise (round-robin pairing, all p/2 pairs of a round in
// parallel, one half-wavefront per pair) until every pair x, y satisfies
// |x^H y| <= p eps ||x|| ||y|| (eps = 2^-52: what a length-p FP64 dot product
// resolves), pairs whose norm product is below 1e-30 ||Mx||_F^2 counting as
// orthogonal (their singular values are below 1e-15 s_1).  Then s_j = ||col_j||,
// U'[:, j] = col_j / s_j, W'[:, j] = the accumulated rotations, sorted by
// decreasing s (ties by index).
constexpr int kJacThreads = 1024;
constexpr int kJacLd = 64;
__global__ void __launch_bounds__(kJacThreads) k_svd_jacobi(const SvdJacobiOp* __restrict__ ops) {
  const SvdJacobiOp op = ops[0];
  const int p = op.p;
  const int np = p + (p & 1);  // even number of players (the pad column stays zero)
  extern __shared__ char smem_raw[];
  c2* A = reinterpret_cast<c2*>(smem_raw);  // column j at A[j * kJacLd]
  c2* V = A + 64 * kJacLd;
  __shared__ int rotated;
  __shared__ double sig[64];
  __shared__ double fro2;
  __shared__ int order[64];
  const int tid = threadIdx.x, h = tid >> 5, l = tid & 31;
  const c2* __restrict__ R = reinterpret_cast<const c2*>(op.R);
  for (int e = tid; e < 64 * 64; e += kJacThreads) {
    const int j = e / 64, i = e % 64;  // Mx[i, j] = conj(R[j, i])
    c2 v{0.0, 0.0};
    if (i < p && j < p) {
      const c2 t = R[(long)j * p + i];
      v = c2{t.r, -t.i};
    }
    A[j * kJacLd + i] = v;
    V[j * kJacLd + i] = c2{i == j && j < p ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  if (tid < 64) {
    double f = 0.0;
    for (int j = 0; j < p; ++j) {
      const c2 v = A[j * kJacLd + tid];
      f += v.r * v.r + v.i * v.i;
    }
    for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off, 64);
    if (tid == 0) fro2 = f;
  }
  __syncthreads();
  const double tol = p * 2.220446049250313e-16;
  const double tiny = 1e-30 * fro2;
  for (int sweep = 0; sweep < op.max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      if (h < np / 2) {
        int a, b;
        if (h == 0) {
          a = r;
          b = np - 1;
        } else {
          a = (r + h) % (np - 1);
          b = (r - h + (np - 1)) % (np - 1);
        }
        c2* x = A + a * kJacLd;
        c2* y = A + b * kJacLd;
        const c2 x0 = x[l], x1 = x[l + 32], y0 = y[l], y1 = y[l + 32];
        double al = x0.r * x0.r + x0.i * x0.i + x1.r * x1.r + x1.i * x1.i;
        double be = y0.r * y0.r + y0.i * y0.i + y1.r * y1.r + y1.i * y1.i;
        double gr = x0.r * y0.r + x0.i * y0.i + x1.r * y1.r + x1.i * y1.i;  // x^H y
        double gi = x0.r * y0.i - x0.i * y0.r + x1.r * y1.i - x1.i * y1.r;
        for (int off = 16; off > 0; off >>= 1) {
          al += __shfl_xor(al, off, 32);
          be += __shfl_xor(be, off, 32);
          gr += __shfl_xor(gr, off, 32);
          gi += __shfl_xor(gi, off, 32);
        }
        const double g = sqrt(gr * gr + gi * gi);
        const double nn = sqrt(al * be);
        if (g > 0.0 && nn > tiny && g > tol * nn) {
          // x' = c x - s e^{-i phi} y, y' = s e^{i phi} x + c y with
          // x^H y = g e^{i phi}: makes x'^H y' = 0
          const double zeta = (be - al) / (2.0 * g);
          const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          const c2 ep{gr / g, gi / g}, em{gr / g, -gi / g};
          const c2 sm{s * em.r, s * em.i}, sp{s * ep.r, s * ep.i};
          auto rot = [&](c2* X, c2* Y, int i) {
            const c2 u = X[i], w = Y[i];
            const c2 smw = cmul(sm, w), spu = cmul(sp, u);
            X[i] = c2{c * u.r - smw.r, c * u.i - smw.i};
            Y[i] = c2{spu.r + c * w.r, spu.i + c * w.i};
          };
          rot(x, y, l);
          rot(x, y, l + 32);
          rot(V + a * kJacLd, V + b * kJacLd, l);
          rot(V + a * kJacLd, V + b * kJacLd, l + 32);
          if (l == 0) rotated = 1;
        }
      }
      __syncthreads();
    }
    // every thread reads the flag before thread 0 may clear it again
    const int again = rotated;
    __syncthreads();
    if (!again) break;
  }
  if (tid < p) {
    double s = 0.0;
    for (int i = 0; i < p; ++i) {
      const c2 v = A[tid * kJacLd + i];
      s += v.r * v.r + v.i * v.i;
    }
    sig[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < p) {
    int rk = 0;
    for (int j = 0; j < p; ++j) rk += (sig[j] > sig[tid] || (sig[j] == sig[tid] && j < tid)) ? 1 : 0;
    order[tid] = rk;
    op.sigma[rk] = sig[tid];
  }
  __syncthreads();
  c2* __restrict__ Up = reinterpret_cast<c2*>(op.Up);
  c2* __restrict__ Wp = reinterpret_cast<c2*>(op.Wp);
  for (int e = tid; e < p * p; e += kJacThreads) {
    const int j = e / p, i = e % p;
    const double s = sig[j];
    const c2 v = A[j * kJacLd + i];
    Up[(long)order[j] * p + i] = s > 0.0 ? c2{v.r / s, v.i / s} : c2{0.0, 0.0};
    Wp[(long)order[j] * p + i] = V[j * kJacLd + i];
  }
}

// Singular vectors of the isometry side, row-major (n_iso x p):
// iso 0: U = Q U' (Q: rows x p), iso 1: V = W W' (W: cols x p).  Workgroup 0
// also takes the truncation decision (all in FP64).  The tail after r
// directions is the suffix sum m + sum_{r <= i < p} s_i^2, summed from the
// smallest term up, where m, the energy outside the captured subspace
// (||Theta||_F^2 - sum_i s_i^2), counts only when the subspace may be
// incomplete (p below the smaller side and s_{p-1} above 1e-13 s_1; else it is
// rounding).  r_eps is the smallest r whose tail is at most eps^2 times the
// total (r_eps >= 1; eps = 0 keeps every direction); the kept rank is
// r' = max(1, min(max_rank, cap_r, min(rows, cols), r_eps + 1)); k counts
// the singular values above 1e-10 s_1, at most r'.  rec_i = {r', k, r_eps},
// rec_d = {total, m}.  With ratio > 0 the count r_atol of singular values
// above atol (at least 1) replaces r_eps, and r' = max(1, min(max_rank,
// cap_r, min(rows, cols), ceil(ratio r_atol))).
__global__ void __launch_bounds__(256) k_svd_finish(const SvdFinishOp* __restrict__ ops) {
  const SvdFinishOp op = ops[0];
  const int p = op.p;
  const int n_iso = op.iso == 0 ? op.rows : op.cols;
  const c2* __restrict__ Qm = reinterpret_cast<const c2*>(op.iso == 0 ? op.Q : op.W);
  const c2* __restrict__ Sm = reinterpret_cast<const c2*>(op.iso == 0 ? op.Up : op.Wp);
  c2* __restrict__ out = reinterpret_cast<c2*>(op.out);
  for (long e = blockIdx.x * 256L + threadIdx.x; e < (long)n_iso * p; e += 256L * gridDim.x) {
    const int i = (int)(e / p), j = (int)(e % p);
    double sr = 0.0, si = 0.0;
    for (int q = 0; q < p; ++q) {
      const c2 a = Qm[(long)q * n_iso + i], b = Sm[(long)j * p + q];
      sr = fma(a.r, b.r, fma(-a.i, b.i, sr));
      si = fma(a.r, b.i, fma(a.i, b.r, si));
    }
    out[e] = c2{sr, si};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double tot = 0.0;
    for (int q = 0; q < op.n_norm_part; ++q) tot += op.norm_part[q];
    const double* s = op.sigma;
    const int avail = min(op.rows, op.cols);
    double cap2 = 0.0;
    for (int i = p - 1; i >= 0; --i) cap2 += s[i] * s[i];
    const bool partial = p < avail && s[p - 1] > 1e-13 * s[0];
    const double m = partial ? fmax(tot - cap2, 0.0) : 0.0;
    double suf[65];
    suf[p] = m;
    for (int i = p - 1; i >= 0; --i) suf[i] = suf[i + 1] + s[i] * s[i];
    const double thr = op.eps * op.eps * suf[0];
    int r_eps = avail;
    if (op.eps > 0.0)
      for (int r = 0; r <= p; ++r)
        if (suf[r] <= thr) {
          r_eps = r;
          break;
        }
    r_eps = max(1, r_eps);
    int want = r_eps + 1;
    if (op.ratio > 0.0) {
      int r_atol = 0;
      for (int i = 0; i < p; ++i) r_atol += s[i] > op.atol ? 1 : 0;
      r_eps = max(1, r_atol);
      want = (int)ceil(op.ratio * (double)r_eps);
    }
    const int rp = max(1, min(min(op.max_rank, op.cap_r), min(avail, want)));
    int k = 0;
    if (s[0] > 0.0)
      for (int i = 0; i < p; ++i) k += s[i] > 1e-10 * s[0] ? 1 : 0;
    op.rec_i[0] = rp;
    op.rec_i[1] = min(k, rp);
    op.rec_i[2] = r_eps;
    op.rec_d[0] = tot;
    op.rec_d[1] = m;
  }
}

hipError_t launch_svd_gemm(const SvdGemmOp* op, int M_tiles, int nsplit, hipStream_t s) {
  hipLaunchKernelGGL(k_svd_gemm, dim3(M_tiles, nsplit), dim3(256), 0, s, op);
  return hipGetLastError();
}

hipError_t launch_svd_reduce(const SvdGemmOp* op, long n_complex, hipStream_t s) {
  const long blocks = std::min<long>(1024, (2 * n_complex + 255) / 256);
  hipLaunchKernelGGL(k_svd_reduce, dim3((unsigned)std::max<long>(1, blocks)), dim3(256), 0, s, op);
  return hipGetLastError();
}

hipError_t launch_svd_jacobi(const SvdJacobiOp* op, hipStream_t s) {
  static bool attr = false;
  const int lds = 2 * 64 * kJacLd * (int)sizeof(c2);
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_svd_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    attr = true;
  }
  hipLaunchKernelGGL(k_svd_jacobi, dim3(1), dim3(kJacThreads), lds, s, op);
  return hipGetLastError();
}

hipError_t launch_svd_finish(const SvdFinishOp* op, long n_iso_p, hipStream_t s) {
  const long blocks = std::min<long>(512, (n_iso_p + 255) / 256);
  hipLaunchKernelGGL(k_svd_finish, dim3((unsigned)std::max<long>(1, blocks)), dim3(256), 0, s, op);
  return hipGetLastError();
}

}  // namespace tenso
