// HIP kernels for CDNA4 (gfx950) of the TTN-HEOM propagation library.
//
// apply  : Y_f += sum_m coef_m(t) A_m X_f B_m^T over the free index f of a
//          core viewed as [P0, d1, P1, d2, P2] (effective generator of the SOP
//          form, paper Eq. master_lvn, contracted at one node / bond / edge),
//          complex real-split on 16x16x4 MFMA (FP32 or FP64), one wavefront per
//          (f, 16-column block) unit, intermediate X_f B^T staged in LDS.
// presum : weighted sums of matrices (single-leg terms summed once per stage).
// combine: RK4 stage bookkeeping into the FP64 master state.
// qr     : Householder QR in FP64 (gauge moves of the projector splitting).
// absorb : in-place FP64 mode product of a bond matrix into a core.
// gram   : environment finalisation E = conj(C)_(open) T_(open)^T.
// rho    : bottom-up vacuum contraction for rho_S = <0|Omega>.
#include <hip/hip_runtime.h>
#include <math.h>
#include <algorithm>
#include "tenso_internal.h"

namespace tenso {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct MT;
template <> struct MT<float> {
  typedef v4f v4;
  static constexpr int NT = 4;  // accumulator tiles per wavefront
  __device__ static inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of accumulator register r in lane group g (measured on gfx950)
  __device__ static inline int drow(int g, int r) { return 4 * g + r; }
};
template <> struct MT<double> {
  typedef v4d v4;
  static constexpr int NT = 4;
  __device__ static inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the FP64 variant interleaves rows across lane groups (measured on gfx950)
  __device__ static inline int drow(int g, int r) { return g + 4 * r; }
};

template <typename T> struct cpx { T re, im; };

template <typename Tin, typename T>
__device__ inline cpx<T> ldc(const void* base, long idx) {
  const Tin* p = reinterpret_cast<const Tin*>(base) + 2 * idx;
  return cpx<T>{(T)p[0], (T)p[1]};
}

__device__ inline void coef_at(const TermRef& t, const double* drive, int ld, int j,
                               double& cr, double& ci) {
  cr = t.cre;
  ci = t.cim;
  if (t.slot >= 0 && drive) {
    double f = drive[(long)t.slot * ld + j];
    cr *= f;
    ci *= f;
  }
}

// ---------------------------------------------------------------------------
// apply
// ---------------------------------------------------------------------------
// Wavefront-level complex 16x16x4 product: acc += a * b, with a, b given as
// (re, im) operand values of this lane.
template <typename T>
__device__ inline void cmma(typename MT<T>::v4& cr, typename MT<T>::v4& ci, T ar, T ai, T br,
                            T bi) {
  // the two products into the same accumulator are issued apart so that the
  // dependent MFMAs interleave with the independent ones
  cr = MT<T>::mma(ar, br, cr);
  ci = MT<T>::mma(ar, bi, ci);
  cr = MT<T>::mma(-ai, bi, cr);
  ci = MT<T>::mma(ai, br, ci);
}

struct UnitGeo {
  long base;
  int col;
};

__device__ inline UnitGeo unit_geo(const ApplyGroup& G, int u, int njb, int c) {
  const int f = u / njb, jb = u % njb;
  const int p2 = f % G.P2;
  const int p1 = (f / G.P2) % G.P1;
  const int p0 = f / (G.P2 * G.P1);
  UnitGeo r;
  r.base = (long)p0 * G.d1 * G.P1 * G.d2 * G.P2 + (long)p1 * G.d2 * G.P2 + p2;
  r.col = 16 * jb + c;
  return r;
}

template <typename T>
__device__ inline void load_scaled(const T* M, int d, int row, int kk, double cr, double ci, T& ar,
                                   T& ai) {
  ar = 0;
  ai = 0;
  if (row < d && kk < d) {
    const double a0 = M[2 * ((long)row * d + kk)], a1 = M[2 * ((long)row * d + kk) + 1];
    ar = (T)(a0 * cr - a1 * ci);
    ai = (T)(a0 * ci + a1 * cr);
  }
}

// LDS layout of one apply tile (T elements; complex values interleaved):
//   X : nfl x D1 x (D2 + 1)     the tile's input slices X_f, zero padded
//   A : D1 x (D1 + 1)           coefficient-scaled operand of the current term
//   B : D2 x (D2 + 1)
//   Z : 4 wavefronts x D1 x 16  per-wave X_f B^T of one unit
// with D = 16 * ceil(d / 16).  Every MFMA operand is then one LDS vector load
// without bounds checks.
__host__ __device__ inline long apply_lds_elems(int nfl, int d1, int d2, int) {
  const long D1 = 16 * ((d1 + 15) / 16), D2 = 16 * ((d2 + 15) / 16);
  return 2 * (nfl * D1 * (D2 + 1) + D1 * (D1 + 1) + D2 * (D2 + 1) + 4 * D1 * 16);
}

template <typename T> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };

template <typename T, typename Tin>
__global__ void __launch_bounds__(256, 2) k_apply(const ApplyGroup* __restrict__ groups,
                                               const ApplyTile* __restrict__ tiles,
                                               const int* __restrict__ step_ctr) {
  typedef typename MT<T>::v4 v4;
  typedef typename V2<T>::t c2;
  constexpr int NT = MT<T>::NT;
  extern __shared__ char smem_raw[];
  c2* smem = reinterpret_cast<c2*>(smem_raw);
  const ApplyTile tile = tiles[blockIdx.x];
  const ApplyGroup& G = groups[tile.group];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane & 15;   // MFMA row / column within a 16-block
  const int g = lane >> 4;   // K sub-index (0..3)
  const int d1 = G.d1, d2 = G.d2;
  const int nib = (d1 + 15) >> 4, njb = (d2 + 15) >> 4;
  const int D1 = 16 * nib, D2 = 16 * njb;
  const int xs1 = D2 + 1, as1 = D1 + 1, bs1 = D2 + 1;  // padded row strides
  const int nq1 = (d2 + 3) >> 2;  // K steps of X_f B^T
  const int nq2 = (d1 + 3) >> 2;  // K steps of A Z
  const long sb = G.P2;
  const long sa = (long)G.P1 * d2 * G.P2;
  const int step = step_ctr ? *step_ctr : 0;
  const int jdrv = 4 * step + G.rel;
  const int f_first = tile.u0 / njb;
  const int nfl = (tile.u0 + tile.nu - 1) / njb - f_first + 1;
  c2* xs = smem;
  c2* as = xs + (long)nfl * D1 * xs1;
  c2* bs = as + (long)D1 * as1;
  c2* zs = bs + (long)D2 * bs1 + (long)wave * D1 * 16;

  // stage the tile's input slices (zero padded, compute precision)
  for (long e = threadIdx.x; e < (long)nfl * D1 * D2; e += 256) {
    const int fl = (int)(e / ((long)D1 * D2));
    const int rem = (int)(e % ((long)D1 * D2));
    const int a = rem / D2, bcol = rem % D2;
    c2 v;
    v.x = 0;
    v.y = 0;
    if (a < d1 && bcol < d2) {
      const UnitGeo ug = unit_geo(G, (f_first + fl) * njb, njb, 0);
      const cpx<T> x = ldc<Tin, T>(G.X, ug.base + a * sa + bcol * sb);
      v.x = x.re;
      v.y = x.im;
    }
    xs[((long)fl * D1 + a) * xs1 + bcol] = v;
  }

  int n_my = tile.nu > wave ? (tile.nu - wave + 3) / 4 : 0;
  if (n_my * nib > NT) n_my = NT / nib;
  v4 yr[NT], yi[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    yr[t] = v4{0, 0, 0, 0};
    yi[t] = v4{0, 0, 0, 0};
  }

  for (int m = 0; m < G.n_terms; ++m) {
    const TermRef tr = G.terms[m];
    double cr, ci;
    coef_at(tr, G.drive, G.drive_ld, jdrv, cr, ci);
    const T* Am = reinterpret_cast<const T*>(tr.A);
    const T* Bm = reinterpret_cast<const T*>(tr.B);
    __syncthreads();  // previous term's operands are no longer read
    if (Am) {  // A carries the coefficient
      for (int e = threadIdx.x; e < D1 * D1; e += 256) {
        const int i = e / D1, j = e % D1;
        c2 v;
        v.x = 0;
        v.y = 0;
        if (i < d1 && j < d1) {
          const double a0 = Am[2 * (i * d1 + j)], a1 = Am[2 * (i * d1 + j) + 1];
          v.x = (T)(a0 * cr - a1 * ci);
          v.y = (T)(a0 * ci + a1 * cr);
        }
        as[i * as1 + j] = v;
      }
    }
    if (Bm) {  // B carries it only for one-sided B terms
      const double br0 = Am ? 1.0 : cr, bi0 = Am ? 0.0 : ci;
      for (int e = threadIdx.x; e < D2 * D2; e += 256) {
        const int i = e / D2, j = e % D2;
        c2 v;
        v.x = 0;
        v.y = 0;
        if (i < d2 && j < d2) {
          const double b0 = Bm[2 * (i * d2 + j)], b1 = Bm[2 * (i * d2 + j) + 1];
          v.x = (T)(b0 * br0 - b1 * bi0);
          v.y = (T)(b0 * bi0 + b1 * br0);
        }
        bs[i * bs1 + j] = v;
      }
    }
    __syncthreads();
    for (int uu = 0; uu < n_my; ++uu) {
      const int u = tile.u0 + wave + 4 * uu;
      const int fl = u / njb - f_first, jb = u % njb;
      const c2* xf = xs + (long)fl * D1 * xs1;
      const int col = 16 * jb + c;
      const int t_lo = uu * nib;
      if (Am && Bm) {
        v4 zra[NT], zia[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          zra[t] = v4{0, 0, 0, 0};
          zia[t] = v4{0, 0, 0, 0};
        }
        for (int q = 0; q < nq1; ++q) {
          const int kk = 4 * q + g;
          const c2 bv = bs[col * bs1 + kk];
#pragma unroll
          for (int t = 0; t < NT; ++t) {
            if (t < nib) {
              const c2 xv = xf[(16 * t + c) * xs1 + kk];
              cmma<T>(zra[t], zia[t], xv.x, xv.y, bv.x, bv.y);
            }
          }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (t < nib) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              c2 v;
              v.x = zra[t][r];
              v.y = zia[t][r];
              zs[(16 * t + MT<T>::drow(g, r)) * 16 + c] = v;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int q = 0; q < nq2; ++q) {
          const int kk = 4 * q + g;
          const c2 zv = zs[kk * 16 + c];
#pragma unroll
          for (int ti = 0; ti < NT; ++ti) {
            if (ti >= t_lo && ti < t_lo + nib) {
              const c2 av = as[(16 * (ti - t_lo) + c) * as1 + kk];
              cmma<T>(yr[ti], yi[ti], av.x, av.y, zv.x, zv.y);
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      } else if (Am) {
        for (int q = 0; q < nq2; ++q) {
          const int kk = 4 * q + g;
          const c2 xv = xf[kk * xs1 + col];
#pragma unroll
          for (int ti = 0; ti < NT; ++ti) {
            if (ti >= t_lo && ti < t_lo + nib) {
              const c2 av = as[(16 * (ti - t_lo) + c) * as1 + kk];
              cmma<T>(yr[ti], yi[ti], av.x, av.y, xv.x, xv.y);
            }
          }
        }
      } else if (Bm) {
        for (int q = 0; q < nq1; ++q) {
          const int kk = 4 * q + g;
          const c2 bv = bs[col * bs1 + kk];
#pragma unroll
          for (int ti = 0; ti < NT; ++ti) {
            if (ti >= t_lo && ti < t_lo + nib) {
              const c2 xv = xf[(16 * (ti - t_lo) + c) * xs1 + kk];
              cmma<T>(yr[ti], yi[ti], xv.x, xv.y, bv.x, bv.y);
            }
          }
        }
      }
    }
  }
  T* Y = reinterpret_cast<T*>(G.Y);
#pragma unroll
  for (int ti = 0; ti < NT; ++ti) {
    if (ti < n_my * nib) {
      const int uu = ti / nib, t = ti % nib;
      const UnitGeo ug = unit_geo(G, tile.u0 + wave + 4 * uu, njb, c);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * t + MT<T>::drow(g, r);
        if (row < d1 && ug.col < d2) {
          const long o = 2 * (ug.base + row * sa + (long)ug.col * sb);
          if (G.accumulate) {
            Y[o] += yr[ti][r];
            Y[o + 1] += yi[ti][r];
          } else {
            Y[o] = yr[ti][r];
            Y[o + 1] = yi[ti][r];
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// presum: out = sum_i coef_i(t) M_i
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_presum(const PresumOp* __restrict__ ops,
                                                const int* __restrict__ step_ctr) {
  const PresumOp& op = ops[blockIdx.x];
  const int step = step_ctr ? *step_ctr : 0;
  const int j = 4 * step + op.rel;
  const int n = op.dim * op.dim;
  T* out = reinterpret_cast<T*>(op.out);
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double sr = 0, si = 0;
    for (int m = 0; m < op.n_terms; ++m) {
      const TermRef& t = op.terms[m];
      double cr, ci;
      coef_at(t, op.drive, op.drive_ld, j, cr, ci);
      const T* M = reinterpret_cast<const T*>(t.A);
      const double a = M[2 * e], b = M[2 * e + 1];
      sr += a * cr - b * ci;
      si += a * ci + b * cr;
    }
    out[2 * e] = (T)sr;
    out[2 * e + 1] = (T)si;
  }
}

// ---------------------------------------------------------------------------
// combine: RK4 stage update (FP64 master, compute-precision stage input)
// ---------------------------------------------------------------------------
struct CombineTile {
  int op;
  int pad;
  long e0, e1;
};

template <typename T>
__global__ void __launch_bounds__(256) k_combine(const CombineOp* __restrict__ ops,
                                                 const CombineTile* __restrict__ tiles) {
  const CombineTile tl = tiles[blockIdx.x];
  const CombineOp& op = ops[tl.op];
  const T* parts = reinterpret_cast<const T*>(op.parts);
  T* xin = reinterpret_cast<T*>(op.xin);
  for (long e = tl.e0 + threadIdx.x; e < tl.e1; e += blockDim.x) {
    double kr = 0, ki = 0;
    for (int p = 0; p < op.n_parts; ++p) {
      kr += (double)parts[2 * (p * op.n + e)];
      ki += (double)parts[2 * (p * op.n + e) + 1];
    }
    if (op.stage == 0) {  // plain evaluation: y0 = k
      op.y0[2 * e] = kr;
      op.y0[2 * e + 1] = ki;
      continue;
    }
    const double yr = op.y0[2 * e], yi = op.y0[2 * e + 1];
    if (op.stage == 1) {
      op.acc[2 * e] = kr;
      op.acc[2 * e + 1] = ki;
      xin[2 * e] = (T)(yr + 0.5 * op.h * kr);
      xin[2 * e + 1] = (T)(yi + 0.5 * op.h * ki);
    } else if (op.stage == 2 || op.stage == 3) {
      op.acc[2 * e] += 2.0 * kr;
      op.acc[2 * e + 1] += 2.0 * ki;
      const double s = op.stage == 2 ? 0.5 * op.h : op.h;
      xin[2 * e] = (T)(yr + s * kr);
      xin[2 * e + 1] = (T)(yi + s * ki);
    } else {
      op.y0[2 * e] = yr + (op.h / 6.0) * (op.acc[2 * e] + kr);
      op.y0[2 * e + 1] = yi + (op.h / 6.0) * (op.acc[2 * e + 1] + ki);
    }
  }
}

// ---------------------------------------------------------------------------
// FP64 Householder QR (LAPACK zgeqr2 + zung2r conventions)
// ---------------------------------------------------------------------------
struct z2 {
  double r, i;
};
// Relative rank threshold of the gauge-move QR: a residual column with norm at
// or below QR_RANK_TOL * ||A||_F is treated as exactly zero (identity
// reflector), so the completion of a rank-deficient core does not follow
// rounding noise.
constexpr double QR_RANK_TOL = 1e-10;
__device__ inline z2 zmul(z2 a, z2 b) { return z2{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline z2 zconjmul(z2 a, z2 b) {  // conj(a) * b
  return z2{a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ void __launch_bounds__(256) k_qr(const QrOp* __restrict__ ops) {
  const QrOp op = ops[blockIdx.x];
  const int m = op.m, n = op.n, k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[8];  // [0..3] column norms, [4..7] Frobenius norm
  __shared__ double sh_tau[2], sh_scale[2], sh_beta[2];
  __shared__ int sh_skip;
  z2* V = reinterpret_cast<z2*>(op.V);  // column-major m x n
  z2* tau = reinterpret_cast<z2*>(op.tau);
  z2* C = reinterpret_cast<z2*>(op.C);
  auto cidx = [&](int row, int col) -> long {
    const int pre = row / op.Ppost, post = row % op.Ppost;
    return (long)pre * n * op.Ppost + (long)col * op.Ppost + post;
  };
  double fro = 0;
  for (long e = tid; e < (long)m * n; e += 256) {
    const int row = e % m, col = e / m;
    const z2 v = C[cidx(row, col)];
    V[e] = v;
    fro += v.r * v.r + v.i * v.i;
  }
  fro = wave_sum(fro);
  if (lane == 0) red[4 + wave] = fro;
  __syncthreads();
  // residual columns at or below this squared norm count as exact zeros
  const double thr2 = QR_RANK_TOL * QR_RANK_TOL * (red[4] + red[5] + red[6] + red[7]);
  for (int j = 0; j < k; ++j) {
    // xnorm of V[j+1:m, j]
    double s = 0;
    for (int i = j + 1 + tid; i < m; i += 256) {
      z2 v = V[(long)j * m + i];
      s += v.r * v.r + v.i * v.i;
    }
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      const double xn2 = red[0] + red[1] + red[2] + red[3];
      const z2 alpha = V[(long)j * m + j];
      if (alpha.r * alpha.r + alpha.i * alpha.i + xn2 <= thr2) {
        sh_skip = 2;  // numerically zero residual: identity reflector, zero column
        tau[j] = z2{0, 0};
      } else if (xn2 == 0.0 && alpha.i == 0.0) {
        sh_skip = 1;
        tau[j] = z2{0, 0};
        sh_tau[0] = 0;
        sh_tau[1] = 0;
      } else {
        const double nrm = sqrt(alpha.r * alpha.r + alpha.i * alpha.i + xn2);
        // beta = -sign(Re alpha) * nrm (LAPACK zlarfg; a zero counts as positive)
        const double beta = alpha.r >= 0.0 ? -nrm : nrm;
        const z2 t{(beta - alpha.r) / beta, -alpha.i / beta};
        tau[j] = t;
        sh_tau[0] = t.r;
        sh_tau[1] = t.i;
        // scale = 1 / (alpha - beta)
        const double dr = alpha.r - beta, di = alpha.i;
        const double den = dr * dr + di * di;
        sh_scale[0] = dr / den;
        sh_scale[1] = -di / den;
        sh_beta[0] = beta;
        sh_skip = 0;
      }
    }
    __syncthreads();
    if (sh_skip == 2) {
      for (int i = j + tid; i < m; i += 256) V[(long)j * m + i] = z2{0, 0};
    }
    if (!sh_skip) {
      const z2 sc{sh_scale[0], sh_scale[1]};
      for (int i = j + 1 + tid; i < m; i += 256) V[(long)j * m + i] = zmul(V[(long)j * m + i], sc);
      if (tid == 0) V[(long)j * m + j] = z2{sh_beta[0], 0.0};
      __syncthreads();
      // apply H^H = I - conj(tau) v v^H to columns j+1..n-1
      const z2 ct{sh_tau[0], -sh_tau[1]};
      for (int col = j + 1 + wave; col < n; col += 4) {
        double wr = 0, wi = 0;
        for (int i = j + lane; i < m; i += 64) {
          const z2 v = i == j ? z2{1.0, 0.0} : V[(long)j * m + i];
          const z2 a = V[(long)col * m + i];
          const z2 p = zconjmul(v, a);
          wr += p.r;
          wi += p.i;
        }
        wr = wave_sum(wr);
        wi = wave_sum(wi);
        const z2 fct = zmul(ct, z2{wr, wi});
        for (int i = j + lane; i < m; i += 64) {
          const z2 v = i == j ? z2{1.0, 0.0} : V[(long)j * m + i];
          const z2 pv = zmul(fct, v);
          V[(long)col * m + i].r -= pv.r;
          V[(long)col * m + i].i -= pv.i;
        }
      }
    }
    __syncthreads();
  }
  // R (n x n upper; rows >= k zero) into op.R, before Q overwrites V
  z2* R = reinterpret_cast<z2*>(op.R);
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, col = e % n;
    z2 v = (i <= col && i < k) ? V[(long)col * m + i] : z2{0, 0};
    if (op.transposeR) R[(long)col * n + i] = v;
    else R[(long)i * n + col] = v;
  }
  __syncthreads();
  // Q = H_0 ... H_{k-1} applied to the first min(m,n) unit columns (zung2r)
  const int nq = k;  // Q is m x k
  for (int i = k - 1; i >= 0; --i) {
    const z2 t = tau[i];
    if (i < nq - 1) {
      for (int col = i + 1 + wave; col < nq; col += 4) {
        double wr = 0, wi = 0;
        for (int r = i + lane; r < m; r += 64) {
          const z2 v = r == i ? z2{1.0, 0.0} : V[(long)i * m + r];
          const z2 p = zconjmul(v, V[(long)col * m + r]);
          wr += p.r;
          wi += p.i;
        }
        wr = wave_sum(wr);
        wi = wave_sum(wi);
        const z2 fct = zmul(t, z2{wr, wi});
        for (int r = i + lane; r < m; r += 64) {
          const z2 v = r == i ? z2{1.0, 0.0} : V[(long)i * m + r];
          const z2 pv = zmul(fct, v);
          V[(long)col * m + r].r -= pv.r;
          V[(long)col * m + r].i -= pv.i;
        }
      }
    }
    __syncthreads();
    for (int r = i + 1 + tid; r < m; r += 256) {
      const z2 v = V[(long)i * m + r];
      const z2 p = zmul(t, v);
      V[(long)i * m + r] = z2{-p.r, -p.i};
    }
    if (tid == 0) V[(long)i * m + i] = z2{1.0 - t.r, -t.i};
    for (int r = tid; r < i; r += 256) V[(long)i * m + r] = z2{0, 0};
    __syncthreads();
  }
  // phases: make diag(R) real non-negative
  __shared__ double ph[2 * 64];
  if (tid < n) {
    const int j = tid;
    z2 d = op.transposeR ? R[(long)j * n + j] : R[(long)j * n + j];
    const double a = sqrt(d.r * d.r + d.i * d.i);
    ph[2 * j] = a > 0 ? d.r / a : 1.0;
    ph[2 * j + 1] = a > 0 ? d.i / a : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, col = e % n;
    const z2 cph{ph[2 * i], -ph[2 * i + 1]};
    const long o = op.transposeR ? (long)col * n + i : (long)i * n + col;
    R[o] = zmul(cph, R[o]);
  }
  for (long e = tid; e < (long)m * n; e += 256) {
    const int row = e % m, col = e / m;
    z2 q = col < nq ? zmul(V[(long)col * m + row], z2{ph[2 * col], ph[2 * col + 1]}) : z2{0, 0};
    C[cidx(row, col)] = q;
  }
}

// ---------------------------------------------------------------------------
// absorb: C[pre, a, post] <- sum_a' Mx[a, a'] C[pre, a', post]   (FP64)
// ---------------------------------------------------------------------------
struct AbsorbTile {
  int op;
  int f0, f1;  // fiber range (fiber = (pre, post))
};

__global__ void __launch_bounds__(256) k_absorb(const AbsorbOp* __restrict__ ops,
                                                const AbsorbTile* __restrict__ tiles) {
  const AbsorbTile tl = tiles[blockIdx.x];
  const AbsorbOp op = ops[tl.op];
  extern __shared__ char smem_raw[];
  z2* buf = reinterpret_cast<z2*>(smem_raw);
  z2* C = reinterpret_cast<z2*>(op.C);
  const z2* M = reinterpret_cast<const z2*>(op.M);
  const int n = op.n;
  const int nf = tl.f1 - tl.f0;
  auto off = [&](int fib, int a) -> long {
    const int pre = fib / op.Ppost, post = fib % op.Ppost;
    return (long)pre * n * op.Ppost + (long)a * op.Ppost + post;
  };
  for (int e = threadIdx.x; e < nf * n; e += blockDim.x) {
    const int fl = e / n, a = e % n;
    buf[e] = C[off(tl.f0 + fl, a)];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nf * n; e += blockDim.x) {
    const int fl = e / n, a = e % n;
    double sr = 0, si = 0;
    for (int b = 0; b < n; ++b) {
      const z2 mv = op.transposeM ? M[(long)b * n + a] : M[(long)a * n + b];
      const z2 x = buf[fl * n + b];
      sr += mv.r * x.r - mv.i * x.i;
      si += mv.r * x.i + mv.i * x.r;
    }
    C[off(tl.f0 + fl, a)] = z2{sr, si};
  }
}

// ---------------------------------------------------------------------------
// gram: E[a', a] = sum_k conj(C[pre, a', post]) T[pre, a, post],  k = (pre, post)
// ---------------------------------------------------------------------------
// One workgroup per environment matrix.  Work items = (16x16 output tile,
// K part); with fewer than four tiles K is split across wavefronts and the
// partial tiles are summed in LDS.
template <typename T>
__global__ void __launch_bounds__(256) k_gram(const GramOp* __restrict__ ops) {
  typedef typename MT<T>::v4 v4;
  const GramOp op = ops[blockIdx.x];
  const int r = op.r;
  const long K = (long)op.Ppre * op.Ppost;
  const T* Tm = reinterpret_cast<const T*>(op.T);
  T* E = reinterpret_cast<T*>(op.E);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int nb = (r + 15) >> 4, nt = nb * nb;
  const int kparts = nt >= 4 ? 1 : 4 / nt;
  const int n_items = nt * kparts;
  const long kchunk = (K + kparts - 1) / kparts;
  __shared__ T red[2][4][256];
  v4 accr[4], acci[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    accr[j] = v4{0, 0, 0, 0};
    acci[j] = v4{0, 0, 0, 0};
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int item = wave + 4 * j;
    if (item < n_items) {
      const int tile = item % nt, kp = item / nt;
      const int ti = tile / nb, tj = tile % nb;
      const int arow = 16 * ti + c, bcol = 16 * tj + c;
      const long k0 = kp * kchunk, k1 = k0 + kchunk < K ? k0 + kchunk : K;
      for (long kb = k0; kb < k1; kb += 4) {
        const long k = kb + g;
        T ar = 0, ai = 0, br = 0, bi = 0;
        if (k < k1) {
          const long pre = k / op.Ppost, post = k % op.Ppost;
          const long base = pre * r * op.Ppost + post;
          if (arow < r) {
            const long o = base + (long)arow * op.Ppost;
            ar = (T)op.C[2 * o];
            ai = -(T)op.C[2 * o + 1];  // conj(C)
          }
          if (bcol < r) {
            const long o = base + (long)bcol * op.Ppost;
            br = Tm[2 * o];
            bi = Tm[2 * o + 1];
          }
        }
        cmma<T>(accr[j], acci[j], ar, ai, br, bi);
      }
    }
  }
  if (kparts == 1) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int item = wave + 4 * j;
      if (item < n_items) {
        const int ti = item / nb, tj = item % nb;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = 16 * ti + MT<T>::drow(g, q), col = 16 * tj + c;
          if (row < r && col < r) {
            E[2 * ((long)row * r + col)] = accr[j][q];
            E[2 * ((long)row * r + col) + 1] = acci[j][q];
          }
        }
      }
    }
    return;
  }
  // nt < 4: each wave holds one partial of some tile in accr[0]
  const int item = wave;
  const int tile = item % nt, kp = item / nt;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    red[0][wave][MT<T>::drow(g, q) * 16 + c] = accr[0][q];
    red[1][wave][MT<T>::drow(g, q) * 16 + c] = acci[0][q];
  }
  __syncthreads();
  (void)tile;
  (void)kp;
  for (int e = threadIdx.x; e < nt * 256; e += 256) {
    const int t = e / 256, w = e % 256;
    T sr = 0, si = 0;
    for (int p = 0; p < kparts; ++p) {
      sr += red[0][t + p * nt][w];
      si += red[1][t + p * nt][w];
    }
    const int ti = t / nb, tj = t % nb;
    const int row = 16 * ti + w / 16, col = 16 * tj + w % 16;
    if (row < r && col < r) {
      E[2 * ((long)row * r + col)] = sr;
      E[2 * ((long)row * r + col) + 1] = si;
    }
  }
}

// ---------------------------------------------------------------------------
// rho: bottom-up vacuum contraction, FP64, one workgroup per program
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rho(const RhoProg* __restrict__ progs) {
  const RhoProg P = progs[blockIdx.x];
  for (int ni = 0; ni < P.n_nodes; ++ni) {
    const RhoNode nd = P.nodes[ni];
    // output index space: parent leg (dim r) or the two system ends (M*M)
    int out_dims[2] = {1, 1}, out_legs[2] = {-1, -1}, n_out = 0;
    int strides[8];
    long st = 1;
    for (int l = nd.n_legs - 1; l >= 0; --l) {
      strides[l] = (int)st;
      st *= nd.dims[l];
    }
    for (int l = 0; l < nd.n_legs; ++l)
      if (nd.kind[l] == 0 || nd.kind[l] == 2) {
        out_legs[n_out] = l;
        out_dims[n_out] = nd.dims[l];
        ++n_out;
      }
    // summed legs: child bonds
    int sum_legs[8], n_sum = 0;
    long n_terms = 1;
    for (int l = 0; l < nd.n_legs; ++l)
      if (nd.kind[l] == 3) {
        sum_legs[n_sum++] = l;
        n_terms *= nd.dims[l];
      }
    const int n_outv = out_dims[0] * out_dims[1];
    for (int o = threadIdx.x; o < n_outv; o += blockDim.x) {
      long base = 0;
      if (n_out > 0) base += (long)(o / out_dims[1]) * strides[out_legs[0]];
      if (n_out > 1) base += (long)(o % out_dims[1]) * strides[out_legs[1]];
      double sr = 0, si = 0;
      for (long t = 0; t < n_terms; ++t) {
        long rem = t, off = base;
        double wr = 1, wi = 0;
        for (int s = n_sum - 1; s >= 0; --s) {
          const int l = sum_legs[s];
          const int b = rem % nd.dims[l];
          rem /= nd.dims[l];
          off += (long)b * strides[l];
          const double* v = P.vecs + 2 * ((long)nd.child_slot[l] * P.vec_ld + b);
          const double nr = wr * v[0] - wi * v[1], nim = wr * v[1] + wi * v[0];
          wr = nr;
          wi = nim;
        }
        const double cr = nd.C[2 * off], ci = nd.C[2 * off + 1];
        sr += cr * wr - ci * wi;
        si += cr * wi + ci * wr;
      }
      double* dst = nd.out_slot >= 0 ? P.vecs + 2 * ((long)nd.out_slot * P.vec_ld + o)
                                     : P.rho_out + 2 * o;
      dst[0] = sr;
      dst[1] = si;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// ps2: merge, Gram eigen-decomposition, split (FP64, single workgroup)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_merge(const MergeOp* __restrict__ ops) {
  const MergeOp op = ops[blockIdx.y];
  const z2* S = reinterpret_cast<const z2*>(op.Cs);
  const z2* Cc = reinterpret_cast<const z2*>(op.Cc);
  z2* Th = reinterpret_cast<z2*>(op.Theta);
  const long n = (long)op.rows * op.cols;
  for (long e = blockIdx.x * 256L + threadIdx.x; e < n; e += 256L * gridDim.x) {
    const int row = (int)(e / op.cols), col = (int)(e % op.cols);
    const int pre = row / op.Ppost, post = row % op.Ppost;
    double sr = 0, si = 0;
    for (int a = 0; a < op.r; ++a) {
      const z2 x = S[(long)pre * op.r * op.Ppost + (long)a * op.Ppost + post];
      const z2 y = Cc[(long)a * op.cols + col];
      sr += x.r * y.r - x.i * y.i;
      si += x.r * y.i + x.i * y.r;
    }
    Th[e] = z2{sr, si};
  }
}

// Cyclic Jacobi on the n x n Hermitian Gram matrix held in LDS (n <= 64),
// parallel rounds of the circle-method pairing.
__global__ void __launch_bounds__(256) k_eig(const EigOp* __restrict__ ops) {
  const EigOp op = ops[blockIdx.x];
  const int n = op.side == 0 ? op.rows : op.cols;
  const int m = op.side == 0 ? op.cols : op.rows;
  const z2* Th = reinterpret_cast<const z2*>(op.Theta);
  __shared__ z2 G[64 * 64];
  __shared__ z2 U[64 * 64];
  __shared__ double rot[32][4];  // c, s, cos(phi), sin(phi)
  __shared__ int pr[32][2];
  __shared__ double offmax, diagmax;
  const int tid = threadIdx.x;
  // Gram: side 0: G[i][j] = sum_c Th[i][c] conj(Th[j][c]); side 1: sum_r conj(Th[r][i]) Th[r][j]
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    double sr = 0, si = 0;
    for (int q = 0; q < m; ++q) {
      z2 x, y;
      if (op.side == 0) {
        x = Th[(long)i * op.cols + q];
        y = Th[(long)j * op.cols + q];
        sr += x.r * y.r + x.i * y.i;  // x * conj(y)
        si += x.i * y.r - x.r * y.i;
      } else {
        x = Th[(long)q * op.cols + i];
        y = Th[(long)q * op.cols + j];
        sr += x.r * y.r + x.i * y.i;  // conj(x) * y
        si += x.r * y.i - x.i * y.r;
      }
    }
    G[i * 64 + j] = z2{sr, si};
    U[i * 64 + j] = z2{i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int np = (n + 1) / 2;            // pairs per round (a dummy player when n is odd)
  const int nplay = 2 * np;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) {
      double om = 0, dm = 0;
      for (int i = 0; i < n; ++i) {
        dm = fmax(dm, fabs(G[i * 64 + i].r));
        for (int j = i + 1; j < n; ++j) {
          const z2 g = G[i * 64 + j];
          om = fmax(om, sqrt(g.r * g.r + g.i * g.i));
        }
      }
      offmax = om;
      diagmax = dm;
    }
    __syncthreads();
    if (offmax <= 1e-15 * diagmax || offmax == 0.0) break;
    for (int round = 0; round < nplay - 1; ++round) {
      if (tid < np) {
        int p, q;
        if (tid == 0) {
          p = round;
          q = nplay - 1;
        } else {
          p = (round + tid) % (nplay - 1);
          q = (round - tid + (nplay - 1)) % (nplay - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        pr[tid][0] = p;
        pr[tid][1] = q;
        double c = 1, sn = 0, cph = 1, sph = 0;
        if (q < n) {
          const z2 g = G[p * 64 + q];
          const double h = sqrt(g.r * g.r + g.i * g.i);
          if (h > 1e-300) {
            const double a = G[p * 64 + p].r, b = G[q * 64 + q].r;
            const double zeta = (b - a) / (2.0 * h);
            const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            cph = g.r / h;
            sph = g.i / h;
          }
        }
        rot[tid][0] = c;
        rot[tid][1] = sn;
        rot[tid][2] = cph;
        rot[tid][3] = sph;
      }
      __syncthreads();
      // columns: G <- G J and U <- U J, J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]]
      for (int e = tid; e < np * n; e += 256) {
        const int k = e / n, row = e % n;
        const int p = pr[k][0], q = pr[k][1];
        if (q >= n) continue;
        const double c = rot[k][0], sn = rot[k][1], cph = rot[k][2], sph = rot[k][3];
        const z2 emi{cph, -sph};  // e^{-i phi}
        for (int w = 0; w < 2; ++w) {
          z2* A = w == 0 ? G : U;
          const z2 xp = A[row * 64 + p], xq = A[row * 64 + q];
          const z2 xq_e = zmul(xq, emi);
          A[row * 64 + p] = z2{c * xp.r - sn * xq_e.r, c * xp.i - sn * xq_e.i};
          A[row * 64 + q] = z2{sn * xp.r + c * xq_e.r, sn * xp.i + c * xq_e.i};
        }
      }
      __syncthreads();
      // rows: G <- J^H G
      for (int e = tid; e < np * n; e += 256) {
        const int k = e / n, col = e % n;
        const int p = pr[k][0], q = pr[k][1];
        if (q >= n) continue;
        const double c = rot[k][0], sn = rot[k][1], cph = rot[k][2], sph = rot[k][3];
        const z2 epi{cph, sph};  // e^{i phi}
        const z2 xp = G[p * 64 + col], xq = G[q * 64 + col];
        const z2 xq_e = zmul(xq, epi);
        G[p * 64 + col] = z2{c * xp.r - sn * xq_e.r, c * xp.i - sn * xq_e.i};
        G[q * 64 + col] = z2{sn * xp.r + c * xq_e.r, sn * xp.i + c * xq_e.i};
      }
      __syncthreads();
    }
  }
  // descending order: rank of each eigenvalue (ties by index)
  for (int j = tid; j < n; j += 256) {
    const double lj = G[j * 64 + j].r;
    int rank = 0;
    for (int i = 0; i < n; ++i) {
      const double li = G[i * 64 + i].r;
      if (li > lj || (li == lj && i < j)) ++rank;
    }
    op.evals[rank] = lj;
    for (int row = 0; row < n; ++row) {
      const z2 v = U[row * 64 + j];
      op.evecs[2 * ((long)row * n + rank)] = v.r;
      op.evecs[2 * ((long)row * n + rank) + 1] = v.i;
    }
  }
}

__global__ void __launch_bounds__(256) k_split(const SplitOp* __restrict__ ops) {
  const SplitOp op = ops[blockIdx.x];
  const z2* Th = reinterpret_cast<const z2*>(op.Theta);
  const z2* E = reinterpret_cast<const z2*>(op.evecs);
  z2* W = reinterpret_cast<z2*>(op.W);
  const int n = op.side == 0 ? op.rows : op.cols;       // spectral side
  const int miso = op.iso == 0 ? op.rows : op.cols;     // isometry side
  const int k = op.k, rp = op.rp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[2][4];
  __shared__ double sh_norm;
  // first k columns of W: spectral vectors on the isometry side
  for (long e = tid; e < (long)miso * k; e += 256) {
    const int i = (int)(e / k), j = (int)(e % k);
    z2 v;
    if (op.side == op.iso) {
      v = E[(long)i * n + j];
    } else {
      // map through Theta: other side vector = Theta^(H) u_j / sigma_j
      const double sig = sqrt(fmax(op.evals[j], 0.0));
      double sr = 0, si = 0;
      if (op.iso == 1) {  // spectral on rows: w_j = Theta^H u_j / s_j (cols)
        for (int r = 0; r < op.rows; ++r) {
          const z2 t = Th[(long)r * op.cols + i];
          const z2 u = E[(long)r * n + j];
          sr += t.r * u.r + t.i * u.i;  // conj(t) * u
          si += t.r * u.i - t.i * u.r;
        }
      } else {  // spectral on cols: w_j = Theta v_j / s_j (rows)
        for (int c = 0; c < op.cols; ++c) {
          const z2 t = Th[(long)i * op.cols + c];
          const z2 u = E[(long)c * n + j];
          sr += t.r * u.r - t.i * u.i;
          si += t.r * u.i + t.i * u.r;
        }
      }
      v = z2{sr / sig, si / sig};
    }
    W[(long)i * rp + j] = v;
  }
  __syncthreads();
  // re-orthonormalise the mapped columns (only needed when mapped through Theta)
  if (op.side != op.iso) {
    for (int j = 0; j < k; ++j) {
      for (int pass = 0; pass < 2; ++pass) {
        for (int q = 0; q < j; ++q) {
          double dr = 0, di = 0;
          for (int i = lane; i < miso; i += 64) {
            const z2 a = W[(long)i * rp + q], b = W[(long)i * rp + j];
            dr += a.r * b.r + a.i * b.i;
            di += a.r * b.i - a.i * b.r;
          }
          dr = wave_sum(dr);
          di = wave_sum(di);
          __syncthreads();
          if (wave == 0)
            for (int i = lane; i < miso; i += 64) {
              const z2 a = W[(long)i * rp + q];
              W[(long)i * rp + j].r -= a.r * dr - a.i * di;
              W[(long)i * rp + j].i -= a.r * di + a.i * dr;
            }
          __syncthreads();
        }
      }
      double s2 = 0;
      for (int i = tid; i < miso; i += 256) {
        const z2 b = W[(long)i * rp + j];
        s2 += b.r * b.r + b.i * b.i;
      }
      s2 = wave_sum(s2);
      if (lane == 0) red[0][wave] = s2;
      __syncthreads();
      if (tid == 0) sh_norm = sqrt(red[0][0] + red[0][1] + red[0][2] + red[0][3]);
      __syncthreads();
      for (int i = tid; i < miso; i += 256) {
        W[(long)i * rp + j].r /= sh_norm;
        W[(long)i * rp + j].i /= sh_norm;
      }
      __syncthreads();
    }
  }
  // completion: unit vectors e_0, e_1, ... projected out of span(W[:, :j]),
  // twice, accepted when the residual norm exceeds 0.5
  int j = k;
  for (int cand = 0; cand < miso && j < rp; ++cand) {
    for (int i = tid; i < miso; i += 256) W[(long)i * rp + j] = z2{i == cand ? 1.0 : 0.0, 0.0};
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < j; ++q) {
        double dr = 0, di = 0;
        for (int i = lane; i < miso; i += 64) {
          const z2 a = W[(long)i * rp + q], b = W[(long)i * rp + j];
          dr += a.r * b.r + a.i * b.i;
          di += a.r * b.i - a.i * b.r;
        }
        dr = wave_sum(dr);
        di = wave_sum(di);
        __syncthreads();
        if (wave == 0)
          for (int i = lane; i < miso; i += 64) {
            const z2 a = W[(long)i * rp + q];
            W[(long)i * rp + j].r -= a.r * dr - a.i * di;
            W[(long)i * rp + j].i -= a.r * di + a.i * dr;
          }
        __syncthreads();
      }
    }
    double s2 = 0;
    for (int i = tid; i < miso; i += 256) {
      const z2 b = W[(long)i * rp + j];
      s2 += b.r * b.r + b.i * b.i;
    }
    s2 = wave_sum(s2);
    if (lane == 0) red[1][wave] = s2;
    __syncthreads();
    if (tid == 0) sh_norm = sqrt(red[1][0] + red[1][1] + red[1][2] + red[1][3]);
    __syncthreads();
    if (sh_norm > 0.5) {
      for (int i = tid; i < miso; i += 256) {
        W[(long)i * rp + j].r /= sh_norm;
        W[(long)i * rp + j].i /= sh_norm;
      }
      ++j;
    }
    __syncthreads();
  }
  // new cores
  z2* Cs = reinterpret_cast<z2*>(op.Cs);
  z2* Cc = reinterpret_cast<z2*>(op.Cc);
  auto cs_at = [&](int row, int a) -> long {
    const int pre = row / op.Ppost_s, post = row % op.Ppost_s;
    return (long)pre * rp * op.Ppost_s + (long)a * op.Ppost_s + post;
  };
  if (op.iso == 0) {
    for (long e = tid; e < (long)op.rows * rp; e += 256) {
      const int row = (int)(e / rp), a = (int)(e % rp);
      Cs[cs_at(row, a)] = W[(long)row * rp + a];
    }
    for (long e = tid; e < (long)rp * op.cols; e += 256) {  // Cc = W^H Theta
      const int a = (int)(e / op.cols), col = (int)(e % op.cols);
      double sr = 0, si = 0;
      for (int row = 0; row < op.rows; ++row) {
        const z2 w = W[(long)row * rp + a], t = Th[(long)row * op.cols + col];
        sr += w.r * t.r + w.i * t.i;
        si += w.r * t.i - w.i * t.r;
      }
      Cc[e] = z2{sr, si};
    }
  } else {
    for (long e = tid; e < (long)rp * op.cols; e += 256) {  // Cc = W^H
      const int a = (int)(e / op.cols), col = (int)(e % op.cols);
      const z2 w = W[(long)col * rp + a];
      Cc[e] = z2{w.r, -w.i};
    }
    for (long e = tid; e < (long)op.rows * rp; e += 256) {  // Cs = Theta W
      const int row = (int)(e / rp), a = (int)(e % rp);
      double sr = 0, si = 0;
      for (int col = 0; col < op.cols; ++col) {
        const z2 t = Th[(long)row * op.cols + col], w = W[(long)col * rp + a];
        sr += t.r * w.r - t.i * w.i;
        si += t.r * w.i + t.i * w.r;
      }
      Cs[cs_at(row, a)] = z2{sr, si};
    }
  }
}

__global__ void k_step_inc(int* ctr, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = value < 0 ? *ctr + 1 : value;
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
size_t apply_lds_bytes(int fp64, int nfl, int d1, int d2, int with_ab) {
  return (size_t)apply_lds_elems(nfl, d1, d2, with_ab) * (fp64 ? sizeof(double) : sizeof(float));
}

hipError_t launch_apply(int fp64, int in_fp64, const ApplyGroup* groups, const ApplyTile* tiles,
                        int n_tiles, const int* step_ctr, size_t lds, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    const int cap = 160 * 1024;
    (void)hipFuncSetAttribute((const void*)k_apply<float, float>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void*)k_apply<float, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void*)k_apply<double, double>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    attr_set = true;
  }
  if (fp64) {
    if (in_fp64)
      hipLaunchKernelGGL((k_apply<double, double>), dim3(n_tiles), dim3(256), lds, s, groups, tiles, step_ctr);
    else
      hipLaunchKernelGGL((k_apply<double, double>), dim3(n_tiles), dim3(256), lds, s, groups, tiles, step_ctr);
  } else {
    if (in_fp64)
      hipLaunchKernelGGL((k_apply<float, double>), dim3(n_tiles), dim3(256), lds, s, groups, tiles, step_ctr);
    else
      hipLaunchKernelGGL((k_apply<float, float>), dim3(n_tiles), dim3(256), lds, s, groups, tiles, step_ctr);
  }
  return hipGetLastError();
}

hipError_t launch_presum(int fp64, const PresumOp* ops, int n, const int* step_ctr, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp64) hipLaunchKernelGGL(k_presum<double>, dim3(n), dim3(256), 0, s, ops, step_ctr);
  else hipLaunchKernelGGL(k_presum<float>, dim3(n), dim3(256), 0, s, ops, step_ctr);
  return hipGetLastError();
}

hipError_t launch_combine(int fp64, const CombineOp* ops, const void* tiles, int n_tiles,
                          hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  const CombineTile* t = reinterpret_cast<const CombineTile*>(tiles);
  if (fp64) hipLaunchKernelGGL(k_combine<double>, dim3(n_tiles), dim3(256), 0, s, ops, t);
  else hipLaunchKernelGGL(k_combine<float>, dim3(n_tiles), dim3(256), 0, s, ops, t);
  return hipGetLastError();
}

hipError_t launch_qr(const QrOp* ops, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_qr, dim3(n), dim3(256), 0, s, ops);
  return hipGetLastError();
}

hipError_t launch_absorb(const AbsorbOp* ops, const void* tiles, int n_tiles, size_t lds,
                         hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_absorb, dim3(n_tiles), dim3(256), lds, s, ops,
                     reinterpret_cast<const AbsorbTile*>(tiles));
  return hipGetLastError();
}

hipError_t launch_gram(int fp64, const GramOp* ops, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp64) hipLaunchKernelGGL(k_gram<double>, dim3(n), dim3(256), 0, s, ops);
  else hipLaunchKernelGGL(k_gram<float>, dim3(n), dim3(256), 0, s, ops);
  return hipGetLastError();
}

hipError_t launch_rho(const RhoProg* progs, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rho, dim3(n), dim3(256), 0, s, progs);
  return hipGetLastError();
}

hipError_t launch_step_inc(int* ctr, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(64), 0, s, ctr, value);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeOp* op, long n, hipStream_t s) {
  int blocks = (int)std::min<long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_merge, dim3(blocks, 1), dim3(256), 0, s, op);
  return hipGetLastError();
}
hipError_t launch_eig(const EigOp* op, hipStream_t s) {
  hipLaunchKernelGGL(k_eig, dim3(1), dim3(256), 0, s, op);
  return hipGetLastError();
}
hipError_t launch_split(const SplitOp* op, hipStream_t s) {
  hipLaunchKernelGGL(k_split, dim3(1), dim3(256), 0, s, op);
  return hipGetLastError();
}

size_t combine_tile_bytes() { return sizeof(CombineTile); }
size_t absorb_tile_bytes() { return sizeof(AbsorbTile); }

}  // namespace tenso
