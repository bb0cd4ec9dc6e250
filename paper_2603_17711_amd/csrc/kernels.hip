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
#include <hip/hip_ext.h>
#include <math.h>
#include <algorithm>
#include <type_traits>
#include <utility>
#include "tenso_internal.h"

namespace tenso {

// Pointers read from op descriptors in memory are generic: the compiler would
// access them with FLAT instructions, whose completion is counted together
// with LDS traffic, so every wait for an LDS result would also wait for all
// outstanding HBM loads.  Every such pointer refers to device global memory;
// gmem() gives it the global address space, and accesses through it become
// global loads/stores.
// (The host compilation pass, which only parses device code, sees plain
// pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define TENSO_GLOBAL __attribute__((address_space(1)))
#else
#define TENSO_GLOBAL
#endif
template <class T>
using gp = TENSO_GLOBAL T*;
template <class T>
__device__ inline gp<T> gmem(T* p) {
  return (gp<T>)p;
}
template <class T>
__device__ inline gp<const T> gmem(const T* p) {
  return (gp<const T>)p;
}

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct MT;
template <> struct MT<float> {
  typedef v4f v4;
  static constexpr int NT = kApplyAccTiles;  // accumulator tiles per wavefront
  __device__ static inline v4 mma(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of accumulator register r in lane group g (measured on gfx950)
  __device__ static inline int drow(int g, int r) { return 4 * g + r; }
};
template <> struct MT<double> {
  typedef v4d v4;
  static constexpr int NT = kApplyAccTiles;
  __device__ static inline v4 mma(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // the FP64 variant interleaves rows across lane groups (measured on gfx950)
  __device__ static inline int drow(int g, int r) { return g + 4 * r; }
};

template <typename T> struct cpx { T re, im; };

template <typename Tin, typename T>
__device__ inline cpx<T> ldc(const void* base, long idx) {
  const gp<const Tin> p = gmem(reinterpret_cast<const Tin*>(base)) + 2 * idx;
  return cpx<T>{(T)p[0], (T)p[1]};
}

// Input kind of an RK4 stage whose update is formed while the input is
// staged (in_fp64 = 2): (T)(y0 + xp_s * k), k the previous stage's partial
// outputs summed in order, in FP64, as the stage-combine kernel sums them.
struct StageIn {};

template <typename Tin, typename T>
__device__ inline cpx<T> ld_input(const ApplyGroup& G, long idx) {
  if constexpr (std::is_same<Tin, StageIn>::value) {
    const gp<const double> y = gmem(reinterpret_cast<const double*>(G.X)) + 2 * idx;
    const gp<const T> pp = gmem(reinterpret_cast<const T*>(G.xp)) + 2 * idx;
    double kr = 0, ki = 0;
    for (int p = 0; p < G.xp_np; ++p) {
      kr += (double)pp[2 * (long)p * G.xp_n];
      ki += (double)pp[2 * (long)p * G.xp_n + 1];
    }
    return cpx<T>{(T)(y[0] + G.xp_s * kr), (T)(y[1] + G.xp_s * ki)};
  } else {
    return ldc<Tin, T>(G.X, idx);
  }
}

__device__ inline void coef_at(const TermRef& t, const double* drive, int ld, int j,
                               double& cr, double& ci) {
  cr = t.cre;
  ci = t.cim;
  if (t.slot >= 0 && drive) {
    double f = gmem(drive)[(long)t.slot * ld + j];
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

// Compile-time loop: f(std::integral_constant<int, I>) for I = 0 .. N - 1, so
// that register arrays indexed by I are addressed statically.
template <typename F, int... I>
__device__ __forceinline__ void static_for_(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_(f, std::make_integer_sequence<int, N>{});
}

// LDS layout of one apply tile (T elements; complex values interleaved):
//   X : nfl x D1 x (D2 + 1)     the tile's input slices X_f, zero padded
//   A : 2 x D1 x (D1 + 1)       coefficient-scaled operand, two buffers: term m
//   B : 2 x D2 x (D2 + 1)       is read from one while term m + 1 is written
//                               to the other
//   Z : 4 wavefronts x D1 x 16  per-wave X_f B^T of one unit
// with D = 16 * ceil(d / 16).  Every MFMA operand is then one LDS vector load
// without bounds checks.
// Row stride of a wavefront's X_f B^T slab in LDS (padded: rows 4 apart map
// to different banks).
constexpr int ZS1 = 17;

__host__ __device__ inline long apply_lds_elems(int nfl, int d1, int d2) {
  const long D1 = 16 * ((d1 + 15) / 16), D2 = 16 * ((d2 + 15) / 16);
  return 2 * (nfl * D1 * (D2 + 1) + 2 * (D1 * (D1 + 1) + D2 * (D2 + 1)) +
              kApplyWaves * D1 * ZS1);
}

template <typename T> struct V2;
template <> struct V2<float> { typedef float2 t; };
template <> struct V2<double> { typedef double2 t; };

// Rounding of an FP32 value to the nearest BF16 value (ties to even), kept in
// FP32: products of two such values are exact in FP32, so an FP32 MFMA on
// them gives the products of a BF16 MFMA with FP32 accumulation.
__device__ inline float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}
__device__ inline double bf16_round(double x) { return x; }

// K loop of one unit product, acc[TLO + t] += Aop_t Bop over nq k-steps of 4:
// lane (c, g) reads Aop_t[c][k] at ar[t * ars16 + k] (ar already offset to
// row c) and Bop[k][col] at bc[k * bks] (bc offset to the lane's column),
// k = 4 q + g.  Operands of k-step q + 1 are read from LDS into the second
// register set while the MFMAs of step q run (two sets used in turn, so no
// register copies between steps).  NIB and TLO are compile-time so that every
// register array is indexed statically.
// With M3 the complex product takes three real products (Gauss): accr
// collects Re a Re b, accx Im a Im b and acci (Re a + Im a)(Re b + Im b); the
// product is Re = accr - accx, Im = acci - accr - accx (m3_re, m3_im).
template <typename T, int NIB, int TLO, int NA, bool M3, typename C2>
__device__ __forceinline__ void mma_loop(typename MT<T>::v4 (&accr)[NA],
                                         typename MT<T>::v4 (&acci)[NA],
                                         typename MT<T>::v4 (&accx)[NA], const C2* ar, int ars16,
                                         const C2* bc, int bks, int nq, int g) {
  C2 b0, b1, a0[NIB], a1[NIB];
  auto ld = [&](int q, C2& b, C2(&a)[NIB]) {
    const int kk = 4 * q + g;
    b = bc[kk * bks];
#pragma unroll
    for (int t = 0; t < NIB; ++t) a[t] = ar[t * ars16 + kk];
  };
  auto mm = [&](const C2& b, const C2(&a)[NIB]) {
    if constexpr (M3) {
      const T bs = b.x + b.y;
#pragma unroll
      for (int t = 0; t < NIB; ++t) {
        accr[TLO + t] = MT<T>::mma(a[t].x, b.x, accr[TLO + t]);
        accx[TLO + t] = MT<T>::mma(a[t].y, b.y, accx[TLO + t]);
        acci[TLO + t] = MT<T>::mma(a[t].x + a[t].y, bs, acci[TLO + t]);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NIB; ++t) cmma<T>(accr[TLO + t], acci[TLO + t], a[t].x, a[t].y, b.x, b.y);
    }
  };
  // both products of an iteration are unconditional, so the accumulators
  // stay in place across iterations; an odd last step follows the loop
  ld(0, b0, a0);
  int q = 0;
  for (; q + 1 < nq; q += 2) {
    ld(q + 1, b1, a1);
    mm(b0, a0);
    if (q + 2 < nq) ld(q + 2, b0, a0);
    mm(b1, a1);
  }
  if (q < nq) mm(b0, a0);
}

// Operand staging: lanes over the columns of a row, 64 / D rows per
// wavefront pass for D = 16, 32, 64 (one row for D = 48, lanes 48..63 idle).
// For D <= 32 a thread holds at most kApplyPf entries (rows i0, i0 + step,
// ...); those are read from global memory one term ahead, while the current
// term is multiplied.
constexpr int kApplyPf = 4;

struct OpLane {
  int i0, step, j;
  bool on;
};
__device__ inline OpLane op_lane(int D, int lane, int wave) {
  const bool p2 = (D & (D - 1)) == 0;
  const int rpw = p2 ? 64 / D : 1;
  OpLane o;
  o.i0 = wave * rpw + (p2 ? lane / D : 0);
  o.step = kApplyWaves * rpw;
  o.j = p2 ? (lane & (D - 1)) : lane;
  o.on = o.j < D;
  return o;
}

template <typename T, typename C2>
__device__ __forceinline__ void op_fetch(const T* M, int d, int D, const OpLane& o,
                                         C2 (&r)[kApplyPf]) {
#pragma unroll
  for (int k = 0; k < kApplyPf; ++k) {
    const int i = o.i0 + k * o.step;
    C2 v;
    v.x = 0;
    v.y = 0;
    if (o.on && i < D && i < d && o.j < d) {
      const gp<const T> e = gmem(M) + 2 * (i * d + o.j);
      v.x = e[0];
      v.y = e[1];
    }
    r[k] = v;
  }
}

// entries scaled by the coefficient unless it is exactly 1 (in the compute
// precision: one rounding, as for the operand itself)
template <typename T, typename C2>
__device__ __forceinline__ C2 op_scale(C2 v, bool unit, T sr, T si) {
  if (!unit) {
    const T a0 = v.x, a1 = v.y;
    v.x = a0 * sr - a1 * si;
    v.y = a0 * si + a1 * sr;
  }
  return v;
}

template <typename T, bool RB, typename C2>
__device__ __forceinline__ C2 op_round(C2 v) {
  if constexpr (RB) {
    v.x = bf16_round(v.x);
    v.y = bf16_round(v.y);
  }
  return v;
}

template <typename T, bool RB, typename C2>
__device__ __forceinline__ void op_put(const C2 (&r)[kApplyPf], int D, int ld, const OpLane& o,
                                       C2* dst, double sr, double si) {
  if (!o.on) return;
  const bool unit = sr == 1.0 && si == 0.0;
#pragma unroll
  for (int k = 0; k < kApplyPf; ++k) {
    const int i = o.i0 + k * o.step;
    if (i < D) dst[i * ld + o.j] = op_round<T, RB>(op_scale<T>(r[k], unit, (T)sr, (T)si));
  }
}

// D > 32: read and written in one pass (no look-ahead)
template <typename T, bool RB, typename C2>
__device__ void op_stage(const T* M, int d, int D, int ld, const OpLane& o, C2* dst, double sr,
                         double si) {
  if (!o.on) return;
  const bool unit = sr == 1.0 && si == 0.0;
  for (int i = o.i0; i < D; i += o.step) {
    C2 v;
    v.x = 0;
    v.y = 0;
    if (i < d && o.j < d) {
      const gp<const T> e = gmem(M) + 2 * (i * d + o.j);
      v.x = e[0];
      v.y = e[1];
    }
    dst[i * ld + o.j] = op_round<T, RB>(op_scale<T>(v, unit, (T)sr, (T)si));
  }
}

#define TENSO_WAVE_SYNC()                                \
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); \
  __builtin_amdgcn_wave_barrier();                       \
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront")

// One tile with NIB 16-row blocks of leg 1: each wavefront owns up to
// MT<T>::NT / NIB units of the tile and accumulates them over all terms.
template <typename T> __device__ inline T m3_re(T r, T i, T x) { return r - x; }
template <typename T> __device__ inline T m3_im(T r, T i, T x) { return i - r - x; }


// AMODE: 0 complex products from four real MFMA products, 1 from three
// (Gauss), 2 four products on operands rounded to BF16 (X slices, scaled
// operator entries and the intermediate X B^T).
template <typename T, typename Tin, int NIB, int AMODE>
__device__ __forceinline__ void apply_tile(const ApplyGroup& G, const ApplyTile& tile,
                                           char* smem_raw, long* sbase, int step) {
  typedef typename MT<T>::v4 v4;
  typedef typename V2<T>::t c2;
  constexpr int UPW = MT<T>::NT / NIB;  // units per wavefront
  constexpr int NA = UPW * NIB;         // accumulator tiles used
  constexpr int AW = kApplyWaves;
  constexpr int D1 = 16 * NIB;
  constexpr int as1 = D1 + 1;
  constexpr bool M3 = AMODE == 1;
  constexpr bool RB = AMODE == 2;
  auto rbf = [](c2 v) {  // BF16 rounding of staged operands (AMODE 2)
    if constexpr (RB) {
      v.x = bf16_round(v.x);
      v.y = bf16_round(v.y);
    }
    return v;
  };
  c2* smem = reinterpret_cast<c2*>(smem_raw);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int c = lane & 15;  // MFMA row / column within a 16-block
  const int g = lane >> 4;  // K sub-index (0..3)
  const int d1 = G.d1, d2 = G.d2;
  const int njb = (d2 + 15) >> 4;
  const int D2 = 16 * njb;
  const int xs1 = D2 + 1, bs1 = D2 + 1;  // padded row strides
  const int nq1 = (d2 + 3) >> 2;         // K steps of X_f B^T
  const int nq2 = (d1 + 3) >> 2;         // K steps of A Z
  const long sb = G.P2;
  const long sa = (long)G.P1 * d2 * G.P2;
  const int jdrv = 4 * step + G.rel;
  const int f_first = tile.u0 / njb;
  const int nfl = (tile.u0 + tile.nu - 1) / njb - f_first + 1;
  c2* xs = smem;
  c2* asb = xs + (long)nfl * D1 * xs1;
  c2* bsb = asb + 2 * D1 * as1;
  c2* zs = bsb + 2 * (long)D2 * bs1 + (long)wave * D1 * ZS1;

  // stage the tile's input slices (zero padded, compute precision): slice
  // bases once, then lanes over the columns of a row (D2 = 16, 32, 64: 64/D2
  // rows per wavefront pass; D2 = 48: one row, lanes 48..63 idle)
  if ((int)threadIdx.x < nfl)
    sbase[threadIdx.x] = unit_geo(G, (f_first + (int)threadIdx.x) * njb, njb, 0).base;
  __syncthreads();
  {
    const bool p2 = (D2 & (D2 - 1)) == 0;
    const int rpw = p2 ? 64 / D2 : 1;
    const int sub = p2 ? lane / D2 : 0;
    const int bcol = p2 ? (lane & (D2 - 1)) : lane;
    if (bcol < D2 && (p2 || lane < D2)) {
      // rows (fl, a) in steps of AW * rpw
      const int stp = AW * rpw;
      int fl = 0, a = wave * rpw + sub;
      c2* dst = xs + (long)a * xs1 + bcol;
      while (a >= D1) {  // the first row may already lie in a later slice
        a -= D1;
        ++fl;
      }
      long src = fl < nfl ? sbase[fl] + (long)bcol * sb : 0;
      const bool colok = bcol < d2;
#pragma unroll 4
      for (int ra = a; ra < nfl * D1; ra += stp) {
        c2 v;
        v.x = 0;
        v.y = 0;
        if (a < d1 && colok) {
          const cpx<T> x = ld_input<Tin, T>(G, src + a * sa);
          v.x = x.re;
          v.y = x.im;
        }
        *dst = rbf(v);
        dst += (long)stp * xs1;
        a += stp;
        if (a >= D1) {
          do {
            a -= D1;
            ++fl;
          } while (a >= D1);
          if (fl < nfl) src = sbase[fl] + (long)bcol * sb;
        }
      }
    }
  }

  // this wavefront's units (at most UPW: the host sizes tiles to fit)
  int n_my = tile.nu > wave ? (tile.nu - wave + AW - 1) / AW : 0;
  if (n_my > UPW) n_my = UPW;
  int xoff[UPW], ucol[UPW];
  long ubase[UPW];
  static_for<UPW>([&](auto uc) {
    constexpr int UU = decltype(uc)::value;
    const int u = tile.u0 + wave + AW * UU;
    xoff[UU] = (u / njb - f_first) * D1 * xs1;
    ucol[UU] = 16 * (u % njb) + c;
    ubase[UU] = unit_geo(G, u, njb, c).base;
  });
  v4 yr[NA], yi[NA], yx[NA];  // yx: M3 only
#pragma unroll
  for (int t = 0; t < NA; ++t) {
    yr[t] = v4{0, 0, 0, 0};
    yi[t] = v4{0, 0, 0, 0};
    yx[t] = v4{0, 0, 0, 0};
  }

  // write the wavefront's accumulators (its units of this tile) to Yb
  auto store_out = [&](gp<T> Yb) {
    static_for<UPW>([&](auto uc) {
      constexpr int UU = decltype(uc)::value;
      if (UU < n_my) {
        const int col = ucol[UU];
#pragma unroll
        for (int t = 0; t < NIB; ++t) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int row = 16 * t + MT<T>::drow(g, r);
            if (row < d1 && col < d2) {
              const long o = 2 * (ubase[UU] + row * sa + (long)col * sb);
              T vr = yr[UU * NIB + t][r], vi = yi[UU * NIB + t][r];
              if constexpr (M3) {
                const T vx = yx[UU * NIB + t][r];
                vi = m3_im(vr, vi, vx);
                vr = m3_re(vr, vi, vx);
              }
              if (G.accumulate) {
                Yb[o] += vr;
                Yb[o + 1] += vi;
              } else {
                Yb[o] = vr;
                Yb[o + 1] = vi;
              }
            }
          }
        }
      }
    });
  };

  // operands: term m + 1 is read (D <= 32) while term m is multiplied, and
  // written to the other LDS buffer after it
  const OpLane oa = op_lane(D1, lane, wave), ob = op_lane(D2, lane, wave);
  const bool pfa = D1 <= 32, pfb = D2 <= 32;
  c2 ra[kApplyPf], rb[kApplyPf];
  auto fetch = [&](const TermRef& t) {
    if (t.A && pfa) op_fetch<T>(reinterpret_cast<const T*>(t.A), d1, D1, oa, ra);
    if (t.B && pfb) op_fetch<T>(reinterpret_cast<const T*>(t.B), d2, D2, ob, rb);
  };
  auto put = [&](const TermRef& t, double cr, double ci, int buf) {
    c2* as = asb + buf * D1 * as1;
    c2* bs = bsb + (long)buf * D2 * bs1;
    if (t.A) {  // A carries the coefficient
      if (pfa) op_put<T, RB>(ra, D1, as1, oa, as, cr, ci);
      else op_stage<T, RB>(reinterpret_cast<const T*>(t.A), d1, D1, as1, oa, as, cr, ci);
    }
    if (t.B) {  // B only when alone
      const double sr = t.A ? 1.0 : cr, si = t.A ? 0.0 : ci;
      if (pfb) op_put<T, RB>(rb, D2, bs1, ob, bs, sr, si);
      else op_stage<T, RB>(reinterpret_cast<const T*>(t.B), d2, D2, bs1, ob, bs, sr, si);
    }
  };
  TermRef tr{};
  if (G.n_terms > 0) {
    double cr, ci;
    tr = gmem(G.terms)[0];
    coef_at(tr, G.drive, G.drive_ld, jdrv, cr, ci);
    fetch(tr);
    put(tr, cr, ci, 0);
  }
  __syncthreads();
  for (int m = 0; m < G.n_terms; ++m) {
    const int buf = m & 1;
    const bool more = m + 1 < G.n_terms;
    TermRef tn{};
    double cnr = 0, cni = 0;
    if (more) {
      tn = gmem(G.terms)[m + 1];
      coef_at(tn, G.drive, G.drive_ld, jdrv, cnr, cni);
      fetch(tn);
    }
    const c2* as = asb + buf * D1 * as1;
    const c2* bs = bsb + (long)buf * D2 * bs1;
    const int kind = (tr.A ? 1 : 0) | (tr.B ? 2 : 0);
    // Y += A X_f B^T (kind 3: Z = X_f B^T for the unit's 16 columns into the
    // wavefront's slab first, then A Z), A X_f (kind 1) or X_f B^T (kind 2):
    // every unit's accumulators are updated at one place in the code
    const bool two = kind == 3;
    const int nq = kind == 2 ? nq1 : nq2;
    const int ars16 = 16 * (kind == 2 ? xs1 : as1);
    const int bks = kind == 3 ? ZS1 : kind == 1 ? xs1 : 1;
    static_for<UPW>([&](auto uc) {
      constexpr int UU = decltype(uc)::value;
      if (UU < n_my) {
        const c2* xf = xs + xoff[UU];
        const int col = ucol[UU];
        if (two) {
          v4 zr[NIB], zi[NIB], zx[NIB];
#pragma unroll
          for (int t = 0; t < NIB; ++t) {
            zr[t] = v4{0, 0, 0, 0};
            zi[t] = v4{0, 0, 0, 0};
            zx[t] = v4{0, 0, 0, 0};
          }
          mma_loop<T, NIB, 0, NIB, M3>(zr, zi, zx, xf + c * xs1, 16 * xs1, bs + col * bs1, 1, nq1, g);
#pragma unroll
          for (int t = 0; t < NIB; ++t) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              c2 v;
              v.x = zr[t][r];
              v.y = zi[t][r];
              if constexpr (M3) {
                v.y = m3_im(zr[t][r], zi[t][r], zx[t][r]);
                v.x = m3_re(zr[t][r], zi[t][r], zx[t][r]);
              }
              zs[(16 * t + MT<T>::drow(g, r)) * ZS1 + c] = rbf(v);
            }
          }
          TENSO_WAVE_SYNC();
        }
        const c2* ar = kind == 2 ? xf + c * xs1 : as + c * as1;
        const c2* bc = two ? zs + c : kind == 1 ? xf + col : bs + col * bs1;
        mma_loop<T, NIB, UU * NIB, NA, M3>(yr, yi, yx, ar, ars16, bc, bks, nq, g);
        if (two) TENSO_WAVE_SYNC();
      }
    });
    if (G.per_term_out) {  // this term's result goes to its own slab
      store_out(gmem(reinterpret_cast<T*>(G.Y)) + 2 * (long)G.F * d1 * d2 * m);
#pragma unroll
      for (int t = 0; t < NA; ++t) {
        yr[t] = v4{0, 0, 0, 0};
        yi[t] = v4{0, 0, 0, 0};
        yx[t] = v4{0, 0, 0, 0};
      }
    }
    if (more) put(tn, cnr, cni, buf ^ 1);
    __syncthreads();  // the next term's operands are in place; this term's are free
    tr = tn;
  }
  if (!G.per_term_out) store_out(gmem(reinterpret_cast<T*>(G.Y)));
}
#undef TENSO_WAVE_SYNC

template <typename T, typename Tin, int AMODE>
__global__ void __launch_bounds__(64 * kApplyWaves) k_apply(const ApplyGroup* __restrict__ groups,
                                                            const ApplyTile* __restrict__ tiles,
                                                            const int* __restrict__ step_ctr) {
  extern __shared__ char smem_raw[];
  __shared__ long sbase[kApplyMaxUnits + 1];
  const ApplyTile tile = tiles[blockIdx.x];
  const ApplyGroup& G = groups[tile.group];
  const int step = step_ctr ? gmem(step_ctr)[0] : 0;
  switch ((G.d1 + 15) >> 4) {  // uniform per tile
    case 1: apply_tile<T, Tin, 1, AMODE>(G, tile, smem_raw, sbase, step); break;
    case 2: apply_tile<T, Tin, 2, AMODE>(G, tile, smem_raw, sbase, step); break;
    case 3: apply_tile<T, Tin, 3, AMODE>(G, tile, smem_raw, sbase, step); break;
    default: apply_tile<T, Tin, 4, AMODE>(G, tile, smem_raw, sbase, step); break;
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
  const gp<T> out = gmem(reinterpret_cast<T*>(op.out));
  const gp<const TermRef> terms = gmem(op.terms);
  const gp<const double> drive = op.drive ? gmem(op.drive) : nullptr;
  // term matrices and coefficients (drive factor included) staged once;
  // the host keeps n_terms <= PRESUM_MAX_TERMS
  __shared__ const T* mats[PRESUM_MAX_TERMS];
  __shared__ double cfs[PRESUM_MAX_TERMS][2];
  for (int m = threadIdx.x; m < op.n_terms; m += blockDim.x) {
    const TermRef t = terms[m];
    double cr = t.cre, ci = t.cim;
    if (t.slot >= 0 && drive) {
      const double f = drive[(long)t.slot * op.drive_ld + j];
      cr *= f;
      ci *= f;
    }
    mats[m] = reinterpret_cast<const T*>(t.A);
    cfs[m][0] = cr;
    cfs[m][1] = ci;
  }
  __syncthreads();
  const int nm = op.n_terms;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    double ar = 0, ai = 0;
    int m = 0;
    for (; m + 4 <= nm; m += 4) {  // four independent loads per batch
      T v[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const gp<const T> M = gmem(mats[m + u]);
        v[u][0] = M[2 * e];
        v[u][1] = M[2 * e + 1];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double a = v[u][0], b = v[u][1];
        ar += a * cfs[m + u][0] - b * cfs[m + u][1];
        ai += a * cfs[m + u][1] + b * cfs[m + u][0];
      }
    }
    for (; m < nm; ++m) {
      const gp<const T> M = gmem(mats[m]);
      const double a = M[2 * e], b = M[2 * e + 1];
      ar += a * cfs[m][0] - b * cfs[m][1];
      ai += a * cfs[m][1] + b * cfs[m][0];
    }
    out[2 * e] = (T)ar;
    out[2 * e + 1] = (T)ai;
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
    if (op.stage == 5) {  // a sum in compute precision (an environment channel)
      xin[2 * e] = (T)kr;
      xin[2 * e + 1] = (T)ki;
      continue;
    }
    if (op.stage == 6) {  // the whole RK4 update from the four stages' parts
      // (kr, ki: stage 1's sum; the accumulator as stages 1-3 would build it)
      double ar = kr, ai = ki;
      double qr = 0, qi = 0;
      for (int st = 1; st < 4; ++st) {
        qr = 0;
        qi = 0;
        const T* ps = parts + 2 * st * op.stage_stride;
        for (int p = 0; p < op.n_parts; ++p) {
          qr += (double)ps[2 * (p * op.n + e)];
          qi += (double)ps[2 * (p * op.n + e) + 1];
        }
        if (st < 3) {
          ar += 2.0 * qr;
          ai += 2.0 * qi;
        }
      }
      op.y0[2 * e] = op.y0[2 * e] + (op.h / 6.0) * (ar + qr);
      op.y0[2 * e + 1] = op.y0[2 * e + 1] + (op.h / 6.0) * (ai + qi);
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
// Rank threshold of the QR (per op, QrOp::tol): a residual column with norm at
// or below tol * ||A||_F is treated as exactly zero (identity reflector), so
// the completion of a rank-deficient core does not follow rounding noise.
__device__ inline z2 zmul(z2 a, z2 b) { return z2{a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ inline z2 zconjmul(z2 a, z2 b) {  // conj(a) * b
  return z2{a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}

// One DPP move of a double across lanes (both 32-bit halves, same pattern).
template <int CTRL>
__device__ inline double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp((int)b, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(b >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes of a wavefront, returned to every lane; all lanes
// must be active.  Within each row of 16 lanes: swap neighbours, swap pairs
// (quad permutes), mirror halves of 8, mirror the row; each exchange pairs
// two partial sums, so every lane of a row ends with the row sum.  The four
// row sums are then read as scalars and added.
__device__ inline double wave_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Quotient n / d for 0 <= n < 2^31 and 1 <= d <= 2^12 through a
// double-precision reciprocal: the product is within 2^-21 of n / d, so one
// correction step gives the exact quotient.
__device__ inline int qr_div(int n, int d, double dinv) {
  int q = (int)((double)n * dinv);
  const int r = n - q * d;
  if (r >= d) ++q;
  else if (r < 0) --q;
  return q;
}

// Blocked form of the Householder QR (LAPACK zgeqrf / zungqr structure), for
// m <= QR_MAX_M.  Panels of pb <= QR_PB columns are factored with the
// unblocked algorithm, and the columns right of a panel (and later the Q
// columns) are updated once per panel with the compact WY form
// H_p ... H_{p+pb-1} = I - V T V^H.  Reflectors, taus and the rank rule are
// those of the column-by-column algorithm; only the rounding order of the
// updates differs.
//   Thread t owns rows p + t + QR_NT j of each panel and keeps them in
// registers.  Panel column jj needs one block reduction, of |x|^2 and of the
// raw products x^H a_c for the later panel columns (then
// v^H a_c = a_c[jj] + conj(1 / (alpha - beta)) x^H a_c); every thread derives
// beta, tau and the scale from the same sums and updates its own rows: one
// barrier per column.  The Gram products of the reflectors (for T) come from
// the same registers.
//   Column updates: the explicit reflectors go to LDS; one wavefront per
// column holds the column's rows in registers (QR_RPL per lane), forms
// w = V^H x with a wave reduction and writes x - V (S w).
constexpr int QR_NT = 512;               // threads per QR (8 wavefronts)
constexpr int QR_NW = QR_NT / 64;
constexpr int QR_PB = 4;                 // panel width
constexpr int QR_RPL = 16;               // rows per lane of a column update
constexpr int QR_RPT = 2;                // panel rows per thread
constexpr int QR_MAX_M = 64 * QR_RPL;    // 1024 = QR_NT * QR_RPT
constexpr int QR_NPAIR = QR_PB * (QR_PB - 1) / 2;
static_assert(QR_MAX_M == kQrBlockedMaxM, "blocked QR height");

// x <- (I - V S V^H) x for one column, x[r] at X[off[q]] for r = q * 64 + lane
// (rows past mp - 1 are clamped to mp - 1 in off); V explicit (unit
// diagonal, zeros above) in LDS with leading dimension QR_MAX_M, finite
// (zero) in rows >= mp and columns >= pb, so that every read is the lane's
// base plus a constant offset; S is QR_PB x QR_PB in LDS, zero outside
// pb x pb.
__device__ inline void qr_apply_col(const z2* __restrict__ Lv, int mp, int pb,
                                    const z2* __restrict__ S, gp<z2> __restrict__ X,
                                    const int* off, int lane, double* tail) {
  // 16-byte panel reads: one ds_read_b128 with a constant offset each
  const double2* __restrict__ Ll = reinterpret_cast<const double2*>(Lv) + lane;
  auto lv = [&](int i, int q) {
    const double2 t = Ll[i * QR_MAX_M + q * 64];
    return z2{t.x, t.y};
  };
  z2 xs[QR_RPL];
#pragma unroll
  for (int q = 0; q < QR_RPL; ++q) xs[q] = X[off[q]];
  double w[2 * QR_PB];
#pragma unroll
  for (int i = 0; i < 2 * QR_PB; ++i) w[i] = 0;
#pragma unroll
  for (int q = 0; q < QR_RPL; ++q) {
    const int r = q * 64 + lane;
    if (r >= mp) xs[q] = z2{0.0, 0.0};  // clamped duplicate: no contribution
    z2 vv[QR_PB];
#pragma unroll
    for (int i = 0; i < QR_PB; ++i) vv[i] = lv(i, q);
#pragma unroll
    for (int i = 0; i < QR_PB; ++i) {  // w_i += conj(v_i) x
      w[2 * i] = fma(vv[i].r, xs[q].r, fma(vv[i].i, xs[q].i, w[2 * i]));
      w[2 * i + 1] = fma(vv[i].r, xs[q].i, fma(-vv[i].i, xs[q].r, w[2 * i + 1]));
    }
    // keep the scheduler from hoisting every reflector load of the column
    // (they would not fit in registers)
    if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int i = 0; i < 2 * QR_PB; ++i) w[i] = wave_sum(w[i]);
  // u = S w (w is the same in every lane): lane 2 i + h forms the real
  // (h = 0) or imaginary (h = 1) part of u_i, then all lanes read it
  double uc = 0;
  {
    const int ui = (lane >> 1) & (QR_PB - 1), uh = lane & 1;
#pragma unroll
    for (int l = 0; l < QR_PB; ++l) {
      const z2 t = S[ui * QR_PB + l];
      uc = uh ? fma(t.r, w[2 * l + 1], fma(t.i, w[2 * l], uc))
              : fma(t.r, w[2 * l], fma(-t.i, w[2 * l + 1], uc));
    }
  }
  double u[2 * QR_PB];
#pragma unroll
  for (int e = 0; e < 2 * QR_PB; ++e) u[e] = readlane_d(uc, e);
  double t2 = 0;  // squared norm of the result below the panel's rows
#pragma unroll
  for (int q = 0; q < QR_RPL; ++q) {
    const int r = q * 64 + lane;
    if (r < mp) {
      z2 vv[QR_PB];
#pragma unroll
      for (int i = 0; i < QR_PB; ++i) vv[i] = lv(i, q);
      double ar = xs[q].r, ai = xs[q].i;
#pragma unroll
      for (int i = 0; i < QR_PB; ++i) {  // x -= v_i u_i
        ar = fma(-vv[i].r, u[2 * i], fma(vv[i].i, u[2 * i + 1], ar));
        ai = fma(-vv[i].r, u[2 * i + 1], fma(-vv[i].i, u[2 * i], ai));
      }
      if (r >= pb) t2 = fma(ar, ar, fma(ai, ai, t2));
      X[off[q]] = z2{ar, ai};
    }
    if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
  }
  if (tail) {
    t2 = wave_sum(t2);
    if (lane == 0) *tail = t2;
  }
}

// Column-by-column form, all in global memory: used for matrices too tall
// for the LDS panel of the blocked form.
__device__ void qr_unblocked(const QrOp& op) {
  const int m = op.m, n = op.n, k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[2 * QR_NW];  // [0, NW) column norms, [NW, 2 NW) Frobenius norm
  __shared__ double sh_tau[2], sh_scale[2], sh_beta[2];
  __shared__ int sh_skip;
  const gp<z2> V = gmem(reinterpret_cast<z2*>(op.V));  // column-major m x n
  const gp<z2> tau = gmem(reinterpret_cast<z2*>(op.tau));
  const gp<z2> C = gmem(reinterpret_cast<z2*>(op.C));
  auto cidx = [&](int row, int col) -> long {
    const int pre = row / op.Ppost, post = row % op.Ppost;
    return (long)pre * n * op.Ppost + (long)col * op.Ppost + post;
  };
  double fro = 0;
  for (long e = tid; e < (long)m * n; e += QR_NT) {
    const int row = e % m, col = e / m;
    const z2 v = C[cidx(row, col)];
    V[e] = v;
    fro += v.r * v.r + v.i * v.i;
  }
  fro = wave_sum(fro);
  if (lane == 0) red[QR_NW + wave] = fro;
  __syncthreads();
  // residual columns at or below this squared norm count as exact zeros
  double fsum = 0;
  for (int w = 0; w < QR_NW; ++w) fsum += red[QR_NW + w];
  const double thr2 = op.tol * op.tol * fsum;
  for (int j = 0; j < k; ++j) {
    // xnorm of V[j+1:m, j]
    double s = 0;
    for (int i = j + 1 + tid; i < m; i += QR_NT) {
      z2 v = V[(long)j * m + i];
      s += v.r * v.r + v.i * v.i;
    }
    s = wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) {
      double xn2 = 0;
      for (int w = 0; w < QR_NW; ++w) xn2 += red[w];
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
      for (int i = j + tid; i < m; i += QR_NT) V[(long)j * m + i] = z2{0, 0};
    }
    if (!sh_skip) {
      const z2 sc{sh_scale[0], sh_scale[1]};
      for (int i = j + 1 + tid; i < m; i += QR_NT) V[(long)j * m + i] = zmul(V[(long)j * m + i], sc);
      if (tid == 0) V[(long)j * m + j] = z2{sh_beta[0], 0.0};
      __syncthreads();
      // apply H^H = I - conj(tau) v v^H to columns j+1..n-1
      const z2 ct{sh_tau[0], -sh_tau[1]};
      for (int col = j + 1 + wave; col < n; col += QR_NW) {
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
  const gp<z2> R = gmem(reinterpret_cast<z2*>(op.R));
  for (int e = tid; e < n * n; e += QR_NT) {
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
      for (int col = i + 1 + wave; col < nq; col += QR_NW) {
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
    for (int r = i + 1 + tid; r < m; r += QR_NT) {
      const z2 v = V[(long)i * m + r];
      const z2 p = zmul(t, v);
      V[(long)i * m + r] = z2{-p.r, -p.i};
    }
    if (tid == 0) V[(long)i * m + i] = z2{1.0 - t.r, -t.i};
    for (int r = tid; r < i; r += QR_NT) V[(long)i * m + r] = z2{0, 0};
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
  for (int e = tid; e < n * n; e += QR_NT) {
    const int i = e / n, col = e % n;
    const z2 cph{ph[2 * i], -ph[2 * i + 1]};
    const long o = op.transposeR ? (long)col * n + i : (long)i * n + col;
    R[o] = zmul(cph, R[o]);
  }
  for (long e = tid; e < (long)m * n; e += QR_NT) {
    const int row = e % m, col = e / m;
    z2 q = col < nq ? zmul(V[(long)col * m + row], z2{ph[2 * col], ph[2 * col + 1]}) : z2{0, 0};
    C[cidx(row, col)] = q;
  }
}


// Column-by-column form on a column-major working copy L of the matrix: in
// LDS (m <= kQrLdsMaxM, m * n <= kQrLdsElems) or the scratch V in global
// memory (m <= QR_MAX_M; V apart from C).  Columns are dealt to the wavefronts
// in turn.  Every wavefront forms reflector j itself from column j (the same
// arithmetic on the same data in each, so no broadcast is needed) and applies
// it to its own later columns; one barrier per column (the owner writes the
// finished column after it, once every wavefront has read the column).  The orthonormal
// factor is formed column by column from the stored reflectors
// (Q e_c = H_0 ... H_c e_c, the LAPACK zung2r result), each column by its
// owner in registers, with no barrier.  A lane holds rows lane + 64 q
// (q < RPL, m <= 64 RPL) of a column in registers.  Reflectors, taus, the
// rank rule and the phases of R are those of the other forms; only the
// rounding order differs.
static_assert(kQrLdsElems * 16 <= 128 * 1024, "LDS form within the CU's LDS");
// The same algorithm runs on the scratch copy V in global memory (L2
// resident) for the larger ops, m <= QR_MAX_M.

template <int RPL, typename ZP>
__device__ void qr_cols(const QrOp& op, ZP L) {
  const int m = op.m, n = op.n, k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[QR_NW];
  __shared__ z2 tauS[64];
  __shared__ double phS[2 * 64];
  const gp<z2> C = gmem(reinterpret_cast<z2*>(op.C));
  const gp<z2> R = gmem(reinterpret_cast<z2*>(op.R));
  const int ppost = op.Ppost;
  const int cstride = n * ppost;
  const double pinv = 1.0 / ppost;
  auto crow = [=](int row) -> int {
    const int q = qr_div(row, ppost, pinv);
    return q * cstride + (row - q * ppost);
  };
  // C -> L and the Frobenius norm (16 columns of a row read at once)
  __syncthreads();  // a previous op of this workgroup no longer reads L
  double fro = 0;
  for (int row = tid; row < m; row += QR_NT) {
    const int cb = crow(row);
    for (int c0 = 0; c0 < n; c0 += 16) {
      z2 t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = c0 + u < n ? C[cb + (c0 + u) * ppost] : z2{0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + u < n) {
          L[(c0 + u) * m + row] = t[u];
          fro += t[u].r * t[u].r + t[u].i * t[u].i;
        }
    }
  }
  fro = wave_sum(fro);
  if (lane == 0) red[wave] = fro;
  __syncthreads();
  double fsum = 0;
  for (int w = 0; w < QR_NW; ++w) fsum += red[w];
  // residual columns at or below this squared norm count as exact zeros
  const double thr2 = op.tol * op.tol * fsum;
  // rows r >= r0 of a column into registers (zeros elsewhere); row r0 reads
  // as 1 when `unit` (the reflector's implicit leading entry)
  auto ldcol = [&](ZP Lc, int r0, bool unit, z2(&y)[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      y[q] = r >= r0 && r < m ? Lc[r] : z2{0.0, 0.0};
      if (unit && r == r0) y[q] = z2{1.0, 0.0};
    }
  };
  auto stcol = [&](ZP Lc, int r0, const z2(&y)[RPL]) {
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (r >= r0 && r < m) Lc[r] = y[q];
    }
  };
  // w = v^H y over the lane's rows, summed over the wavefront
  auto vdot = [&](const z2(&v)[RPL], const z2(&y)[RPL]) {
    double wr = 0, wi = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const z2 p = zconjmul(v[q], y[q]);
      wr += p.r;
      wi += p.i;
    }
    return z2{wave_sum(wr), wave_sum(wi)};
  };
  // v^H ya and v^H yb: the four wave reductions are independent chains
  auto vdot2 = [&](const z2(&v)[RPL], const z2(&ya)[RPL], const z2(&yb)[RPL], z2& da, z2& db) {
    double ar = 0, ai = 0, br = 0, bi = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const z2 pa = zconjmul(v[q], ya[q]), pb = zconjmul(v[q], yb[q]);
      ar += pa.r;
      ai += pa.i;
      br += pb.r;
      bi += pb.i;
    }
    da = z2{wave_sum(ar), wave_sum(ai)};
    db = z2{wave_sum(br), wave_sum(bi)};
  };
  auto axpy = [&](z2(&y)[RPL], const z2(&v)[RPL], z2 f) {  // y -= f v
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const z2 pv = zmul(f, v[q]);
      y[q] = z2{y[q].r - pv.r, y[q].i - pv.i};
    }
  };

  // The owner's store of a finished column waits for the next barrier, so
  // that every wavefront has read the column first: the owner keeps the
  // reflector in v (unit leading entry) and writes it with beta in front.
  z2 v[RPL];
  int pj = -1;       // column whose store is pending (-1: none)
  double pbeta = 0;  // its diagonal entry; pzero: the column is zero
  bool pzero = false;
  auto flush = [&]() {
    if (pj < 0) return;
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (pzero) v[q] = z2{0.0, 0.0};
      else if (r == pj) v[q] = z2{pbeta, 0.0};
    }
    stcol(L + pj * m, pj, v);
    pj = -1;
  };
  for (int j = 0; j < k; ++j) {
    flush();
    ZP Lj = L + j * m;
    ldcol(Lj, j, false, v);
    double xn2 = 0;
#pragma unroll
    for (int q = 0; q < RPL; ++q)
      if (lane + 64 * q > j) xn2 = fma(v[q].r, v[q].r, fma(v[q].i, v[q].i, xn2));
    xn2 = wave_sum(xn2);
    const z2 alpha = Lj[j];
    const bool own_j = wave == j % QR_NW;
    z2 t{0.0, 0.0};
    bool apply = false;
    if (alpha.r * alpha.r + alpha.i * alpha.i + xn2 <= thr2) {
      // numerically zero residual: identity reflector, zero column
      if (own_j) {
        pj = j;
        pzero = true;
      }
    } else if (!(xn2 == 0.0 && alpha.i == 0.0)) {
      apply = true;
      const double nrm = sqrt(alpha.r * alpha.r + alpha.i * alpha.i + xn2);
      // beta = -sign(Re alpha) * nrm (LAPACK zlarfg; a zero counts as positive)
      const double beta = alpha.r >= 0.0 ? -nrm : nrm;
      t = z2{(beta - alpha.r) / beta, -alpha.i / beta};
      const double dr = alpha.r - beta, di = alpha.i;
      const double den = dr * dr + di * di;
      const z2 sc{dr / den, -di / den};  // 1 / (alpha - beta)
#pragma unroll
      for (int q = 0; q < RPL; ++q) {
        const int r = lane + 64 * q;
        v[q] = r == j ? z2{beta, 0.0} : zmul(v[q], sc);
      }
      if (own_j) {
        pj = j;
        pbeta = beta;
        pzero = false;
      }
#pragma unroll
      for (int q = 0; q < RPL; ++q)
        if (lane + 64 * q == j) v[q] = z2{1.0, 0.0};
    }
    if (own_j && lane == 0) {
      tauS[j] = t;
      gmem(reinterpret_cast<z2*>(op.tau))[j] = t;
    }
    if (apply) {
      // H^H = I - conj(tau) v v^H on this wavefront's later columns
      const z2 ct{t.r, -t.i};
      int c = j + 1 + ((wave - (j + 1)) % QR_NW + QR_NW) % QR_NW;  // first own column
      // two columns at a time where the registers allow
      for (; RPL <= 4 && c + QR_NW < n; c += 2 * QR_NW) {
        ZP La = L + c * m, Lb = L + (c + QR_NW) * m;
        z2 ya[RPL], yb[RPL], da, db;
        ldcol(La, j, false, ya);
        ldcol(Lb, j, false, yb);
        vdot2(v, ya, yb, da, db);
        axpy(ya, v, zmul(ct, da));
        axpy(yb, v, zmul(ct, db));
        stcol(La, j, ya);
        stcol(Lb, j, yb);
      }
      for (; c < n; c += QR_NW) {
        ZP Lc = L + c * m;
        z2 y[RPL];
        ldcol(Lc, j, false, y);
        axpy(y, v, zmul(ct, vdot(v, y)));
        stcol(Lc, j, y);
      }
    }
    __syncthreads();
  }
  flush();
  __syncthreads();
  // phases that make diag(R) real non-negative; R with its rows rephased
  if (tid < n) {
    const z2 dd = tid < k ? L[tid * m + tid] : z2{0.0, 0.0};
    const double a = sqrt(dd.r * dd.r + dd.i * dd.i);
    phS[2 * tid] = a > 0 ? dd.r / a : 1.0;
    phS[2 * tid + 1] = a > 0 ? dd.i / a : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < n * n; e += QR_NT) {
    const int i = e / n, c = e % n;
    const z2 x = (i <= c && i < k) ? zmul(z2{phS[2 * i], -phS[2 * i + 1]}, L[c * m + i])
                                   : z2{0.0, 0.0};
    if (op.transposeR) R[c * n + i] = x;
    else R[i * n + c] = x;
  }
  // Q column c = H_0 ... H_c e_c: e_c - tau_c v_c, then H_{c-1}, ..., H_0 in
  // turn; the reflectors in L are only read from here on.  For m <= 256 a
  // wavefront builds its columns two at a time (ca < cb): cb alone down to
  // H_ca, then both from H_{ca-1}, each reflector read once for the two.
  auto qinit = [&](int c, z2(&y)[RPL]) {
    z2 vc[RPL];
    ldcol(L + c * m, c, true, vc);
    const z2 tc = tauS[c];
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      const z2 p = zmul(tc, vc[q]);
      y[q] = r >= c ? z2{(r == c ? 1.0 : 0.0) - p.r, -p.i} : z2{0.0, 0.0};
    }
  };
  auto qstore = [&](int c, const z2(&y)[RPL]) {  // with the phase of R's row c
    const z2 ph{phS[2 * c], phS[2 * c + 1]};
#pragma unroll
    for (int q = 0; q < RPL; ++q) {
      const int r = lane + 64 * q;
      if (r < m) C[crow(r) + c * ppost] = zmul(y[q], ph);
    }
  };
  for (int ca = wave; ca < k; ca += (RPL <= 4 ? 2 : 1) * QR_NW) {
    const int cb = ca + QR_NW;
    z2 ya[RPL];
    if (RPL <= 4 && cb < k) {
      z2 yb[RPL];
      qinit(cb, yb);
      for (int i = cb - 1; i >= ca; --i) {
        const z2 ti = tauS[i];
        if (ti.r == 0.0 && ti.i == 0.0) continue;
        z2 vi[RPL];
        ldcol(L + i * m, i, true, vi);
        axpy(yb, vi, zmul(ti, vdot(vi, yb)));
      }
      qinit(ca, ya);
      for (int i = ca - 1; i >= 0; --i) {
        const z2 ti = tauS[i];
        if (ti.r == 0.0 && ti.i == 0.0) continue;
        z2 vi[RPL], da, db;
        ldcol(L + i * m, i, true, vi);
        vdot2(vi, ya, yb, da, db);
        axpy(ya, vi, zmul(ti, da));
        axpy(yb, vi, zmul(ti, db));
      }
      qstore(cb, yb);
    } else {
      qinit(ca, ya);
      for (int i = ca - 1; i >= 0; --i) {
        const z2 ti = tauS[i];
        if (ti.r == 0.0 && ti.i == 0.0) continue;
        z2 vi[RPL];
        ldcol(L + i * m, i, true, vi);
        axpy(ya, vi, zmul(ti, vdot(vi, ya)));
      }
    }
    qstore(ca, ya);
  }
}

__global__ void __launch_bounds__(QR_NT) k_qr(const QrOp* __restrict__ ops) {
  const QrOp op = ops[blockIdx.x];
  if (op.m > QR_MAX_M) {
    qr_unblocked(op);
    return;
  }
  const gp<z2> V = gmem(reinterpret_cast<z2*>(op.V));
  if (op.m <= 128) qr_cols<2>(op, V);  // uniform per workgroup
  else if (op.m <= 256) qr_cols<4>(op, V);
  else qr_cols<8>(op, V);
}

// Launches with an op taller than kQrLdsMaxM: the blocked form (and the
// column-by-column form in global memory above QR_MAX_M).
// SPLIT: stop once R is written and leave Q to k_qr_formq, which forms its
// columns in parallel from the reflectors in V and tau (not when V is the
// core itself: then Q is formed here, over the reflectors).
template <bool SPLIT>
__global__ void __launch_bounds__(QR_NT) k_qr_blocked(const QrOp* __restrict__ ops) {
  const QrOp op = ops[blockIdx.x];
  if (op.m > QR_MAX_M) {
    qr_unblocked(op);
    return;
  }
  const int m = op.m, n = op.n, k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  constexpr int NRED = 2 * QR_PB + 2 * QR_NPAIR;  // per-wave partial sums
  __shared__ double red[2][QR_NW][NRED];          // double-buffered
  __shared__ z2 rowjj[2][QR_PB];                  // row jj of the panel, copied by its owner
  __shared__ z2 S[QR_PB * QR_PB];                 // T^H (factoring) or T (forming Q)
  __shared__ z2 tauL[64];
  __shared__ double tailn[64];  // per column: squared norm below the last factored panel
  __shared__ double ph[2 * 64];
  extern __shared__ char smem_raw[];
  z2* __restrict__ L = reinterpret_cast<z2*>(smem_raw);  // explicit panel, QR_MAX_M x QR_PB
  const gp<z2> __restrict__ V = gmem(reinterpret_cast<z2*>(op.V));  // column-major m x n
  const gp<z2> __restrict__ C = gmem(reinterpret_cast<z2*>(op.C));
  const gp<z2> __restrict__ R = gmem(reinterpret_cast<z2*>(op.R));
  const int ppost = op.Ppost;
  const int cstride = n * ppost;
  const double pinv = 1.0 / ppost;
  auto crow = [=](int row) -> int {
    const int q = qr_div(row, ppost, pinv);
    return q * cstride + (row - q * ppost);
  };

  // C -> V and the Frobenius norm (V may be C itself: a core whose QR leg is
  // its slowest index is already column-major m x n)
  const bool in_place = op.V == op.C;
  double fro = 0;
  for (int row = tid; row < m; row += QR_NT) {
    const int cb = crow(row);
    for (int c0 = 0; c0 < n; c0 += 16) {
      z2 t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = c0 + u < n ? C[cb + (c0 + u) * ppost] : z2{0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + u < n) {
          if (!in_place) V[(c0 + u) * m + row] = t[u];
          fro += t[u].r * t[u].r + t[u].i * t[u].i;
        }
    }
  }
  fro = wave_sum(fro);
  if (lane == 0) red[0][wave][0] = fro;
  __syncthreads();
  // residual columns at or below this squared norm count as exact zeros
  double fsum = 0;
  for (int w = 0; w < QR_NW; ++w) fsum += red[0][w][0];
  const double thr2 = op.tol * op.tol * fsum;
  const int nbk = (k + QR_PB - 1) / QR_PB;
  int nbf = nbk;  // panels actually factored (fewer after an early exit)
  int par = 1;
  const bool split = SPLIT && !in_place && k <= 64;  // k_qr_formq's grid covers 64 columns

  for (int st = 0; st < (split ? nbk + 1 : 2 * nbk); ++st) {
    const bool fact = st < nbk;
    if (fact && st >= nbf) continue;  // past an early exit (uniform)
    const int bk = fact ? st : 2 * nbk - 1 - st;
    const int p = bk * QR_PB, pb = min(QR_PB, k - p), mp = m - p;
    if (st == nbk) {
      // phases that make diag(R) real non-negative; R with its rows rephased
      if (tid < n) {
        const z2 dd = tid < k ? V[tid * m + tid] : z2{0.0, 0.0};
        const double a = sqrt(dd.r * dd.r + dd.i * dd.i);
        ph[2 * tid] = a > 0 ? dd.r / a : 1.0;
        ph[2 * tid + 1] = a > 0 ? dd.i / a : 0.0;
      }
      __syncthreads();
      for (int e = tid; e < n * n; e += QR_NT) {
        const int i = e / n, c = e % n;
        const z2 v = (i <= c && i < k) ? zmul(z2{ph[2 * i], -ph[2 * i + 1]}, V[c * m + i])
                                       : z2{0.0, 0.0};
        if (op.transposeR) R[c * n + i] = v;
        else R[i * n + c] = v;
      }
      if (split) return;  // V keeps the reflectors for k_qr_formq
      // Q is formed in V (column-major): column c starts as the unit column
      // e_c once its reflector has been read; the columns of the identity
      // blocks (past an early exit) start so now, after R has been read out
      __syncthreads();
      for (int c = nbf * QR_PB; c < k; ++c)
        for (int row = tid; row < m; row += QR_NT) V[c * m + row] = z2{row == c ? 1.0 : 0.0, 0.0};
    }
    if (!fact && bk >= nbf) {  // identity reflectors (all tau zero): nothing to apply
      __syncthreads();
      continue;
    }
    // own panel rows (relative row tid + QR_NT j) into registers
    z2 P[QR_RPT][QR_PB];
#pragma unroll
    for (int j = 0; j < QR_RPT; ++j) {
      const int row = tid + QR_NT * j;
#pragma unroll
      for (int c = 0; c < QR_PB; ++c)
        P[j][c] = row < mp && c < pb ? V[(p + c) * m + p + row] : z2{0.0, 0.0};
    }
    if (fact) {
#pragma unroll
      for (int jj = 0; jj < QR_PB; ++jj) {
        if (jj >= pb) break;
        double d[2 * QR_PB];  // slot 0: |x|^2; slots 2c, 2c+1: x^H a_c for c > jj
#pragma unroll
        for (int c = 0; c < 2 * QR_PB; ++c) d[c] = 0;
#pragma unroll
        for (int j = 0; j < QR_RPT; ++j) {
          if (tid + QR_NT * j <= jj) continue;  // rows past mp hold zeros
          const z2 x = P[j][jj];
          d[0] = fma(x.r, x.r, fma(x.i, x.i, d[0]));
#pragma unroll
          for (int c = jj + 1; c < QR_PB; ++c) {
            d[2 * c] = fma(x.r, P[j][c].r, fma(x.i, P[j][c].i, d[2 * c]));
            d[2 * c + 1] = fma(x.r, P[j][c].i, fma(-x.i, P[j][c].r, d[2 * c + 1]));
          }
        }
        d[0] = wave_sum(d[0]);
#pragma unroll
        for (int c = jj + 1; c < QR_PB; ++c) {
          d[2 * c] = wave_sum(d[2 * c]);
          d[2 * c + 1] = wave_sum(d[2 * c + 1]);
        }
        // row jj before this column's update; its owner (thread jj) updates
        // it after the barrier while the others still read it
        if (tid == jj) {
#pragma unroll
          for (int c = jj; c < QR_PB; ++c) rowjj[par][c] = P[0][c];
        }
        if (lane == 0) {
          red[par][wave][0] = d[0];
#pragma unroll
          for (int c = jj + 1; c < QR_PB; ++c) {
            red[par][wave][2 * c] = d[2 * c];
            red[par][wave][2 * c + 1] = d[2 * c + 1];
          }
        }
        __syncthreads();
        double xn2 = 0;
        for (int w = 0; w < QR_NW; ++w) xn2 += red[par][w][0];
        const z2 alpha = rowjj[par][jj];
        z2 t{0.0, 0.0};
        if (alpha.r * alpha.r + alpha.i * alpha.i + xn2 <= thr2) {
          // numerically zero residual: identity reflector, zero column
#pragma unroll
          for (int j = 0; j < QR_RPT; ++j)
            if (tid + QR_NT * j >= jj) P[j][jj] = z2{0.0, 0.0};
        } else if (!(xn2 == 0.0 && alpha.i == 0.0)) {
          const double nrm = sqrt(alpha.r * alpha.r + alpha.i * alpha.i + xn2);
          // beta = -sign(Re alpha) * nrm (LAPACK zlarfg; a zero counts as positive)
          const double beta = alpha.r >= 0.0 ? -nrm : nrm;
          t = z2{(beta - alpha.r) / beta, -alpha.i / beta};
          const double dr = alpha.r - beta, di = alpha.i;
          const double den = dr * dr + di * di;
          const z2 sc{dr / den, -di / den};  // 1 / (alpha - beta)
          const z2 ct{t.r, -t.i};
          z2 f[QR_PB];
#pragma unroll
          for (int c = jj + 1; c < QR_PB; ++c) {
            z2 D{0.0, 0.0};
            for (int w = 0; w < QR_NW; ++w) {
              D.r += red[par][w][2 * c];
              D.i += red[par][w][2 * c + 1];
            }
            const z2 cd = zmul(z2{sc.r, -sc.i}, D);
            const z2 a0 = rowjj[par][c];
            f[c] = zmul(ct, z2{a0.r + cd.r, a0.i + cd.i});
          }
#pragma unroll
          for (int j = 0; j < QR_RPT; ++j) {
            const int row = tid + QR_NT * j;
            if (row < jj) continue;
            const z2 v = row == jj ? z2{1.0, 0.0} : zmul(P[j][jj], sc);
#pragma unroll
            for (int c = jj + 1; c < QR_PB; ++c) {
              P[j][c].r = fma(-f[c].r, v.r, fma(f[c].i, v.i, P[j][c].r));
              P[j][c].i = fma(-f[c].r, v.i, fma(-f[c].i, v.r, P[j][c].i));
            }
            P[j][jj] = row == jj ? z2{beta, 0.0} : v;
          }
        }
        if (tid == 0) {
          tauL[p + jj] = t;
          gmem(reinterpret_cast<z2*>(op.tau))[p + jj] = t;
        }
        par ^= 1;
      }
      // factored panel (R entries and reflectors) back to V
#pragma unroll
      for (int j = 0; j < QR_RPT; ++j) {
        const int row = tid + QR_NT * j;
        if (row < mp) {
#pragma unroll
          for (int c = 0; c < QR_PB; ++c)
            if (c < pb) V[(p + c) * m + p + row] = P[j][c];
        }
      }
    }
    const int c0 = fact ? p + pb : p, c1 = fact ? n : k;
    if (c0 < c1) {
      // explicit reflectors: unit diagonal, zeros above; to LDS for the
      // column updates, and their Gram products y_ij = v_i^H v_j (i < j)
      double g[2 * QR_NPAIR];
#pragma unroll
      for (int e = 0; e < 2 * QR_NPAIR; ++e) g[e] = 0;
#pragma unroll
      for (int j = 0; j < QR_RPT; ++j) {
        const int row = tid + QR_NT * j;
#pragma unroll
        for (int c = 0; c < QR_PB; ++c) {
          if (row == c) P[j][c] = z2{1.0, 0.0};
          else if (row < c) P[j][c] = z2{0.0, 0.0};
        }
        // every row and column of the LDS panel (zeros past mp and pb)
#pragma unroll
        for (int c = 0; c < QR_PB; ++c) L[c * QR_MAX_M + row] = P[j][c];
        int e = 0;
#pragma unroll
        for (int jc = 1; jc < QR_PB; ++jc)
#pragma unroll
          for (int ic = 0; ic < jc; ++ic, ++e) {
            g[2 * e] = fma(P[j][ic].r, P[j][jc].r, fma(P[j][ic].i, P[j][jc].i, g[2 * e]));
            g[2 * e + 1] = fma(P[j][ic].r, P[j][jc].i, fma(-P[j][ic].i, P[j][jc].r, g[2 * e + 1]));
          }
      }
#pragma unroll
      for (int e = 0; e < 2 * QR_NPAIR; ++e) g[e] = wave_sum(g[e]);
      if (lane == 0) {
#pragma unroll
        for (int e = 0; e < 2 * QR_NPAIR; ++e) red[par][wave][2 * QR_PB + e] = g[e];
      }
      __syncthreads();
      if (!fact) {  // every thread holds its panel rows: the reflectors' columns become e_c
        for (int c = p; c < p + pb; ++c)
          for (int row = tid; row < m; row += QR_NT) V[c * m + row] = z2{row == c ? 1.0 : 0.0, 0.0};
      }
      if (tid == 0) {
        // T (forward column-wise): T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] y[0:j, j]
        z2 T[QR_PB][QR_PB];
#pragma unroll
        for (int i = 0; i < QR_PB; ++i)
#pragma unroll
          for (int j = 0; j < QR_PB; ++j) T[i][j] = z2{0.0, 0.0};
        int e0 = 0;
#pragma unroll
        for (int j = 0; j < QR_PB; ++j) {
          if (j < pb) {
            const z2 tj = tauL[p + j];
            z2 y[QR_PB];
#pragma unroll
            for (int l = 0; l < j; ++l) {
              const int o = 2 * QR_PB + 2 * (e0 + l);
              y[l] = z2{0.0, 0.0};
              for (int w = 0; w < QR_NW; ++w) {
                y[l].r += red[par][w][o];
                y[l].i += red[par][w][o + 1];
              }
            }
#pragma unroll
            for (int i = 0; i < j; ++i) {
              double sr = 0, si = 0;
#pragma unroll
              for (int l = i; l < j; ++l) {
                const z2 pr = zmul(T[i][l], y[l]);
                sr += pr.r;
                si += pr.i;
              }
              const z2 pr = zmul(tj, z2{sr, si});
              T[i][j] = z2{-pr.r, -pr.i};
            }
            T[j][j] = tj;
          }
          e0 += j;
        }
        // the factor applied: T^H while factoring (H^H is applied), T while forming Q
#pragma unroll
        for (int i = 0; i < QR_PB; ++i)
#pragma unroll
          for (int l = 0; l < QR_PB; ++l)
            S[i * QR_PB + l] = fact ? z2{T[l][i].r, -T[l][i].i} : T[i][l];
      }
      par ^= 1;
      __syncthreads();
      // columns of V (reflectors while factoring, Q while forming it)
      int off[QR_RPL];
#pragma unroll
      for (int q = 0; q < QR_RPL; ++q) {
        const int r = q * 64 + lane;
        off[q] = p + (r < mp ? r : mp - 1);
      }
      for (int cc = c0 + wave; cc < c1; cc += QR_NW)
        qr_apply_col(L, mp, pb, S, V + cc * m, off, lane, fact ? tailn + cc : nullptr);
    }
    __syncthreads();
    if (fact && c0 < c1) {
      // Early exit by the rank rule: if every remaining column's norm below
      // this panel is at or under the threshold, each of them would in turn
      // be found numerically zero (identity reflectors change nothing, and a
      // column's norm from its diagonal down is at most its norm from here
      // down).  Do that at once: zero each from its diagonal down, tau = 0.
      double mx = 0;
      for (int cc = c0; cc < c1; ++cc) mx = fmax(mx, tailn[cc]);
      if (mx <= thr2) {
        for (int cc = c0; cc < c1; ++cc)
          for (int row = cc + tid; row < m; row += QR_NT) V[cc * m + row] = z2{0.0, 0.0};
        if (tid >= c0 && tid < k) {
          tauL[tid] = z2{0.0, 0.0};
          gmem(reinterpret_cast<z2*>(op.tau))[tid] = z2{0.0, 0.0};
        }
        nbf = st + 1;
        __syncthreads();
      }
    }
  }
  // Q (the first k columns of V) into the core, with the phases of R
  for (int row = tid; row < m; row += QR_NT) {
    const int cb = crow(row);
    for (int c0 = 0; c0 < k; c0 += 16) {
      z2 t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) t[u] = c0 + u < k ? V[(c0 + u) * m + row] : z2{0.0, 0.0};
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = c0 + u;
        if (c < k) C[cb + c * ppost] = zmul(t[u], z2{ph[2 * c], ph[2 * c + 1]});
      }
    }
  }
}

// Q of a factorisation that k_qr_blocked<true> left in V (reflectors below
// the diagonal, R on and above it) and tau.  Column c of Q is H_0 ... H_c e_c
// and needs no other column, so the columns are dealt to wavefronts of
// several workgroups (grid: ops x groups of QR_NW columns).  A workgroup takes
// the panels from that of its last column down to the first: the panel's
// explicit reflectors go to LDS, thread 0 forms its T factor from their Gram
// products, and every wavefront whose column has started (at its own panel,
// as e_c) applies I - V T V^H to it, the column held in registers (row
// lane + 64 q).  The finished columns go into the core with the phases that
// make diag(R) real non-negative.  Panels whose taus are all zero (past an
// early exit of the rank rule) are identities and are skipped.
__global__ void __launch_bounds__(QR_NT) k_qr_formq(const QrOp* __restrict__ ops) {
  const QrOp op = ops[blockIdx.x];
  const int m = op.m, n = op.n, k = m < n ? m : n;
  if (m > QR_MAX_M || op.V == op.C || k > 64) return;  // formed by the factoring kernel
  const int c_lo = (int)blockIdx.y * QR_NW;
  if (c_lo >= k) return;
  const int c_hi = min(k, c_lo + QR_NW);  // this workgroup's columns [c_lo, c_hi)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int c = c_lo + wave;  // this wavefront's column (none when c >= c_hi)
  __shared__ double red[QR_NW][2 * QR_NPAIR];
  __shared__ z2 S[QR_PB * QR_PB];
  extern __shared__ char smem_raw[];
  z2* __restrict__ L = reinterpret_cast<z2*>(smem_raw);  // QR_MAX_M x QR_PB, absolute rows
  const gp<const z2> V = gmem(reinterpret_cast<const z2*>(op.V));
  const gp<const z2> tau = gmem(reinterpret_cast<const z2*>(op.tau));
  const gp<z2> C = gmem(reinterpret_cast<z2*>(op.C));
  z2 x[QR_RPL];
#pragma unroll
  for (int q = 0; q < QR_RPL; ++q) x[q] = z2{0.0, 0.0};
  for (int bk = (c_hi - 1) / QR_PB; bk >= 0; --bk) {
    const int p = bk * QR_PB, pb = min(QR_PB, k - p);
    z2 tp[QR_PB];
    bool any = false;
#pragma unroll
    for (int i = 0; i < QR_PB; ++i) {
      tp[i] = z2{0.0, 0.0};
      if (i < pb) tp[i] = tau[p + i];
      any = any || tp[i].r != 0.0 || tp[i].i != 0.0;
    }
    if (c < c_hi && c >= p && c < p + pb) {  // the column starts at its own panel
#pragma unroll
      for (int q = 0; q < QR_RPL; ++q) x[q] = z2{lane + 64 * q == c ? 1.0 : 0.0, 0.0};
    }
    if (!any) continue;  // identity reflectors (the same taus in every thread)
    __syncthreads();     // the previous panel's LDS reads are done
    double g[2 * QR_NPAIR];
#pragma unroll
    for (int e = 0; e < 2 * QR_NPAIR; ++e) g[e] = 0;
#pragma unroll
    for (int j = 0; j < QR_RPT; ++j) {
      const int row = tid + QR_NT * j;  // < QR_MAX_M
      z2 v[QR_PB];
#pragma unroll
      for (int i = 0; i < QR_PB; ++i) {
        const int d = p + i;  // the reflector's unit entry
        if (i >= pb || row < d || row >= m) v[i] = z2{0.0, 0.0};
        else if (row == d) v[i] = z2{1.0, 0.0};
        else v[i] = V[(long)d * m + row];
        L[i * QR_MAX_M + row] = v[i];
      }
      int e = 0;
#pragma unroll
      for (int jc = 1; jc < QR_PB; ++jc)
#pragma unroll
        for (int ic = 0; ic < jc; ++ic, ++e) {  // y_ic,jc = v_ic^H v_jc
          g[2 * e] = fma(v[ic].r, v[jc].r, fma(v[ic].i, v[jc].i, g[2 * e]));
          g[2 * e + 1] = fma(v[ic].r, v[jc].i, fma(-v[ic].i, v[jc].r, g[2 * e + 1]));
        }
    }
#pragma unroll
    for (int e = 0; e < 2 * QR_NPAIR; ++e) g[e] = wave_sum(g[e]);
    if (lane == 0) {
#pragma unroll
      for (int e = 0; e < 2 * QR_NPAIR; ++e) red[wave][e] = g[e];
    }
    __syncthreads();
    if (tid == 0) {
      // T (forward column-wise): T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] y[0:j, j]
      z2 T[QR_PB][QR_PB];
#pragma unroll
      for (int i = 0; i < QR_PB; ++i)
#pragma unroll
        for (int j = 0; j < QR_PB; ++j) T[i][j] = z2{0.0, 0.0};
      int e0 = 0;
#pragma unroll
      for (int j = 0; j < QR_PB; ++j) {
        if (j < pb) {
          z2 y[QR_PB];
#pragma unroll
          for (int l = 0; l < j; ++l) {
            y[l] = z2{0.0, 0.0};
            for (int w = 0; w < QR_NW; ++w) {
              y[l].r += red[w][2 * (e0 + l)];
              y[l].i += red[w][2 * (e0 + l) + 1];
            }
          }
#pragma unroll
          for (int i = 0; i < j; ++i) {
            double sr = 0, si = 0;
#pragma unroll
            for (int l = i; l < j; ++l) {
              const z2 pr = zmul(T[i][l], y[l]);
              sr += pr.r;
              si += pr.i;
            }
            const z2 pr = zmul(tp[j], z2{sr, si});
            T[i][j] = z2{-pr.r, -pr.i};
          }
          T[j][j] = tp[j];
        }
        e0 += j;
      }
#pragma unroll
      for (int i = 0; i < QR_PB; ++i)
#pragma unroll
        for (int l = 0; l < QR_PB; ++l) S[i * QR_PB + l] = T[i][l];
    }
    __syncthreads();
    if (c < c_hi && c >= p) {
      // w = V^H x, u = T w, x -= V u
      const double2* __restrict__ Ll = reinterpret_cast<const double2*>(L) + lane;
      double w[2 * QR_PB];
#pragma unroll
      for (int i = 0; i < 2 * QR_PB; ++i) w[i] = 0;
#pragma unroll
      for (int q = 0; q < QR_RPL; ++q) {
#pragma unroll
        for (int i = 0; i < QR_PB; ++i) {
          const double2 t = Ll[i * QR_MAX_M + q * 64];
          w[2 * i] = fma(t.x, x[q].r, fma(t.y, x[q].i, w[2 * i]));
          w[2 * i + 1] = fma(t.x, x[q].i, fma(-t.y, x[q].r, w[2 * i + 1]));
        }
        if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int i = 0; i < 2 * QR_PB; ++i) w[i] = wave_sum(w[i]);
      double u[2 * QR_PB];
#pragma unroll
      for (int i = 0; i < QR_PB; ++i) {
        double ur = 0, ui = 0;
#pragma unroll
        for (int l = 0; l < QR_PB; ++l) {
          const z2 t = S[i * QR_PB + l];
          ur = fma(t.r, w[2 * l], fma(-t.i, w[2 * l + 1], ur));
          ui = fma(t.r, w[2 * l + 1], fma(t.i, w[2 * l], ui));
        }
        u[2 * i] = ur;
        u[2 * i + 1] = ui;
      }
#pragma unroll
      for (int q = 0; q < QR_RPL; ++q) {
        double ar = x[q].r, ai = x[q].i;
#pragma unroll
        for (int i = 0; i < QR_PB; ++i) {  // x -= v_i u_i
          const double2 t = Ll[i * QR_MAX_M + q * 64];
          ar = fma(-t.x, u[2 * i], fma(t.y, u[2 * i + 1], ar));
          ai = fma(-t.x, u[2 * i + 1], fma(-t.y, u[2 * i], ai));
        }
        x[q] = z2{ar, ai};
        if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  if (c < c_hi) {
    const z2 dd = V[(long)c * m + c];
    const double a = sqrt(dd.r * dd.r + dd.i * dd.i);
    const z2 ph{a > 0 ? dd.r / a : 1.0, a > 0 ? dd.i / a : 0.0};
    const int ppost = op.Ppost, cstride = n * ppost;
    const double pinv = 1.0 / ppost;
#pragma unroll
    for (int q = 0; q < QR_RPL; ++q) {
      const int row = lane + 64 * q;
      if (row < m) {
        const int qq = qr_div(row, ppost, pinv);
        C[qq * cstride + (row - qq * ppost) + c * ppost] = zmul(x[q], ph);
      }
    }
  }
}

// Launches whose every op fits the LDS form (m <= kQrLdsMaxM, m n <= kQrLdsElems).
__global__ void __launch_bounds__(QR_NT) k_qr_lds(const QrOp* __restrict__ ops) {
  const QrOp op = ops[blockIdx.x];
  extern __shared__ char qr_smem[];
  z2* L = reinterpret_cast<z2*>(qr_smem);
  if (op.m <= 128) qr_cols<2>(op, L);  // uniform per workgroup
  else if (op.m <= 256) qr_cols<4>(op, L);
  else qr_cols<8>(op, L);
}

// ---------------------------------------------------------------------------
// absorb: C[pre, a, post] <- sum_a' Mx[a, a'] C[pre, a', post]   (FP64)
// ---------------------------------------------------------------------------
struct AbsorbTile {
  int op;
  int f0, f1;  // fiber range (fiber = (pre, post))
};

// The operator (as Mx, row a in column a of the LDS copy, so that lanes with
// consecutive a read consecutive words) and the tile's fibers are staged in
// LDS; thread (g, a) forms output row a of fibers g, g + G, ... (G = 256 / n
// fiber groups), reading each operator entry once for all its fibers.  Every
// output is the same sum over a' in the same order as a plain loop.
__global__ void __launch_bounds__(256) k_absorb(const AbsorbOp* __restrict__ ops,
                                                const AbsorbTile* __restrict__ tiles) {
  const AbsorbTile tl = tiles[blockIdx.x];
  const AbsorbOp op = ops[tl.op];
  extern __shared__ char smem_raw[];
  const int n = op.n;
  const int nf = tl.f1 - tl.f0;
  z2* Mt = reinterpret_cast<z2*>(smem_raw);  // Mt[b * n + a] = Mx[a][b]
  z2* buf = Mt + n * n;                      // buf[fl * n + b]
  z2* C = reinterpret_cast<z2*>(op.C);
  const z2* M = reinterpret_cast<const z2*>(op.M);
  auto off = [&](int fib, int a) -> long {
    const int pre = fib / op.Ppost, post = fib % op.Ppost;
    return (long)pre * n * op.Ppost + (long)a * op.Ppost + post;
  };
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int a = e / n, b = e % n;  // reads of M row by row
    Mt[b * n + a] = op.transposeM ? M[(long)b * n + a] : M[(long)a * n + b];
  }
  for (int e = threadIdx.x; e < nf * n; e += blockDim.x) {
    const int fl = e / n, a = e % n;
    buf[e] = C[off(tl.f0 + fl, a)];
  }
  __syncthreads();
  constexpr int kMaxFib = 16;  // fibers per thread per pass
  const int G = (int)blockDim.x / n;
  const int g = (int)threadIdx.x / n, a = (int)threadIdx.x % n;
  if (g >= G) return;
  for (int f0 = g; f0 < nf; f0 += G * kMaxFib) {
    double sr[kMaxFib], si[kMaxFib];
#pragma unroll
    for (int k = 0; k < kMaxFib; ++k) sr[k] = si[k] = 0.0;
    for (int b = 0; b < n; ++b) {
      const z2 mv = Mt[b * n + a];
#pragma unroll
      for (int k = 0; k < kMaxFib; ++k) {
        const int fl = f0 + k * G;
        if (fl < nf) {
          const z2 x = buf[fl * n + b];
          sr[k] += mv.r * x.r - mv.i * x.i;
          si[k] += mv.r * x.i + mv.i * x.r;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < kMaxFib; ++k) {
      const int fl = f0 + k * G;
      if (fl < nf) C[off(tl.f0 + fl, a)] = z2{sr[k], si[k]};
    }
  }
}

// ---------------------------------------------------------------------------
// gram: E[a', a] = sum_k conj(C[pre, a', post]) T[pre, a, post],  k = (pre, post)
// ---------------------------------------------------------------------------
// One workgroup per environment matrix.  Work items = (16x16 output tile,
// K part); with fewer than four tiles K is split across wavefronts and the
// partial tiles are summed in LDS.
// Operands of one k-step of the Gram product for one accumulator tile:
// conj(C)[arow, k] and T[bcol, k], k = pre * Ppost + post.
template <typename T>
struct GramOpnd {
  T ar, ai, br, bi;
};

// Quotient n / d for 0 <= n < 2^31, d >= 1, through a double-precision
// reciprocal and integer correction.
__device__ inline long gram_div(long n, long d, double dinv) {
  long q = (long)((double)n * dinv);
  while (q * d > n) --q;
  while ((q + 1) * d <= n) ++q;
  return q;
}

// Workgroups are dealt to the 8 XCDs (each with its own L2) in turn by
// block index.  Consecutive ops of a launch usually read the same core, so
// block b runs op (b % 8) * per + b / 8: a run of `per` consecutive ops stays
// on one XCD and shares its L2.  The grid has 8 * per blocks; blocks past
// the last op exit.
constexpr int N_XCD = 8;
__device__ inline int xcd_op(int b, int n) {
  const int per = (n + N_XCD - 1) / N_XCD;
  return (b % N_XCD) * per + b / N_XCD;
}

// Gram product for r <= 32 (NB = 1 or 2 row tiles): K is split across the
// four wavefronts, each accumulating every output tile over its quarter (the
// operand rows of a k-step are loaded once and serve NB x NB tiles); the
// partials are summed through LDS.
template <typename T, int NB>
__device__ void gram_small(const GramOp& op, long K, long Ppost, double pinv, gp<const double> Cm,
                           gp<const T> Tm, gp<T> E, T* red /* [4][NB*NB][2][256] */) {
  typedef typename MT<T>::v4 v4;
  const int r = op.r;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = lane & 15, g = lane >> 4;
  constexpr int KU = 4;
  const long kq = 16 * ((K + 63) / 64);  // multiple of 4 * KU
  const long k0 = wave * kq, k1 = k0 + kq < K ? k0 + kq : K;
  v4 accr[NB * NB], acci[NB * NB];
#pragma unroll
  for (int t = 0; t < NB * NB; ++t) {
    accr[t] = v4{0, 0, 0, 0};
    acci[t] = v4{0, 0, 0, 0};
  }
  struct Opnd {
    T ar[NB], ai[NB], br[NB], bi[NB];
  };
  auto load = [&](long kb, Opnd (&o)[KU]) {
#pragma unroll
    for (int u = 0; u < KU; ++u) {
      const long k = kb + 4 * u + g;
#pragma unroll
      for (int t = 0; t < NB; ++t) o[u].ar[t] = o[u].ai[t] = o[u].br[t] = o[u].bi[t] = 0;
      if (k < k1) {
        const long pre = gram_div(k, Ppost, pinv), post = k - pre * Ppost;
        const long base = pre * r * Ppost + post;
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const int row = 16 * t + c;
          if (row < r) {
            const long o2 = base + (long)row * Ppost;
            o[u].ar[t] = (T)Cm[2 * o2];
            o[u].ai[t] = -(T)Cm[2 * o2 + 1];  // conj(C)
            o[u].br[t] = Tm[2 * o2];
            o[u].bi[t] = Tm[2 * o2 + 1];
          }
        }
      }
    }
  };
  Opnd cur[KU], nxt[KU];
  if (k0 < k1) load(k0, cur);
  for (long kb = k0; kb < k1; kb += 4 * KU) {
    if (kb + 4 * KU < k1) load(kb + 4 * KU, nxt);
#pragma unroll
    for (int u = 0; u < KU; ++u)
#pragma unroll
      for (int ti = 0; ti < NB; ++ti)
#pragma unroll
        for (int tj = 0; tj < NB; ++tj)
          cmma<T>(accr[ti * NB + tj], acci[ti * NB + tj], cur[u].ar[ti], cur[u].ai[ti], cur[u].br[tj],
                  cur[u].bi[tj]);
#pragma unroll
    for (int u = 0; u < KU; ++u) cur[u] = nxt[u];
  }
#pragma unroll
  for (int t = 0; t < NB * NB; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = MT<T>::drow(g, q) * 16 + c;
      red[((wave * NB * NB + t) * 2 + 0) * 256 + e] = accr[t][q];
      red[((wave * NB * NB + t) * 2 + 1) * 256 + e] = acci[t][q];
    }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB * 256; e += 256) {
    const int t = e / 256, w = e % 256;
    T sr = 0, si = 0;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      sr += red[((p * NB * NB + t) * 2 + 0) * 256 + w];
      si += red[((p * NB * NB + t) * 2 + 1) * 256 + w];
    }
    const int ti = t / NB, tj = t % NB;
    const int row = 16 * ti + w / 16, col = 16 * tj + w % 16;
    if (row < r && col < r) {
      E[2 * ((long)row * r + col)] = sr;
      E[2 * ((long)row * r + col) + 1] = si;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gram(const GramOp* __restrict__ ops, int n_ops) {
  typedef typename MT<T>::v4 v4;
  const int oi = xcd_op(blockIdx.x, n_ops);
  if (oi >= n_ops) return;
  const GramOp op = ops[oi];
  const int r = op.r;
  const long K = (long)op.Ppre * op.Ppost;
  const long Ppost = op.Ppost;
  const double pinv = 1.0 / (double)Ppost;
  const gp<const T> Tm = gmem(reinterpret_cast<const T*>(op.T));
  const gp<const double> Cm = gmem(op.C);
  const gp<T> E = gmem(reinterpret_cast<T*>(op.E));
  if (r <= 32) {  // uniform per block
    __shared__ T red_small[4 * 4 * 2 * 256];
    if (r <= 16) gram_small<T, 1>(op, K, Ppost, pinv, Cm, Tm, E, red_small);
    else gram_small<T, 2>(op, K, Ppost, pinv, Cm, Tm, E, red_small);
    return;
  }
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
  // KU k-steps per batch; the next batch is read while the current one is
  // multiplied
  constexpr int KU = 4;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int item = wave + 4 * j;
    if (item < n_items) {
      const int tile = item % nt, kp = item / nt;
      const int ti = tile / nb, tj = tile % nb;
      const int arow = 16 * ti + c, bcol = 16 * tj + c;
      const long k0 = kp * kchunk, k1 = k0 + kchunk < K ? k0 + kchunk : K;
      auto load = [&](long kb, GramOpnd<T>(&o)[KU]) {
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const long k = kb + 4 * u + g;
          o[u] = GramOpnd<T>{0, 0, 0, 0};
          if (k < k1) {
            const long pre = gram_div(k, Ppost, pinv), post = k - pre * Ppost;
            const long base = pre * r * Ppost + post;
            if (arow < r) {
              const long oa = base + (long)arow * Ppost;
              o[u].ar = (T)Cm[2 * oa];
              o[u].ai = -(T)Cm[2 * oa + 1];  // conj(C)
            }
            if (bcol < r) {
              const long ob = base + (long)bcol * Ppost;
              o[u].br = Tm[2 * ob];
              o[u].bi = Tm[2 * ob + 1];
            }
          }
        }
      };
      GramOpnd<T> cur[KU], nxt[KU];
      load(k0, cur);
      for (long kb = k0; kb < k1; kb += 4 * KU) {
        if (kb + 4 * KU < k1) load(kb + 4 * KU, nxt);
#pragma unroll
        for (int u = 0; u < KU; ++u) cmma<T>(accr[j], acci[j], cur[u].ar, cur[u].ai, cur[u].br, cur[u].bi);
#pragma unroll
        for (int u = 0; u < KU; ++u) cur[u] = nxt[u];
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

// One workgroup of kSplitThreads lanes: the element-parallel parts (copying
// the singular vectors, the projections) spread over all of them; the
// Gram-Schmidt steps of the completion reduce per wavefront and over the
// workgroup.
constexpr int kSplitThreads = 1024;
constexpr int kSplitWaves = kSplitThreads / 64;
__global__ void __launch_bounds__(kSplitThreads) k_split(const SplitOp* __restrict__ ops) {
  const SplitOp op = ops[blockIdx.x];
  const z2* Th = reinterpret_cast<const z2*>(op.Theta);
  const z2* E = reinterpret_cast<const z2*>(op.E);
  z2* W = reinterpret_cast<z2*>(op.W);
  const int miso = op.iso == 0 ? op.rows : op.cols;     // isometry side
  const int k = op.k, rp = op.rp;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double red[2][kSplitWaves];
  __shared__ double sh_norm;
  // first k columns of W: the leading singular vectors of the isometry side
  for (long e = tid; e < (long)miso * k; e += kSplitThreads) {
    const int i = (int)(e / k), j = (int)(e % k);
    W[(long)i * rp + j] = E[(long)i * op.ld_e + j];
  }
  __syncthreads();
  // completion: unit vectors e_0, e_1, ... projected out of span(W[:, :j]),
  // twice, accepted when the residual norm exceeds 0.5
  int j = k;
  for (int cand = 0; cand < miso && j < rp; ++cand) {
    for (int i = tid; i < miso; i += kSplitThreads) W[(long)i * rp + j] = z2{i == cand ? 1.0 : 0.0, 0.0};
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
    for (int i = tid; i < miso; i += kSplitThreads) {
      const z2 b = W[(long)i * rp + j];
      s2 += b.r * b.r + b.i * b.i;
    }
    s2 = wave_sum(s2);
    if (lane == 0) red[1][wave] = s2;
    __syncthreads();
    if (tid == 0) {
      double t = 0;
      for (int w = 0; w < kSplitWaves; ++w) t += red[1][w];
      sh_norm = sqrt(t);
    }
    __syncthreads();
    if (sh_norm > 0.5) {
      for (int i = tid; i < miso; i += kSplitThreads) {
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
    for (long e = tid; e < (long)op.rows * rp; e += kSplitThreads) {
      const int row = (int)(e / rp), a = (int)(e % rp);
      Cs[cs_at(row, a)] = W[(long)row * rp + a];
    }
    for (long e = tid; e < (long)rp * op.cols; e += kSplitThreads) {  // Cc = W^H Theta
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
    for (long e = tid; e < (long)rp * op.cols; e += kSplitThreads) {  // Cc = W^H
      const int a = (int)(e / op.cols), col = (int)(e % op.cols);
      const z2 w = W[(long)col * rp + a];
      Cc[e] = z2{w.r, -w.i};
    }
    for (long e = tid; e < (long)op.rows * rp; e += kSplitThreads) {  // Cs = Theta W
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

// Non-finite values in FP64 states: block (op, chunk) scans a 1/16 share of
// op's doubles and sets the op's flag (plain vector stores of 1).
__global__ void __launch_bounds__(256) k_finite(const FiniteOp* __restrict__ ops) {
  const FiniteOp op = ops[blockIdx.x];
  const gp<const double> p = gmem(op.p);
  bool bad = false;
  for (long i = (long)blockIdx.y * 256 + threadIdx.x; i < op.n; i += 256L * gridDim.y)
    bad = bad || !isfinite(p[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) *gmem(op.flag) = 1;
}

__global__ void k_clear_flags(int* flags, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) gmem(flags)[i] = 0;
}

__global__ void k_step_inc(int* ctr, int value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ctr = value < 0 ? *ctr + 1 : value;
}

// ---------------------------------------------------------------------------
// launchers (host)
// ---------------------------------------------------------------------------
size_t apply_lds_bytes(int fp64, int nfl, int d1, int d2) {
  return (size_t)apply_lds_elems(nfl, d1, d2) * (fp64 ? sizeof(double) : sizeof(float));
}

// With t0/t1 given, the events are taken by the kernel's own dispatch (start
// and end of its execution), not by separate stream markers.
// mode: 0 complex FP32 (four real products), 1 complex FP64, 2 complex FP32
// with three real products per complex product, 3 complex FP32 on operands
// rounded to BF16
hipError_t launch_apply(int mode, int in_fp64, const ApplyGroup* groups, const ApplyTile* tiles,
                        int n_tiles, const int* step_ctr, size_t lds, hipStream_t s,
                        hipEvent_t t0, hipEvent_t t1) {
  if (n_tiles <= 0) return hipSuccess;
  static bool attr_set = false;
  if (!attr_set) {
    const int cap = kApplyLdsBudget;
    const void* ks[] = {(const void*)k_apply<float, float, 0>, (const void*)k_apply<float, double, 0>,
                        (const void*)k_apply<double, double, 0>, (const void*)k_apply<float, float, 1>,
                        (const void*)k_apply<float, double, 1>, (const void*)k_apply<float, float, 2>,
                        (const void*)k_apply<float, double, 2>, (const void*)k_apply<float, StageIn, 0>,
                        (const void*)k_apply<double, StageIn, 0>, (const void*)k_apply<float, StageIn, 1>,
                        (const void*)k_apply<float, StageIn, 2>};
    for (const void* k : ks) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    attr_set = true;
  }
  auto go = [&](auto kern) {
    if (t0 && t1)
      hipExtLaunchKernelGGL(kern, dim3(n_tiles), dim3(64 * kApplyWaves), (uint32_t)lds, s, t0, t1, 0, groups, tiles,
                            step_ctr);
    else
      hipLaunchKernelGGL(kern, dim3(n_tiles), dim3(64 * kApplyWaves), lds, s, groups, tiles, step_ctr);
  };
  // in_fp64: 0 compute-precision input, 1 the FP64 master, 2 an RK4 stage
  // input formed while staged
  if (mode == 1) {
    if (in_fp64 == 2) go(k_apply<double, StageIn, 0>);
    else go(k_apply<double, double, 0>);
  } else if (mode == 2) {
    if (in_fp64 == 2) go(k_apply<float, StageIn, 1>);
    else if (in_fp64) go(k_apply<float, double, 1>);
    else go(k_apply<float, float, 1>);
  } else if (mode == 3) {
    if (in_fp64 == 2) go(k_apply<float, StageIn, 2>);
    else if (in_fp64) go(k_apply<float, double, 2>);
    else go(k_apply<float, float, 2>);
  } else if (in_fp64 == 2) go(k_apply<float, StageIn, 0>);
  else if (in_fp64) go(k_apply<float, double, 0>);
  else go(k_apply<float, float, 0>);
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

hipError_t launch_qr(const QrOp* ops, int n, int form, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute((const void*)k_qr_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kQrLdsElems * 16);
    (void)hipFuncSetAttribute((const void*)k_qr_blocked<true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, QR_MAX_M * QR_PB * 16);
    (void)hipFuncSetAttribute((const void*)k_qr_formq,
                              hipFuncAttributeMaxDynamicSharedMemorySize, QR_MAX_M * QR_PB * 16);
    attr = true;
  }
  if (form == kQrFormLds) hipLaunchKernelGGL(k_qr_lds, dim3(n), dim3(QR_NT), kQrLdsElems * 16, s, ops);
  else if (form == kQrFormColumns) hipLaunchKernelGGL(k_qr, dim3(n), dim3(QR_NT), 0, s, ops);
  else {
    hipLaunchKernelGGL(k_qr_blocked<true>, dim3(n), dim3(QR_NT), QR_MAX_M * QR_PB * 16, s, ops);
    // Q: columns in groups of QR_NW (n <= 64 columns), after the factoring
    hipLaunchKernelGGL(k_qr_formq, dim3(n, 64 / QR_NW), dim3(QR_NT), QR_MAX_M * QR_PB * 16, s,
                       ops);
  }
  return hipGetLastError();
}

hipError_t launch_absorb(const AbsorbOp* ops, const void* tiles, int n_tiles, size_t lds,
                         hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  static bool attr = false;
  if (!attr) {  // the operator (up to 64 x 64) plus the tile's fibers
    (void)hipFuncSetAttribute((const void*)k_absorb, hipFuncAttributeMaxDynamicSharedMemorySize,
                              kAbsorbLdsMax);
    attr = true;
  }
  hipLaunchKernelGGL(k_absorb, dim3(n_tiles), dim3(256), lds, s, ops,
                     reinterpret_cast<const AbsorbTile*>(tiles));
  return hipGetLastError();
}

hipError_t launch_gram(int fp64, const GramOp* ops, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = N_XCD * ((n + N_XCD - 1) / N_XCD);
  if (fp64) hipLaunchKernelGGL(k_gram<double>, dim3(blocks), dim3(256), 0, s, ops, n);
  else hipLaunchKernelGGL(k_gram<float>, dim3(blocks), dim3(256), 0, s, ops, n);
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

hipError_t launch_finite(const FiniteOp* ops, int n, int* flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_clear_flags, dim3((n + 255) / 256), dim3(256), 0, s, flags, n);
  hipLaunchKernelGGL(k_finite, dim3(n, 16), dim3(256), 0, s, ops);
  return hipGetLastError();
}

hipError_t launch_merge(const MergeOp* op, long n, hipStream_t s) {
  int blocks = (int)std::min<long>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_merge, dim3(blocks, 1), dim3(256), 0, s, op);
  return hipGetLastError();
}
hipError_t launch_split(const SplitOp* op, hipStream_t s) {
  hipLaunchKernelGGL(k_split, dim3(1), dim3(kSplitThreads), 0, s, op);
  return hipGetLastError();
}

size_t combine_tile_bytes() { return sizeof(CombineTile); }
size_t absorb_tile_bytes() { return sizeof(AbsorbTile); }

}  // namespace tenso
