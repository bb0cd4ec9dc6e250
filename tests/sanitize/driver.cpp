// Host-only driver for an AddressSanitizer / UndefinedBehaviorSanitizer build
// of the plan compiler (tenso_host.cpp built with g++, no device code).
// It runs tree construction, generator tables and the device-free plan
// compiler (tenso_plan_query) on real workload term tables, then on a
// deterministic fuzz of malformed trees and generators, and checks that every
// call returns a status instead of crashing.  Kernel launchers are stubs: no
// host-only entry point reaches them.
//
//   driver <table file>...
// Table file (text): M K n_ary rank, K feature dims, n_terms, then per term
// "coef_re coef_im slot n_factors", per factor "end d" and d*d "re im" pairs.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../include/tenso.h"
#include "../../paper_2603_17711_amd/csrc/checks.h"
#include "../../paper_2603_17711_amd/csrc/tenso_internal.h"
#include "../../paper_2603_17711_amd/csrc/vmf.h"

namespace tenso {
#define STUB(...) { std::fprintf(stderr, "kernel launcher reached\n"); std::abort(); }
hipError_t launch_apply(int, int, const ApplyGroup*, const ApplyTile*, int, const int*, size_t,
                        hipStream_t, hipEvent_t, hipEvent_t) STUB()
hipError_t launch_merge(const MergeOp*, long, hipStream_t) STUB()
hipError_t launch_svd_gemm(const SvdGemmOp*, int, int, hipStream_t) STUB()
hipError_t launch_svd_reduce(const SvdGemmOp*, long, hipStream_t) STUB()
hipError_t launch_svd_jacobi(const SvdJacobiOp*, hipStream_t) STUB()
hipError_t launch_svd_finish(const SvdFinishOp*, long, hipStream_t) STUB()
hipError_t launch_split(const SplitOp*, hipStream_t) STUB()
hipError_t launch_presum(int, const PresumOp*, int, const int*, hipStream_t) STUB()
hipError_t launch_combine(int, const CombineOp*, const void*, int, hipStream_t) STUB()
hipError_t launch_qr(const QrOp*, int, int, hipStream_t) STUB()
hipError_t launch_absorb(const AbsorbOp*, const void*, int, size_t, hipStream_t) STUB()
hipError_t launch_gram(int, const GramOp*, int, hipStream_t) STUB()
hipError_t launch_rho(const RhoProg*, int, hipStream_t) STUB()
hipError_t launch_step_inc(int*, int, hipStream_t) STUB()
hipError_t launch_finite(const FiniteOp*, int, int*, hipStream_t) STUB()
hipError_t launch_norms(const NormOp*, int, double*, hipStream_t) STUB()
hipError_t launch_isometry(const IsoOp*, int, double*, hipStream_t) STUB()
hipError_t launch_rho_pure(const double*, int, long, double*, hipStream_t) STUB()
hipError_t launch_zero(void*, size_t, hipStream_t) STUB()
hipError_t launch_reginv(const RegInvOp*, int, hipStream_t) STUB()
hipError_t launch_vproj(const VProjOp*, int, long, hipStream_t) STUB()
hipError_t launch_lincomb(const LinCombOp&, int, hipStream_t) STUB()
hipError_t launch_errnorm(const ErrNormOp&, hipStream_t) STUB()
hipError_t launch_sum_partials(const double*, int, double*, hipStream_t) STUB()
// Shared-memory footprint of an apply tile: the planner only compares it with
// its budget, so any monotone size serves this host-only build.
size_t apply_lds_bytes(int fp64, int nfl, int d1, int d2) {
  const long D1 = 16 * ((d1 + 15) / 16), D2 = 16 * ((d2 + 15) / 16);
  return (size_t)(2 * (nfl * D1 * (D2 + 1) + D1 * (D1 + 1) + D2 * (D2 + 1) + 4 * D1 * 17)) *
         (fp64 ? 8 : 4);
}
}  // namespace tenso

static int g_fail = 0;
#define CHECK(cond)                                                  \
  do {                                                               \
    if (!(cond)) {                                                   \
      std::fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
      ++g_fail;                                                      \
    }                                                                \
  } while (0)

struct Table {
  int M = 0, K = 0, n_ary = 0, rank = 0;
  std::vector<int32_t> dims, slot, nfac, fend;
  std::vector<tenso_c128> coef, mats;
};

static bool read_table(const char* path, Table& T) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  int nt = 0;
  bool ok = std::fscanf(f, "%d %d %d %d", &T.M, &T.K, &T.n_ary, &T.rank) == 4;
  for (int k = 0; ok && k < T.K; ++k) {
    int d;
    ok = std::fscanf(f, "%d", &d) == 1;
    T.dims.push_back(d);
  }
  ok = ok && std::fscanf(f, "%d", &nt) == 1;
  for (int m = 0; ok && m < nt; ++m) {
    tenso_c128 c;
    int s, nf;
    ok = std::fscanf(f, "%lf %lf %d %d", &c.re, &c.im, &s, &nf) == 4;
    T.coef.push_back(c);
    T.slot.push_back(s);
    T.nfac.push_back(nf);
    for (int j = 0; ok && j < nf; ++j) {
      int e, d;
      ok = std::fscanf(f, "%d %d", &e, &d) == 2;
      T.fend.push_back(e);
      for (int q = 0; ok && q < d * d; ++q) {
        tenso_c128 v;
        ok = std::fscanf(f, "%lf %lf", &v.re, &v.im) == 2;
        T.mats.push_back(v);
      }
    }
  }
  std::fclose(f);
  return ok;
}

static void run_table(const Table& T) {
  tenso_tree* tr = nullptr;
  int rc = T.n_ary == 1 ? tenso_tree_train(T.M, T.K, T.dims.data(), T.rank, &tr)
                        : tenso_tree_nary(T.M, T.K, T.dims.data(), T.n_ary, T.rank, &tr);
  CHECK(rc == 0 && tr);
  if (!tr) return;
  tenso_gen* g = nullptr;
  rc = tenso_build_generator(tr, (int)T.coef.size(), T.coef.data(), T.slot.data(), T.nfac.data(),
                             T.fend.data(), T.mats.data(), &g);
  CHECK(rc == 0 && g);
  for (int prec = 0; prec < 2 && g; ++prec)
    for (int method = 0; method < 2; ++method) {
      tenso_plan_opts o{prec, method, method ? 4 : 0};
      size_t sb = 0, wb = 0;
      int64_t nl = 0;
      double fl = 0;
      rc = tenso_plan_query(tr, g, &o, &sb, &wb, &nl, &fl);
      CHECK(rc == 0 || rc == TENSO_EUNSUPPORTED);
      if (rc == 0) CHECK(sb > 0 && wb > 0 && (method == 1 || (nl > 0 && fl > 0)));
    }
  // truncated and perturbed copies of the table: every call returns a status
  std::mt19937 rng(7);
  for (int trial = 0; trial < 200 && g; ++trial) {
    std::vector<int32_t> nfac = T.nfac, fend = T.fend, slot = T.slot;
    int nt = (int)T.coef.size();
    switch (trial % 4) {
      case 0: fend[rng() % fend.size()] = (int32_t)(rng() % 64) - 8; break;
      case 1: nfac[rng() % nfac.size()] = (int32_t)(rng() % 5) - 1; break;
      case 2: nt = (int)(rng() % (T.coef.size() + 1)); break;
      default: slot[rng() % slot.size()] = (int32_t)(rng() % 4) - 2; break;
    }
    // keep the factor count within the arrays the caller really provides
    long need = 0, mats = 0;
    bool inside = true;
    for (int m = 0; m < nt && inside; ++m) {
      if (nfac[m] < 0) break;
      for (int j = 0; j < nfac[m]; ++j) {
        if (need >= (long)fend.size()) { inside = false; break; }
        int e = fend[need++];
        int d = e >= 2 && e - 2 < T.K ? T.dims[e - 2] : (e >= 0 && e < 2 ? T.M : 0);
        mats += (long)d * d;
      }
    }
    if (!inside || mats > (long)T.mats.size()) continue;
    tenso_gen* g2 = nullptr;
    rc = tenso_build_generator(tr, nt, T.coef.data(), slot.data(), nfac.data(), fend.data(),
                               T.mats.data(), &g2);
    CHECK(rc == 0 || rc == TENSO_EINVAL || rc == TENSO_EUNSUPPORTED);
    if (rc == 0) {
      tenso_plan_opts o{1, 0, 0};
      rc = tenso_plan_query(tr, g2, &o, nullptr, nullptr, nullptr, nullptr);
      CHECK(rc == 0 || rc == TENSO_EUNSUPPORTED);
      tenso_gen_destroy(g2);
    }
  }
  tenso_gen_destroy(g);
  tenso_tree_destroy(tr);
}

static void fuzz_trees() {
  std::mt19937 rng(11);
  for (int trial = 0; trial < 2000; ++trial) {
    int n = 1 + (int)(rng() % 9), ne = (int)(rng() % 10);
    std::vector<int32_t> parent(n), end_node(ne), end_dim(ne), br(n);
    for (int s = 0; s < n; ++s) parent[s] = s == 0 ? -1 : (int32_t)(rng() % (n + 2)) - 1;
    for (int e = 0; e < ne; ++e) {
      end_node[e] = (int32_t)(rng() % (n + 1)) - (trial % 17 == 0);
      end_dim[e] = (int32_t)(rng() % 6) - (trial % 13 == 0);
    }
    for (int s = 0; s < n; ++s) br[s] = (int32_t)(rng() % 9);
    tenso_tree* t = nullptr;
    int rc = tenso_build_tree(n, parent.data(), ne, end_node.data(), end_dim.data(),
                              (int)(rng() % 8), trial % 2 ? br.data() : nullptr, &t);
    CHECK(rc == 0 || rc == TENSO_EINVAL);
    if (rc == 0) {
      CHECK(t != nullptr);
      std::vector<int32_t> r(n);
      CHECK(tenso_tree_ranks(t, r.data()) == 0);
      tenso_tree_destroy(t);
    }
  }
}

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) {
    Table T;
    if (!read_table(argv[i], T)) {
      std::fprintf(stderr, "cannot read %s\n", argv[i]);
      return 2;
    }
    run_table(T);
  }
  fuzz_trees();
  std::printf("sanitizer driver: %d failed checks\n", g_fail);
  return g_fail ? 1 : 0;
}
