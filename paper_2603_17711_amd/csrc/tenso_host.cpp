// Host side of the TTN-HEOM library: trees, generators, plan compilation,
// operation lists for the projector-splitting sweeps, descriptor binding and
// the C ABI of include/tenso.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <set>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/tenso.h"
#include "tenso_internal.h"
#include "checks.h"
#include "vmf.h"

namespace tenso {
hipError_t launch_apply(int mode, int in_fp64, const ApplyGroup* groups, const ApplyTile* tiles,
                        int n_tiles, const int* step_ctr, size_t lds, hipStream_t s,
                        hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr);
size_t apply_lds_bytes(int fp64, int nfl, int d1, int d2);
hipError_t launch_merge(const MergeOp* op, long n, hipStream_t s);
hipError_t launch_svd_gemm(const SvdGemmOp* op, int M_tiles, int nsplit, hipStream_t s);
hipError_t launch_svd_reduce(const SvdGemmOp* op, long n_complex, hipStream_t s);
hipError_t launch_svd_jacobi(const SvdJacobiOp* op, hipStream_t s);
hipError_t launch_svd_finish(const SvdFinishOp* op, long n_iso_p, hipStream_t s);
hipError_t launch_split(const SplitOp* op, hipStream_t s);
hipError_t launch_presum(int fp64, const PresumOp* ops, int n, const int* step_ctr, hipStream_t s);
hipError_t launch_combine(int fp64, const CombineOp* ops, const void* tiles, int n_tiles,
                          hipStream_t s);
hipError_t launch_qr(const QrOp* ops, int n, int form, hipStream_t s);
hipError_t launch_absorb(const AbsorbOp* ops, const void* tiles, int n_tiles, size_t lds,
                         hipStream_t s);
hipError_t launch_gram(int fp64, const GramOp* ops, int n, hipStream_t s);
hipError_t launch_rho(const RhoProg* progs, int n, hipStream_t s);
hipError_t launch_step_inc(int* ctr, int value, hipStream_t s);
hipError_t launch_finite(const FiniteOp* ops, int n, int* flags, hipStream_t s);
}  // namespace tenso

using namespace tenso;
using cd = std::complex<double>;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;
struct TErr {
  int code;
  std::string msg;
};
[[noreturn]] static void fail(int code, const std::string& m) { throw TErr{code, m}; }
static void hipchk(hipError_t e, const char* where) {
  if (e != hipSuccess) fail(TENSO_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}
template <class F>
static int guard(F&& f) {
  try {
    f();
    return TENSO_OK;
  } catch (const TErr& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return TENSO_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return TENSO_EINVAL;
  }
}

// ---------------------------------------------------------------------------
// tree
// ---------------------------------------------------------------------------
struct Leg {
  int kind;  // 0 parent bond, 1 end, 2 child bond
  int id;    // parent node / end index / child node
};

struct tenso_tree {
  int n = 0, n_ends = 0;
  std::vector<int> parent, end_node, end_dim, rank;
  std::vector<std::vector<int>> children, ends;
  std::vector<std::vector<Leg>> legs;
  std::vector<std::vector<char>> in_sub;  // [node][end]

  int leg_dim(int s, const Leg& l) const {
    if (l.kind == 0) return rank[s];
    if (l.kind == 1) return end_dim[l.id];
    return rank[l.id];
  }
  std::vector<int> shape(int s) const {
    std::vector<int> d;
    for (auto& l : legs[s]) d.push_back(leg_dim(s, l));
    return d;
  }
  long size(int s) const {
    long p = 1;
    for (int d : shape(s)) p *= d;
    return p;
  }
  int leg_of_child(int s, int c) const {
    for (size_t i = 0; i < legs[s].size(); ++i)
      if (legs[s][i].kind == 2 && legs[s][i].id == c) return (int)i;
    fail(TENSO_EINVAL, "child not found");
  }
  void finish(int max_rank, const int32_t* bond_rank) {
    children.assign(n, {});
    ends.assign(n, {});
    for (int s = 1; s < n; ++s) children[parent[s]].push_back(s);
    for (int e = 0; e < n_ends; ++e) ends[end_node[e]].push_back(e);
    legs.assign(n, {});
    for (int s = 0; s < n; ++s) {
      if (s > 0) legs[s].push_back({0, parent[s]});
      for (int e : ends[s]) legs[s].push_back({1, e});
      for (int c : children[s]) legs[s].push_back({2, c});
      if (legs[s].size() > 8) fail(TENSO_EUNSUPPORTED, "a core has more than 8 legs");
      if (legs[s].size() < 2) fail(TENSO_EINVAL, "a core needs at least two legs");
    }
    in_sub.assign(n, std::vector<char>(n_ends, 0));
    for (int s = n - 1; s >= 0; --s) {
      for (int e : ends[s]) in_sub[s][e] = 1;
      for (int c : children[s])
        for (int e = 0; e < n_ends; ++e) in_sub[s][e] |= in_sub[c][e];
    }
    rank.assign(n, 0);
    for (int c = 1; c < n; ++c) {
      int r = bond_rank ? bond_rank[c] : max_rank;
      if (r < 1) fail(TENSO_EINVAL, "bond ranks must be >= 1");
      rank[c] = r;
    }
    clamp();
  }
  void clamp() {
    bool changed = true;
    while (changed) {
      changed = false;
      for (int c = 1; c < n; ++c) {
        int p = parent[c];
        long lo = 1, hi = 1;
        for (size_t i = 1; i < legs[c].size(); ++i) lo *= leg_dim(c, legs[c][i]);
        for (auto& l : legs[p])
          if (!(l.kind == 2 && l.id == c)) hi *= leg_dim(p, l);
        long r = std::min<long>(rank[c], std::min(lo, hi));
        if (r != rank[c]) {
          rank[c] = (int)r;
          changed = true;
        }
      }
    }
  }
};

static tenso_tree* make_tree(int n, const int32_t* parent, int n_ends, const int32_t* end_node,
                             const int32_t* end_dim, int max_rank, const int32_t* bond_rank) {
  if (n < 1 || n_ends < 2) fail(TENSO_EINVAL, "need >= 1 node and >= 2 ends");
  if (parent[0] != -1) fail(TENSO_EINVAL, "parent[0] must be -1");
  for (int s = 1; s < n; ++s)
    if (parent[s] < 0 || parent[s] >= s) fail(TENSO_EINVAL, "parent[s] must be in [0, s)");
  for (int e = 0; e < n_ends; ++e) {
    if (end_node[e] < 0 || end_node[e] >= n) fail(TENSO_EINVAL, "end attached to a bad node");
    if (end_dim[e] < 1) fail(TENSO_EINVAL, "end dims must be >= 1");
  }
  if (end_node[0] != 0 || end_node[1] != 0) fail(TENSO_EINVAL, "ket and bra ends must sit on the root");
  if (end_dim[1] != end_dim[0] && end_dim[1] != 1)
    fail(TENSO_EINVAL, "the bra end has the ket's dimension (a density) or 1 (a wavefunction)");
  if (max_rank < 1 && !bond_rank) fail(TENSO_EINVAL, "max_rank must be >= 1");
  auto t = std::make_unique<tenso_tree>();
  t->n = n;
  t->n_ends = n_ends;
  t->parent.assign(parent, parent + n);
  t->end_node.assign(end_node, end_node + n_ends);
  t->end_dim.assign(end_dim, end_dim + n_ends);
  t->finish(max_rank, bond_rank);
  return t.release();
}

// ---------------------------------------------------------------------------
// generator
// ---------------------------------------------------------------------------
typedef std::vector<std::pair<int, int>> Key;  // sorted (end, matrix id)

struct tenso_gen {
  struct Term {
    cd coef;
    int slot;
    Key f;
  };
  std::vector<Term> terms;
  std::vector<std::vector<cd>> mats;
  std::vector<int> mat_dim;
  int n_slots = 0;
  int n_ends = 0;
  std::vector<int> end_dim;
};

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
static const uint64_t OFF_MASK = (1ull << 56) - 1;
// Largest ps2 two-site tensor (elements at the rank cap): ENOMEM beyond.
static constexpr long kPs2ThetaMax = 1L << 26;
// Most summed-index ranges of one ps2 SVD product.
static constexpr int kSvdMaxSplit = 8;
enum { TAG_ABS = 0, TAG_STATE = 2, TAG_WS = 3, TAG_TERM = 4, TAG_RNODE = 5 };
static inline void* tagp(int tag, uint64_t off) { return (void*)(((uint64_t)tag << 56) | off); }

struct LaunchRec {
  int kind;
  int in_fp64;
  int first, count;    // descriptors
  int tfirst, tcount;  // tiles
  size_t lds;
  double flops = 0;    // algorithmic flops of an apply launch (8 per complex MAC)
  double bytes = 0;    // algorithmic HBM bytes of an apply launch
  int amode = 0;       // apply launches of FP32 plans: 0 four real products per complex
                       // one, 2 three (TENSO_FP32_3M), 3 BF16-rounded operands (TENSO_BF16)
};
enum { LK_APPLY, LK_PRESUM, LK_COMBINE, LK_QR, LK_ABSORB, LK_GRAM, LK_RHO, LK_REGINV, LK_VPROJ };

// Elements per combine workgroup (256 threads, one element each), so that
// loads of its elements' partial outputs are in flight together instead of
// one element's round trip after another
constexpr long kCombineTile = 256;
// Core elements per absorb workgroup (the fibres of a tile times the leg):
// short tiles for a single instance, whose chain of launches is latency-bound;
// longer ones in a batch, where the workgroups of many instances fill the GPU
inline int absorb_tile_elems(int par_target) { return par_target >= 64 ? 256 : 1024; }

struct CombineTileH {
  int op;
  int pad;
  long e0, e1;
};
struct AbsorbTileH {
  int op;
  int f0, f1;
};

struct Program {
  std::vector<TermRef> terms;
  std::vector<double> credit;  // per term: generator terms it stands for (work accounting)
  std::vector<ApplyGroup> groups;
  std::vector<ApplyTile> atiles;
  std::vector<PresumOp> presums;
  std::vector<CombineOp> combines;
  std::vector<CombineTileH> ctiles;
  std::vector<QrOp> qrs;
  std::vector<AbsorbOp> absorbs;
  std::vector<AbsorbTileH> abtiles;
  std::vector<GramOp> grams;
  std::vector<RhoNode> rnodes;
  std::vector<RhoProg> rprogs;
  std::vector<RegInvOp> reginvs;
  std::vector<VProjOp> vprojs;
  std::vector<LaunchRec> launches;
};

// Device copy of a program (descriptor arena).
struct DevProgram {
  char* arena = nullptr;
  size_t bytes = 0;
  bool external = false;  // arena owned by the caller: never grown or freed here
  size_t o_terms, o_groups, o_atiles, o_presums, o_combines, o_ctiles, o_qrs, o_absorbs, o_abtiles,
      o_grams, o_rnodes, o_rprogs, o_reginvs, o_vprojs;
  std::vector<LaunchRec> launches;
  DevProgram() = default;
  DevProgram(char* a, size_t b) : arena(a), bytes(b), external(true) {}
  DevProgram(const DevProgram&) = delete;
  DevProgram& operator=(const DevProgram&) = delete;
  ~DevProgram() {
    if (arena && !external) (void)hipFree(arena);
  }
};

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Drive table of one dopri5 step: the value of slot k at stage i (time
// t + c_i h) sits at [k][4 i], read by the contraction with the step counter
// set to i; the ps2 steps of the mixed strategy use [k][0..4] (quarter steps).
static constexpr int kVmfDriveLd = 4 * 6 + 1;

// operand reference resolved when a program is built
struct ORef {
  int kind = 0;  // 0 identity, 1 factor, 2 down slot, 3 up slot, 4 bond density (vmf),
                 // 5 down channel D0 of `node`, 6 up channel U0 of `node`,
                 // 7 partner channel `idx` of `node`
  int node = 0, idx = 0;
};

struct Recipe {  // effective generator on one tensor (node core, bond or edge)
  struct G {
    int l1, l2;
    std::vector<std::pair<int, std::pair<ORef, ORef>>> pair_terms;  // (term, (A, B))
    std::vector<std::pair<int, ORef>> sa, sb;                       // singles on l1 / l2
  };
  std::vector<int> dims;
  std::vector<G> groups;
};

// Term grouping: pair terms of a group that carry the same operator on one
// leg satisfy sum_m c_m(t) A (x) B_m = A (x) (sum_m c_m(t) B_m), so each such
// cluster costs one pair of products on a presummed operator.  The shared
// side is the one with fewer distinct operators.
struct PairCluster {
  int shared_side;  // 0: operator on l1 shared, others on l2; 1: the reverse
  ORef shared;
  std::vector<std::pair<int, ORef>> others;  // (term, operator on the other leg)
};

static bool same_ref(const ORef& a, const ORef& b) {
  return a.kind == b.kind && a.node == b.node && a.idx == b.idx;
}

static std::vector<PairCluster> cluster_pairs(const Recipe::G& g) {
  auto distinct = [&](int side) {
    std::vector<ORef> seen;
    for (auto& pt : g.pair_terms) {
      const ORef& o = side == 0 ? pt.second.first : pt.second.second;
      bool found = false;
      for (auto& x : seen) found = found || same_ref(x, o);
      if (!found) seen.push_back(o);
    }
    return seen.size();
  };
  const int side = distinct(1) < distinct(0) ? 1 : 0;
  std::vector<PairCluster> out;
  for (auto& pt : g.pair_terms) {
    const ORef& key = side == 0 ? pt.second.first : pt.second.second;
    const ORef& oth = side == 0 ? pt.second.second : pt.second.first;
    PairCluster* c = nullptr;
    for (auto& x : out)
      if (same_ref(x.shared, key)) c = &x;
    if (!c) {
      out.push_back({side, key, {}});
      c = &out.back();
    }
    c->others.push_back({pt.first, oth});
  }
  return out;
}

// One step of a compiled program (its launches plus the step-counter
// advance) captured as a HIP graph, so that a step costs one graph launch
// instead of hundreds of kernel launches.  Capture happens on a private
// stream (the caller's may be the null stream, which cannot capture); the
// graph is launched on the caller's stream.  The captured launches hold
// device addresses bound at capture time: any re-upload of the program
// resets the graph.
// A step may consist of several independent programs (parts of a batch):
// they are captured as parallel branches (fork from the capture stream, one
// side stream per further part, join before the counter advance).
struct StepGraph {
  bool enabled = true;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev;  // [0] fork, [k] join of part k
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
  }
  ~StepGraph() {
    reset();
    if (cap) (void)hipStreamDestroy(cap);
    for (auto x : side) (void)hipStreamDestroy(x);
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

struct tenso_plan {
  tenso_tree tree;   // current ranks
  tenso_tree cap;    // capacity ranks (sizes every buffer; = tree for ps1)
  tenso_gen gen;
  tenso_plan_opts opts;
  std::vector<int> slot_r;  // env slot stride (capacity rank) per node
  int fp64 = 0;
  int amode = 0;   // launch_apply mode of the FP32 contractions (2: TENSO_FP32_3M, 3: TENSO_BF16)
  size_t tsz = 8;  // bytes per complex in compute precision
  int max_dim = 1;
  // env slots
  std::vector<std::vector<Key>> dkeys, ukeys;
  std::vector<std::map<Key, int>> dmap, umap;
  std::vector<std::vector<int>> term_d, term_u;  // [node][term] -> slot, -1 (no factor on
                                                 // that side) or kInChannel
  // Channels of the operator on every bond (the tree-operator form of the
  // generator): the sum, with coefficients, of every time-independent term
  // entirely inside the subtree (down, D0) or entirely outside it (up, U0)
  // costs one environment instead of one per distinct operator.
  std::vector<char> has_d0, has_u0;
  // Partner channels of the down side: a time-independent term with one
  // factor inside the subtree and every other factor on the root's ends
  // (a system operator P) is summed, with its coefficient, into the channel
  // D_P of the bond; P's environment stays a plain up slot.  gkeys[x]: the
  // keys P, term_g[x][m]: the term's channel (-1: none).
  std::vector<std::vector<Key>> gkeys;
  std::vector<std::map<Key, int>> gmap;
  std::vector<std::vector<int>> term_g;
  // constant buffer (factor matrices in both precisions)
  void* cbuf = nullptr;
  std::vector<size_t> mat_off64, mat_off32;
  // state layout
  std::vector<size_t> core_off;  // bytes
  size_t state_bytes = 0;
  // workspace layout
  std::vector<size_t> envd_off, envu_off;
  size_t ws_presum = 0, ws_xin = 0, ws_acc = 0, ws_parts = 0, ws_envscr = 0, ws_bond = 0,
         ws_qrv = 0, ws_qrtau = 0, ws_rhovec = 0, ws_rhoout = 0, ws_ctr = 0, ws_drive = 0,
         ws_check = 0, ws_bytes = 0;
  size_t presum_cap = 0, parts_cap = 0, envscr_cap = 0, qrv_cap = 0;
  size_t ws_theta = 0, ws_W = 0, theta_cap = 0, W_cap = 0, svd_side = 0;
  // ps2 SVD scratch: range-finder and projection blocks (side x 64, column-
  // major), split-K partials, QR scratch for sides above the blocked QR,
  // the small factors, singular values, isometry-side vectors, and the
  // decision record
  size_t ws_svd_y = 0, ws_svd_z = 0, ws_svd_part = 0, ws_svd_qrv = 0, ws_svd_r = 0,
         ws_svd_up = 0, ws_svd_wp = 0, ws_svd_sig = 0, ws_svd_tau = 0, ws_svd_norm = 0,
         ws_svd_e = 0, ws_svd_rec = 0;
  void* opbuf = nullptr;  // device scratch for single-op descriptors (ps2): 8 slots of
                          // 512 bytes, then 4 slots for the SVD
  int par_target = 64;  // tiles wanted per apply (single-instance latency)
  // RK4 sub-flows form each stage's input inside the next contraction (one
  // combine per sub-flow) rather than with a combine per stage: fewer launches
  // on a latency-bound chain, more input traffic; batches turn it off
  bool fuse_stages = true;
  // ... up to this many partial-output elements per stage (parts x core
  // size): every contraction tile re-reads the parts of the slice it stages,
  // which outgrows one combine pass on large cores (measured: cores of 4096
  // elements in up to 8 parts gain, cores of 64000 in 5 parts lose)
  long fuse_max_elems = 1L << 16;
  int built_target = -1;  // par_target the cached programs were built with
  bool built_fuse = true;  // fuse_stages the cached programs were built with
  double tile_work = 16e6;        // flops per apply tile
  bool tile_work_set = false;     // set by the caller (else batches use their default)
  double built_tile_work = -1;    // tile_work the cached programs were built with
  // compiled programs (host descriptors with tagged pointers, device copies)
  std::unique_ptr<Program> prog_step, prog_init;
  std::unique_ptr<DevProgram> dev_step, dev_init;
  std::map<int, std::unique_ptr<DevProgram>> dev_apply;
  std::unique_ptr<DevProgram> dev_rho;
  // ps2: uploaded sub-flow programs keyed by sub-flow and current bond ranks,
  // valid for one binding (buffers, dt, drive, tile size)
  std::map<std::string, std::unique_ptr<DevProgram>> ps2_progs;
  const void* ps2_state = nullptr;
  const void* ps2_ws = nullptr;
  const double* ps2_drive = nullptr;
  double ps2_dt = 0, ps2_tile = -1;
  int ps2_ld = -1;
  // binding of the step program
  void* b_state = nullptr;
  void* b_ws = nullptr;
  double b_dt = -1;
  const double* b_drive = nullptr;
  int b_ld = -1;
  std::vector<int32_t> rank_log;
  StepGraph graph;  // captured step program (replayed per step)
  // direct (vmf) integration: while a vmf program is built, a parent leg with
  // no factor of a term outside the subtree carries the bond density rather
  // than the identity (the non-root cores are not orthonormal toward it)
  bool vmf_rho = false;
  bool vmf_ok = false;  // layout holds the vmf areas (FP64 ps1 / ps2 / vmf plans)
  std::vector<size_t> vmf_rho_off, vmf_rinv_off, vmf_s_off, vmf_node_parts, vmf_node_presum;
  size_t ws_vmf_ys = 0, ws_vmf_k = 0, ws_vmf_kout = 0, ws_vmf_part = 0, ws_vmf_err = 0,
         ws_vmf_segs = 0, ws_vmf_dtab = 0;
  int vmf_chunks = 1;      // workgroup chunks of the largest core (segment kernels)
  std::unique_ptr<DevProgram> dev_vmf;
  StepGraph vmf_graph;     // the derivative program captured once it has run eagerly
  bool vmf_eager_done = false;
  std::vector<int> vmf_ranks;   // ranks the cached vmf program was built for
  double vmf_reg = -1;
  const void* vmf_ws = nullptr;
  int64_t vmf_accepted = 0, vmf_rejected = 0;
  double vmf_h = 0;        // proposed dopri5 step (0: none yet)
  int mix_phase = 0;       // mixed strategy: 0 auxiliary ps2, 1 vmf
  int mix_switch = -1;     // steps of ps2 before the switch (-1: not yet)
  int mix_ps2_steps = 0;
  double ps2_atol = 0, ps2_ratio = 0;  // ps2 truncation by an absolute threshold (ratio > 0)
  void reset_integrators() {
    vmf_accepted = vmf_rejected = 0;
    vmf_h = 0;
    mix_phase = 0;
    mix_switch = -1;
    mix_ps2_steps = 0;
  }

  ~tenso_plan() {
    if (cbuf) (void)hipFree(cbuf);
    if (opbuf) (void)hipFree(opbuf);
  }
};

// -- slot analysis ----------------------------------------------------------
static Key restrict_key(const tenso_tree& t, const Key& k, int node, bool inside) {
  Key r;
  for (auto& p : k)
    if ((bool)t.in_sub[node][p.first] == inside) r.push_back(p);
  return r;
}

static int key_mat(const Key& k, int end) {
  for (auto& p : k)
    if (p.first == end) return p.second;
  return -1;
}

// Env slots per bond: one per distinct restricted key of the terms that act on
// both sides of the bond (or carry a drive slot); the time-independent terms
// on one side only go into that side's channel (term_d / term_u =
// kInChannel).  Every slot a bond's environments need from a neighbouring
// bond exists there: a term with factors on both sides of bond x also has
// factors on both sides of every bond between them.
static constexpr int kInChannel = -2;
static constexpr int kInGroup = -3;  // term_d: the term is in a partner channel (term_g)
// Recipe term indices: m >= 0 a generator term; m = -w a channel standing for
// w generator terms (coefficient 1, no drive; credited as w terms of work).
static double term_weight(int m) { return m < 0 ? (double)-m : 1.0; }
static void analyse_slots(tenso_plan& P) {
  const tenso_tree& t = P.tree;
  const int nt = (int)P.gen.terms.size();
  P.dkeys.assign(t.n, {});
  P.ukeys.assign(t.n, {});
  P.dmap.assign(t.n, {});
  P.umap.assign(t.n, {});
  P.term_d.assign(t.n, std::vector<int>(nt, -1));
  P.term_u.assign(t.n, std::vector<int>(nt, -1));
  P.has_d0.assign(t.n, 0);
  P.has_u0.assign(t.n, 0);
  P.gkeys.assign(t.n, {});
  P.gmap.assign(t.n, {});
  P.term_g.assign(t.n, std::vector<int>(nt, -1));
  for (int x = 1; x < t.n; ++x) {
    for (int m = 0; m < nt; ++m) {
      const Key& k = P.gen.terms[m].f;
      Key kd = restrict_key(t, k, x, true), ku = restrict_key(t, k, x, false);
      const bool fixed = P.gen.terms[m].slot < 0;
      bool at_root = !ku.empty();
      for (auto& f : ku) at_root = at_root && t.end_node[f.first] == 0;
      if (fixed && kd.size() == 1 && at_root) {  // a partner channel
        auto gi = P.gmap[x].find(ku);
        if (gi == P.gmap[x].end()) {
          gi = P.gmap[x].emplace(ku, (int)P.gkeys[x].size()).first;
          P.gkeys[x].push_back(ku);
        }
        P.term_g[x][m] = gi->second;
        P.term_d[x][m] = kInGroup;
        auto it = P.umap[x].find(ku);
        if (it == P.umap[x].end()) {
          it = P.umap[x].emplace(ku, (int)P.ukeys[x].size()).first;
          P.ukeys[x].push_back(ku);
        }
        P.term_u[x][m] = it->second;
        continue;
      }
      if (fixed && ku.empty()) {
        P.term_d[x][m] = kInChannel;
        P.has_d0[x] = 1;
        continue;
      }
      if (fixed && kd.empty()) {
        P.term_u[x][m] = kInChannel;
        P.has_u0[x] = 1;
        continue;
      }
      if (!kd.empty()) {
        auto it = P.dmap[x].find(kd);
        if (it == P.dmap[x].end()) {
          it = P.dmap[x].emplace(kd, (int)P.dkeys[x].size()).first;
          P.dkeys[x].push_back(kd);
        }
        P.term_d[x][m] = it->second;
      }
      if (!ku.empty()) {
        auto it = P.umap[x].find(ku);
        if (it == P.umap[x].end()) {
          it = P.umap[x].emplace(ku, (int)P.ukeys[x].size()).first;
          P.ukeys[x].push_back(ku);
        }
        P.term_u[x][m] = it->second;
      }
    }
  }
}

// operand of a restricted key on leg `l` of node s (the key lives on the legs of s)
static ORef leg_ref_for_key(const tenso_plan& P, int s, const Leg& l, const Key& key) {
  const tenso_tree& t = P.tree;
  ORef r;
  if (l.kind == 1) {
    int m = key_mat(key, l.id);
    if (m >= 0) {
      r.kind = 1;
      r.idx = m;
    }
  } else if (l.kind == 2) {
    Key k = restrict_key(t, key, l.id, true);
    if (!k.empty()) {
      r.kind = 2;
      r.node = l.id;
      r.idx = P.dmap[l.id].at(k);
    }
  } else {
    Key k = restrict_key(t, key, s, false);
    if (!k.empty()) {
      r.kind = 3;
      r.node = s;
      r.idx = P.umap[s].at(k);
    } else if (P.vmf_rho) {
      r.kind = 4;
      r.node = s;
    }
  }
  return r;
}

// Group the per-term leg operands of a tensor with legs of dimensions `dims`:
// pair terms by leg pair, single-leg terms into the presummed sides of a group
// holding their leg (term indices as for term_weight).
static Recipe build_groups(const std::vector<int>& dims,
                           const std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>>& tl) {
  Recipe R;
  R.dims = dims;
  std::map<std::pair<int, int>, int> gidx;
  std::vector<std::vector<std::pair<int, ORef>>> singles(dims.size());
  for (auto& te : tl) {
    const int m = te.first;
    const auto& nz = te.second;
    if (nz.empty()) fail(TENSO_EINVAL, "term with no factor in the network");
    if (nz.size() > 2)
      fail(TENSO_EUNSUPPORTED, "a term acts on more than two legs of one core");
    if (nz.size() == 1) {
      singles[nz[0].first].push_back({m, nz[0].second});
    } else {
      auto key = std::make_pair(nz[0].first, nz[1].first);
      auto it = gidx.find(key);
      if (it == gidx.end()) {
        it = gidx.emplace(key, (int)R.groups.size()).first;
        Recipe::G g;
        g.l1 = key.first;
        g.l2 = key.second;
        R.groups.push_back(g);
      }
      R.groups[it->second].pair_terms.push_back({m, {nz[0].second, nz[1].second}});
    }
  }
  for (int l = 0; l < (int)dims.size(); ++l) {
    if (singles[l].empty()) continue;
    int gi = -1;
    bool first_leg = false;
    for (int i = 0; i < (int)R.groups.size(); ++i) {
      if (R.groups[i].l1 == l) {
        gi = i;
        first_leg = true;
        break;
      }
      if (R.groups[i].l2 == l) {
        gi = i;
        first_leg = false;
        break;
      }
    }
    if (gi < 0) {
      Recipe::G g;
      int other = l == 0 ? 1 : 0;
      g.l1 = std::min(l, other);
      g.l2 = std::max(l, other);
      R.groups.push_back(g);
      gi = (int)R.groups.size() - 1;
      first_leg = g.l1 == l;
    }
    auto& dst = first_leg ? R.groups[gi].sa : R.groups[gi].sb;
    dst.insert(dst.end(), singles[l].begin(), singles[l].end());
  }
  return R;
}

// Channel operands on a list of legs: D0 of every child leg's subtree and U0
// of every parent leg's node.  A D0 channel on a leg of node s also carries
// the density rho_s on s's parent leg while a vmf program is built (the
// channel's terms have nothing outside s), unless that leg is `open`.
static void add_channels(const tenso_plan& P, const std::vector<std::pair<int, Leg>>& legs, int open,
                         std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>>& tl) {
  for (int i = 0; i < (int)legs.size(); ++i) {
    if (i == open) continue;
    const int node = legs[i].first;
    const Leg& l = legs[i].second;
    if (l.kind == 2 && P.has_d0[l.id]) {
      int w = 0;
      for (int m = 0; m < (int)P.gen.terms.size(); ++m) w += P.term_d[l.id][m] == kInChannel;
      ORef o;
      o.kind = 5;
      o.node = l.id;
      std::vector<std::pair<int, ORef>> nz{{i, o}};
      if (P.vmf_rho && node != 0)
        for (int j = 0; j < (int)legs.size(); ++j)
          if (j != open && legs[j].first == node && legs[j].second.kind == 0) {
            ORef r;
            r.kind = 4;
            r.node = node;
            nz.push_back({j, r});
            if (nz[1].first < nz[0].first) std::swap(nz[0], nz[1]);
          }
      tl.push_back({-w, nz});
    } else if (l.kind == 0 && P.has_u0[node]) {
      int w = 0;
      for (int m = 0; m < (int)P.gen.terms.size(); ++m) w += P.term_u[node][m] == kInChannel;
      ORef o;
      o.kind = 6;
      o.node = node;
      tl.push_back({-w, {{i, o}}});
    }
  }
}

// A partner channel that holds term m on one of the legs (a child leg whose
// bond sums m into its channel D_P): (leg, child, channel), or leg -1.
static int group_size(const tenso_plan& P, int x, int gi) {
  int w = 0;
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) w += P.term_g[x][m] == gi;
  return w;
}

struct GroupUse {
  int leg, child, idx;
  bool operator<(const GroupUse& o) const {
    return std::tie(leg, child, idx) < std::tie(o.leg, o.child, o.idx);
  }
};
static GroupUse held_by_group(const tenso_plan& P, const std::vector<std::pair<int, Leg>>& legs,
                              int open, int m) {
  for (int i = 0; i < (int)legs.size(); ++i) {
    const Leg& l = legs[i].second;
    if (i != open && l.kind == 2 && P.term_g[l.id][m] >= 0) return {i, l.id, P.term_g[l.id][m]};
  }
  return {-1, 0, 0};
}

// The partner channels used on a list of legs, each as one term: D_P of the
// child leg, with P's operators on the other legs (its up slot on a parent
// leg, its factors on the root's ends).
static void add_groups(const tenso_plan& P, const std::vector<std::pair<int, Leg>>& legs, int open,
                       const std::set<GroupUse>& used,
                       std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>>& tl) {
  for (const GroupUse& u : used) {
    std::vector<std::pair<int, ORef>> nz;
    for (int j = 0; j < (int)legs.size(); ++j) {
      if (j == open) continue;
      if (j == u.leg) {
        ORef o;
        o.kind = 7;
        o.node = u.child;
        o.idx = u.idx;
        nz.push_back({j, o});
        continue;
      }
      ORef o = leg_ref_for_key(P, legs[j].first, legs[j].second, P.gkeys[u.child][u.idx]);
      if (o.kind) nz.push_back({j, o});
    }
    tl.push_back({-group_size(P, u.child, u.idx), nz});
  }
}

// Whether term m sits in a channel on one of the legs (all its factors
// inside a child leg's subtree, or all outside a parent leg's node).
static bool in_channel(const tenso_plan& P, const std::vector<std::pair<int, Leg>>& legs, int m) {
  for (auto& nl : legs) {
    const Leg& l = nl.second;
    if (l.kind == 2 && P.term_d[l.id][m] == kInChannel) return true;
    if (l.kind == 0 && P.term_u[nl.first][m] == kInChannel) return true;
  }
  return false;
}

// Effective-generator recipe over a list of (node, leg) legs: every term not
// held by a channel, plus the channels.
static Recipe make_recipe(const tenso_plan& P, const std::vector<std::pair<int, Leg>>& legs,
                          const std::vector<int>& dims) {
  std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>> tl;
  std::set<GroupUse> used;
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) {
    if (in_channel(P, legs, m)) continue;
    const GroupUse g = held_by_group(P, legs, -1, m);
    if (g.leg >= 0) {
      used.insert(g);
      continue;
    }
    const Key& k = P.gen.terms[m].f;
    std::vector<std::pair<int, ORef>> nz;
    for (int i = 0; i < (int)legs.size(); ++i) {
      ORef o = leg_ref_for_key(P, legs[i].first, legs[i].second, k);
      if (o.kind) nz.push_back({i, o});
    }
    tl.push_back({m, nz});
  }
  add_channels(P, legs, -1, tl);
  add_groups(P, legs, -1, used, tl);
  return build_groups(dims, tl);
}

// The sum that defines a channel, as a recipe over the legs of `node` with
// leg `open` left alone: D0(x) on core x (open = its parent leg): the
// channels D0 of its children and every channel term of x that no child's
// channel holds; U0(x) on core p = parent(x) (open = the leg to x): U0(p),
// the D0 of x's siblings, and every term of U0(x) that neither holds.
static Recipe channel_recipe(const tenso_plan& P, int node, int open, int x, bool down) {
  const tenso_tree& t = P.tree;
  std::vector<std::pair<int, Leg>> legs;
  for (auto& l : t.legs[node]) legs.push_back({node, l});
  std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>> tl;
  std::set<GroupUse> used;
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) {
    if ((down ? P.term_d[x][m] : P.term_u[x][m]) != kInChannel) continue;
    const GroupUse gu = held_by_group(P, legs, open, m);
    if (gu.leg >= 0) {
      used.insert(gu);
      continue;
    }
    bool held = false;
    for (int i = 0; i < (int)legs.size(); ++i) {
      if (i == open) continue;
      const Leg& l = legs[i].second;
      if (l.kind == 2 && P.term_d[l.id][m] == kInChannel) held = true;
      if (l.kind == 0 && P.term_u[node][m] == kInChannel) held = true;
    }
    if (held) continue;
    const Key& k = P.gen.terms[m].f;
    std::vector<std::pair<int, ORef>> nz;
    for (int i = 0; i < (int)legs.size(); ++i) {
      if (i == open) continue;
      ORef o = leg_ref_for_key(P, node, legs[i].second, k);
      if (o.kind) nz.push_back({i, o});
    }
    tl.push_back({m, nz});
  }
  add_channels(P, legs, open, tl);
  add_groups(P, legs, open, used, tl);
  return build_groups(t.shape(node), tl);
}

// The sum that defines partner channel gi of bond x, over the legs of core
// x (its parent leg left alone): the same channel of every child that holds
// some of its terms, and c_m F_m for its terms whose factor sits on an end
// of x.
static Recipe group_recipe(const tenso_plan& P, int x, int gi) {
  const tenso_tree& t = P.tree;
  std::vector<std::pair<int, Leg>> legs;
  for (auto& l : t.legs[x]) legs.push_back({x, l});
  std::vector<std::pair<int, std::vector<std::pair<int, ORef>>>> tl;
  std::set<std::pair<int, int>> kids;  // (leg, child)
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) {
    if (P.term_g[x][m] != gi) continue;
    const GroupUse gu = held_by_group(P, legs, 0, m);
    if (gu.leg >= 0) {
      kids.insert({gu.leg, gu.child});
      continue;
    }
    std::vector<std::pair<int, ORef>> nz;
    for (int i = 1; i < (int)legs.size(); ++i) {
      ORef o = leg_ref_for_key(P, x, legs[i].second, P.gen.terms[m].f);
      if (o.kind) nz.push_back({i, o});
    }
    tl.push_back({m, nz});
  }
  for (auto& k : kids) {
    ORef o;
    o.kind = 7;
    o.node = k.second;
    o.idx = P.gmap[k.second].at(P.gkeys[x][gi]);
    tl.push_back({-group_size(P, k.second, o.idx), {{k.first, o}}});
  }
  return build_groups(t.shape(x), tl);
}

static Recipe node_recipe(const tenso_plan& P, int s) {
  std::vector<std::pair<int, Leg>> legs;
  for (auto& l : P.tree.legs[s]) legs.push_back({s, l});
  return make_recipe(P, legs, P.tree.shape(s));
}

static Recipe bond_recipe(const tenso_plan& P, int c) {
  // bond matrix B[a_parent_side, a_child_side]: leg 0 carries the up-env of c,
  // leg 1 the down-env of c.
  Recipe R;
  R.dims = {P.tree.rank[c], P.tree.rank[c]};
  Recipe::G g;
  g.l1 = 0;
  g.l2 = 1;
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) {
    if (P.term_d[c][m] == kInGroup) continue;  // in a partner channel (below)
    ORef a, b;
    if (P.term_u[c][m] >= 0) {
      a.kind = 3;
      a.node = c;
      a.idx = P.term_u[c][m];
    }
    if (P.term_d[c][m] >= 0) {
      b.kind = 2;
      b.node = c;
      b.idx = P.term_d[c][m];
    }
    if (a.kind && b.kind) g.pair_terms.push_back({m, {a, b}});
    else if (a.kind) g.sa.push_back({m, a});
    else if (b.kind) g.sb.push_back({m, b});
  }
  // partner channels: P's up slot with the channel D_P
  for (int gi = 0; gi < (int)P.gkeys[c].size(); ++gi) {
    ORef a, b;
    a.kind = 3;
    a.node = c;
    a.idx = P.umap[c].at(P.gkeys[c][gi]);
    b.kind = 7;
    b.node = c;
    b.idx = gi;
    g.pair_terms.push_back({-group_size(P, c, gi), {a, b}});
  }
  // the channels: everything outside c on the parent side, everything
  // inside on the child side
  int wu = 0, wd = 0;
  for (int m = 0; m < (int)P.gen.terms.size(); ++m) {
    wu += P.term_u[c][m] == kInChannel;
    wd += P.term_d[c][m] == kInChannel;
  }
  if (P.has_u0[c]) {
    ORef a;
    a.kind = 6;
    a.node = c;
    g.sa.push_back({-wu, a});
  }
  if (P.has_d0[c]) {
    ORef b;
    b.kind = 5;
    b.node = c;
    g.sb.push_back({-wd, b});
  }
  R.groups.push_back(g);
  return R;
}

static Recipe edge_recipe(const tenso_plan& P, int s, int c) {
  const tenso_tree& t = P.tree;
  const int i = t.leg_of_child(s, c);
  std::vector<std::pair<int, Leg>> legs;
  std::vector<int> dims;
  for (int j = 0; j < (int)t.legs[s].size(); ++j)
    if (j != i) {
      legs.push_back({s, t.legs[s][j]});
      dims.push_back(t.leg_dim(s, t.legs[s][j]));
    }
  for (int j = 1; j < (int)t.legs[c].size(); ++j) {
    legs.push_back({c, t.legs[c][j]});
    dims.push_back(t.leg_dim(c, t.legs[c][j]));
  }
  return make_recipe(P, legs, dims);
}

// -- layouts ------------------------------------------------------------------
static long prod(const std::vector<int>& d, int a, int b) {
  long p = 1;
  for (int i = a; i < b; ++i) p *= d[i];
  return p;
}

static void* oref_ptr(const tenso_plan& P, const ORef& o) {
  switch (o.kind) {
    case 1:
      return (char*)P.cbuf + (P.fp64 ? P.mat_off64[o.idx] : P.mat_off32[o.idx]);
    case 2: {
      size_t r = P.slot_r[o.node];
      return tagp(TAG_WS, P.envd_off[o.node] + (size_t)o.idx * r * r * P.tsz);
    }
    case 3: {
      size_t r = P.slot_r[o.node];
      return tagp(TAG_WS, P.envu_off[o.node] + (size_t)o.idx * r * r * P.tsz);
    }
    case 4:
      return tagp(TAG_WS, P.vmf_rho_off[o.node]);
    case 5: {
      size_t r = P.slot_r[o.node];
      return tagp(TAG_WS, P.envd_off[o.node] + P.dkeys[o.node].size() * r * r * P.tsz);
    }
    case 6: {
      size_t r = P.slot_r[o.node];
      return tagp(TAG_WS, P.envu_off[o.node] + P.ukeys[o.node].size() * r * r * P.tsz);
    }
    case 7: {
      size_t r = P.slot_r[o.node];
      return tagp(TAG_WS, P.envd_off[o.node] +
                              (P.dkeys[o.node].size() + P.has_d0[o.node] + o.idx) * r * r * P.tsz);
    }
  }
  return nullptr;
}

static void layout(tenso_plan& P) {
  // every size below is taken at the capacity ranks
  tenso_tree cur = P.tree;
  P.tree = P.cap;
  const tenso_tree& t = P.tree;
  P.slot_r.assign(t.n, 1);
  for (int c = 1; c < t.n; ++c) P.slot_r[c] = t.rank[c];
  P.core_off.assign(t.n, 0);
  size_t off = 0;
  long maxP = 1;
  for (int s = 0; s < t.n; ++s) {
    P.core_off[s] = off;
    off += align256((size_t)t.size(s) * 16);
    maxP = std::max(maxP, t.size(s));
  }
  P.state_bytes = off;
  int maxr = 1;
  for (int c = 1; c < t.n; ++c) maxr = std::max(maxr, t.rank[c]);
  for (int e = 0; e < t.n_ends; ++e) P.max_dim = std::max(P.max_dim, t.end_dim[e]);
  P.max_dim = std::max(P.max_dim, maxr);
  size_t presum = 0, parts = 0, envscr = 0, qrv = 0, theta = 0, wcap = 0, side = 0;
  // presum elements and partial-output elements of a recipe on n elements
  auto recipe_need = [&](const Recipe& R, long n) {
    size_t ps = 0;
    for (auto& g : R.groups) {
      if (!g.sa.empty()) ps += (size_t)R.dims[g.l1] * R.dims[g.l1];
      if (!g.sb.empty()) ps += (size_t)R.dims[g.l2] * R.dims[g.l2];
      for (auto& c : cluster_pairs(g))
        if (c.others.size() > 1) {
          const size_t d = R.dims[c.shared_side == 0 ? g.l2 : g.l1];
          ps += d * d;
        }
    }
    return std::make_pair(ps, (size_t)R.groups.size() * 8 * (size_t)n);
  };
  auto recipe_caps = [&](const Recipe& R, long n) {
    size_t ps = 0;
    for (auto& g : R.groups) {
      if (!g.sa.empty()) ps += (size_t)R.dims[g.l1] * R.dims[g.l1];
      if (!g.sb.empty()) ps += (size_t)R.dims[g.l2] * R.dims[g.l2];
      for (auto& c : cluster_pairs(g))
        if (c.others.size() > 1) {
          const size_t d = R.dims[c.shared_side == 0 ? g.l2 : g.l1];
          ps += d * d;
        }
    }
    presum = std::max(presum, ps);
    parts = std::max(parts, (size_t)R.groups.size() * 8 * (size_t)n);
  };
  P.vmf_ok = P.fp64 != 0;
  for (int s = 0; s < t.n; ++s) {
    recipe_caps(node_recipe(P, s), t.size(s));
    if (s > 0) {
      const int p = t.parent[s];
      {  // the down channels of one environment update share the areas
        std::pair<size_t, size_t> need{0, 0};
        auto addn = [&](const Recipe& R) {
          const auto q = recipe_need(R, t.size(s));
          need.first += q.first;
          need.second += q.second;
        };
        if (P.has_d0[s]) addn(channel_recipe(P, s, 0, s, true));
        for (int gi = 0; gi < (int)P.gkeys[s].size(); ++gi) addn(group_recipe(P, s, gi));
        presum = std::max(presum, need.first);
        parts = std::max(parts, need.second);
      }
      if (P.has_u0[s]) recipe_caps(channel_recipe(P, p, t.leg_of_child(p, s), s, false), t.size(p));
      if (P.vmf_ok && P.has_u0[s]) {  // the vmf form of the up channel (with densities)
        P.vmf_rho = true;
        try {
          recipe_caps(channel_recipe(P, p, t.leg_of_child(p, s), s, false), t.size(p));
        } catch (const TErr&) {
          P.vmf_ok = false;
        }
        P.vmf_rho = false;
      }
      // one slab per key, one for the channel (vmf: one more, the bond density)
      envscr = std::max(envscr, (P.dkeys[s].size() + P.has_d0[s] + P.gkeys[s].size()) *
                                    (size_t)t.size(s));
      envscr = std::max(envscr, (P.ukeys[s].size() + P.has_u0[s] + (P.vmf_ok ? 1 : 0)) *
                                    (size_t)t.size(t.parent[s]));
      size_t r = t.rank[s];
      qrv = std::max(qrv, (size_t)t.size(s));
      qrv = std::max(qrv, (size_t)t.size(t.parent[s]));
      presum = std::max(presum, 2 * r * r);
      parts = std::max(parts, 8 * r * r);
      recipe_caps(bond_recipe(P, s), (long)r * r);
      if (P.opts.method == TENSO_PS2) {
        const int p = t.parent[s];
        const long rows = t.size(p) / t.rank[s], cols = t.size(s) / t.rank[s];
        if (rows * cols > kPs2ThetaMax)
          fail(TENSO_ENOMEM, "ps2 two-site tensor of " + std::to_string(rows * cols) +
                                 " elements at the rank cap (budget 2^26)");
        theta = std::max(theta, (size_t)(rows * cols));
        side = std::max(side, (size_t)std::max(rows, cols));
        wcap = std::max(wcap, (size_t)std::max(rows, cols) * (size_t)maxr);
        recipe_caps(edge_recipe(P, p, s), rows * cols);
        maxP = std::max<long>(maxP, rows * cols);
      }
    }
  }
  size_t w = 0;
  auto take = [&](size_t bytes) {
    size_t o = w;
    w += align256(bytes);
    return o;
  };
  P.envd_off.assign(t.n, 0);
  P.envu_off.assign(t.n, 0);
  for (int x = 1; x < t.n; ++x) {
    size_t r = t.rank[x];
    P.envd_off[x] = take(std::max<size_t>(1, P.dkeys[x].size() + P.has_d0[x] + P.gkeys[x].size()) *
                         r * r * P.tsz);
    P.envu_off[x] = take(std::max<size_t>(1, P.ukeys[x].size() + P.has_u0[x]) * r * r * P.tsz);
  }
  P.presum_cap = presum;
  P.parts_cap = parts;
  P.envscr_cap = envscr;
  P.qrv_cap = qrv;
  P.theta_cap = theta;
  P.W_cap = wcap;
  P.ws_presum = take(std::max<size_t>(1, presum) * P.tsz);
  P.ws_xin = take((size_t)maxP * P.tsz);
  P.ws_acc = take((size_t)maxP * 16);
  // four stage areas: an RK4 sub-flow keeps every stage's partial outputs
  P.ws_parts = take(4 * std::max<size_t>(1, parts) * P.tsz);
  P.ws_envscr = take(std::max<size_t>(1, envscr) * P.tsz);
  P.ws_bond = take((size_t)maxr * maxr * 16);
  P.ws_qrv = take(std::max<size_t>(1, qrv) * 16);
  P.ws_qrtau = take((size_t)P.max_dim * 16);
  P.ws_rhovec = take((size_t)t.n * maxr * 16);
  P.ws_rhoout = take((size_t)t.end_dim[0] * t.end_dim[0] * 16);
  P.ws_ctr = take(256);  // step counter at 0, finiteness flag at 64, its descriptor at 128,
                         // the root-norm descriptor at 160, norms before / after at 192 / 200
  // drive values of a one-off apply (one per slot), and the isometry-check
  // descriptors and results of the canonical-center test (one per node)
  P.ws_drive = take((size_t)std::max(1, P.gen.n_slots) * sizeof(double));
  P.ws_check = take(align256((size_t)t.n * sizeof(IsoOp)) + (size_t)t.n * sizeof(double));
  if (P.opts.method == TENSO_PS2) {
    const size_t blk = std::max<size_t>(1, side) * kSvdP * 16;
    P.svd_side = side;
    P.ws_theta = take(std::max<size_t>(1, theta) * 16);
    P.ws_svd_y = take(blk);
    P.ws_svd_z = take(blk);
    P.ws_svd_part = take(kSvdMaxSplit * blk);
    P.ws_svd_qrv = take(blk);
    P.ws_svd_r = take(kSvdP * kSvdP * 16);
    P.ws_svd_up = take(kSvdP * kSvdP * 16);
    P.ws_svd_wp = take(kSvdP * kSvdP * 16);
    P.ws_svd_sig = take(kSvdP * 8);
    P.ws_svd_tau = take(kSvdP * 16);
    P.ws_svd_norm = take(((side + 63) / 64) * kSvdMaxSplit * 8);
    P.ws_svd_e = take(blk);
    P.ws_svd_rec = take(256);
    P.ws_W = take(std::max<size_t>(1, wcap) * 16);
  }
  // direct integration needs every node's vmf recipe (a term may then carry
  // the density on the parent leg besides its own legs): without them the
  // plan simply has no vmf areas
  std::vector<size_t> vparts(t.n, 1), vpresum(t.n, 1);
  long vmaxsz = 1;
  if (P.vmf_ok) {
    P.vmf_rho = true;
    try {
      for (int s = 0; s < t.n; ++s) {
        const Recipe R = node_recipe(P, s);
        size_t ps = 0;
        for (auto& g : R.groups) {
          if (!g.sa.empty()) ps += (size_t)R.dims[g.l1] * R.dims[g.l1];
          if (!g.sb.empty()) ps += (size_t)R.dims[g.l2] * R.dims[g.l2];
          for (auto& c : cluster_pairs(g))
            if (c.others.size() > 1) {
              const size_t d = R.dims[c.shared_side == 0 ? g.l2 : g.l1];
              ps += d * d;
            }
        }
        vparts[s] = std::max<size_t>(1, R.groups.size() * 8 * (size_t)t.size(s));
        vpresum[s] = std::max<size_t>(1, ps);
        vmaxsz = std::max(vmaxsz, t.size(s));
      }
      for (int x = 1; x < t.n; ++x)
        if (t.rank[x] > kVmfMaxRank) fail(TENSO_EUNSUPPORTED, "bond above the vmf inverse's size");
    } catch (const TErr&) {
      P.vmf_ok = false;
    }
    P.vmf_rho = false;
  }
  if (P.vmf_ok) {
    // direct integration: bond densities, their regularised inverses and the
    // projection coefficients per bond; the stage input, seven dopri5 stages
    // and the derivative (state-shaped); partial outputs and presums of the
    // one contraction launch that serves every node; segment list, error
    // partials and the ps2 drive table of the mixed strategy
    P.vmf_rho_off.assign(t.n, 0);
    P.vmf_rinv_off.assign(t.n, 0);
    P.vmf_s_off.assign(t.n, 0);
    for (int x = 1; x < t.n; ++x) {
      const size_t r = t.rank[x];
      P.vmf_rho_off[x] = take(r * r * 16);
      P.vmf_rinv_off[x] = take(r * r * 16);
      P.vmf_s_off[x] = take(r * r * 16);
    }
    P.ws_vmf_ys = take(P.state_bytes);
    P.ws_vmf_k = take(7 * P.state_bytes);
    P.ws_vmf_kout = take(P.state_bytes);
    P.vmf_node_parts.assign(t.n, 0);
    P.vmf_node_presum.assign(t.n, 0);
    for (int s = 0; s < t.n; ++s) {
      P.vmf_node_parts[s] = take(vparts[s] * 16);
      P.vmf_node_presum[s] = take(vpresum[s] * 16);
    }
    P.vmf_chunks = (int)((vmaxsz + kVmfChunk - 1) / kVmfChunk);
    P.ws_vmf_segs = take((size_t)t.n * sizeof(VecSeg));
    P.ws_vmf_part = take((size_t)t.n * P.vmf_chunks * sizeof(double));
    P.ws_vmf_err = take(256);
    P.ws_vmf_dtab = take((size_t)std::max(1, P.gen.n_slots) * kVmfDriveLd * sizeof(double));
  }
  P.ws_bytes = w;
  P.tree = cur;
}

// -- program building ---------------------------------------------------------
struct Builder {
  tenso_plan& P;
  Program& G;
  tenso_plan& P_;
  Builder(tenso_plan& p, Program& g) : P(p), G(g), P_(p) {}

  void launch(int kind, int in_fp64, int first, int count, int tfirst, int tcount, size_t lds = 0) {
    LaunchRec L{kind, in_fp64, first, count, tfirst, tcount, lds};
    if (kind == LK_APPLY) {
      L.amode = P_.amode;
      size_t mx = 0;
      for (int t = tfirst; t < tfirst + tcount; ++t) {
        const ApplyTile& tl = G.atiles[t];
        const ApplyGroup& g = G.groups[first + tl.group];
        const int njb = (g.d2 + 15) / 16;
        const int nfl = (tl.u0 + tl.nu - 1) / njb - tl.u0 / njb + 1;
        mx = std::max(mx, apply_lds_bytes(P_.fp64, nfl, g.d1, g.d2));
      }
      L.lds = mx;
      // useful work (no padding): pair term F*d1*d2*(d1+d2) complex MACs,
      // one-sided terms F*d1*d1*d2 or F*d1*d2*d2; bytes: input read, output
      // written (one slab per term for per-term outputs), operand matrices
      // read once per group
      for (int gi = first; gi < first + count; ++gi) {
        const ApplyGroup& g = G.groups[gi];
        const double F = g.F, d1 = g.d1, d2 = g.d2, P = F * d1 * d2;
        const double esz = in_fp64 ? 16.0 : (double)P_.tsz;
        L.bytes += P * esz + P * P_.tsz * (g.per_term_out ? g.n_terms : 1);
        const int t0 = (int)(((uint64_t)g.terms) & OFF_MASK);
        for (int m = t0; m < t0 + g.n_terms; ++m) {
          // credited per generator term the entry stands for (grouped and
          // presummed terms count as the separate terms they replace)
          const TermRef& t = G.terms[m];
          const double w = G.credit[m];
          if (t.A && t.B) L.flops += w * 8.0 * F * d1 * d2 * (d1 + d2);
          else if (t.A) L.flops += w * 8.0 * F * d1 * d1 * d2;
          else L.flops += w * 8.0 * F * d1 * d2 * d2;
          if (t.A) L.bytes += w * d1 * d1 * P_.tsz;
          if (t.B) L.bytes += w * d2 * d2 * P_.tsz;
        }
      }
    }
    G.launches.push_back(L);
  }

  void* core(int s) { return tagp(TAG_STATE, P.core_off[s]); }
  void* ws(size_t off) { return tagp(TAG_WS, off); }

  int term_index(const TermRef& tr, double credit = 1.0) {
    G.terms.push_back(tr);
    G.credit.push_back(credit);
    return (int)G.terms.size() - 1;
  }

  // m < 0: a channel (coefficient 1, no drive)
  TermRef term_ref(int m, void* A, void* B) {
    TermRef tr{};
    tr.cre = m < 0 ? 1.0 : P.gen.terms[m].coef.real();
    tr.cim = m < 0 ? 0.0 : P.gen.terms[m].coef.imag();
    tr.slot = m < 0 ? -1 : P.gen.terms[m].slot;
    tr.A = A;
    tr.B = B;
    return tr;
  }

  // Padded MFMA work (flops) of one unit (f, 16-column block) for one term.
  static double unit_work(int d1, int d2) {
    const int D1 = 16 * ((d1 + 15) / 16);
    const int k1 = 4 * ((d2 + 3) / 4), k2 = 4 * ((d1 + 3) / 4);
    return 8.0 * 16 * D1 * (k1 + k2);
  }

  // Tiles for one group of units: about `tile_work` flops per tile (at most
  // kApplyMaxUnits / nib units), at least `target` tiles, and the
  // tile's input slices and operand matrices within the LDS budget.
  // Units per tile for a group (see add_tiles).
  long tile_units(int d1, int d2, long F, int target, int n_terms) {
    const int nib = (d1 + 15) / 16, njb = (d2 + 15) / 16;
    const int NT = kApplyAccTiles;  // accumulator tiles per wavefront in the kernel
    const size_t budget = kApplyLdsBudget;
    if (nib > NT || d1 > 64 || d2 > 64 || apply_lds_bytes(P.fp64, 1, d1, d2) > budget)
      fail(TENSO_EUNSUPPORTED, "leg dimensions too large for the apply kernel in this precision");
    const long units = F * njb;
    const double per_unit = unit_work(d1, d2) * std::max(1, n_terms);
    long want = std::max<long>(target, (long)std::ceil(units * per_unit / P.tile_work));
    long per = std::max<long>(1, (units + want - 1) / want);
    per = std::min<long>(per, (long)(kApplyWaves * (NT / nib)));  // each wavefront's accumulators
    while (per > 1 && apply_lds_bytes(P.fp64, (int)((per + njb - 1) / njb + 1), d1, d2) > budget)
      per /= 2;
    // (the FP64 kernel's registers allow one workgroup per CU anyway)
    while (!P.fp64 && per > 1 &&
           apply_lds_bytes(P.fp64, (int)((per + njb - 1) / njb + 1), d1, d2) > (size_t)kApplyLdsShare)
      per /= 2;
    return per;
  }

  void add_tiles(int gi, int d1, int d2, long F, int target, int n_terms) {
    const int njb = (d2 + 15) / 16;
    const long units = F * njb;
    const long per = tile_units(d1, d2, F, target, n_terms);
    for (long u = 0; u < units; u += per) {
      ApplyTile tl{};
      tl.group = gi;
      tl.u0 = (int)u;
      tl.nu = (int)std::min<long>(per, units - u);
      tl.pad = 1;
      G.atiles.push_back(tl);
    }
  }

  // Workspace areas of one contraction: partial outputs and presummed
  // operators (byte offsets; capacities in elements).
  struct ApplyArea {
    size_t parts, presum, parts_cap, presum_cap;
  };
  // Input of an RK4 stage formed while staged (in_fp64 = 2): X plus
  // sign * h (half: h / 2) times the sum of the np partial outputs at parts.
  struct StageSrc {
    void* parts;
    long n;
    int np;
    double sign;
    int half;
  };

  // Emit apply launches of recipe R on input X -> parts (chunked), with the
  // presum launch in front.  Returns the number of partial slabs written.
  int emit_apply(const Recipe& R, void* X, int in_fp64, long Pn, int rel, int presum_now,
                 int target, size_t parts_off = 0, const StageSrc* src = nullptr) {
    const int pfirst = (int)G.presums.size();
    const int gfirst = (int)G.groups.size(), tfirst = (int)G.atiles.size();
    const int part = add_apply(R, X, in_fp64, Pn, rel, presum_now, target,
                               ApplyArea{parts_off ? parts_off : P.ws_parts, P.ws_presum,
                                         P.parts_cap, P.presum_cap},
                               gfirst, nullptr, src);
    const int np = (int)G.presums.size() - pfirst;
    if (np) launch(LK_PRESUM, 0, pfirst, np, 0, 0);
    launch(LK_APPLY, in_fp64, gfirst, (int)G.groups.size() - gfirst, tfirst,
           (int)G.atiles.size() - tfirst);
    return part;
  }

  // The presums and contraction groups of recipe R on input X, appended
  // without a launch: presums to G.presums, groups and tiles after gfirst
  // (the first group of the launch they will join), partial slabs from A.parts.
  // Returns the number of partial slabs.
  int add_apply(const Recipe& R, void* X, int in_fp64, long Pn, int rel, int presum_now,
                int target, const ApplyArea& A, int gfirst, size_t* presum_bytes = nullptr,
                const StageSrc* src = nullptr) {
    // presums
    size_t poff = A.presum;
    std::vector<void*> sa_buf(R.groups.size(), nullptr), sb_buf(R.groups.size(), nullptr);
    for (size_t gi = 0; gi < R.groups.size(); ++gi) {
      auto& g = R.groups[gi];
      for (int side = 0; side < 2; ++side) {
        auto& lst = side == 0 ? g.sa : g.sb;
        if (lst.empty()) continue;
        int d = R.dims[side == 0 ? g.l1 : g.l2];
        void* out = ws(poff);
        poff += (size_t)d * d * P.tsz;
        (side == 0 ? sa_buf : sb_buf)[gi] = out;
        PresumOp op{};
        op.out = out;
        int first = -1;
        for (auto& st : lst) {
          int k = term_index(term_ref(st.first, oref_ptr(P, st.second), nullptr));
          if (first < 0) first = k;
        }
        op.terms = (const TermRef*)tagp(TAG_TERM, first);
        op.n_terms = (int)lst.size();
        op.dim = d;
        op.rel = rel;
        if (op.n_terms > PRESUM_MAX_TERMS) fail(TENSO_EUNSUPPORTED, "more than 512 terms in one presum");
        if (presum_now) G.presums.push_back(op);
      }
    }
    // grouped pair terms: presum of the non-shared operators of each cluster
    std::vector<std::vector<void*>> cl_buf(R.groups.size());
    std::vector<std::vector<PairCluster>> clusters(R.groups.size());
    for (size_t gi = 0; gi < R.groups.size(); ++gi) {
      auto& g = R.groups[gi];
      clusters[gi] = cluster_pairs(g);
      for (auto& c : clusters[gi]) {
        if (c.others.size() < 2) {
          cl_buf[gi].push_back(nullptr);
          continue;
        }
        const int d = R.dims[c.shared_side == 0 ? g.l2 : g.l1];
        void* out = ws(poff);
        poff += (size_t)d * d * P.tsz;
        cl_buf[gi].push_back(out);
        PresumOp op{};
        op.out = out;
        int first = -1;
        for (auto& o : c.others) {
          int k = term_index(term_ref(o.first, oref_ptr(P, o.second), nullptr));
          if (first < 0) first = k;
        }
        op.terms = (const TermRef*)tagp(TAG_TERM, first);
        op.n_terms = (int)c.others.size();
        op.dim = d;
        op.rel = rel;
        if (op.n_terms > PRESUM_MAX_TERMS) fail(TENSO_EUNSUPPORTED, "more than 512 terms in one presum");
        if (presum_now) G.presums.push_back(op);
      }
    }
    if (poff - A.presum > A.presum_cap * P.tsz + 1) fail(TENSO_EINVAL, "presum capacity");
    if (presum_bytes) *presum_bytes = poff - A.presum;
    // groups, chunked over terms
    int part = 0;
    long free_total = 0;
    for (auto& g : R.groups) free_total += Pn / ((long)R.dims[g.l1] * R.dims[g.l2]);
    for (size_t gi = 0; gi < R.groups.size(); ++gi) {
      auto& g = R.groups[gi];
      std::vector<TermRef> trs;
      std::vector<double> trc;  // generator terms per entry
      for (size_t ci = 0; ci < clusters[gi].size(); ++ci) {
        const PairCluster& c = clusters[gi][ci];
        if (!cl_buf[gi][ci]) {  // a cluster of one: the plain pair term
          const auto& o = c.others[0];
          void* sh = oref_ptr(P, c.shared);
          void* ot = oref_ptr(P, o.second);
          trs.push_back(c.shared_side == 0 ? term_ref(o.first, sh, ot) : term_ref(o.first, ot, sh));
          trc.push_back(term_weight(o.first));
          continue;
        }
        TermRef tr{};
        tr.cre = 1;
        tr.slot = -1;
        tr.A = c.shared_side == 0 ? oref_ptr(P, c.shared) : cl_buf[gi][ci];
        tr.B = c.shared_side == 0 ? cl_buf[gi][ci] : oref_ptr(P, c.shared);
        trs.push_back(tr);
        double w = 0;
        for (auto& o : c.others) w += term_weight(o.first);
        trc.push_back(w);
      }
      if (sa_buf[gi]) {
        TermRef tr{};
        tr.cre = 1;
        tr.slot = -1;
        tr.A = sa_buf[gi];
        trs.push_back(tr);
        double w = 0;
        for (auto& o : g.sa) w += term_weight(o.first);
        trc.push_back(w);
      }
      if (sb_buf[gi]) {
        TermRef tr{};
        tr.cre = 1;
        tr.slot = -1;
        tr.B = sb_buf[gi];
        trs.push_back(tr);
        double w = 0;
        for (auto& o : g.sb) w += term_weight(o.first);
        trc.push_back(w);
      }
      const int d1 = R.dims[g.l1], d2 = R.dims[g.l2];
      const long F = Pn / ((long)d1 * d2);
      const long units = F * ((d2 + 15) / 16);
      // Term chunks (each with its own partial output): when even 4-unit
      // tiles would exceed the tile work, or the launch wants more tiles
      // than the units allow.
      int nchunk = 1;
      {
        const double w_all = (double)units * unit_work(d1, d2) * (double)trs.size();
        const long tiles_units = std::max<long>(1, (units + 3) / 4);
        long want = std::max<long>((long)std::ceil(w_all / P.tile_work),
                                   target > 1 ? (long)target / (long)R.groups.size() : 1);
        nchunk = (int)std::min<long>(8, std::max<long>(1, (want + tiles_units - 1) / tiles_units));
        nchunk = std::min<int>(nchunk, std::max<int>(1, (int)trs.size() / 2));
      }
      size_t per = (trs.size() + nchunk - 1) / nchunk;
      for (int ch = 0; ch < nchunk; ++ch) {
        size_t a = ch * per, b = std::min(trs.size(), a + per);
        if (a >= b && ch > 0) break;
        ApplyGroup ag{};
        ag.X = X;
        ag.Y = ws(A.parts + (size_t)part * Pn * P.tsz);
        ++part;
        int first = (int)G.terms.size();
        for (size_t i = a; i < b; ++i) {
          G.terms.push_back(trs[i]);
          G.credit.push_back(trc[i]);
        }
        ag.terms = (const TermRef*)tagp(TAG_TERM, first);
        ag.in_fp64 = in_fp64;
        if (src) {
          ag.xp = src->parts;
          ag.xp_n = src->n;
          ag.xp_np = src->np;
          ag.xp_s = src->sign;  // times h or h / 2 at bind time
          ag.xp_half = src->half;
        }
        ag.n_terms = (int)(b - a);
        ag.d1 = d1;
        ag.d2 = d2;
        ag.P1 = (int)prod(R.dims, g.l1 + 1, g.l2);
        ag.P2 = (int)prod(R.dims, g.l2 + 1, (int)R.dims.size());
        ag.F = (int)F;
        ag.rel = rel;
        ag.accumulate = 0;
        G.groups.push_back(ag);
        add_tiles((int)G.groups.size() - 1 - gfirst, d1, d2, F,
                  target > 1 ? std::max(1, target / (nchunk * (int)R.groups.size())) : 1,
                  (int)(b - a));
      }
    }
    if ((size_t)part * Pn > A.parts_cap) fail(TENSO_EINVAL, "parts capacity exceeded");
    return part;
  }

  void emit_combine(void* y0, long n, int n_parts, int stage, double h_sign_half) {
    CombineOp op{};
    op.y0 = (double*)y0;
    op.xin = ws(P.ws_xin);
    op.acc = (double*)ws(P.ws_acc);
    op.parts = ws(P.ws_parts);
    op.n = n;
    op.n_parts = n_parts;
    op.stage = stage;
    op.h = h_sign_half;  // sign; multiplied by dt/2 at bind time
    int oi = (int)G.combines.size();
    G.combines.push_back(op);
    int tf = (int)G.ctiles.size();
    for (long e = 0; e < n; e += kCombineTile) G.ctiles.push_back({oi, 0, e, std::min(n, e + kCombineTile)});
    launch(LK_COMBINE, 0, oi, 1, tf, (int)G.ctiles.size() - tf);
  }

  // RK4 sub-flow of sign * L_eff over half a step on y0 (FP64 master).
  void emit_rk4(const Recipe& R, void* y0, long n, double sign, int half) {
    const int rel0 = half == 0 ? 0 : 2;
    const int rels[4] = {rel0, rel0 + 1, rel0 + 1, rel0 + 2};
    bool td = false;
    for (auto& g : R.groups) {  // presummed coefficients that change within the sub-flow
      for (auto& s : g.sa) td |= s.first >= 0 && P.gen.terms[s.first].slot >= 0;
      for (auto& s : g.sb) td |= s.first >= 0 && P.gen.terms[s.first].slot >= 0;
      for (auto& s : g.pair_terms) td |= s.first >= 0 && P.gen.terms[s.first].slot >= 0;
    }
    // stage 1 (input y0) leaves its partial outputs in the first part area
    const int np1 = emit_apply(R, y0, 1, n, rels[0], 1, P.par_target);
    if (!P.fuse_stages || (long)np1 * n > P.fuse_max_elems) {
      // a combine per stage: the next input in xin
      emit_combine(y0, n, np1, 1, sign);
      for (int st = 2; st <= 4; ++st) {
        int np = emit_apply(R, ws(P.ws_xin), 0, n, rels[st - 1], td, P.par_target);
        emit_combine(y0, n, np, st, sign);
      }
      return;
    }
    // every stage keeps its partial outputs (stage s at s - 1 part areas
    // from the first): the next stage's input y0 + c k_s is formed while its
    // contraction stages it, and one combine at the end applies the update
    const size_t stride = std::max<size_t>(1, P.parts_cap);  // elements
    int np_prev = np1;
    for (int st = 2; st <= 4; ++st) {
      StageSrc src{};
      src.parts = ws(P.ws_parts + (size_t)(st - 2) * stride * P.tsz);
      src.n = n;
      src.np = np_prev;
      src.sign = sign;
      src.half = st <= 3;
      const int np = emit_apply(R, y0, 2, n, rels[st - 1], td, P.par_target,
                                P.ws_parts + (size_t)(st - 1) * stride * P.tsz, &src);
      if (np != np1) fail(TENSO_EINVAL, "RK4 stages split into different parts");
      np_prev = np;
    }
    CombineOp op{};
    op.y0 = (double*)y0;
    op.xin = ws(P.ws_xin);
    op.acc = (double*)ws(P.ws_acc);
    op.parts = ws(P.ws_parts);
    op.n = n;
    op.n_parts = np1;
    op.stage = 6;
    op.h = sign;  // multiplied by dt/2 at bind time
    op.stage_stride = (long)stride;
    const int oi = (int)G.combines.size();
    G.combines.push_back(op);
    const int tf = (int)G.ctiles.size();
    for (long e = 0; e < n; e += kCombineTile) G.ctiles.push_back({oi, 0, e, std::min(n, e + kCombineTile)});
    launch(LK_COMBINE, 0, oi, 1, tf, (int)G.ctiles.size() - tf);
  }

  void emit_env_down(int x) { emit_env(x, true, false); }
  void emit_env_up(int x) { emit_env(x, false, false); }

  // Environments of bond x on one side: the slots of its keys (down: from
  // core x, open leg its parent leg; up: from the parent core p, open leg
  // the one to x) and the side's channel, in one contraction launch (per-key
  // results in their own slabs, the channel's terms summed into partial
  // outputs), the channel's partial sum, then one Gram launch for all.
  // with_rho (up side of a vmf program): also the bond density rho_x, from
  // p's core with rho_p on its parent leg (p's plain Gram at the root).
  void emit_env(int x, bool down, bool with_rho) {
    const tenso_tree& t = P.tree;
    const std::vector<Key>& keys = down ? P.dkeys[x] : P.ukeys[x];
    const bool chan = down ? P.has_d0[x] : P.has_u0[x];
    if (keys.empty() && !chan && !with_rho && !(down && !P.gkeys[x].empty())) return;
    const int node = down ? x : t.parent[x];
    const std::vector<int> dims = t.shape(node);
    const long Pn = t.size(node);
    const int open = down ? 0 : t.leg_of_child(node, x);
    const int pfirst = (int)G.presums.size();
    const int gfirst = (int)G.groups.size(), tfirst = (int)G.atiles.size();
    std::vector<std::vector<std::pair<int, ORef>>> nzs;
    for (size_t k = 0; k < keys.size(); ++k) {
      std::vector<std::pair<int, ORef>> nz;
      for (int i = 0; i < (int)t.legs[node].size(); ++i) {
        if (i == open) continue;
        ORef o = leg_ref_for_key(P, node, t.legs[node][i], keys[k]);
        if (o.kind) nz.push_back({i, o});
      }
      nzs.push_back(nz);
    }
    const bool rho_direct = with_rho && node == 0;
    if (with_rho && !rho_direct) {
      ORef o;
      o.kind = 4;
      o.node = node;
      nzs.push_back({{0, o}});
    }
    const std::vector<size_t> slab = add_env_groups(dims, Pn, open, nzs, node, gfirst);
    // channels: D0 / U0, then (down side) the partner channels, each summed
    // into partial outputs of its own and then into its slab
    std::vector<Recipe> chans;
    if (chan) chans.push_back(channel_recipe(P, node, open, x, down));
    if (down)
      for (int gi = 0; gi < (int)P.gkeys[x].size(); ++gi) chans.push_back(group_recipe(P, x, gi));
    std::vector<int> nparts(chans.size());
    std::vector<size_t> pbase(chans.size());
    size_t used_parts = 0, used_presum = 0;
    for (size_t ci = 0; ci < chans.size(); ++ci) {
      pbase[ci] = used_parts;
      size_t pb = 0;
      nparts[ci] = add_apply(chans[ci], core(node), 1, Pn, 0, 1, P.par_target,
                             ApplyArea{P.ws_parts + used_parts * Pn * P.tsz,
                                       P.ws_presum + used_presum,
                                       P.parts_cap - std::min(P.parts_cap, used_parts * Pn),
                                       P.presum_cap - std::min(P.presum_cap, used_presum / P.tsz)},
                             gfirst, &pb);
      used_parts += nparts[ci];
      used_presum += pb;
    }
    const int np = (int)G.presums.size() - pfirst;
    if (np) launch(LK_PRESUM, 0, pfirst, np, 0, 0);
    if ((int)G.groups.size() > gfirst)
      launch(LK_APPLY, 1, gfirst, (int)G.groups.size() - gfirst, tfirst,
             (int)G.atiles.size() - tfirst);
    const size_t chan_slab = nzs.size();
    if (!chans.empty()) {  // each channel's partial outputs summed into its slab
      const int cf = (int)G.combines.size(), tf = (int)G.ctiles.size();
      for (size_t ci = 0; ci < chans.size(); ++ci) {
        CombineOp op{};
        op.y0 = (double*)ws(P.ws_acc);
        op.xin = ws(P.ws_envscr + (chan_slab + ci) * Pn * P.tsz);
        op.acc = (double*)ws(P.ws_acc);
        op.parts = ws(P.ws_parts + pbase[ci] * Pn * P.tsz);
        op.n = Pn;
        op.n_parts = nparts[ci];
        op.stage = 5;
        const int oi = (int)G.combines.size();
        G.combines.push_back(op);
        for (long e = 0; e < Pn; e += kCombineTile) G.ctiles.push_back({oi, 0, e, std::min(Pn, e + kCombineTile)});
      }
      launch(LK_COMBINE, 0, cf, (int)chans.size(), tf, (int)G.ctiles.size() - tf);
    }
    const int qf = (int)G.grams.size();
    const size_t rr = (size_t)P.slot_r[x] * P.slot_r[x] * P.tsz;
    const size_t base = down ? P.envd_off[x] : P.envu_off[x];
    auto gram = [&](const void* T, size_t e_off) {
      GramOp go{};
      go.C = (const double*)core(node);
      go.T = T;
      go.E = ws(e_off);
      go.r = t.rank[x];
      go.Ppre = (int)prod(dims, 0, open);
      go.Ppost = (int)prod(dims, open + 1, (int)dims.size());
      G.grams.push_back(go);
    };
    for (size_t k = 0; k < keys.size(); ++k) gram(ws(P.ws_envscr + slab[k] * Pn * P.tsz), base + k * rr);
    // channel slabs: D0 / U0 right after the keys, then the partner channels
    for (size_t ci = 0; ci < chans.size(); ++ci)
      gram(ws(P.ws_envscr + (chan_slab + ci) * Pn * P.tsz), base + (keys.size() + ci) * rr);
    if (with_rho)
      gram(rho_direct ? core(node) : ws(P.ws_envscr + slab.back() * Pn * P.tsz), P.vmf_rho_off[x]);
    launch(LK_GRAM, 0, qf, (int)G.grams.size() - qf, 0, 0);
  }

  // Environment operators on core `node` (one per env slot k, acting on one
  // or two of its legs besides `open`): slots with the same leg pair share
  // one apply group whose terms each write their own result slab, so the
  // core is staged once per tile for all of them.  Returns the scratch slab
  // of every slot (slabs of a group are consecutive).
  std::vector<size_t> add_env_groups(const std::vector<int>& dims, long Pn, int open,
                                     const std::vector<std::vector<std::pair<int, ORef>>>& nzs,
                                     int node, int gfirst) {
    struct Item {
      int l1, l2;
      void *A, *B;
    };
    std::vector<Item> items;
    for (auto& nz : nzs) {
      if (nz.empty() || nz.size() > 2)
        fail(TENSO_EUNSUPPORTED, "environment operator acts on more than two legs");
      Item it{};
      if (nz.size() == 2) {
        it.l1 = nz[0].first;
        it.l2 = nz[1].first;
        it.A = oref_ptr(P, nz[0].second);
        it.B = oref_ptr(P, nz[1].second);
      } else {
        const int l = nz[0].first;
        it.l1 = std::min(l, open);
        it.l2 = std::max(l, open);
        if (it.l1 == l) it.A = oref_ptr(P, nz[0].second);
        else it.B = oref_ptr(P, nz[0].second);
      }
      items.push_back(it);
    }
    std::vector<size_t> slab(items.size());
    std::vector<bool> done(items.size(), false);
    size_t next = 0;
    const int target = std::max(1, P.par_target / 8);
    for (size_t k0 = 0; k0 < items.size(); ++k0) {
      if (done[k0]) continue;
      const int l1 = items[k0].l1, l2 = items[k0].l2;
      std::vector<size_t> ks;
      for (size_t k = k0; k < items.size(); ++k) {
        if (done[k] || items[k].l1 != l1 || items[k].l2 != l2) continue;
        done[k] = true;
        ks.push_back(k);
      }
      const int d1 = dims[l1], d2 = dims[l2];
      const long F = Pn / ((long)d1 * d2);
      // term chunks (separate groups) while one chunk would give fewer tiles
      // than the plan's parallelism target
      const long units = F * ((d2 + 15) / 16);
      const long per = tile_units(d1, d2, F, target, (int)ks.size());
      const long tiles_all = (units + per - 1) / per;
      const int nchunk = (int)std::min<long>((long)ks.size(),
                                             std::max<long>(1, (P.par_target + tiles_all - 1) / tiles_all));
      const size_t cper = (ks.size() + nchunk - 1) / nchunk;
      for (size_t a = 0; a < ks.size(); a += cper) {
        const size_t b = std::min(ks.size(), a + cper);
        const size_t s0 = next;
        const int first = (int)G.terms.size();
        for (size_t i = a; i < b; ++i) {
          slab[ks[i]] = next++;
          TermRef tr{};
          tr.cre = 1;
          tr.slot = -1;
          tr.A = items[ks[i]].A;
          tr.B = items[ks[i]].B;
          term_index(tr);
        }
        ApplyGroup ag{};
        ag.X = core(node);
        ag.Y = ws(P.ws_envscr + s0 * Pn * P.tsz);
        ag.terms = (const TermRef*)tagp(TAG_TERM, first);
        ag.in_fp64 = 1;
        ag.n_terms = (int)(b - a);
        ag.per_term_out = 1;
        ag.d1 = d1;
        ag.d2 = d2;
        ag.P1 = (int)prod(dims, l1 + 1, l2);
        ag.P2 = (int)prod(dims, l2 + 1, (int)dims.size());
        ag.F = (int)F;
        ag.rel = 0;
        G.groups.push_back(ag);
        add_tiles((int)G.groups.size() - 1 - gfirst, d1, d2, F, target, ag.n_terms);
      }
    }
    return slab;
  }

  void emit_qr(int node, int leg, int transposeR) {
    const tenso_tree& t = P.tree;
    std::vector<int> d = t.shape(node);
    QrOp q{};
    q.C = (double*)core(node);
    q.R = (double*)ws(P.ws_bond);
    q.V = (double*)ws(P.ws_qrv);
    q.tau = (double*)ws(P.ws_qrtau);
    q.n = d[leg];
    q.m = (int)(t.size(node) / d[leg]);
    q.Ppost = (int)prod(d, leg + 1, (int)d.size());
    q.transposeR = transposeR;
    q.tol = kQrRankTol;
    if (q.m < q.n) fail(TENSO_EUNSUPPORTED, "QR with fewer rows than columns");
    if (q.n > 64) fail(TENSO_EUNSUPPORTED, "QR of a bond wider than 64");
    int qi = (int)G.qrs.size();
    G.qrs.push_back(q);
    launch(LK_QR, 0, qi, 1, 0, 0);
  }

  void emit_absorb(int node, int leg, int transposeM) {
    const tenso_tree& t = P.tree;
    std::vector<int> d = t.shape(node);
    AbsorbOp a{};
    a.C = (double*)core(node);
    a.M = (const double*)ws(P.ws_bond);
    a.n = d[leg];
    if (a.n > kAbsorbMaxN) fail(TENSO_EUNSUPPORTED, "bond wider than 64 in a gauge move");
    a.Ppost = (int)prod(d, leg + 1, (int)d.size());
    a.Ppre = (int)prod(d, 0, leg);
    a.transposeM = transposeM;
    int ai = (int)G.absorbs.size();
    G.absorbs.push_back(a);
    int tf = (int)G.abtiles.size();
    int fibers = a.Ppre * a.Ppost;
    int per = std::max(1, absorb_tile_elems(P.par_target) / a.n);
    for (int f = 0; f < fibers; f += per) G.abtiles.push_back({ai, f, std::min(fibers, f + per)});
    launch(LK_ABSORB, 0, ai, 1, tf, (int)G.abtiles.size() - tf, absorb_lds(a.n, per));
  }

  // ps1 first-order sweep and its adjoint (mirrors the recursive subflows)
  void V(int s, int half) {
    const tenso_tree& t = P.tree;
    for (int c : t.children[s]) {
      int i = t.leg_of_child(s, c);
      emit_qr(s, i, 0);
      emit_absorb(c, 0, 0);
      emit_env_up(c);
      V(c, half);
      emit_qr(c, 0, 1);
      emit_env_down(c);
      emit_rk4(bond_recipe(P, c), ws(P.ws_bond), (long)t.rank[c] * t.rank[c], -1.0, half);
      emit_absorb(s, i, 1);
    }
    emit_rk4(node_recipe(P, s), core(s), t.size(s), +1.0, half);
  }
  void Vstar(int s, int half) {
    const tenso_tree& t = P.tree;
    emit_rk4(node_recipe(P, s), core(s), t.size(s), +1.0, half);
    const auto& ch = t.children[s];
    for (int k = (int)ch.size() - 1; k >= 0; --k) {
      int c = ch[k];
      int i = t.leg_of_child(s, c);
      emit_qr(s, i, 0);
      emit_env_up(c);
      emit_rk4(bond_recipe(P, c), ws(P.ws_bond), (long)t.rank[c] * t.rank[c], -1.0, half);
      emit_absorb(c, 0, 0);
      Vstar(c, half);
      emit_qr(c, 0, 0);
      emit_absorb(s, i, 0);
      emit_env_down(c);
    }
  }

  void env_init_toward(int center) {
    const tenso_tree& t = P.tree;
    std::vector<char> on_path(t.n, 0);
    std::vector<int> path;
    for (int x = center; x >= 0; x = x == 0 ? -1 : t.parent[x]) {
      on_path[x] = 1;
      path.push_back(x);
    }
    for (int x = t.n - 1; x >= 1; --x)
      if (!on_path[x] || x == center) {
        if (x == center) continue;
          emit_env_down(x);
      }
    // children of center are off-path: done above.  Up envs along the path.
    for (int k = (int)path.size() - 2; k >= 0; --k) {
      emit_env_up(path[k]);
    }
  }

  void rho_prog() {
    const tenso_tree& t = P.tree;
    int first = (int)G.rnodes.size();
    for (int s = t.n - 1; s >= 0; --s) {
      RhoNode nd{};
      nd.C = (const double*)core(s);
      nd.n_legs = (int)t.legs[s].size();
      for (int l = 0; l < nd.n_legs; ++l) {
        const Leg& lg = t.legs[s][l];
        nd.dims[l] = t.leg_dim(s, lg);
        if (lg.kind == 0) nd.kind[l] = 0;
        else if (lg.kind == 1) nd.kind[l] = (s == 0 && lg.id < 2) ? 2 : 1;
        else {
          nd.kind[l] = 3;
          nd.child_slot[l] = lg.id;
        }
      }
      nd.out_slot = s == 0 ? -1 : s;
      G.rnodes.push_back(nd);
    }
    RhoProg rp{};
    rp.nodes = (const RhoNode*)tagp(TAG_RNODE, first);
    rp.n_nodes = t.n;
    rp.vecs = (double*)ws(P.ws_rhovec);
    int maxr = 1;
    for (int c = 1; c < t.n; ++c) maxr = std::max(maxr, P.slot_r[c]);
    rp.vec_ld = maxr;
    rp.rho_out = (double*)ws(P.ws_rhoout);
    G.rprogs.push_back(rp);
    launch(LK_RHO, 0, (int)G.rprogs.size() - 1, 1, 0, 0);
  }

  // -- direct (vmf) integration -------------------------------------------
  // Mean fields of bond x from its parent core p, which is not an isometry
  // toward x: the up-environment slots of x, each weighted by the density of
  // p's own bond (a key with nothing outside p carries that density on p's
  // parent leg), and the bond density rho_x itself (p's core with rho_p on
  // its parent leg; the plain Gram of the root core when p is the root).
  void emit_vmf_up(int x) { emit_env(x, false, true); }

  // The time derivative of every core of the state at TAG_STATE into the
  // derivative buffer (same layout): down environments (children first),
  // mean fields and densities (parents first), the regularised inverses, one
  // contraction launch for every node's effective generator, the partial
  // sums, then for every non-root core the inverse density on its parent leg
  // and the projection off its own span.
  void vmf_deriv(double reg) {
    const tenso_tree& t = P.tree;
    struct Flag {
      bool& f;
      explicit Flag(bool& x) : f(x) { f = true; }
      ~Flag() { f = false; }
    } on(P.vmf_rho);
    for (int x = t.n - 1; x >= 1; --x) emit_env_down(x);
    for (int x = 1; x < t.n; ++x) emit_vmf_up(x);
    if (t.n > 1) {
      const int rf = (int)G.reginvs.size();
      for (int x = 1; x < t.n; ++x) {
        RegInvOp q{};
        q.rho = (const double*)ws(P.vmf_rho_off[x]);
        q.M = (double*)ws(P.vmf_rinv_off[x]);
        q.reg = reg;
        q.r = t.rank[x];
        G.reginvs.push_back(q);
      }
      launch(LK_REGINV, 0, rf, t.n - 1, 0, 0);
    }
    // every node's effective generator in one contraction launch
    const int pfirst = (int)G.presums.size();
    const int gfirst = (int)G.groups.size(), tfirst = (int)G.atiles.size();
    std::vector<int> nparts(t.n);
    for (int s = 0; s < t.n; ++s) {
      const Recipe R = node_recipe(P, s);
      // capacities were taken at the capacity ranks (the current ones are not larger)
      nparts[s] = add_apply(R, core(s), 1, t.size(s), 0, 1, std::max(1, P.par_target / t.n),
                            ApplyArea{P.vmf_node_parts[s], P.vmf_node_presum[s],
                                      (size_t)1 << 40, (size_t)1 << 40},
                            gfirst);
    }
    const int np = (int)G.presums.size() - pfirst;
    if (np) launch(LK_PRESUM, 0, pfirst, np, 0, 0);
    launch(LK_APPLY, 1, gfirst, (int)G.groups.size() - gfirst, tfirst,
           (int)G.atiles.size() - tfirst);
    // partial sums into the derivative buffer
    const int cf = (int)G.combines.size(), ctf = (int)G.ctiles.size();
    for (int s = 0; s < t.n; ++s) {
      CombineOp op{};
      const long n = t.size(s);
      op.y0 = (double*)ws(P.ws_vmf_kout + P.core_off[s]);
      op.xin = ws(P.ws_xin);
      op.acc = (double*)ws(P.ws_acc);
      op.parts = ws(P.vmf_node_parts[s]);
      op.n = n;
      op.n_parts = nparts[s];
      op.stage = 0;
      const int oi = (int)G.combines.size();
      G.combines.push_back(op);
      for (long e = 0; e < n; e += kCombineTile) G.ctiles.push_back({oi, 0, e, std::min(n, e + kCombineTile)});
    }
    launch(LK_COMBINE, 0, cf, t.n, ctf, (int)G.ctiles.size() - ctf);
    if (t.n == 1) return;
    // (rho_x + reg)^-1 on the parent leg of every non-root derivative
    const int af = (int)G.absorbs.size(), atf = (int)G.abtiles.size();
    size_t lds = 0;
    for (int x = 1; x < t.n; ++x) {
      AbsorbOp a{};
      a.C = (double*)ws(P.ws_vmf_kout + P.core_off[x]);
      a.M = (const double*)ws(P.vmf_rinv_off[x]);
      a.n = t.rank[x];
      a.Ppre = 1;
      a.Ppost = (int)(t.size(x) / t.rank[x]);
      a.transposeM = 0;
      const int ai = (int)G.absorbs.size();
      G.absorbs.push_back(a);
      const int fibers = a.Ppost;
      const int per = std::max(1, absorb_tile_elems(P.par_target) / a.n);
      for (int f = 0; f < fibers; f += per) G.abtiles.push_back({ai, f, std::min(fibers, f + per)});
      lds = std::max(lds, absorb_lds(a.n, per));
    }
    launch(LK_ABSORB, 0, af, t.n - 1, atf, (int)G.abtiles.size() - atf, lds);
    // S_x = U_x^H dU_x over the non-parent legs, then dU_x -= U_x S_x
    const int qf = (int)G.grams.size();
    for (int x = 1; x < t.n; ++x) {
      GramOp go{};
      go.C = (const double*)core(x);
      go.T = ws(P.ws_vmf_kout + P.core_off[x]);
      go.E = ws(P.vmf_s_off[x]);
      go.r = t.rank[x];
      go.Ppre = 1;
      go.Ppost = (int)(t.size(x) / t.rank[x]);
      G.grams.push_back(go);
    }
    launch(LK_GRAM, 0, qf, t.n - 1, 0, 0);
    const int vf = (int)G.vprojs.size();
    long mx = 1;
    for (int x = 1; x < t.n; ++x) {
      VProjOp v{};
      v.Y = (double*)ws(P.ws_vmf_kout + P.core_off[x]);
      v.U = (const double*)core(x);
      v.S = (const double*)ws(P.vmf_s_off[x]);
      v.r = t.rank[x];
      v.post = t.size(x) / t.rank[x];
      G.vprojs.push_back(v);
      mx = std::max(mx, t.size(x));
    }
    launch(LK_VPROJ, 0, vf, t.n - 1, 0, 0, (size_t)mx);
  }
};

// -- resolution & upload ------------------------------------------------------
static void* res(void* p, void* state, void* ws) {
  uint64_t v = (uint64_t)p;
  int tag = (int)(v >> 56);
  uint64_t off = v & OFF_MASK;
  if (tag == TAG_STATE) return (char*)state + off;
  if (tag == TAG_WS) return (char*)ws + off;
  return p;
}

template <class T>
static size_t put(std::vector<char>& buf, const std::vector<T>& v) {
  size_t o = align256(buf.size());
  buf.resize(o + v.size() * sizeof(T));
  if (!v.empty()) memcpy(buf.data() + o, v.data(), v.size() * sizeof(T));
  return o;
}

// Resolve state / workspace tags and per-step scalars of one instance's
// program (term and rho-node references stay as indices).
static void resolve(Program& G, void* state, void* ws, double dt, const double* drive,
                    int drive_ld) {
  for (auto& t : G.terms) {
    t.A = res((void*)t.A, state, ws);
    t.B = res((void*)t.B, state, ws);
  }
  for (auto& g : G.groups) {
    g.X = res((void*)g.X, state, ws);
    g.Y = res(g.Y, state, ws);
    g.drive = drive;
    g.drive_ld = drive_ld;
    if (g.in_fp64 == 2) {  // the stage coefficient as the combine kernel forms it
      g.xp = res((void*)g.xp, state, ws);
      const double h = g.xp_s * 0.5 * dt;
      g.xp_s = g.xp_half ? 0.5 * h : h;
    }
  }
  for (auto& p : G.presums) {
    p.out = res(p.out, state, ws);
    p.drive = drive;
    p.drive_ld = drive_ld;
  }
  for (auto& c : G.combines) {
    c.y0 = (double*)res(c.y0, state, ws);
    c.xin = res(c.xin, state, ws);
    c.acc = (double*)res(c.acc, state, ws);
    c.parts = res((void*)c.parts, state, ws);
    c.h = c.h * 0.5 * dt;
  }
  for (auto& q : G.qrs) {
    q.C = (double*)res(q.C, state, ws);
    q.R = (double*)res(q.R, state, ws);
    q.V = (double*)res(q.V, state, ws);
    q.tau = (double*)res(q.tau, state, ws);
  }
  for (auto& a : G.absorbs) {
    a.C = (double*)res(a.C, state, ws);
    a.M = (const double*)res((void*)a.M, state, ws);
  }
  for (auto& g : G.grams) {
    g.C = (const double*)res((void*)g.C, state, ws);
    g.T = res((void*)g.T, state, ws);
    g.E = res(g.E, state, ws);
  }
  for (auto& n : G.rnodes) n.C = (const double*)res((void*)n.C, state, ws);
  for (auto& r : G.rprogs) {
    r.vecs = (double*)res(r.vecs, state, ws);
    r.rho_out = (double*)res(r.rho_out, state, ws);
  }
  for (auto& q : G.reginvs) {
    q.rho = (const double*)res((void*)q.rho, state, ws);
    q.M = (double*)res(q.M, state, ws);
  }
  for (auto& v : G.vprojs) {
    v.Y = (double*)res(v.Y, state, ws);
    v.U = (const double*)res((void*)v.U, state, ws);
    v.S = (const double*)res((void*)v.S, state, ws);
  }
}

// Upload a resolved program, turning term / rho-node indices into pointers.
// Copy a resolved program's descriptors into D's device arena (grown when
// too small).  Without `hold` the call waits for the copy; with it, the host
// buffer is kept in *hold and the caller must synchronise the stream before
// clearing it (the arena itself is reused in stream order).
static void upload_resolved(DevProgram& D, const Program& G, hipStream_t s,
                            std::vector<std::vector<char>>* hold = nullptr) {
  std::vector<char> buf;
  D.o_terms = put(buf, G.terms);
  D.o_groups = put(buf, G.groups);
  D.o_atiles = put(buf, G.atiles);
  D.o_presums = put(buf, G.presums);
  D.o_combines = put(buf, G.combines);
  D.o_ctiles = put(buf, G.ctiles);
  D.o_qrs = put(buf, G.qrs);
  D.o_absorbs = put(buf, G.absorbs);
  D.o_abtiles = put(buf, G.abtiles);
  D.o_grams = put(buf, G.grams);
  D.o_rnodes = put(buf, G.rnodes);
  D.o_rprogs = put(buf, G.rprogs);
  D.o_reginvs = put(buf, G.reginvs);
  D.o_vprojs = put(buf, G.vprojs);
  if (D.external && D.bytes < buf.size())
    fail(TENSO_ENOMEM, "launch descriptors exceed the scratch space left for them");
  if (!D.arena || D.bytes < buf.size()) {
    if (D.arena) hipchk(hipFree(D.arena), "hipFree");
    D.arena = nullptr;
    hipchk(hipMalloc((void**)&D.arena, std::max<size_t>(buf.size(), 256)), "hipMalloc(program)");
    D.bytes = std::max<size_t>(buf.size(), 256);
  }
  char* base = D.arena;
  auto term_ptr = [&](const TermRef* p) -> const TermRef* {
    uint64_t v = (uint64_t)p;
    if ((int)(v >> 56) != TAG_TERM) return p;
    return (const TermRef*)(base + D.o_terms + (v & OFF_MASK) * sizeof(TermRef));
  };
  ApplyGroup* gp = (ApplyGroup*)(buf.data() + D.o_groups);
  for (size_t i = 0; i < G.groups.size(); ++i) gp[i].terms = term_ptr(gp[i].terms);
  PresumOp* pp = (PresumOp*)(buf.data() + D.o_presums);
  for (size_t i = 0; i < G.presums.size(); ++i) pp[i].terms = term_ptr(pp[i].terms);
  RhoProg* rp = (RhoProg*)(buf.data() + D.o_rprogs);
  for (size_t i = 0; i < G.rprogs.size(); ++i) {
    uint64_t v = (uint64_t)rp[i].nodes;
    rp[i].nodes = (const RhoNode*)(base + D.o_rnodes + (v & OFF_MASK) * sizeof(RhoNode));
  }
  hipchk(hipMemcpyAsync(D.arena, buf.data(), buf.size(), hipMemcpyHostToDevice, s), "upload program");
  if (hold) hold->push_back(std::move(buf));
  else hipchk(hipStreamSynchronize(s), "sync upload");
  D.launches = G.launches;
  for (auto& L : D.launches)  // QR launches: lds holds the form that serves every op
    if (L.kind == LK_QR) {
      int f = kQrFormLds;
      for (int k = L.first; k < L.first + L.count; ++k) f = qr_form_join(f, qr_form(G.qrs[k]));
      L.lds = (size_t)f;
    }
}

static void upload(DevProgram& D, const Program& G0, void* state, void* ws, double dt,
                   const double* drive, int drive_ld, hipStream_t s,
                   std::vector<std::vector<char>>* hold = nullptr) {
  Program G = G0;
  resolve(G, state, ws, dt, drive, drive_ld);
  upload_resolved(D, G, s, hold);
}

// Merge resolved per-instance programs into one launch sequence: at each
// phase the kernel type whose waiting instances have the most remaining
// launches (critical path first) is issued for all instances waiting on it.
static Program merge_programs(std::vector<Program>& progs) {
  Program M;
  const size_t n = progs.size();
  std::vector<int> term_off(n), rn_off(n);
  for (size_t i = 0; i < n; ++i) {
    term_off[i] = (int)M.terms.size();
    M.terms.insert(M.terms.end(), progs[i].terms.begin(), progs[i].terms.end());
    rn_off[i] = (int)M.rnodes.size();
    M.rnodes.insert(M.rnodes.end(), progs[i].rnodes.begin(), progs[i].rnodes.end());
  }
  auto shift_term = [](const TermRef* p, int off) -> const TermRef* {
    uint64_t v = (uint64_t)p;
    if ((int)(v >> 56) != TAG_TERM) return p;
    return (const TermRef*)tagp(TAG_TERM, (v & OFF_MASK) + off);
  };
  std::vector<size_t> pos(n, 0);
  auto type_of = [](const LaunchRec& L) { return L.kind * 4 + L.in_fp64; };
  while (true) {
    std::map<int, long> weight;
    for (size_t i = 0; i < n; ++i)
      if (pos[i] < progs[i].launches.size())
        weight[type_of(progs[i].launches[pos[i]])] += (long)(progs[i].launches.size() - pos[i]);
    if (weight.empty()) break;
    int best = -1;
    long bw = -1;
    for (auto& kv : weight)
      if (kv.second > bw) {
        bw = kv.second;
        best = kv.first;
      }
    LaunchRec ML{best / 4, best % 4, 0, 0, 0, 0, 0};
    const int kind = best / 4;
    switch (kind) {
      case LK_APPLY: ML.first = (int)M.groups.size(); ML.tfirst = (int)M.atiles.size(); break;
      case LK_PRESUM: ML.first = (int)M.presums.size(); break;
      case LK_COMBINE: ML.first = (int)M.combines.size(); ML.tfirst = (int)M.ctiles.size(); break;
      case LK_QR: ML.first = (int)M.qrs.size(); break;
      case LK_ABSORB: ML.first = (int)M.absorbs.size(); ML.tfirst = (int)M.abtiles.size(); break;
      case LK_GRAM: ML.first = (int)M.grams.size(); break;
      case LK_RHO: ML.first = (int)M.rprogs.size(); break;
    }
    for (size_t i = 0; i < n; ++i) {
      if (pos[i] >= progs[i].launches.size()) continue;
      const LaunchRec& L = progs[i].launches[pos[i]];
      if (type_of(L) != best) continue;
      ++pos[i];
      Program& P = progs[i];
      ML.flops += L.flops;
      ML.bytes += L.bytes;
      ML.amode = L.amode;
      ML.lds = std::max(ML.lds, L.lds);
      switch (kind) {
        case LK_APPLY: {
          const int goff = (int)M.groups.size() - ML.first;
          for (int g = L.first; g < L.first + L.count; ++g) {
            ApplyGroup ag = P.groups[g];
            ag.terms = shift_term(ag.terms, term_off[i]);
            M.groups.push_back(ag);
          }
          for (int t = L.tfirst; t < L.tfirst + L.tcount; ++t) {
            ApplyTile tl = P.atiles[t];
            tl.group += goff;
            M.atiles.push_back(tl);
          }
          break;
        }
        case LK_PRESUM:
          for (int k = L.first; k < L.first + L.count; ++k) {
            PresumOp op = P.presums[k];
            op.terms = shift_term(op.terms, term_off[i]);
            M.presums.push_back(op);
          }
          break;
        case LK_COMBINE: {
          const int base = (int)M.combines.size();
          for (int k = L.first; k < L.first + L.count; ++k) M.combines.push_back(P.combines[k]);
          for (int t = L.tfirst; t < L.tfirst + L.tcount; ++t) {
            CombineTileH ct = P.ctiles[t];
            ct.op = base + (ct.op - L.first);
            M.ctiles.push_back(ct);
          }
          break;
        }
        case LK_QR:
          for (int k = L.first; k < L.first + L.count; ++k) M.qrs.push_back(P.qrs[k]);
          break;
        case LK_ABSORB: {
          const int base = (int)M.absorbs.size();
          for (int k = L.first; k < L.first + L.count; ++k) M.absorbs.push_back(P.absorbs[k]);
          for (int t = L.tfirst; t < L.tfirst + L.tcount; ++t) {
            AbsorbTileH at = P.abtiles[t];
            at.op = base + (at.op - L.first);
            M.abtiles.push_back(at);
          }
          break;
        }
        case LK_GRAM:
          for (int k = L.first; k < L.first + L.count; ++k) M.grams.push_back(P.grams[k]);
          break;
        case LK_RHO:
          for (int k = L.first; k < L.first + L.count; ++k) {
            RhoProg rp = P.rprogs[k];
            uint64_t v = (uint64_t)rp.nodes;
            rp.nodes = (const RhoNode*)tagp(TAG_RNODE, (v & OFF_MASK) + rn_off[i]);
            M.rprogs.push_back(rp);
          }
          break;
      }
    }
    switch (kind) {
      case LK_APPLY:
        ML.count = (int)M.groups.size() - ML.first;
        ML.tcount = (int)M.atiles.size() - ML.tfirst;
        break;
      case LK_PRESUM: ML.count = (int)M.presums.size() - ML.first; break;
      case LK_COMBINE:
        ML.count = (int)M.combines.size() - ML.first;
        ML.tcount = (int)M.ctiles.size() - ML.tfirst;
        break;
      case LK_QR: ML.count = (int)M.qrs.size() - ML.first; break;
      case LK_ABSORB:
        ML.count = (int)M.absorbs.size() - ML.first;
        ML.tcount = (int)M.abtiles.size() - ML.tfirst;
        break;
      case LK_GRAM: ML.count = (int)M.grams.size() - ML.first; break;
      case LK_RHO: ML.count = (int)M.rprogs.size() - ML.first; break;
    }
    M.launches.push_back(ML);
  }
  return M;
}

// Optional timing of the apply kernel (the SOP contraction): HIP start/stop
// events taken by every apply launch's own dispatch on the caller's stream,
// with its algorithmic work.
struct Prof {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  std::vector<std::pair<double, double>> work;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      hipchk(hipEventCreate(&e), "hipEventCreate");
      pool.push_back(e);
    }
    return pool[used++];
  }
};
static Prof g_prof;

static void run(const DevProgram& D, int fp64, const int* ctr, hipStream_t s) {
  char* b = D.arena;
  for (const auto& L : D.launches) {
    hipError_t e = hipSuccess;
    switch (L.kind) {
      case LK_APPLY:
        if (g_prof.on) {
          hipEvent_t e0 = g_prof.get(), e1 = g_prof.get();
          e = launch_apply(fp64 ? 1 : L.amode, L.in_fp64,
                           (const ApplyGroup*)(b + D.o_groups) + L.first,
                           (const ApplyTile*)(b + D.o_atiles) + L.tfirst, L.tcount, ctr, L.lds, s,
                           e0, e1);
          g_prof.ev.push_back({e0, e1});
          g_prof.work.push_back({L.flops, L.bytes});
          break;
        }
        e = launch_apply(fp64 ? 1 : L.amode, L.in_fp64,
                         (const ApplyGroup*)(b + D.o_groups) + L.first,
                         (const ApplyTile*)(b + D.o_atiles) + L.tfirst, L.tcount, ctr, L.lds, s);
        break;
      case LK_PRESUM:
        e = launch_presum(fp64, (const PresumOp*)(b + D.o_presums) + L.first, L.count, ctr, s);
        break;
      case LK_COMBINE:
        e = launch_combine(fp64, (const CombineOp*)(b + D.o_combines),
                           (const CombineTileH*)(b + D.o_ctiles) + L.tfirst, L.tcount, s);
        break;
      case LK_QR:
        e = launch_qr((const QrOp*)(b + D.o_qrs) + L.first, L.count, (int)L.lds, s);
        break;
      case LK_ABSORB:
        e = launch_absorb((const AbsorbOp*)(b + D.o_absorbs),
                          (const AbsorbTileH*)(b + D.o_abtiles) + L.tfirst, L.tcount, L.lds, s);
        break;
      case LK_GRAM:
        e = launch_gram(fp64, (const GramOp*)(b + D.o_grams) + L.first, L.count, s);
        break;
      case LK_RHO:
        e = launch_rho((const RhoProg*)(b + D.o_rprogs) + L.first, L.count, s);
        break;
      case LK_REGINV:
        e = launch_reginv((const RegInvOp*)(b + D.o_reginvs) + L.first, L.count, s);
        break;
      case LK_VPROJ:  // lds: the largest core of the launch (complex elements)
        e = launch_vproj((const VProjOp*)(b + D.o_vprojs) + L.first, L.count, (long)L.lds, s);
        break;
    }
    hipchk(e, "kernel launch");
  }
}

// Capture one step (program launches, then the step-counter advance).
static void capture_step(StepGraph& G, const std::vector<const DevProgram*>& parts, int fp64,
                         int* ctr) {
  if (!G.cap) hipchk(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking), "hipStreamCreate");
  while (G.side.size() + 1 < parts.size()) {
    hipStream_t x;
    hipchk(hipStreamCreateWithFlags(&x, hipStreamNonBlocking), "hipStreamCreate");
    G.side.push_back(x);
  }
  while (G.ev.size() < parts.size()) {
    hipEvent_t e;
    hipchk(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    G.ev.push_back(e);
  }
  hipGraph_t g = nullptr;
  hipchk(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  try {
    if (parts.size() > 1) hipchk(hipEventRecord(G.ev[0], G.cap), "fork");
    for (size_t k = 1; k < parts.size(); ++k) {
      hipchk(hipStreamWaitEvent(G.side[k - 1], G.ev[0], 0), "fork wait");
      run(*parts[k], fp64, ctr, G.side[k - 1]);
      hipchk(hipEventRecord(G.ev[k], G.side[k - 1]), "join");
    }
    run(*parts[0], fp64, ctr, G.cap);
    for (size_t k = 1; k < parts.size(); ++k) hipchk(hipStreamWaitEvent(G.cap, G.ev[k], 0), "join wait");
    hipchk(launch_step_inc(ctr, -1, G.cap), "ctr");
  } catch (...) {
    (void)hipStreamEndCapture(G.cap, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  hipchk(hipStreamEndCapture(G.cap, &g), "hipStreamEndCapture");
  const hipError_t e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  hipchk(e, "hipGraphInstantiate");
}

// n_steps steps of program D: graph replays when enabled (the first step of
// a fresh binding runs eagerly, which also performs the kernels' one-time
// attribute setup outside any capture), eager launches otherwise or while
// the apply kernels are being timed.
static void step_loop(StepGraph& G, const std::vector<const DevProgram*>& parts, int fp64,
                      int* ctr, int n_steps, hipStream_t s) {
  const bool use = G.enabled && !g_prof.on;
  for (int k = 0; k < n_steps; ++k) {
    if (use && G.exec) {
      hipchk(hipGraphLaunch(G.exec, s), "hipGraphLaunch");
      continue;
    }
    for (auto* D : parts) run(*D, fp64, ctr, s);  // eager: parts one after another
    hipchk(launch_step_inc(ctr, -1, s), "ctr");
    if (use) capture_step(G, parts, fp64, ctr);
  }
}

// Norm of the plan's root core (the state's norm: the state is canonical
// toward the root between step calls) into the workspace slot `slot` (0:
// before the call, 1: after it).
static void plan_root_norm(tenso_plan* p, void* d_state, void* d_ws, int slot, hipStream_t s) {
  char* base = (char*)d_ws + p->ws_ctr;
  NormOp op{};
  op.p = (const double*)((const char*)d_state + p->core_off[0]);
  op.n = 2 * p->tree.size(0);
  hipchk(hipMemcpyAsync(base + 160, &op, sizeof(op), hipMemcpyHostToDevice, s), "norm op");
  hipchk(launch_norms((const NormOp*)(base + 160), 1, (double*)(base + 192) + slot, s), "root norm");
}

// After stepping: non-finite values in the plan's state, or a norm grown by
// more than kNormGrowthLimit over the call, are ENUMERIC.  Two small
// launches and one synchronisation per step call.
static void check_plan_finite(tenso_plan* p, void* d_state, void* d_ws, hipStream_t s) {
  char* base = (char*)d_ws + p->ws_ctr;
  FiniteOp op{};
  op.p = (const double*)d_state;
  op.n = (long)(p->state_bytes / sizeof(double));
  op.flag = (int*)(base + 64);
  hipchk(hipMemcpyAsync(base + 128, &op, sizeof(op), hipMemcpyHostToDevice, s), "finite op");
  hipchk(launch_finite((const FiniteOp*)(base + 128), 1, op.flag, s), "finite check");
  plan_root_norm(p, d_state, d_ws, 1, s);
  int flag = 0;
  double norms[2] = {0, 0};
  hipchk(hipMemcpyAsync(&flag, op.flag, sizeof(int), hipMemcpyDeviceToHost, s), "finite flag");
  hipchk(hipMemcpyAsync(norms, base + 192, sizeof(norms), hipMemcpyDeviceToHost, s), "norms");
  hipchk(hipStreamSynchronize(s), "sync");
  if (flag) fail(TENSO_ENUMERIC, "non-finite values in the state after stepping");
  if (norms[1] > kNormGrowthLimit * norms[0])
    fail(TENSO_ENUMERIC, "state norm grew by more than a factor 1e6 over the step call");
}

// Tile group indices are relative to the first group of their launch.
static void fix_tile_groups(Program& G) {
  for (auto& L : G.launches) {
    if (L.kind != LK_APPLY) continue;
    // tiles already carry indices relative to the launch's first group
    (void)L;
  }
}

static void build_step(tenso_plan& P, Program& G) {
  Builder b(P, G);
  b.V(0, 0);
  b.Vstar(0, 1);
  fix_tile_groups(G);
}

static void build_init(tenso_plan& P, Program& G) {
  Builder b(P, G);
  for (int x = P.tree.n - 1; x >= 1; --x) {
    b.emit_env_down(x);
  }
}

// ---------------------------------------------------------------------------
// ps2 split: FP64 SVD of the two-site tensor and the truncation decision
// ---------------------------------------------------------------------------
// Device scratch of one SVD (see svd.hip for the method).  Sizes for sides up
// to `side`: y, z, qrv, e hold side x 64 complex; part kSvdMaxSplit times that;
// r, up, wp 64 x 64; sig 64 doubles; tau 64 complex; norm
// ceil(side / 64) * kSvdMaxSplit doubles; rec 256 bytes; opbuf 4 x 512 bytes.
struct SvdScratch {
  double *y, *z, *part, *qrv, *r, *up, *wp, *sig, *tau, *norm, *e;
  char* rec;
  char* opbuf;
};

static SvdScratch svd_scratch(const tenso_plan& P, void* ws) {
  char* w = (char*)ws;
  return SvdScratch{(double*)(w + P.ws_svd_y),   (double*)(w + P.ws_svd_z),
                    (double*)(w + P.ws_svd_part), (double*)(w + P.ws_svd_qrv),
                    (double*)(w + P.ws_svd_r),    (double*)(w + P.ws_svd_up),
                    (double*)(w + P.ws_svd_wp),   (double*)(w + P.ws_svd_sig),
                    (double*)(w + P.ws_svd_tau),  (double*)(w + P.ws_svd_norm),
                    (double*)(w + P.ws_svd_e),    w + P.ws_svd_rec, nullptr};
}

// Single-op descriptor upload into slot `slot` of sc.opbuf; the host bytes
// stay in `hold` until the caller's next synchronisation.
template <class T>
static const T* svd_put(const SvdScratch& sc, int slot, const T& op, hipStream_t s,
                        std::vector<std::vector<char>>& hold) {
  char* dst = sc.opbuf + slot * 512;
  std::vector<char> bytes(sizeof(T));
  memcpy(bytes.data(), &op, sizeof(T));
  hipchk(hipMemcpyAsync(dst, bytes.data(), sizeof(T), hipMemcpyHostToDevice, s), "op upload");
  hold.push_back(std::move(bytes));
  return (const T*)dst;
}

// SVD of theta (rows x cols, row-major complex FP64) and the truncation
// decision for (eps, max_rank, cap_r): sc.e receives the leading singular
// vectors of the isometry side (iso 0: left, rows x p; iso 1: right, cols x p;
// row-major with leading dimension p), sc.sig the p singular values; the
// width p is returned.  rec_i = {r', k, r_eps}, rec_d = {||theta||_F^2,
// energy outside the captured subspace when it may be incomplete, else 0}.
// Synchronises `s` once per pass (the decision is read back).
//   Width: first svd_width(...) test columns (the kept rank plus room, at most
// 64).  When p is below the smaller side and s_{p-1} exceeds 1e-13 s_1 (the
// numerical rank may exceed p), power steps are added until the leading
// min(p, cap_r + 1) singular values move by at most 1e-14 s_1 between passes
// (at most kSvdMaxPower); but if after the first pass s_{p-1} exceeds 0.01
// s_{keep-1} (a flat spectrum, where power steps converge slowly), the
// factorisation restarts at the full width min(64, rows, cols).
static int svd_width(long rows, long cols, int max_rank, int cap_r) {
  const long keep = std::min(max_rank, cap_r);
  return (int)std::min<long>({(long)kSvdP, rows, cols, 2 * keep + 8});
}

static int svd_truncate(const SvdScratch& sc, const double* theta, long rows, long cols, int iso,
                        double eps, int max_rank, int cap_r, hipStream_t s,
                        std::vector<std::vector<char>>& hold, int rec_i[3], double rec_d[2],
                        double atol = 0.0, double ratio = 0.0) {
  const int full = (int)std::min<long>({(long)kSvdP, rows, cols});
  int p = svd_width(rows, cols, max_rank, cap_r);
  const int keep = std::max(1, std::min({max_rank, cap_r, p}));
  for (;;) {
    int n_norm = 0;
    // out = theta B (mode 0) or theta^H B (mode 1); B null: the test matrix
    auto gemm = [&](int mode, const double* B, double* out, bool norm) {
      const int M = (int)(mode == 0 ? rows : cols), K = (int)(mode == 0 ? cols : rows);
      const int mt = (M + 63) / 64;
      int nsplit = std::min(kSvdMaxSplit, std::max(1, K / 256));
      const int kchunk = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
      nsplit = (K + kchunk - 1) / kchunk;
      SvdGemmOp g{theta, B, out, sc.part, norm ? sc.norm : nullptr, (int)rows, (int)cols, p, mode,
                  nsplit, kchunk, 0x5EEDu, 0};
      const SvdGemmOp* d = svd_put(sc, 0, g, s, hold);
      hipchk(launch_svd_gemm(d, mt, nsplit, s), "svd product");
      if (nsplit > 1) hipchk(launch_svd_reduce(d, (long)M * p, s), "svd reduce");
      if (norm) n_norm = mt * nsplit;
    };
    auto qr = [&](double* A, int m) {
      QrOp q{};
      q.C = A;
      q.R = sc.r;
      q.V = sc.qrv;
      q.tau = sc.tau;
      q.m = m;
      q.n = p;
      q.Ppost = m;
      q.transposeR = 0;
      q.tol = 0.0;
      hipchk(launch_qr(svd_put(sc, 1, q, s, hold), 1, qr_form(q), s), "svd qr");
    };
    // range finder on theta's column space, then the projection Z = theta^H Q
    gemm(0, nullptr, sc.y, true);
    qr(sc.y, (int)rows);
    const int nwatch = std::min(p, cap_r + 1);
    double sig[kSvdP], prev[kSvdP];
    bool widen = false;
    for (int power = 0;; ++power) {
      gemm(1, sc.y, sc.z, false);
      qr(sc.z, (int)cols);
      SvdJacobiOp jo{sc.r, sc.up, sc.wp, sc.sig, p, kSvdMaxSweeps};
      hipchk(launch_svd_jacobi(svd_put(sc, 2, jo, s, hold), s), "svd jacobi");
      SvdFinishOp fo{sc.y, sc.z, sc.up, sc.wp, sc.sig, sc.norm, sc.e, (int*)sc.rec,
                     (double*)(sc.rec + 64), eps, n_norm, (int)rows, (int)cols, p, iso, max_rank,
                     cap_r, 0, atol, ratio};
      hipchk(launch_svd_finish(svd_put(sc, 3, fo, s, hold), (iso == 0 ? rows : cols) * (long)p, s),
             "svd finish");
      hipchk(hipMemcpyAsync(rec_i, sc.rec, 3 * sizeof(int), hipMemcpyDeviceToHost, s), "decision");
      hipchk(hipMemcpyAsync(rec_d, sc.rec + 64, 2 * sizeof(double), hipMemcpyDeviceToHost, s),
             "decision");
      hipchk(hipMemcpyAsync(sig, sc.sig, p * sizeof(double), hipMemcpyDeviceToHost, s), "sigma");
      hipchk(hipStreamSynchronize(s), "sync");
      hold.clear();
      // captured subspace complete (p is the smaller side, or the last captured
      // singular value is at rounding level): done
      if (p == std::min(rows, cols) || sig[p - 1] <= 1e-13 * sig[0]) break;
      if (power == 0 && p < full && sig[p - 1] > 0.01 * sig[keep - 1]) {
        widen = true;
        break;
      }
      if (power >= kSvdMaxPower) break;
      if (power > 0) {
        double moved = 0;
        for (int j = 0; j < nwatch; ++j) moved = std::max(moved, std::fabs(sig[j] - prev[j]));
        if (moved <= 1e-14 * sig[0]) break;
      }
      for (int j = 0; j < nwatch; ++j) prev[j] = sig[j];
      gemm(0, sc.z, sc.y, false);
      qr(sc.y, (int)rows);
    }
    if (!widen) return p;
    p = full;
  }
}

// ---------------------------------------------------------------------------
// ps2: host-driven two-site sweep (ranks decided on the device per edge and
// read back, since they set the shapes of the following sub-flows)
// ---------------------------------------------------------------------------
struct Ps2Exec {
  tenso_plan& P;
  void* state;
  void* ws;
  double dt;
  const double* drive;
  int ld;
  hipStream_t s;
  int max_rank;
  double eps;
  int* ctr = nullptr;
  // host copies of the programs uploaded since the last synchronisation (the
  // eigenvalue read of each edge, the end of the call); uploads do not wait
  std::vector<std::vector<char>> hold;
  // on every exit, error paths included, no copy may still read `hold`
  ~Ps2Exec() { (void)hipStreamSynchronize(s); }

  char* wsb(size_t off) { return (char*)ws + off; }
  double* core(int x) { return (double*)((char*)state + P.core_off[x]); }

  // A sub-flow's program depends only on the plan, the binding and the current
  // bond ranks: it is built and uploaded the first time and replayed after
  // (ranks settle at the cap within a few steps).
  template <class F>
  void exec_cached(const std::string& tag, F build) {
    std::string key = tag;
    for (int r : P.tree.rank) {
      key += ',';
      key += std::to_string(r);
    }
    auto it = P.ps2_progs.find(key);
    if (it == P.ps2_progs.end()) {
      if (P.ps2_progs.size() >= 4096) {  // bound the cache (ranks still moving)
        hipchk(hipStreamSynchronize(s), "sync");
        P.ps2_progs.clear();
      }
      Program G;
      build(G);
      auto D_ = std::make_unique<DevProgram>();
      upload(*D_, G, state, ws, dt, drive, ld, s, &hold);
      it = P.ps2_progs.emplace(key, std::move(D_)).first;
    }
    run(*it->second, P.fp64, ctr, s);
  }
  static std::string tag(char k, std::initializer_list<int> a) {
    std::string t(1, k);
    for (int v : a) {
      t += ':';
      t += std::to_string(v);
    }
    return t + '|';
  }

  void env_down(int x) {
    exec_cached(tag('D', {x}), [&](Program& G) {
      Builder b(P, G);
      b.emit_env_down(x);
    });
  }
  void env_up(int x) {
    exec_cached(tag('U', {x}), [&](Program& G) {
      Builder b(P, G);
      b.emit_env_up(x);
    });
  }
  void node_bwd(int x, int half) {
    exec_cached(tag('N', {x, half}), [&](Program& G) {
      Builder b(P, G);
      b.emit_rk4(node_recipe(P, x), b.core(x), P.tree.size(x), -1.0, half);
    });
  }
  // QR of core `a` toward leg `la`, R absorbed into core `b` on leg `lb`
  void move(int a, int la, int b_, int lb) {
    exec_cached(tag('M', {a, la, b_, lb}), [&](Program& G) {
      Builder b(P, G);
      b.emit_qr(a, la, 0);
      b.emit_absorb(b_, lb, 0);
    });
  }
  // single-op descriptors: the host bytes go into `hold` (alive until the next
  // synchronisation), like the programs' host buffers
  template <class T>
  const T* put_op(const T& op, size_t slot) {
    char* dst = (char*)P.opbuf + slot * 512;
    std::vector<char> bytes(sizeof(T));
    memcpy(bytes.data(), &op, sizeof(T));
    hipchk(hipMemcpyAsync(dst, bytes.data(), sizeof(T), hipMemcpyHostToDevice, s), "op upload");
    hold.push_back(std::move(bytes));
    return (const T*)dst;
  }

  void edge(int sn, int c, int half, bool center_to_child) {
    tenso_tree& t = P.tree;
    const int i = t.leg_of_child(sn, c);
    const int r = t.rank[c];
    const std::vector<int> ds = t.shape(sn);
    const long rows = t.size(sn) / r, cols = t.size(c) / r;
    long ppost = 1;
    for (int j = i + 1; j < (int)ds.size(); ++j) ppost *= ds[j];
    double* theta = (double*)wsb(P.ws_theta);
    MergeOp mo{core(sn), core(c), theta, (int)rows, (int)cols, r, (int)ppost};
    hipchk(launch_merge(put_op(mo, 0), rows * cols, s), "merge");
    exec_cached(tag('E', {sn, c, half}), [&](Program& G) {
      Builder b(P, G);
      b.emit_rk4(edge_recipe(P, sn, c), b.ws(P.ws_theta), rows * cols, +1.0, half);
    });
    const int iso = center_to_child ? 0 : 1;
    SvdScratch sc = svd_scratch(P, ws);
    sc.opbuf = (char*)P.opbuf + 4096;
    int rec_i[3] = {0, 0, 0};
    double rec_d[2] = {0, 0};
    const int p =
        svd_truncate(sc, theta, rows, cols, iso, eps, max_rank, P.cap.rank[c], s, hold, rec_i, rec_d,
                     P.ps2_atol, P.ps2_ratio);
    const int rp = rec_i[0], k = rec_i[1];
    if (rp < 1 || rp > P.cap.rank[c] || k < 0 || k > rp)
      fail(TENSO_ENUMERIC, "ps2 truncation decision out of range");
    // the ranks of the new cores must stay within the capacity layout
    t.rank[c] = rp;
    const std::vector<int> ds2 = t.shape(sn);
    long ppost2 = 1;
    for (int j = i + 1; j < (int)ds2.size(); ++j) ppost2 *= ds2[j];
    SplitOp so{theta, sc.e, (int)rows, (int)cols, iso, k, rp, p,
               (double*)wsb(P.ws_W), core(sn), core(c), (int)ppost2, 0};
    if ((size_t)std::max(rows, cols) * rp > P.W_cap) fail(TENSO_ENOMEM, "ps2 split scratch");
    hipchk(launch_split(put_op(so, 2), s), "split");
    P.rank_log.push_back(rp);
  }

  void W(int sn, int half) {
    tenso_tree& t = P.tree;
    const std::vector<int> kids = t.children[sn];
    for (size_t idx = 0; idx < kids.size(); ++idx) {
      const int c = kids[idx];
      const int i = t.leg_of_child(sn, c);
      edge(sn, c, half, true);
      env_up(c);
      if (!t.children[c].empty()) {
        node_bwd(c, half);
        W(c, half);
      }
      move(c, 0, sn, i);
      env_down(c);
      if (idx + 1 < kids.size()) node_bwd(sn, half);
    }
  }
  void Wstar(int sn, int half) {
    tenso_tree& t = P.tree;
    const std::vector<int> kids = t.children[sn];
    for (int idx = (int)kids.size() - 1; idx >= 0; --idx) {
      const int c = kids[idx];
      const int i = t.leg_of_child(sn, c);
      if (idx + 1 < (int)kids.size()) node_bwd(sn, half);
      move(sn, i, c, 0);
      env_up(c);
      if (!t.children[c].empty()) {
        Wstar(c, half);
        node_bwd(c, half);
      }
      edge(sn, c, half, false);
      env_down(c);
    }
  }
};

// Compile tree + generator into a plan: slot analysis, constant tables,
// buffer layout and recipe validation.  With device = false nothing touches
// the GPU (the constant tables stay on the host; used to query sizes).
static std::unique_ptr<tenso_plan> compile_plan(const tenso_tree* t, const tenso_gen* g,
                                                const tenso_plan_opts* o, bool device) {
  if (!t || !g || !o) fail(TENSO_EINVAL, "null argument");
  if (o->precision != TENSO_FP64 && o->precision != TENSO_FP32 && o->precision != TENSO_FP32_3M &&
      o->precision != TENSO_BF16)
    fail(TENSO_EINVAL, "bad precision");
  if (o->method != TENSO_PS1 && o->method != TENSO_PS2 && o->method != TENSO_VMF)
    fail(TENSO_EINVAL, "bad method");
  if (o->method == TENSO_VMF && o->precision != TENSO_FP64)
    fail(TENSO_EUNSUPPORTED, "direct (vmf) integration runs in FP64 only");
  if (g->n_ends != t->n_ends || g->end_dim != t->end_dim) fail(TENSO_EINVAL, "generator built for another tree");
  auto P = std::make_unique<tenso_plan>();
  P->tree = *t;
  P->gen = *g;
  P->opts = *o;
  P->fp64 = o->precision == TENSO_FP64;
  P->amode = o->precision == TENSO_FP32_3M ? 2 : o->precision == TENSO_BF16 ? 3 : 0;
  P->tsz = P->fp64 ? 16 : 8;
  P->cap = P->tree;
  if (o->method == TENSO_PS2) {
    if (o->max_rank < 2) fail(TENSO_EINVAL, "ps2 needs max_rank >= 2");
    for (int c = 1; c < P->cap.n; ++c) P->cap.rank[c] = o->max_rank;
    P->cap.clamp();
    for (int c = 1; c < P->tree.n; ++c) P->tree.rank[c] = std::min(2, P->cap.rank[c]);
    P->tree.clamp();
  }
  analyse_slots(*P);
  // constant buffer: factor matrices in FP64 and FP32
  std::vector<char> cb;
  for (size_t i = 0; i < P->gen.mats.size(); ++i) {
    const auto& m = P->gen.mats[i];
    size_t o64 = align256(cb.size());
    cb.resize(o64 + m.size() * 16);
    memcpy(cb.data() + o64, m.data(), m.size() * 16);
    size_t o32 = align256(cb.size());
    cb.resize(o32 + m.size() * 8);
    float* f = (float*)(cb.data() + o32);
    for (size_t q = 0; q < m.size(); ++q) {
      f[2 * q] = (float)m[q].real();
      f[2 * q + 1] = (float)m[q].imag();
    }
    P->mat_off64.push_back(o64);
    P->mat_off32.push_back(o32);
  }
  if (device) {
    hipchk(hipMalloc(&P->cbuf, std::max<size_t>(cb.size(), 256)), "hipMalloc(constants)");
    hipchk(hipMalloc(&P->opbuf, 8192), "hipMalloc(op scratch)");
    if (!cb.empty())
      hipchk(hipMemcpy(P->cbuf, cb.data(), cb.size(), hipMemcpyHostToDevice), "upload constants");
  }
  layout(*P);
  // validate that every recipe compiles (throws EUNSUPPORTED otherwise)
  for (int s = 0; s < P->tree.n; ++s) (void)node_recipe(*P, s);
  if (o->method == TENSO_VMF && !P->vmf_ok)
    fail(TENSO_EUNSUPPORTED,
         "direct integration needs at most one factor of a term inside any non-root subtree "
         "and bonds of at most 64");
  return P;
}


// ---------------------------------------------------------------------------
// one-off effective generator (tenso_apply_generator and its variants)
// ---------------------------------------------------------------------------
// Canonical-center test: every core other than the center must be an
// isometry toward it (orthonormal rows along the leg that points to the
// center: the child leg on the root-to-center path, the parent leg
// elsewhere).  One small kernel, one synchronisation.
static constexpr double kIsometryTol = 1e-8;

static void check_canonical(tenso_plan* p, const void* d_state, int center, void* d_ws,
                            hipStream_t s) {
  const tenso_tree& t = p->tree;
  std::vector<int> toward(t.n, 0);
  for (int x = center; x != 0; x = t.parent[x]) toward[t.parent[x]] = t.leg_of_child(t.parent[x], x);
  std::vector<IsoOp> ops;
  std::vector<int> node;
  for (int x = 0; x < t.n; ++x) {
    if (x == center) continue;
    const std::vector<int> d = t.shape(x);
    const int l = toward[x];
    IsoOp op{};
    op.C = (const double*)((const char*)d_state + p->core_off[x]);
    op.p0 = prod(d, 0, l);
    op.d = d[l];
    op.p1 = prod(d, l + 1, (int)d.size());
    ops.push_back(op);
    node.push_back(x);
  }
  if (ops.empty()) return;
  char* base = (char*)d_ws + p->ws_check;
  double* dev = (double*)(base + align256(ops.size() * sizeof(IsoOp)));
  hipchk(hipMemcpyAsync(base, ops.data(), ops.size() * sizeof(IsoOp), hipMemcpyHostToDevice, s),
         "isometry descriptors");
  hipchk(launch_isometry((const IsoOp*)base, (int)ops.size(), dev, s), "isometry check");
  std::vector<double> dv(ops.size());
  hipchk(hipMemcpyAsync(dv.data(), dev, dv.size() * sizeof(double), hipMemcpyDeviceToHost, s),
         "isometry readback");
  hipchk(hipStreamSynchronize(s), "sync");
  for (size_t i = 0; i < dv.size(); ++i)
    if (!(dv[i] <= kIsometryTol))
      fail(TENSO_EINVAL, "state is not canonical toward center " + std::to_string(center) +
                             ": core " + std::to_string(node[i]) +
                             " is not an isometry toward it (deviation " + std::to_string(dv[i]) + ")");
}

// Y = L_eff(center) C_center into d_out, with the workspace d_ws and the
// launch descriptors in D (its own arena, or caller-provided scratch).
static void apply_generator_impl(tenso_plan* p, const void* d_state, int center, const double* drive,
                                 void* d_out, void* d_ws, DevProgram& D, hipStream_t s) {
  if (!p || !d_state || !d_out || !d_ws) fail(TENSO_EINVAL, "null argument");
  if (center < 0 || center >= p->tree.n) fail(TENSO_EINVAL, "bad center");
  if (p->gen.n_slots > 0 && !drive) fail(TENSO_EINVAL, "generator has drive slots: drive values needed");
  check_canonical(p, d_state, center, d_ws, s);
  Program G;
  Builder b(*p, G);
  b.env_init_toward(center);
  Recipe R = node_recipe(*p, center);
  int np = b.emit_apply(R, b.core(center), 1, p->tree.size(center), 0, 1, p->par_target);
  b.emit_combine(d_out, p->tree.size(center), np, 0, 0.0);
  // the combine writes y0 = k at stage 0: y0 is the caller's buffer (absolute)
  G.combines.back().y0 = (double*)d_out;
  // drive values: one row per slot (ld = 1, index 0), in the workspace
  std::vector<double> dv(std::max(1, p->gen.n_slots), 0.0);
  if (drive)
    for (int k = 0; k < p->gen.n_slots; ++k) dv[k] = drive[k];
  double* d_drive = (double*)((char*)d_ws + p->ws_drive);
  hipchk(hipMemcpyAsync(d_drive, dv.data(), dv.size() * sizeof(double), hipMemcpyHostToDevice, s),
         "drive");
  upload(D, G, const_cast<void*>(d_state), d_ws, 0.0, d_drive, 1, s);
  int* ctr = (int*)((char*)d_ws + p->ws_ctr);
  hipchk(launch_step_inc(ctr, 0, s), "ctr");
  run(D, p->fp64, ctr, s);
  hipchk(hipStreamSynchronize(s), "sync");
}

namespace tenso {
// The variant of tenso_apply_generator that allocates nothing: workspace and
// launch descriptors both live in caller-provided device scratch (the
// workspace first, zeroed by a kernel, then the descriptor arena).
int apply_generator_scratch(tenso_plan* p, const void* d_state, int center, const double* drive,
                            void* d_out, void* scratch, size_t scratch_bytes, hipStream_t s) {
  return guard([&] {
    if (!p || !scratch) fail(TENSO_EINVAL, "null argument");
    const size_t ws = align256(p->ws_bytes);
    if (ws + 256 > scratch_bytes)
      fail(TENSO_ENOMEM, "plan workspace (" + std::to_string(p->ws_bytes) +
                             " bytes) exceeds the static scratch (" + std::to_string(scratch_bytes) +
                             " bytes)");
    hipchk(launch_zero(scratch, ws, s), "zero scratch");
    DevProgram D((char*)scratch + ws, scratch_bytes - ws);
    apply_generator_impl(p, d_state, center, drive, d_out, scratch, D, s);
  });
}

int set_last_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}
}  // namespace tenso

// ---------------------------------------------------------------------------
// host-side state helpers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// direct (vmf) integration: dopri5 over every core at once
// ---------------------------------------------------------------------------
// Dormand-Prince 5(4): nodes, stage weights, fifth- and fourth-order weights.
static const double kDpC[7] = {0.0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1.0, 1.0};
static const double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
static const double kDpB[7] = {35.0 / 384, 0.0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784,
                               11.0 / 84, 0.0};
static const double kDpBs[7] = {5179.0 / 57600, 0.0, 7571.0 / 16695, 393.0 / 640,
                                -92097.0 / 339200, 187.0 / 2100, 1.0 / 40};

// Build (or reuse) the derivative program for the plan's current ranks, the
// regularisation and the workspace binding; the stage input buffer plays
// the state.
static void vmf_prepare(tenso_plan* p, void* d_ws, double reg, hipStream_t s) {
  if (!p->vmf_ok)
    fail(TENSO_EUNSUPPORTED,
         "direct integration needs an FP64 plan whose terms leave room for the bond density "
         "(at most one factor of a term inside any non-root subtree) and bonds of at most 64");
  if (p->dev_vmf && p->vmf_ranks == p->tree.rank && p->vmf_reg == reg && p->vmf_ws == d_ws) return;
  p->par_target = 64;
  p->fuse_stages = true;
  Program G;
  Builder b(*p, G);
  b.vmf_deriv(reg);
  if (!p->dev_vmf) p->dev_vmf = std::make_unique<DevProgram>();
  char* ws = (char*)d_ws;
  upload(*p->dev_vmf, G, ws + p->ws_vmf_ys, d_ws, 0.0, (const double*)(ws + p->ws_vmf_dtab),
         kVmfDriveLd, s);
  std::vector<VecSeg> segs(p->tree.n);
  for (int c = 0; c < p->tree.n; ++c) segs[c] = VecSeg{(long)(p->core_off[c] / 16), p->tree.size(c)};
  hipchk(hipMemcpyAsync(ws + p->ws_vmf_segs, segs.data(), segs.size() * sizeof(VecSeg),
                        hipMemcpyHostToDevice, s),
         "vmf segments");
  hipchk(hipStreamSynchronize(s), "sync");
  p->vmf_ranks = p->tree.rank;
  p->vmf_reg = reg;
  p->vmf_ws = d_ws;
  p->vmf_graph.reset();
  p->vmf_eager_done = false;
}

struct VmfRun {
  tenso_plan& P;
  double* y0;
  char* ws;
  hipStream_t s;
  tenso_drive_fn drive;
  void* ctx;
  int* ctr;
  double* K[7];
  double* ys;
  double* kout;
  const VecSeg* segs;
  long n_elems = 0;
  bool k1 = false;  // K[0] holds the derivative at y0
  std::vector<double> tab, vals;

  VmfRun(tenso_plan& p, void* d_state, void* d_ws, hipStream_t st, tenso_drive_fn f, void* c)
      : P(p), y0((double*)d_state), ws((char*)d_ws), s(st), drive(f), ctx(c) {
    ctr = (int*)(ws + P.ws_ctr);
    for (int i = 0; i < 7; ++i) K[i] = (double*)(ws + P.ws_vmf_k + (size_t)i * P.state_bytes);
    ys = (double*)(ws + P.ws_vmf_ys);
    kout = (double*)(ws + P.ws_vmf_kout);
    segs = (const VecSeg*)(ws + P.ws_vmf_segs);
    for (int c2 = 0; c2 < P.tree.n; ++c2) n_elems += P.tree.size(c2);
  }

  void lincomb(double* out, const double* base, int n, double* const* src, const double* c) {
    LinCombOp op{};
    op.out = out;
    op.base = base;
    op.n_src = n;
    for (int j = 0; j < n; ++j) {
      op.src[j] = src[j];
      op.c[j] = c[j];
    }
    op.n_seg = P.tree.n;
    op.segs = segs;
    hipchk(launch_lincomb(op, P.vmf_chunks, s), "lincomb");
  }

  // drive values at the seven stage times of a step (t, h)
  void set_drive(double t, double h) {
    const int ns = P.gen.n_slots;
    if (ns == 0) return;
    tab.assign((size_t)ns * kVmfDriveLd, 0.0);
    vals.assign(ns, 0.0);
    for (int i = 0; i < 7; ++i) {
      drive(t + kDpC[i] * h, vals.data(), ctx);
      for (int k = 0; k < ns; ++k) tab[(size_t)k * kVmfDriveLd + 4 * i] = vals[k];
    }
    hipchk(hipMemcpyAsync(ws + P.ws_vmf_dtab, tab.data(), tab.size() * sizeof(double),
                          hipMemcpyHostToDevice, s),
           "vmf drive");
    hipchk(hipStreamSynchronize(s), "sync");  // the host table is rewritten next step
  }

  // derivative at the stage input (ys) for stage i, into out: replayed from
  // a captured graph (as tenso_step_fixed's steps) once the program has run
  // eagerly, unless graphs are off or the contraction is being timed
  void deriv(int i, double* out) {
    hipchk(launch_step_inc(ctr, i, s), "ctr");
    if (P.graph.enabled && !g_prof.on && P.vmf_eager_done) {
      if (!P.vmf_graph.exec) capture_step(P.vmf_graph, {P.dev_vmf.get()}, 1, ctr);
      hipchk(hipGraphLaunch(P.vmf_graph.exec, s), "hipGraphLaunch");
    } else {
      run(*P.dev_vmf, 1, ctr, s);
      P.vmf_eager_done = true;
    }
    lincomb(out, kout, 0, nullptr, nullptr);
  }

  // One Dormand-Prince step of size h from y0 at t; the fifth-order result
  // is left in ys.  Returns the error norm when asked (one synchronisation).
  double step(double t, double h, bool need_err, double rtol, double atol) {
    set_drive(t, h);
    if (!k1) {
      lincomb(ys, y0, 0, nullptr, nullptr);
      deriv(0, K[0]);
      k1 = true;
    }
    for (int i = 1; i < 7; ++i) {
      double c[6];
      for (int j = 0; j < i; ++j) c[j] = h * kDpA[i][j];
      lincomb(ys, y0, i, K, c);
      deriv(i, K[i]);
    }
    if (!need_err) return 0.0;
    ErrNormOp e{};
    e.y0 = y0;
    e.y1 = ys;
    e.n_src = 7;
    for (int j = 0; j < 7; ++j) {
      e.src[j] = K[j];
      e.c[j] = h * (kDpB[j] - kDpBs[j]);
    }
    e.rtol = rtol;
    e.atol = atol;
    e.n_seg = P.tree.n;
    e.segs = segs;
    e.part = (double*)(ws + P.ws_vmf_part);
    e.chunks = P.vmf_chunks;
    hipchk(launch_errnorm(e, s), "error norm");
    double* out = (double*)(ws + P.ws_vmf_err);
    hipchk(launch_sum_partials(e.part, P.tree.n * P.vmf_chunks, out, s), "error sum");
    double v = 0;
    hipchk(hipMemcpyAsync(&v, out, sizeof(double), hipMemcpyDeviceToHost, s), "error norm");
    hipchk(hipStreamSynchronize(s), "sync");
    return std::sqrt(v / (double)std::max<long>(1, n_elems));
  }

  // take the step: y0 = ys, and the last stage is the next step's first
  void accept() {
    lincomb(y0, ys, 0, nullptr, nullptr);
    std::swap(K[0], K[6]);
  }

  // cover [t0, t0 + dt] with dopri5 steps (readings of the step control:
  // see tenso_step_vmf in the header)
  void advance(double t0, double dt, const tenso_vmf_opts& o, long& substeps) {
    if (o.fixed_substeps > 0) {
      const double h = dt / o.fixed_substeps;
      for (int j = 0; j < o.fixed_substeps; ++j) {
        step(t0 + j * h, h, false, 0, 0);
        accept();
        ++P.vmf_accepted;
      }
      return;
    }
    if (!(P.vmf_h > 0)) P.vmf_h = dt;
    const double t_end = t0 + dt;
    double t = t0;
    while (t < t_end) {
      const double h = std::min(P.vmf_h, t_end - t);
      if (h <= 1e-14 * std::fabs(dt)) fail(TENSO_ENUMERIC, "dopri5 step size underflow");
      if (++substeps > o.max_substeps) fail(TENSO_ENUMERIC, "more dopri5 substeps than max_substeps");
      const bool last = t + h >= t_end;
      const double en = step(t, h, true, o.ode_rtol, o.ode_atol);
      if (!std::isfinite(en)) fail(TENSO_ENUMERIC, "non-finite dopri5 error estimate");
      const double fac = en == 0.0 ? 10.0 : std::min(10.0, std::max(0.2, 0.9 * std::pow(en, -0.2)));
      if (en <= 1.0) {
        t = last ? t_end : t + h;
        accept();
        ++P.vmf_accepted;
        P.vmf_h = h >= P.vmf_h ? h * fac : std::max(P.vmf_h, h * fac);
      } else {
        ++P.vmf_rejected;
        P.vmf_h = h * fac;
      }
    }
  }
};

static void check_vmf_opts(const tenso_vmf_opts* o) {
  if (!o) fail(TENSO_EINVAL, "null vmf options");
  if (!(o->vmf_atol >= 0)) fail(TENSO_EINVAL, "vmf_atol must be >= 0");
  if (o->fixed_substeps < 0) fail(TENSO_EINVAL, "fixed_substeps must be >= 0");
  if (o->fixed_substeps == 0) {
    if (!(o->ode_rtol >= 0) || !(o->ode_atol >= 0) || !(o->ode_rtol + o->ode_atol > 0))
      fail(TENSO_EINVAL, "adaptive steps need ode_rtol, ode_atol >= 0, not both 0");
    if (o->max_substeps < 1) fail(TENSO_EINVAL, "max_substeps must be >= 1");
  }
}

static void vmf_steps(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                      const tenso_vmf_opts& o, tenso_drive_fn drive, void* ctx, void* d_ws,
                      hipStream_t s) {
  vmf_prepare(p, d_ws, o.vmf_atol, s);
  VmfRun R(*p, d_state, d_ws, s, drive, ctx);
  long substeps = 0;
  for (int k = 0; k < n_steps; ++k) R.advance(t0 + k * dt, dt, o, substeps);
}

static std::vector<cd> initial_cores(const tenso_plan& P, const tenso_c128* rho) {
  const tenso_tree& t = P.tree;
  std::vector<cd> h(P.state_bytes / 16, cd(0, 0));
  for (int s = 0; s < t.n; ++s) {
    cd* C = h.data() + P.core_off[s] / 16;
    std::vector<int> d = t.shape(s);
    if (s == 0) {  // ends 0 and 1 are the root's first legs
      const int M1 = t.end_dim[0], M2 = t.end_dim[1];
      long rest = t.size(0) / ((long)M1 * M2);
      for (int i = 0; i < M1; ++i)
        for (int j = 0; j < M2; ++j)
          C[((long)i * M2 + j) * rest] = cd(rho[i * M2 + j].re, rho[i * M2 + j].im);
    } else {
      long cols = t.size(s) / d[0];
      for (int a = 0; a < d[0]; ++a) C[(long)a * cols + a] = 1.0;
    }
  }
  return h;
}

// ---------------------------------------------------------------------------
// ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* tenso_last_error(void) { return g_err.c_str(); }

int tenso_build_tree(int n_nodes, const int32_t* parent, int n_ends, const int32_t* end_node,
                     const int32_t* end_dim, int max_rank, const int32_t* bond_rank,
                     tenso_tree** out) {
  return guard([&] {
    if (!out || !parent || !end_node || !end_dim) fail(TENSO_EINVAL, "null argument");
    *out = make_tree(n_nodes, parent, n_ends, end_node, end_dim, max_rank, bond_rank);
  });
}

int tenso_tree_train(int M, int K, const int32_t* mode_dim, int rank, tenso_tree** out) {
  return guard([&] {
    if (!out || M < 1 || K < 0 || (K > 0 && !mode_dim)) fail(TENSO_EINVAL, "bad train arguments");
    std::vector<int32_t> parent, end_node, end_dim = {M, M};
    for (int k = 0; k < K; ++k) end_dim.push_back(mode_dim[k]);
    if (K <= 1) {
      parent = {-1};
      end_node.assign(2 + K, 0);
    } else {
      parent.push_back(-1);
      for (int s = 1; s < K; ++s) parent.push_back(s - 1);
      end_node = {0, 0};
      for (int k = 0; k < K - 1; ++k) end_node.push_back(k + 1);
      end_node.push_back(K - 1);
    }
    *out = make_tree((int)parent.size(), parent.data(), (int)end_dim.size(), end_node.data(),
                     end_dim.data(), rank, nullptr);
  });
}

int tenso_tree_nary(int M, int K, const int32_t* mode_dim, int n_ary, int rank, tenso_tree** out) {
  return guard([&] {
    if (!out || M < 1 || K < 0 || n_ary < 2 || (K > 0 && !mode_dim)) fail(TENSO_EINVAL, "bad tree arguments");
    std::vector<int32_t> parent = {-1}, end_node(2 + K, 0), end_dim = {M, M};
    for (int k = 0; k < K; ++k) end_dim.push_back(mode_dim[k]);
    // recursive split of a contiguous feature range [a, b) under `holder`
    std::function<void(int, int, int)> build = [&](int a, int b, int holder) {
      int len = b - a;
      if (len == 1) {
        end_node[2 + a] = holder;
        return;
      }
      int me = (int)parent.size();
      parent.push_back(holder);
      if (len <= n_ary) {
        for (int f = a; f < b; ++f) end_node[2 + f] = me;
        return;
      }
      int q = len / n_ary, r = len % n_ary, pos = a;
      for (int j = 0; j < n_ary; ++j) {
        int sz = q + (j < r ? 1 : 0);
        build(pos, pos + sz, me);
        pos += sz;
      }
    };
    if (K > 0) build(0, K, 0);
    *out = make_tree((int)parent.size(), parent.data(), (int)end_dim.size(), end_node.data(),
                     end_dim.data(), rank, nullptr);
  });
}

int tenso_tree_ranks(const tenso_tree* t, int32_t* out) {
  return guard([&] {
    if (!t || !out) fail(TENSO_EINVAL, "null argument");
    for (int s = 0; s < t->n; ++s) out[s] = s == 0 ? 0 : t->rank[s];
  });
}

int tenso_tree_n_nodes(const tenso_tree* t) { return t ? t->n : TENSO_EINVAL; }
void tenso_tree_destroy(tenso_tree* t) { delete t; }

int tenso_build_generator(const tenso_tree* t, int n_terms, const tenso_c128* coef,
                          const int32_t* td_slot, const int32_t* n_factors,
                          const int32_t* factor_end, const tenso_c128* factor_mats,
                          tenso_gen** out) {
  return guard([&] {
    if (!t || !out || n_terms < 0 || (n_terms && (!coef || !n_factors))) fail(TENSO_EINVAL, "null argument");
    auto g = std::make_unique<tenso_gen>();
    g->n_ends = t->n_ends;
    g->end_dim = t->end_dim;
    std::map<std::pair<int, std::vector<double>>, int> dedup;
    long fi = 0, mo = 0;
    for (int m = 0; m < n_terms; ++m) {
      tenso_gen::Term tm;
      tm.coef = cd(coef[m].re, coef[m].im);
      tm.slot = td_slot ? td_slot[m] : -1;
      if (tm.slot >= 0) g->n_slots = std::max(g->n_slots, tm.slot + 1);
      if (n_factors[m] < 1) fail(TENSO_EINVAL, "every term needs at least one factor");
      for (int j = 0; j < n_factors[m]; ++j, ++fi) {
        int e = factor_end[fi];
        if (e < 0 || e >= t->n_ends) fail(TENSO_EINVAL, "factor on a bad end");
        for (auto& p : tm.f)
          if (p.first == e) fail(TENSO_EINVAL, "two factors of one term on the same end");
        int d = t->end_dim[e];
        std::vector<double> key(2 * (size_t)d * d);
        std::vector<cd> mat((size_t)d * d);
        for (long q = 0; q < (long)d * d; ++q) {
          key[2 * q] = factor_mats[mo + q].re;
          key[2 * q + 1] = factor_mats[mo + q].im;
          mat[q] = cd(key[2 * q], key[2 * q + 1]);
        }
        mo += (long)d * d;
        auto k = std::make_pair(d, key);
        auto it = dedup.find(k);
        if (it == dedup.end()) {
          it = dedup.emplace(k, (int)g->mats.size()).first;
          g->mats.push_back(mat);
          g->mat_dim.push_back(d);
        }
        tm.f.push_back({e, it->second});
      }
      std::sort(tm.f.begin(), tm.f.end());
      g->terms.push_back(tm);
    }
    *out = g.release();
  });
}

void tenso_gen_destroy(tenso_gen* g) { delete g; }

int tenso_plan_create(const tenso_tree* t, const tenso_gen* g, const tenso_plan_opts* o,
                      tenso_plan** out) {
  return guard([&] {
    if (!out) fail(TENSO_EINVAL, "null argument");
    *out = compile_plan(t, g, o, true).release();
  });
}

int tenso_plan_query(const tenso_tree* t, const tenso_gen* g, const tenso_plan_opts* o,
                     size_t* state_bytes, size_t* workspace_bytes, int64_t* launches_per_step,
                     double* apply_flops_per_step) {
  return guard([&] {
    auto P = compile_plan(t, g, o, false);
    if (state_bytes) *state_bytes = P->state_bytes;
    if (workspace_bytes) *workspace_bytes = P->ws_bytes;
    int64_t nl = 0;
    double fl = 0;
    if (P->opts.method == TENSO_PS1 || P->opts.method == TENSO_VMF) {
      Program G;
      if (P->opts.method == TENSO_PS1) {
        build_step(*P, G);
      } else {  // one evaluation of the vmf derivative (a dopri5 substep takes six)
        P->par_target = 64;
        P->fuse_stages = true;
        Builder b(*P, G);
        b.vmf_deriv(0.0);
      }
      nl = (int64_t)G.launches.size();
      for (const auto& L : G.launches) fl += L.flops;
    }
    if (launches_per_step) *launches_per_step = nl;
    if (apply_flops_per_step) *apply_flops_per_step = fl;
  });
}

void tenso_plan_destroy(tenso_plan* p) { delete p; }

int tenso_plan_set_graph(tenso_plan* p, int enable) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null plan");
    p->graph.enabled = enable != 0;
    p->graph.reset();
  });
}

int tenso_plan_set_tile_work(tenso_plan* p, double flops) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null plan");
    if (!(flops >= 1e5 && flops <= 1e9)) fail(TENSO_EINVAL, "tile work outside [1e5, 1e9] flops");
    p->tile_work = flops;
    p->tile_work_set = true;
  });
}

int tenso_plan_sizes(const tenso_plan* p, size_t* sb, size_t* wb) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null plan");
    if (sb) *sb = p->state_bytes;
    if (wb) *wb = p->ws_bytes;
  });
}

int tenso_plan_shapes(const tenso_plan* p, int32_t* n_legs, int32_t* dims) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null plan");
    for (int s = 0; s < p->tree.n; ++s) {
      std::vector<int> d = p->tree.shape(s);
      if (n_legs) n_legs[s] = (int)d.size();
      if (dims)
        for (int l = 0; l < 8; ++l) dims[8 * s + l] = l < (int)d.size() ? d[l] : 0;
    }
  });
}

int tenso_state_init(tenso_plan* p, const tenso_c128* rho, void* d_state, hipStream_t s) {
  return guard([&] {
    if (!p || !rho || !d_state) fail(TENSO_EINVAL, "null argument");
    std::vector<cd> h = initial_cores(*p, rho);
    hipchk(hipMemcpyAsync(d_state, h.data(), p->state_bytes, hipMemcpyHostToDevice, s), "state init");
    hipchk(hipStreamSynchronize(s), "sync");
    p->reset_integrators();
  });
}

int tenso_state_import(tenso_plan* p, const tenso_c128* h_cores, void* d_state, hipStream_t s) {
  return guard([&] {
    if (!p || !h_cores || !d_state) fail(TENSO_EINVAL, "null argument");
    std::vector<cd> h(p->state_bytes / 16, cd(0, 0));
    long o = 0;
    for (int c = 0; c < p->tree.n; ++c) {
      long n = p->tree.size(c);
      for (long q = 0; q < n; ++q) h[p->core_off[c] / 16 + q] = cd(h_cores[o + q].re, h_cores[o + q].im);
      o += n;
    }
    hipchk(hipMemcpyAsync(d_state, h.data(), p->state_bytes, hipMemcpyHostToDevice, s), "state import");
    hipchk(hipStreamSynchronize(s), "sync");
    p->reset_integrators();
  });
}

int tenso_state_export(tenso_plan* p, const void* d_state, tenso_c128* h_cores, int32_t* ranks,
                       hipStream_t s) {
  return guard([&] {
    if (!p || !d_state) fail(TENSO_EINVAL, "null argument");
    std::vector<cd> h(p->state_bytes / 16);
    hipchk(hipMemcpyAsync(h.data(), d_state, p->state_bytes, hipMemcpyDeviceToHost, s), "state export");
    hipchk(hipStreamSynchronize(s), "sync");
    long o = 0;
    if (h_cores)
      for (int c = 0; c < p->tree.n; ++c) {
        long n = p->tree.size(c);
        for (long q = 0; q < n; ++q) {
          h_cores[o + q].re = h[p->core_off[c] / 16 + q].real();
          h_cores[o + q].im = h[p->core_off[c] / 16 + q].imag();
        }
        o += n;
      }
    if (ranks)
      for (int c = 0; c < p->tree.n; ++c) ranks[c] = c == 0 ? 0 : p->tree.rank[c];
  });
}

int tenso_apply_generator(tenso_plan* p, const void* d_state, int center, const double* drive,
                          void* d_out, void* d_ws, hipStream_t s) {
  return guard([&] {
    if (!d_ws) fail(TENSO_EINVAL, "null argument");
    DevProgram D;
    apply_generator_impl(p, d_state, center, drive, d_out, d_ws, D, s);
  });
}

int tenso_step_fixed(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                     const double* d_drive_tab, void* d_ws, hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (!(dt > 0)) fail(TENSO_EINVAL, "dt must be > 0");
    if (n_steps < 0) fail(TENSO_EINVAL, "n_steps must be >= 0");
    if (p->opts.method != TENSO_PS1) fail(TENSO_EINVAL, "plan is not a ps1 plan");
    if (p->gen.n_slots > 0 && !d_drive_tab) fail(TENSO_EINVAL, "generator has drive slots: drive table needed");
    (void)t0;
    const int ld = 4 * n_steps + 1;
    if (!p->dev_step) {
      p->dev_step = std::make_unique<DevProgram>();
      p->dev_init = std::make_unique<DevProgram>();
    }
    p->par_target = 64;
    p->fuse_stages = true;
    if (!p->prog_step || p->built_target != p->par_target || p->built_tile_work != p->tile_work ||
        p->built_fuse != p->fuse_stages) {
      p->prog_step = std::make_unique<Program>();
      p->prog_init = std::make_unique<Program>();
      build_step(*p, *p->prog_step);
      build_init(*p, *p->prog_init);
      p->built_target = p->par_target;
      p->built_tile_work = p->tile_work;
      p->built_fuse = p->fuse_stages;
      p->b_state = nullptr;
    }
    // the drive table's row length (4 n_steps + 1) is baked into the launch
    // descriptors; it matters only when the generator has drive slots
    if (p->b_state != d_state || p->b_ws != d_ws || p->b_dt != dt || p->b_drive != d_drive_tab ||
        (p->gen.n_slots > 0 && p->b_ld != ld)) {
      upload(*p->dev_step, *p->prog_step, d_state, d_ws, dt, d_drive_tab, ld, s);
      upload(*p->dev_init, *p->prog_init, d_state, d_ws, dt, d_drive_tab, ld, s);
      p->graph.reset();
      p->b_state = d_state;
      p->b_ws = d_ws;
      p->b_dt = dt;
      p->b_drive = d_drive_tab;
      p->b_ld = ld;
    }
    int* ctr = (int*)((char*)d_ws + p->ws_ctr);
    plan_root_norm(p, d_state, d_ws, 0, s);
    hipchk(launch_step_inc(ctr, 0, s), "ctr");
    run(*p->dev_init, p->fp64, ctr, s);
    step_loop(p->graph, {p->dev_step.get()}, p->fp64, ctr, n_steps, s);
    check_plan_finite(p, d_state, d_ws, s);
  });
}

int tenso_step_adaptive(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                        double eps, int max_rank, const double* d_drive_tab, void* d_ws,
                        hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (!(dt > 0)) fail(TENSO_EINVAL, "dt must be > 0");
    if (n_steps < 0 || eps < 0) fail(TENSO_EINVAL, "bad n_steps or eps");
    if (p->opts.method != TENSO_PS2) fail(TENSO_EINVAL, "plan is not a ps2 plan");
    if (p->gen.n_slots > 0 && !d_drive_tab) fail(TENSO_EINVAL, "generator has drive slots: drive table needed");
    (void)t0;
    const int ld = 4 * n_steps + 1;
    // cached sub-flow programs hold this binding's pointers and dt; the drive
    // table's row length matters only when the generator has drive slots
    if (p->ps2_state != d_state || p->ps2_ws != d_ws || p->ps2_dt != dt ||
        p->ps2_drive != d_drive_tab || p->ps2_tile != p->tile_work ||
        (p->gen.n_slots > 0 && p->ps2_ld != ld)) {
      hipchk(hipStreamSynchronize(s), "sync");
      p->ps2_progs.clear();
      p->ps2_state = d_state;
      p->ps2_ws = d_ws;
      p->ps2_dt = dt;
      p->ps2_drive = d_drive_tab;
      p->ps2_tile = p->tile_work;
      p->ps2_ld = ld;
    }
    Ps2Exec X{*p, d_state, d_ws, dt, d_drive_tab, p->ps2_ld, s, std::min(max_rank, p->opts.max_rank), eps};
    X.ctr = (int*)((char*)d_ws + p->ws_ctr);
    p->rank_log.clear();
    plan_root_norm(p, d_state, d_ws, 0, s);
    X.exec_cached("I|", [&](Program& G) { build_init(*p, G); });
    for (int k = 0; k < n_steps; ++k) {
      hipchk(launch_step_inc(X.ctr, k, s), "ctr");
      X.W(0, 0);
      X.Wstar(0, 1);
    }
    check_plan_finite(p, d_state, d_ws, s);
  });
}

int tenso_step_vmf(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                   const tenso_vmf_opts* o, tenso_drive_fn drive, void* drive_ctx, void* d_ws,
                   hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (!(dt > 0)) fail(TENSO_EINVAL, "dt must be > 0");
    if (n_steps < 0) fail(TENSO_EINVAL, "n_steps must be >= 0");
    check_vmf_opts(o);
    if (p->gen.n_slots > 0 && !drive) fail(TENSO_EINVAL, "generator has drive slots: drive function needed");
    plan_root_norm(p, d_state, d_ws, 0, s);
    vmf_steps(p, d_state, t0, dt, n_steps, *o, drive, drive_ctx, d_ws, s);
    check_plan_finite(p, d_state, d_ws, s);
  });
}

int tenso_vmf_derivative(tenso_plan* p, const void* d_state, double vmf_atol, const double* drive,
                         void* d_out, void* d_ws, hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !d_out || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (!(vmf_atol >= 0)) fail(TENSO_EINVAL, "vmf_atol must be >= 0");
    if (p->gen.n_slots > 0 && !drive) fail(TENSO_EINVAL, "generator has drive slots: drive values needed");
    vmf_prepare(p, d_ws, vmf_atol, s);
    char* ws = (char*)d_ws;
    if (p->gen.n_slots > 0) {
      std::vector<double> tab((size_t)p->gen.n_slots * kVmfDriveLd, 0.0);
      for (int k = 0; k < p->gen.n_slots; ++k) tab[(size_t)k * kVmfDriveLd] = drive[k];
      hipchk(hipMemcpyAsync(ws + p->ws_vmf_dtab, tab.data(), tab.size() * sizeof(double),
                            hipMemcpyHostToDevice, s),
             "drive");
      hipchk(hipStreamSynchronize(s), "sync");
    }
    VmfRun R(*p, const_cast<void*>(d_state), d_ws, s, nullptr, nullptr);
    R.lincomb(R.ys, (const double*)d_state, 0, nullptr, nullptr);
    R.deriv(0, (double*)d_out);
    hipchk(hipStreamSynchronize(s), "sync");
  });
}

int tenso_plan_set_ps2_truncation(tenso_plan* p, double ps2_atol, double ps2_ratio) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null argument");
    if (!(ps2_atol >= 0) || !(ps2_ratio == 0 || ps2_ratio >= 1))
      fail(TENSO_EINVAL, "ps2_atol must be >= 0 and ps2_ratio 0 or >= 1");
    p->ps2_atol = ps2_atol;
    p->ps2_ratio = ps2_ratio;
  });
}

int tenso_vmf_stats(const tenso_plan* p, int64_t* accepted, int64_t* rejected, double* next_h) {
  return guard([&] {
    if (!p) fail(TENSO_EINVAL, "null argument");
    if (accepted) *accepted = p->vmf_accepted;
    if (rejected) *rejected = p->vmf_rejected;
    if (next_h) *next_h = p->vmf_h;
  });
}

int tenso_step_mix(tenso_plan* p, void* d_state, double t0, double dt, int n_steps, double eps,
                   int max_aux_rank, const tenso_vmf_opts* o, tenso_drive_fn drive,
                   void* drive_ctx, void* d_ws, hipStream_t s, int32_t* switch_step) {
  return guard([&] {
    if (!p || !d_state || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (p->opts.method != TENSO_PS2) fail(TENSO_EINVAL, "the mixed strategy needs a ps2 plan");
    if (!(dt > 0) || n_steps < 0 || !(eps >= 0)) fail(TENSO_EINVAL, "bad dt, n_steps or eps");
    if (max_aux_rank < 2 || max_aux_rank > p->opts.max_rank)
      fail(TENSO_EINVAL, "max_aux_rank must lie in [2, the plan's max_rank]");
    check_vmf_opts(o);
    if (!p->vmf_ok) vmf_prepare(p, d_ws, o->vmf_atol, s);  // reports why vmf cannot follow
    if (p->gen.n_slots > 0 && !drive) fail(TENSO_EINVAL, "generator has drive slots: drive function needed");
    char* ws = (char*)d_ws;
    const int ns = p->gen.n_slots;
    std::vector<double> tab, vals(std::max(1, ns));
    for (int k = 0; k < n_steps; ++k) {
      const double t = t0 + k * dt;
      if (p->mix_phase == 0) {
        const double* d_tab = nullptr;
        if (ns > 0) {  // one ps2 step's table: [slot][t + j dt / 4], j = 0..4
          tab.assign((size_t)ns * 5, 0.0);
          for (int j = 0; j < 5; ++j) {
            drive(t + 0.25 * j * dt, vals.data(), drive_ctx);
            for (int q = 0; q < ns; ++q) tab[(size_t)q * 5 + j] = vals[q];
          }
          hipchk(hipMemcpyAsync(ws + p->ws_vmf_dtab, tab.data(), tab.size() * sizeof(double),
                                hipMemcpyHostToDevice, s),
                 "ps2 drive");
          hipchk(hipStreamSynchronize(s), "sync");
          d_tab = (const double*)(ws + p->ws_vmf_dtab);
        }
        const int rc = tenso_step_adaptive(p, d_state, t, dt, 1, eps, max_aux_rank, d_tab, d_ws, s);
        if (rc != TENSO_OK) throw TErr{rc, g_err};
        ++p->mix_ps2_steps;
        int mr = 0;
        for (int c = 1; c < p->tree.n; ++c) mr = std::max(mr, p->tree.rank[c]);
        if (mr >= max_aux_rank) {
          p->mix_phase = 1;
          p->mix_switch = p->mix_ps2_steps;
        }
      } else {
        plan_root_norm(p, d_state, d_ws, 0, s);
        vmf_steps(p, d_state, t, dt, 1, *o, drive, drive_ctx, d_ws, s);
        check_plan_finite(p, d_state, d_ws, s);
      }
    }
    if (switch_step) *switch_step = p->mix_switch;
  });
}

int tenso_reduced_rho(tenso_plan* p, const void* d_state, tenso_c128* h_rho, double* h_trace,
                      void* d_ws, hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !h_rho || !d_ws) fail(TENSO_EINVAL, "null argument");
    if (!p->dev_rho) p->dev_rho = std::make_unique<DevProgram>();
    Program G;
    Builder b(*p, G);
    b.rho_prog();
    upload(*p->dev_rho, G, const_cast<void*>(d_state), d_ws, 0.0, nullptr, 1, s);
    run(*p->dev_rho, p->fp64, nullptr, s);
    const int M = p->tree.end_dim[0];
    hipchk(hipMemcpyAsync(h_rho, (char*)d_ws + p->ws_rhoout, (size_t)M * M * 16, hipMemcpyDeviceToHost, s),
           "rho readback");
    hipchk(hipStreamSynchronize(s), "sync");
    if (h_trace) {
      double tr = 0;
      for (int i = 0; i < M; ++i) tr += h_rho[i * M + i].re;
      *h_trace = tr;
    }
  });
}

int tenso_reduced_rho_pure(tenso_plan* p, const void* d_state, tenso_c128* h_rho, double* h_trace,
                           void* d_ws, hipStream_t s) {
  return guard([&] {
    if (!p || !d_state || !h_rho || !d_ws) fail(TENSO_EINVAL, "null argument");
    const tenso_tree& t = p->tree;
    if (t.end_node.size() < 2 || t.end_node[0] != 0 || t.end_node[1] != 0 || t.end_dim[1] != 1)
      fail(TENSO_EINVAL, "a wavefunction state has ends 0 (system) and 1 (dimension 1) on the root");
    const int M = t.end_dim[0];  // the workspace holds an M x M result (ws_rhoout)
    const double* C = (const double*)((const char*)d_state + p->core_off[0]);
    double* out = (double*)((char*)d_ws + p->ws_rhoout);
    hipchk(launch_rho_pure(C, M, t.size(0) / M, out, s), "rho_pure");
    hipchk(hipMemcpyAsync(h_rho, out, (size_t)M * M * 16, hipMemcpyDeviceToHost, s), "rho readback");
    hipchk(hipStreamSynchronize(s), "sync");
    if (h_trace) {
      double tr = 0;
      for (int i = 0; i < M; ++i) tr += h_rho[i * M + i].re;
      *h_trace = tr;
    }
  });
}

int tenso_rank_trajectory(const tenso_plan* p, int32_t* h, int cap) {
  if (!p) return TENSO_EINVAL;
  int n = std::min<int>(cap, (int)p->rank_log.size());
  for (int i = 0; i < n; ++i) h[i] = p->rank_log[i];
  return n;
}

int tenso_svd_truncate(const void* d_A, int rows, int cols, int iso, double eps, int max_rank,
                       double* h_sigma, void* d_vectors, int32_t* h_decision, double* h_missed,
                       hipStream_t s) {
  return guard([&] {
    if (!d_A || !d_vectors) fail(TENSO_EINVAL, "null argument");
    if (rows < 1 || cols < 1 || (iso != 0 && iso != 1) || !(eps >= 0) || max_rank < 1)
      fail(TENSO_EINVAL, "bad sizes, side, eps or max_rank");
    if ((long)rows * cols > kPs2ThetaMax) fail(TENSO_ENOMEM, "matrix beyond 2^26 elements");
    const size_t side = std::max(rows, cols);
    const size_t blk = align256(side * kSvdP * 16);
    const size_t nrm = align256(((side + 63) / 64) * kSvdMaxSplit * 8);
    const size_t sq = align256((size_t)kSvdP * kSvdP * 16);
    const size_t total = blk * (4 + kSvdMaxSplit) + 3 * sq + 2 * 1024 + nrm + 256 + 4 * 512;
    struct DevMem {
      char* p = nullptr;
      ~DevMem() {
        if (p) (void)hipFree(p);
      }
    } mem;
    hipchk(hipMalloc((void**)&mem.p, total), "hipMalloc(svd scratch)");
    char* w = mem.p;
    auto take = [&](size_t b) {
      char* q = w;
      w += b;
      return q;
    };
    SvdScratch sc{};
    sc.y = (double*)take(blk);
    sc.z = (double*)take(blk);
    sc.qrv = (double*)take(blk);
    sc.part = (double*)take(kSvdMaxSplit * blk);
    sc.r = (double*)take(sq);
    sc.up = (double*)take(sq);
    sc.wp = (double*)take(sq);
    sc.sig = (double*)take(1024);
    sc.tau = (double*)take(1024);
    sc.norm = (double*)take(nrm);
    sc.rec = take(256);
    sc.opbuf = take(4 * 512);
    sc.e = (double*)take(blk);
    std::vector<std::vector<char>> hold;
    int rec_i[3] = {0, 0, 0};
    double rec_d[2] = {0, 0};
    const int pw = svd_truncate(sc, (const double*)d_A, rows, cols, iso, eps, max_rank,
                                std::min(rows, cols), s, hold, rec_i, rec_d);
    // the caller's buffer holds the documented width p <= pw
    const int p = svd_width(rows, cols, max_rank, std::min(rows, cols));
    const size_t n_iso = iso == 0 ? rows : cols;
    hipchk(hipMemcpy2DAsync(d_vectors, p * 16, sc.e, pw * 16, p * 16, n_iso, hipMemcpyDeviceToDevice,
                            s),
           "vectors");
    if (h_sigma)
      hipchk(hipMemcpyAsync(h_sigma, sc.sig, p * sizeof(double), hipMemcpyDeviceToHost, s), "sigma");
    hipchk(hipStreamSynchronize(s), "sync");
    if (h_decision)
      for (int q = 0; q < 3; ++q) h_decision[q] = rec_i[q];
    if (h_missed) *h_missed = rec_d[1] / std::max(rec_d[0], 1e-300);
  });
}

int tenso_profile(int enable) {
  return guard([&] {
    g_prof.on = enable != 0;
    g_prof.ev.clear();
    g_prof.work.clear();
    g_prof.used = 0;
  });
}

int tenso_profile_stats(double* total_ms, int64_t* launches, double* flops, double* bytes) {
  return guard([&] {
    double ms = 0, fl = 0, by = 0;
    for (size_t i = 0; i < g_prof.ev.size(); ++i) {
      hipchk(hipEventSynchronize(g_prof.ev[i].second), "hipEventSynchronize");
      float t = 0;
      hipchk(hipEventElapsedTime(&t, g_prof.ev[i].first, g_prof.ev[i].second), "hipEventElapsedTime");
      ms += t;
      fl += g_prof.work[i].first;
      by += g_prof.work[i].second;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = (int64_t)g_prof.ev.size();
    if (flops) *flops = fl;
    if (bytes) *bytes = by;
  });
}

int tenso_profile_records(int64_t cap, double* ms, double* flops, double* bytes, int64_t* n_out) {
  return guard([&] {
    if (cap < 0 || !n_out) fail(TENSO_EINVAL, "bad arguments");
    const int64_t n = std::min<int64_t>(cap, (int64_t)g_prof.ev.size());
    for (int64_t i = 0; i < n; ++i) {
      hipchk(hipEventSynchronize(g_prof.ev[i].second), "hipEventSynchronize");
      float t = 0;
      hipchk(hipEventElapsedTime(&t, g_prof.ev[i].first, g_prof.ev[i].second), "hipEventElapsedTime");
      if (ms) ms[i] = t;
      if (flops) flops[i] = g_prof.work[i].first;
      if (bytes) bytes[i] = g_prof.work[i].second;
    }
    *n_out = (int64_t)g_prof.ev.size();
  });
}

}  // extern "C"

struct tenso_batch {
  std::vector<tenso_plan*> plans;
  std::vector<void*> states, wss;
  std::vector<double> dts;
  std::vector<const double*> drives;
  int ld = -1;
  int fp64 = 0;
  int* ctr = nullptr;
  double* rho_buf = nullptr;
  std::vector<size_t> rho_off;
  DevProgram init, rho;
  FiniteOp* fin_ops = nullptr;      // per instance: its state, for the finiteness check
  int* fin_flags = nullptr;
  NormOp* norm_ops = nullptr;       // per instance: its root core, for the norm-growth check
  double* norms = nullptr;          // n norms before the step call, then n after it
  std::vector<int> last_flags;      // flags of the last step call
  std::vector<std::unique_ptr<DevProgram>> steps;  // independent parts of one step
  int n_parts = 4;                                 // parts requested
  StepGraph graph;
  std::vector<const DevProgram*> step_parts() const {
    std::vector<const DevProgram*> v;
    for (auto& d : steps) v.push_back(d.get());
    return v;
  }
  ~tenso_batch() {
    if (fin_ops) (void)hipFree(fin_ops);
    if (fin_flags) (void)hipFree(fin_flags);
    if (norm_ops) (void)hipFree(norm_ops);
    if (norms) (void)hipFree(norms);
    if (ctr) (void)hipFree(ctr);
    if (rho_buf) (void)hipFree(rho_buf);
  }
};

static void batch_build(tenso_batch& B, hipStream_t s) {
  const size_t n = B.plans.size();
  std::vector<Program> st(n), in(n), rh(n);
  std::vector<double> cost(n, 0.0);
  std::vector<size_t> chain(n, 0);  // launches of the instance's step program
  for (size_t i = 0; i < n; ++i) {
    tenso_plan& P = *B.plans[i];
    P.par_target = 4;  // the batch supplies the parallelism
    // a batch is throughput-bound: a combine per RK4 stage costs less than
    // staging every stage input from the previous stage's partial outputs
    P.fuse_stages = false;
    // larger tiles in batches: fewer stagings of each term's operands (the
    // tile-size autotuner settles on this value for a 512-instance batch)
    if (!P.tile_work_set) P.tile_work = 64e6;
    if (!P.prog_step || P.built_target != P.par_target || P.built_tile_work != P.tile_work ||
        P.built_fuse != P.fuse_stages) {
      P.prog_step = std::make_unique<Program>();
      P.prog_init = std::make_unique<Program>();
      build_step(P, *P.prog_step);
      build_init(P, *P.prog_init);
      P.built_target = P.par_target;
      P.built_tile_work = P.tile_work;
      P.built_fuse = P.fuse_stages;
      P.b_state = nullptr;
    }
    st[i] = *P.prog_step;
    in[i] = *P.prog_init;
    for (auto& L : st[i].launches) cost[i] += L.flops;
    chain[i] = st[i].launches.size();
    Builder b(P, rh[i]);
    b.rho_prog();
    rh[i].rprogs.back().rho_out = (double*)((char*)B.rho_buf + B.rho_off[i]);
    resolve(st[i], B.states[i], B.wss[i], B.dts[i], B.drives[i], B.ld);
    resolve(in[i], B.states[i], B.wss[i], B.dts[i], B.drives[i], B.ld);
    resolve(rh[i], B.states[i], B.wss[i], B.dts[i], nullptr, 1);
  }
  // Parts of the step: instances sorted by the length of their step's launch
  // chain (then by apply work) and cut into runs of about equal total work, so
  // the deep trees share a part and the shallow ones run beside them on short
  // chains.
  std::vector<size_t> order(n);
  for (size_t i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
    return chain[a] != chain[b] ? chain[a] > chain[b] : cost[a] > cost[b];
  });
  double total = 0;
  for (double c : cost) total += c;
  const int S = (int)std::max<size_t>(1, std::min<size_t>((size_t)B.n_parts, n));
  std::vector<std::vector<Program>> parts(S);
  double acc = 0;
  int k = 0;
  for (size_t j = 0; j < n; ++j) {
    const size_t i = order[j];
    if (k + 1 < S && !parts[k].empty() && acc >= total * (k + 1) / S) ++k;
    parts[k].push_back(std::move(st[i]));
    acc += cost[i];
  }
  B.steps.clear();
  for (auto& pv : parts) {
    if (pv.empty()) continue;
    Program mp = merge_programs(pv);
    B.steps.push_back(std::make_unique<DevProgram>());
    upload_resolved(*B.steps.back(), mp, s);
  }
  Program mi = merge_programs(in), mr = merge_programs(rh);
  upload_resolved(B.init, mi, s);
  upload_resolved(B.rho, mr, s);
  B.graph.reset();
}

// Root-core norms of every instance before a step call.
static void batch_norms_before(tenso_batch* b, hipStream_t s) {
  hipchk(launch_norms(b->norm_ops, (int)b->plans.size(), b->norms, s), "root norms");
}

// Non-finite values in any instance's state, or a norm grown by more than
// kNormGrowthLimit over the call: ENUMERIC (flags kept for tenso_batch_status).
static void check_batch_finite(tenso_batch* b, hipStream_t s) {
  const int n = (int)b->plans.size();
  hipchk(launch_finite(b->fin_ops, n, b->fin_flags, s), "finite check");
  hipchk(launch_norms(b->norm_ops, n, b->norms + n, s), "root norms");
  b->last_flags.assign(n, 0);
  std::vector<double> nb(2 * (size_t)n);
  hipchk(hipMemcpyAsync(b->last_flags.data(), b->fin_flags, n * sizeof(int), hipMemcpyDeviceToHost, s),
         "finite flags");
  hipchk(hipMemcpyAsync(nb.data(), b->norms, 2 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s),
         "norms");
  hipchk(hipStreamSynchronize(s), "sync");
  bool nonfinite = false, grown = false;
  for (int i = 0; i < n; ++i) {
    nonfinite = nonfinite || b->last_flags[i];
    if (!b->last_flags[i] && nb[n + i] > kNormGrowthLimit * nb[i]) {
      b->last_flags[i] = 1;
      grown = true;
    }
  }
  if (nonfinite) fail(TENSO_ENUMERIC, "non-finite values in the state of a batch instance after stepping");
  if (grown) fail(TENSO_ENUMERIC, "the state norm of a batch instance grew by more than a factor 1e6 over the step call");
}

// Check the batch arguments, (re)build the batch programs when the binding
// changed, and advance every instance by n_steps.
static void batch_advance(tenso_batch* b, const double* dt, int n_steps,
                          const double* const* d_drive_tabs, hipStream_t s, bool check = true) {
  if (!b || !dt) fail(TENSO_EINVAL, "null argument");
  if (n_steps < 0) fail(TENSO_EINVAL, "n_steps must be >= 0");
  const size_t n = b->plans.size();
  std::vector<double> dts(dt, dt + n);
  std::vector<const double*> drv(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    if (!(dts[i] > 0)) fail(TENSO_EINVAL, "dt must be > 0");
    if (d_drive_tabs) drv[i] = d_drive_tabs[i];
    if (b->plans[i]->gen.n_slots > 0 && !drv[i]) fail(TENSO_EINVAL, "instance with drive slots needs a drive table");
  }
  const int ld = 4 * n_steps + 1;
  bool stale = false, driven = false;
  for (auto* P : b->plans) {
    stale = stale || P->built_tile_work != P->tile_work;
    driven = driven || P->gen.n_slots > 0;
  }
  // the drive tables' row length is baked into the programs; it matters only
  // for instances with drive slots, so other batches keep their programs and
  // graph when the step count of a call changes
  if (stale || dts != b->dts || drv != b->drives || (driven && ld != b->ld) || b->steps.empty()) {
    b->dts = dts;
    b->drives = drv;
    b->ld = ld;
    batch_build(*b, s);
  }
  if (check) batch_norms_before(b, s);
  hipchk(launch_step_inc(b->ctr, 0, s), "ctr");
  run(b->init, b->fp64, b->ctr, s);
  step_loop(b->graph, b->step_parts(), b->fp64, b->ctr, n_steps, s);
  if (check) check_batch_finite(b, s);
}

extern "C" {

int tenso_batch_create(int n, tenso_plan* const* plans, void* const* d_states,
                       void* const* d_wss, tenso_batch** out) {
  return guard([&] {
    if (n < 1 || !plans || !d_states || !d_wss || !out) fail(TENSO_EINVAL, "bad batch arguments");
    auto B = std::make_unique<tenso_batch>();
    size_t rho_bytes = 0;
    for (int i = 0; i < n; ++i) {
      if (!plans[i] || !d_states[i] || !d_wss[i]) fail(TENSO_EINVAL, "null plan or buffer");
      if (plans[i]->opts.method != TENSO_PS1) fail(TENSO_EINVAL, "batches take ps1 plans");
      if (i > 0 && (plans[i]->fp64 != plans[0]->fp64 || plans[i]->amode != plans[0]->amode))
        fail(TENSO_EINVAL, "mixed precisions in a batch");
      B->plans.push_back(plans[i]);
      B->states.push_back(d_states[i]);
      B->wss.push_back(d_wss[i]);
      B->rho_off.push_back(rho_bytes);
      const size_t M = plans[i]->tree.end_dim[0];
      rho_bytes += align256(M * M * 16);
    }
    B->fp64 = plans[0]->fp64;
    hipchk(hipMalloc((void**)&B->ctr, 256), "hipMalloc(counter)");
    {
      std::vector<FiniteOp> ops(n);
      for (int i = 0; i < n; ++i) {
        ops[i].p = (const double*)d_states[i];
        ops[i].n = (long)(plans[i]->state_bytes / sizeof(double));
      }
      hipchk(hipMalloc((void**)&B->fin_flags, std::max(1, n) * sizeof(int)), "hipMalloc(flags)");
      for (int i = 0; i < n; ++i) ops[i].flag = B->fin_flags + i;
      hipchk(hipMalloc((void**)&B->fin_ops, n * sizeof(FiniteOp)), "hipMalloc(finite ops)");
      hipchk(hipMemcpy(B->fin_ops, ops.data(), n * sizeof(FiniteOp), hipMemcpyHostToDevice), "finite ops");
      std::vector<NormOp> nops(n);
      for (int i = 0; i < n; ++i) {
        nops[i].p = (const double*)((const char*)d_states[i] + plans[i]->core_off[0]);
        nops[i].n = 2 * plans[i]->tree.size(0);
      }
      hipchk(hipMalloc((void**)&B->norm_ops, std::max(1, n) * sizeof(NormOp)), "hipMalloc(norm ops)");
      hipchk(hipMemcpy(B->norm_ops, nops.data(), n * sizeof(NormOp), hipMemcpyHostToDevice), "norm ops");
      hipchk(hipMalloc((void**)&B->norms, std::max(1, 2 * n) * sizeof(double)), "hipMalloc(norms)");
    }
    hipchk(hipMalloc((void**)&B->rho_buf, std::max<size_t>(rho_bytes, 256)), "hipMalloc(rho)");
    *out = B.release();
  });
}

int tenso_batch_step(tenso_batch* b, const double* t0, const double* dt, int n_steps,
                     const double* const* d_drive_tabs, hipStream_t s) {
  return guard([&] {
    (void)t0;
    batch_advance(b, dt, n_steps, d_drive_tabs, s);
  });
}

int tenso_batch_step_record(tenso_batch* b, const double* t0, const double* dt, int n_steps,
                            int every, const double* const* d_drive_tabs, void* d_series,
                            hipStream_t s) {
  return guard([&] {
    if (!b || !dt || !d_series || every < 1) fail(TENSO_EINVAL, "bad arguments");
    if (n_steps < 0) fail(TENSO_EINVAL, "n_steps must be >= 0");
    (void)t0;
    const size_t n = b->plans.size();
    std::vector<double> dts(dt, dt + n);
    std::vector<const double*> drv(n, nullptr);
    for (size_t i = 0; i < n; ++i) {
      if (!(dts[i] > 0)) fail(TENSO_EINVAL, "dt must be > 0");
      if (d_drive_tabs) drv[i] = d_drive_tabs[i];
      if (b->plans[i]->gen.n_slots > 0 && !drv[i]) fail(TENSO_EINVAL, "instance with drive slots needs a drive table");
    }
    const int ld = 4 * n_steps + 1;
    bool stale = false, driven = false;
    for (auto* P : b->plans) {
      stale = stale || P->built_tile_work != P->tile_work;
      driven = driven || P->gen.n_slots > 0;
    }
    if (stale || dts != b->dts || drv != b->drives || (driven && ld != b->ld) || b->steps.empty()) {
      b->dts = dts;
      b->drives = drv;
      b->ld = ld;
      batch_build(*b, s);
    }
    const size_t rec = b->rho_off.back() + align256(b->plans.back()->tree.end_dim[0] *
                                                    b->plans.back()->tree.end_dim[0] * 16);
    batch_norms_before(b, s);
    hipchk(launch_step_inc(b->ctr, 0, s), "ctr");
    run(b->init, b->fp64, b->ctr, s);
    int r = 0;
    run(b->rho, b->fp64, nullptr, s);
    hipchk(hipMemcpyAsync((char*)d_series + (size_t)r++ * rec, b->rho_buf, rec,
                          hipMemcpyDeviceToDevice, s), "record");
    for (int k = 0; k < n_steps; ++k) {
      step_loop(b->graph, b->step_parts(), b->fp64, b->ctr, 1, s);
      if ((k + 1) % every == 0) {
        run(b->rho, b->fp64, nullptr, s);
        hipchk(hipMemcpyAsync((char*)d_series + (size_t)r++ * rec, b->rho_buf, rec,
                              hipMemcpyDeviceToDevice, s), "record");
      }
    }
    check_batch_finite(b, s);
  });
}

int tenso_batch_record_bytes(const tenso_batch* b, size_t* bytes_per_record, size_t* offsets) {
  return guard([&] {
    if (!b) fail(TENSO_EINVAL, "null batch");
    if (bytes_per_record)
      *bytes_per_record = b->rho_off.back() + align256(b->plans.back()->tree.end_dim[0] *
                                                       b->plans.back()->tree.end_dim[0] * 16);
    if (offsets)
      for (size_t i = 0; i < b->rho_off.size(); ++i) offsets[i] = b->rho_off[i];
  });
}

int tenso_batch_reduced_rho(tenso_batch* b, tenso_c128* const* h_rho, hipStream_t s) {
  return guard([&] {
    if (!b || !h_rho) fail(TENSO_EINVAL, "null argument");
    if (!b->rho.arena) fail(TENSO_EINVAL, "batch has not been stepped yet");
    run(b->rho, b->fp64, nullptr, s);
    size_t total = b->rho_off.back() + align256(b->plans.back()->tree.end_dim[0] *
                                                b->plans.back()->tree.end_dim[0] * 16);
    std::vector<char> h(total);
    hipchk(hipMemcpyAsync(h.data(), b->rho_buf, total, hipMemcpyDeviceToHost, s), "rho readback");
    hipchk(hipStreamSynchronize(s), "sync");
    for (size_t i = 0; i < b->plans.size(); ++i) {
      const size_t M = b->plans[i]->tree.end_dim[0];
      memcpy(h_rho[i], h.data() + b->rho_off[i], M * M * 16);
    }
  });
}

int tenso_batch_status(const tenso_batch* b, int32_t* flags) {
  return guard([&] {
    if (!b || !flags) fail(TENSO_EINVAL, "null argument");
    for (size_t i = 0; i < b->plans.size(); ++i)
      flags[i] = i < b->last_flags.size() ? b->last_flags[i] : 0;
  });
}

int tenso_batch_set_parts(tenso_batch* b, int n_parts) {
  return guard([&] {
    if (!b) fail(TENSO_EINVAL, "null batch");
    if (n_parts < 1 || n_parts > 4) fail(TENSO_EINVAL, "n_parts must be in [1, 4]");
    b->n_parts = n_parts;
    b->steps.clear();  // rebuilt at the next step call
    b->graph.reset();
  });
}

int tenso_batch_set_graph(tenso_batch* b, int enable) {
  return guard([&] {
    if (!b) fail(TENSO_EINVAL, "null batch");
    b->graph.enabled = enable != 0;
    b->graph.reset();
  });
}

int tenso_batch_state_bytes(const tenso_batch* b, size_t* bytes) {
  return guard([&] {
    if (!b || !bytes) fail(TENSO_EINVAL, "null argument");
    size_t tot = 0;
    for (auto* P : b->plans) tot += align256(P->state_bytes);
    *bytes = tot;
  });
}

int tenso_batch_autotune(tenso_batch* b, const double* dt, int trial_steps,
                         const double* const* d_drive_tabs, void* d_backup, size_t backup_bytes,
                         double* tile_work_out, hipStream_t s) {
  return guard([&] {
    if (!b || !dt || !d_backup) fail(TENSO_EINVAL, "null argument");
    if (trial_steps < 1) fail(TENSO_EINVAL, "trial_steps must be >= 1");
    const size_t n = b->plans.size();
    std::vector<size_t> off(n);
    size_t tot = 0;
    for (size_t i = 0; i < n; ++i) {
      off[i] = tot;
      tot += align256(b->plans[i]->state_bytes);
    }
    if (backup_bytes < tot) fail(TENSO_ENOMEM, "backup buffer smaller than the batch states");
    auto copy_states = [&](bool save) {
      for (size_t i = 0; i < n; ++i) {
        char* bk = (char*)d_backup + off[i];
        if (save)
          hipchk(hipMemcpyAsync(bk, b->states[i], b->plans[i]->state_bytes, hipMemcpyDeviceToDevice, s), "save");
        else
          hipchk(hipMemcpyAsync(b->states[i], bk, b->plans[i]->state_bytes, hipMemcpyDeviceToDevice, s), "restore");
      }
    };
    copy_states(true);
    static const double cand[] = {4e6, 8e6, 16e6, 32e6, 64e6};
    hipEvent_t e0, e1;
    hipchk(hipEventCreate(&e0), "hipEventCreate");
    hipchk(hipEventCreate(&e1), "hipEventCreate");
    double best = -1, best_ms = 0;
    try {
      for (double w : cand) {
        for (auto* P : b->plans) {
          P->tile_work = w;
          P->tile_work_set = true;
        }
        batch_advance(b, dt, trial_steps, d_drive_tabs, s, false);  // build, capture, warm up
        copy_states(false);
        hipchk(hipEventRecord(e0, s), "hipEventRecord");
        batch_advance(b, dt, trial_steps, d_drive_tabs, s, false);
        hipchk(hipEventRecord(e1, s), "hipEventRecord");
        hipchk(hipEventSynchronize(e1), "hipEventSynchronize");
        float ms = 0;
        hipchk(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        copy_states(false);
        if (best < 0 || ms < best_ms) {
          best = w;
          best_ms = ms;
        }
      }
    } catch (...) {
      copy_states(false);  // the caller gets its states back even on failure
      (void)hipStreamSynchronize(s);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (auto* P : b->plans) P->tile_work = best;
    hipchk(hipStreamSynchronize(s), "sync");
    if (tile_work_out) *tile_work_out = best;
  });
}

void tenso_batch_destroy(tenso_batch* b) { delete b; }

}  // extern "C"
