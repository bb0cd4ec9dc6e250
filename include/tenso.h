/*
 * tenso.h -- C ABI of the MI355X TTN-HEOM propagation library.
 *
 * The library applies a sum-of-products (SOP) generator L(t) to an extended
 * density operator Omega stored as a tree tensor network (TTN) and advances
 * dOmega/dt = L(t) Omega (paper Sec. II B-C: Eqs. heom-std, EDO-eom,
 * master_lvn, omega_tensor, semiunitary) with the fixed-rank (ps1) and
 * adaptive-rank (ps2) projector-splitting integrators (Sec. II C).
 *
 * Conventions shared by every entry point
 *   - Every call returns 0 on success or a negative TENSO_E* code; the
 *     message of the last failure on the calling thread is returned by
 *     tenso_last_error().  No exception crosses this boundary.
 *   - Host arrays passed in are copied during the call; the caller keeps
 *     ownership.  Handles are owned by the library and released with the
 *     matching *_destroy call.  A handle must not be used from two threads
 *     at the same time.
 *   - Device buffers (state, workspace, drive tables) are allocated by the
 *     caller and passed as raw device pointers together with a hipStream_t;
 *     their sizes come from tenso_plan_sizes().  The library allocates device
 *     memory for its constant tables (plan and batch creation) and for its
 *     launch-descriptor arenas: when a step call first runs, or rebuilds, its
 *     programs for a binding (buffers, dt, tile size, drive), and in ps2 calls
 *     for each new combination of sub-flow and bond ranks (the programs are
 *     kept and replayed once the ranks settle).  The caller's buffers are never
 *     reallocated.
 *   - Complex numbers are interleaved {double re, double im} on the host.
 *     The device state layout is private to the library; convert with
 *     tenso_state_import / tenso_state_export.
 *
 * Tree description (Sec. II C, general TTN equation)
 *   Nodes are numbered 0..n_nodes-1; node 0 is the root and parent[s] < s.
 *   Ends (open legs) are numbered 0 = ket (dim M), 1 = bra (dim M),
 *   2 + k = bath feature k (dim N_k); both system ends sit on the root.
 *   The legs of node s are, in order: its bond to parent[s] (if s > 0), the
 *   ends attached to s in increasing end index, its child nodes in increasing
 *   node id.  Core s is stored row-major over its legs.  The bond between
 *   node c and parent[c] has rank r_c; ranks are clamped so that every core
 *   can be semi-unitary (r_c <= product of c's other leg dims and <= product
 *   of parent[c]'s other leg dims).
 */
#ifndef TENSO_H
#define TENSO_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TENSO_OK            0
#define TENSO_EINVAL       -1   /* malformed input (tree, dims, sizes, dt <= 0) */
#define TENSO_ENOMEM       -2   /* workspace too small / size beyond the budget */
#define TENSO_EHIP         -3   /* a HIP runtime error (message carries hipGetErrorString) */
#define TENSO_ENUMERIC     -4   /* NaN or infinity in a state after stepping, or its
                                   norm grown more than 1e6-fold over the step call */
#define TENSO_EUNSUPPORTED -5   /* valid input outside what this library implements */

typedef struct { double re, im; } tenso_c128;
typedef struct tenso_tree tenso_tree;
typedef struct tenso_gen tenso_gen;
typedef struct tenso_plan tenso_plan;
typedef struct tenso_batch tenso_batch;

#define TENSO_FP64 0          /* every contraction in complex FP64 (plain reference path) */
#define TENSO_FP32 1          /* contractions in complex FP32 on MFMA, FP64 master state */
#define TENSO_FP32_3M 2       /* as TENSO_FP32, each complex product of the contraction from
                                 three real MFMA products (Gauss: Re a Re b, Im a Im b,
                                 (Re a + Im a)(Re b + Im b)) instead of four */
#define TENSO_BF16 3          /* precision study: as TENSO_FP32 with every contraction operand
                                 (input slices, scaled operator entries, the intermediate
                                 X B^T) rounded to BF16; the products then equal a BF16 MFMA's
                                 with FP32 accumulation (run on the FP32 MFMA) */

#define TENSO_PS1 0           /* fixed-rank projector splitting */
#define TENSO_PS2 1           /* adaptive-rank projector splitting */
#define TENSO_VMF 2           /* fixed-rank direct integration of every core (FP64 only) */

typedef struct {
  int precision;   /* TENSO_FP64 | TENSO_FP32 | TENSO_FP32_3M | TENSO_BF16 */
  int method;      /* TENSO_PS1 | TENSO_PS2 | TENSO_VMF */
  int max_rank;    /* PS2: cap on any bond rank (also sizes the state) */
} tenso_plan_opts;

/* Last error message of the calling thread ("" if none). */
const char* tenso_last_error(void);

/* Build a tree from a parent array and an end map (general TTN, Sec. II C).
 * parent[0] = -1 and 0 <= parent[s] < s.  end_node[e] / end_dim[e] give the
 * node and dimension of end e (ends 0 and 1 must sit on node 0; end 1 has
 * end 0's dimension for a density state, or 1 for a wavefunction).  bond_rank
 * (nullable, indexed by child node, entry 0 ignored) requests per-bond ranks,
 * otherwise max_rank is requested everywhere; both are clamped (see above).
 * Errors: EINVAL on a malformed tree or dims < 1. */
int tenso_build_tree(int n_nodes, const int32_t* parent, int n_ends,
                     const int32_t* end_node, const int32_t* end_dim,
                     int max_rank, const int32_t* bond_rank, tenso_tree** out);

/* Tensor train (Eq. omega_tensor): root(ket, bra, ->1); node s holds feature
 * s-1 and a bond to s+1; the last node holds the last two features. */
int tenso_tree_train(int M, int K, const int32_t* mode_dim, int rank, tenso_tree** out);

/* Balanced n-ary tree: root(ket, bra, ->tree over all features); a list of
 * features becomes an end if it has one element, a node holding them if it has
 * at most n_ary, else a node over n_ary contiguous near-equal chunks (larger
 * first).  Nodes are numbered in preorder. */
int tenso_tree_nary(int M, int K, const int32_t* mode_dim, int n_ary, int rank,
                    tenso_tree** out);

/* Effective bond ranks after clamping: bond_rank_out[c] for c = 1..n-1
 * (entry 0 is set to 0).  Array length n_nodes. */
int tenso_tree_ranks(const tenso_tree* t, int32_t* bond_rank_out);
int tenso_tree_n_nodes(const tenso_tree* t);
void tenso_tree_destroy(tenso_tree* t);

/* SOP generator (Eq. master_lvn, the paper's SparseSPO): term m is
 * coef[m] * f_slot(t) * (x)_{factors} F, where f_slot = 1 if td_slot[m] < 0.
 * Factor j of term m (in order, n_factors[m] of them) acts on end
 * factor_end[.] with a dense row-major d x d matrix taken consecutively from
 * factor_mats; ends without a factor carry the identity.  Each term needs at
 * least one factor, and at most two legs of any core may carry a non-identity
 * operator for one term (EUNSUPPORTED otherwise; HEOM terms have <= 2
 * factors).  Errors: EINVAL on bad ends / dims. */
int tenso_build_generator(const tenso_tree* t, int n_terms, const tenso_c128* coef,
                          const int32_t* td_slot, const int32_t* n_factors,
                          const int32_t* factor_end, const tenso_c128* factor_mats,
                          tenso_gen** out);
void tenso_gen_destroy(tenso_gen* g);

/* Compile tree + generator into an execution plan (tables uploaded to the
 * current HIP device).  The plan keeps its own copies of tree and generator.
 * Errors: EINVAL (bad options, a generator built for another tree),
 * EUNSUPPORTED (a term with more than two non-identity legs on one core, a
 * ps2 edge beyond what the split supports), EHIP. */
int tenso_plan_create(const tenso_tree* t, const tenso_gen* g, const tenso_plan_opts* opts,
                      tenso_plan** out);

/* Compile the same plan on the host only (no HIP call, no device memory) and
 * report what tenso_plan_create would need: state and workspace bytes (each
 * nullable), and for PS1 plans the kernel launches of one step and their
 * algorithmic apply flops, for VMF plans those of one evaluation of the
 * derivative (a dopri5 substep takes six; 0 for PS2, whose sweep depends on
 * the ranks).
 * Same errors as tenso_plan_create, minus EHIP. */
int tenso_plan_query(const tenso_tree* t, const tenso_gen* g, const tenso_plan_opts* opts,
                     size_t* state_bytes, size_t* workspace_bytes, int64_t* launches_per_step,
                     double* apply_flops_per_step);
void tenso_plan_destroy(tenso_plan* p);

/* Step execution switches (no device work).
 * tenso_plan_set_graph: enable (default) or disable replaying tenso_step_fixed
 * steps from a captured HIP graph; disabled, every step launches its kernels
 * one by one (results are identical either way).
 * tenso_plan_set_tile_work: flops per apply-kernel tile (default 16e6 for a
 * plan stepped alone, 64e6 inside a batch unless set here; range [1e5, 1e9],
 * EINVAL outside); takes effect at the next build of the plan's programs,
 * i.e. the next step call. */
int tenso_plan_set_graph(tenso_plan* p, int enable);
int tenso_plan_set_tile_work(tenso_plan* p, double flops);

/* Device bytes the caller must provide: the state (FP64 master cores) and the
 * workspace (operand copies, environments, stage buffers, QR scratch). */
int tenso_plan_sizes(const tenso_plan* p, size_t* state_bytes, size_t* workspace_bytes);

/* Number of cores and, per core, its current leg dimensions (up to 8 legs,
 * dims_out[8*s + l], unused entries 0).  Host call, no device work. */
int tenso_plan_shapes(const tenso_plan* p, int32_t* n_legs_out, int32_t* dims_out);

/* Write the initial product state rho_S(0) (x) |0..0> (host rho_s, row-major
 * over ends 0 and 1: M x M for a density, M x 1 for a wavefunction psi(0))
 * into d_state: root[i, j, 0..] = rho[i, j]; other cores U[a, beta] =
 * delta(a, flat(beta)).  PS2 plans start at rank 2 on every bond (clamped;
 * with rank 1 a tree whose inner nodes carry no physical leg has two-site
 * tensors with a side of dimension 1, and no bond could ever grow). */
int tenso_state_init(tenso_plan* p, const tenso_c128* rho_s, void* d_state, hipStream_t s);

/* Copy host cores (concatenated, each row-major over its legs at the plan's
 * current ranks) to the device state, and back.  ranks (nullable) receives
 * the current bond ranks (length n_nodes).  Export synchronises the stream. */
int tenso_state_import(tenso_plan* p, const tenso_c128* h_cores, void* d_state, hipStream_t s);
int tenso_state_export(tenso_plan* p, const void* d_state, tenso_c128* h_cores, int32_t* ranks,
                       hipStream_t s);

/* Effective generator at `center` (Sec. II C, the local TDVP right-hand side
 * of Eq. master_lvn on the tree): d_out (complex FP64, the center core's
 * shape, row-major, caller-owned device buffer) =
 * sum_m coef_m f_slot(m) (x)_legs X_{m,l} C_center, with up/down environments
 * on virtual legs, factors on ends and identities skipped.  The time enters
 * only through the drive values: drive is a host array of one value f_slot
 * per slot, taken at the time of interest (nullable if the generator has no
 * slots).  The state must be canonical toward `center`: every other core an
 * isometry toward it (checked on the device to 1e-8; EINVAL otherwise).
 * d_ws is the plan's workspace.  The library allocates the launch
 * descriptors' device arena for the call and frees it before returning
 * (errors included).  Synchronous on `s` for the result. */
int tenso_apply_generator(tenso_plan* p, const void* d_state, int center, const double* drive,
                          void* d_out, void* d_ws, hipStream_t s);

/* The same with no device allocation in the call, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Workspace and launch descriptors live in a static
 * device array of TENSO_NOALLOC_SCRATCH_MIB MiB that each GPU the library
 * runs on holds until the process ends; the caller passes no workspace.
 * The result equals tenso_apply_generator's.  ENOMEM when the plan's
 * workspace plus descriptors exceed the array.  Every call on a GPU shares
 * that GPU's array and clears it first: calls that overlap on one GPU (two
 * streams, two threads) race and must not be issued.  Synchronous on `s`. */
#define TENSO_NOALLOC_SCRATCH_MIB 64
int tenso_apply_generator_noalloc(tenso_plan* p, const void* d_state, int center,
                                  const double* drive, void* d_out, hipStream_t s);

/* Advance n_steps steps of size dt with ps1 (second-order: a first-order
 * sweep over half a step, then its adjoint).  d_drive_tab (nullable when the
 * generator has no slots) holds f_slot at t0 + j*dt/4, j = 0..4*n_steps,
 * as [n_slots][4*n_steps+1] doubles on the device.  The state stays canonical
 * toward the root.  At the end the state is checked for NaN/infinity and
 * for a norm grown more than 1e6-fold over the call (both ENUMERIC; the norm
 * is that of the root core, which carries it in a root-canonical state),
 * which synchronises `s` once per call. */
int tenso_step_fixed(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                     const double* d_drive_tab, void* d_ws, hipStream_t s);

/* Same with ps2 (two-site sweeps, SVD truncation; the SVD and the decision
 * are those of tenso_svd_truncate).  With r_eps the smallest r whose discarded
 * tail sqrt(sum_{i>=r} s_i^2) is at most eps * sqrt(sum s_i^2), every split
 * keeps r' = min(max_rank, available, r_eps + 1) directions, r' >= 1 (one
 * direction beyond r_eps is room for the rank to grow): the leading singular
 * vectors with s_i > 1e-10 s_1, then unit vectors projected onto the
 * orthogonal complement.  The decision is taken on the device and read back
 * once per split (the new rank sets the shapes of the following sub-flows),
 * so the call synchronises the stream per edge.  ENOMEM at plan creation if
 * a two-site tensor exceeds 2^26 elements at the rank cap. */
int tenso_step_adaptive(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                        double eps, int max_rank, const double* d_drive_tab, void* d_ws,
                        hipStream_t s);

/* ---- direct integration (vmf) and the mixed strategy ----------------------
 * Sec. II C: every core is integrated at once by an ODE solver at fixed rank;
 * Sec. VII E: dopri5 with tolerances ode_rtol / ode_atol, and a constant
 * vmf_atol added to the diagonal of the matrix that the non-root equations
 * invert.  The equations are the time-dependent variational principle for
 * dOmega/dt = L Omega in the root gauge (every non-root core U_s an isometry
 * toward its parent, U_s^H dU_s = 0): the root core moves under its
 * effective generator; a non-root core under its effective generator with
 * the mean fields of the rest of the network on its parent leg, followed by
 * (rho_s + vmf_atol I)^-1 on that leg (rho_s: the density on the bond) and
 * the projection off the span of U_s.  Available on every FP64 plan whose
 * terms keep at most one factor inside any non-root subtree and whose bonds
 * are at most 64 (TENSO_VMF plans are checked at creation; on other plans
 * the calls return EUNSUPPORTED).  Every field is used as given; the paper's
 * defaults are ode_rtol 1e-5 and ode_atol 1e-7 (vmf_atol: 1e-7 here). */
typedef struct {
  double ode_rtol;     /* relative tolerance of the adaptive steps */
  double ode_atol;     /* absolute tolerance of the adaptive steps */
  double vmf_atol;     /* diagonal shift of every bond density (>= 0; 0 needs them regular) */
  int fixed_substeps;  /* 0: adaptive steps; n > 0: n equal dopri5 steps per dt, no control */
  int max_substeps;    /* adaptive: ENUMERIC when one call needs more substeps */
} tenso_vmf_opts;

/* Drive callback: f_slots[k] = f_k(t) for every slot k (host, called from
 * the stepping thread). */
typedef void (*tenso_drive_fn)(double t, double* f_slots, void* ctx);

/* Advance n_steps output steps of size dt by direct integration.  Solver:
 * the Dormand-Prince 5(4) pair advancing with the fifth-order solution, the
 * last stage reused as the next step's first.  Adaptive: error norm = root
 * mean square over every complex core entry of |y5 - y4| / (ode_atol +
 * ode_rtol max(|y_old|, |y_new|)); accepted when <= 1; the next size is h
 * 0.9 norm^(-1/5) clipped to [0.2 h, 10 h]; each dt is covered by substeps,
 * the last shortened to end on it (the proposal then stays unless its own
 * is larger); the first substep after tenso_state_init / import tries dt,
 * later calls continue from the last proposal.  The error norm is read back
 * once per substep (a synchronisation).  drive (nullable without slots) is
 * called for the seven stage times of every substep.  The state must be
 * root-canonical, as tenso_state_init, tenso_step_fixed and
 * tenso_step_adaptive leave it.  ENUMERIC on a non-finite state or error
 * estimate, a 1e6-fold norm growth, a step size below 1e-14 dt or more than
 * max_substeps substeps.  The first call per rank pattern builds and uploads
 * the derivative's launch program (device allocation). */
int tenso_step_vmf(tenso_plan* p, void* d_state, double t0, double dt, int n_steps,
                   const tenso_vmf_opts* opts, tenso_drive_fn drive, void* drive_ctx,
                   void* d_ws, hipStream_t s);

/* The time derivative of every core of a root-canonical state (the
 * right-hand side that tenso_step_vmf integrates), into d_out: a device
 * buffer of the plan's state bytes, same layout as the state (read it back
 * with tenso_state_export).  drive: host, one value per slot (nullable
 * without slots).  Synchronous on `s`. */
int tenso_vmf_derivative(tenso_plan* p, const void* d_state, double vmf_atol, const double* drive,
                         void* d_out, void* d_ws, hipStream_t s);

/* The ps2 truncation rule by an absolute threshold (Sec. VII E: ps2_atol and
 * ps2_ratio; paper defaults 1e-7 and 2): with ps2_ratio >= 1 every later ps2
 * split (tenso_step_adaptive, the ps2 part of tenso_step_mix) keeps r' =
 * min(max_rank, available, ceil(ps2_ratio r_atol)) directions, r_atol the
 * number of singular values above ps2_atol (at least 1): the discarded part
 * of the spectrum just below the threshold is partly taken back, in
 * proportion to what was kept.  The eps argument is then ignored.
 * ps2_ratio = 0 restores the eps rule (the default).  No device work.
 * EINVAL on ps2_atol < 0 or 0 < ps2_ratio < 1. */
int tenso_plan_set_ps2_truncation(tenso_plan* p, double ps2_atol, double ps2_ratio);

/* Accepted and rejected dopri5 substeps since tenso_state_init / import,
 * and the next proposed substep size (0 before the first). Each nullable. */
int tenso_vmf_stats(const tenso_plan* p, int64_t* accepted, int64_t* rejected, double* next_h);

/* The mixed strategy (Sec. VI, Sec. VII E) on an FP64 ps2 plan: ps2 steps
 * (the eps rule of tenso_step_adaptive, ranks capped at max_aux_rank) until
 * a bond rank reaches max_aux_rank, then direct integration at the ranks
 * reached for every later step.  The phase persists across calls until
 * tenso_state_init / import.  switch_step (nullable) receives the number of
 * ps2 steps taken before the switch, or -1 while still in ps2.  For the ps2
 * steps drive is sampled at t + j dt / 4, j = 0..4.  Errors as the two
 * methods; EINVAL unless 2 <= max_aux_rank <= the plan's max_rank. */
int tenso_step_mix(tenso_plan* p, void* d_state, double t0, double dt, int n_steps, double eps,
                   int max_aux_rank, const tenso_vmf_opts* opts, tenso_drive_fn drive,
                   void* drive_ctx, void* d_ws, hipStream_t s, int32_t* switch_step);

/* Reduced density matrix rho_S = <0..0|Omega> (Sec. II B) into host h_rho
 * (M x M) and its trace into h_trace (nullable).  Synchronises the stream. */
int tenso_reduced_rho(tenso_plan* p, const void* d_state, tenso_c128* h_rho, double* h_trace,
                      void* d_ws, hipStream_t s);

/* Reduced density of a wavefunction state (Sec. III A 5: ML-MCTDH on the same
 * tree and kernels): the tree's end 1 has dimension 1, and
 * rho_S = Tr_bath |psi><psi| (M x M, host h_rho; its trace into h_trace,
 * nullable), formed on the device from the root core, which holds the
 * state's norm: the state must be canonical toward the root, as it is after
 * tenso_state_init and every step call.  EINVAL if end 1 is not of dimension
 * 1.  Synchronises the stream. */
int tenso_reduced_rho_pure(tenso_plan* p, const void* d_state, tenso_c128* h_rho, double* h_trace,
                           void* d_ws, hipStream_t s);

/* Bond ranks chosen by the last ps2 step, one entry per split in sweep order;
 * returns the number of entries (at most cap) or a negative error. */
int tenso_rank_trajectory(const tenso_plan* p, int32_t* h_ranks, int cap);

/* The SVD behind the ps2 split (Sec. II C: two-site tensors are split by
 * SVD), on its own: A is a device matrix, rows x cols row-major complex FP64
 * (at most 2^26 elements, ENOMEM beyond).  It is factorised in FP64 from A
 * itself (range finder with hashed test columns, Householder QR, one-sided
 * Jacobi on the projected p x p factor; p = min(64, rows, cols,
 * 2 min(max_rank, rows, cols) + 8)), which keeps each singular value accurate
 * to rounding relative to sigma_1.
 *   h_sigma (host, nullable): the p leading singular values, descending.
 *   d_vectors (device, caller-owned, n x p complex row-major): the leading
 *     singular vectors of the left side (iso 0, n = rows) or of the right
 *     side (iso 1, n = cols; columns of V with A = U S V^H).
 *   h_decision (host, nullable, 3 entries): the ps2 truncation for (eps,
 *     max_rank): r' = min(max_rank, min(rows, cols), r_eps + 1), the number k
 *     <= r' of singular values above 1e-10 sigma_1, and r_eps, the smallest r
 *     with sqrt(sum_{i>=r} s_i^2) <= eps * ||A||_F (at least 1; eps = 0
 *     keeps every direction; min(rows, cols) when r_eps exceeds the p
 *     computed directions, which then all lie above the cap).
 *   h_missed (host, nullable): the energy outside the captured p-dimensional
 *     subspace relative to ||A||_F^2, when the subspace may be incomplete
 *     (p below the smaller side and s_p > 1e-13 s_1), else 0.  Then power
 *     steps are added until the leading singular values settle (at most
 *     three).
 * Allocates its device scratch for the call and frees it before returning.
 * Synchronous on `s`.  Errors: EINVAL, ENOMEM, EHIP. */
int tenso_svd_truncate(const void* d_A, int rows, int cols, int iso, double eps, int max_rank,
                       double* h_sigma, void* d_vectors, int32_t* h_decision, double* h_missed,
                       hipStream_t s);

/* ---- measurement ---------------------------------------------------------
 * tenso_profile(1) starts recording HIP events on the launching stream around
 * every launch of the SOP-contraction (apply) kernel, together with its
 * algorithmic work (8 flops per complex multiply-add, no padding; bytes = input
 * read + output written + operand matrices); tenso_profile(0) stops and clears.
 * tenso_profile_stats synchronises on the recorded events and returns the
 * summed kernel time, launch count, flops and bytes.  Process-wide state. */
int tenso_profile(int enable);
int tenso_profile_stats(double* total_ms, int64_t* launches, double* flops, double* bytes);
/* The same per launch, in launch order: the first min(cap, launches) entries
 * of ms / flops / bytes (each nullable; host arrays the caller owns) are
 * filled and *n_out receives the number of recorded launches. */
int tenso_profile_records(int64_t cap, double* ms, double* flops, double* bytes, int64_t* n_out);

/* ---- batched fixed-rank propagation --------------------------------------
 * Many independent ps1 plans (uneven trees, ranks, dims) advance together:
 * one launch per phase serves every instance, and the whole step sequence is
 * captured into a HIP graph and replayed.  All plans must share a precision.
 * d_states[i] / d_wss[i] are each instance's own buffers (sizes from
 * tenso_plan_sizes); t0[i], dt[i] host arrays; d_drive_tabs nullable. */
int tenso_batch_create(int n, tenso_plan* const* plans, void* const* d_states,
                       void* const* d_wss, tenso_batch** out);
int tenso_batch_step(tenso_batch* b, const double* t0, const double* dt, int n_steps,
                     const double* const* d_drive_tabs, hipStream_t s);
/* As tenso_batch_step, recording every instance's rho_S (Sec. II B) on the
 * device before the first step and after every `every` steps into d_series:
 * record j occupies bytes [j*B, (j+1)*B) with B from tenso_batch_record_bytes,
 * instance i's M_i x M_i complex FP64 matrix at byte offset offsets[i] inside a
 * record.  d_series must hold (n_steps/every + 1) records. */
int tenso_batch_step_record(tenso_batch* b, const double* t0, const double* dt, int n_steps,
                            int every, const double* const* d_drive_tabs, void* d_series,
                            hipStream_t s);
int tenso_batch_record_bytes(const tenso_batch* b, size_t* bytes_per_record, size_t* offsets);

/* rho_S of every instance: h_rho[i] points to an M_i x M_i host array. */
int tenso_batch_reduced_rho(tenso_batch* b, tenso_c128* const* h_rho, hipStream_t s);
void tenso_batch_destroy(tenso_batch* b);

/* Per instance, 1 if its state held NaN or infinite values after the last
 * step call, or its norm grew more than 1e6-fold over that call (the call then
 * returned TENSO_ENUMERIC), else 0; flags has n entries.  Host call, no
 * device work. */
int tenso_batch_status(const tenso_batch* b, int32_t* flags);

/* Graph replay of batched steps on (default) or off; results are identical. */
int tenso_batch_set_graph(tenso_batch* b, int enable);

/* Independent parts of a batched step (1..4, default 4; EINVAL outside):
 * instances sorted by step work are cut into parts of about equal work, each
 * part a phase-merged launch sequence of its own; in graph replay the parts
 * are parallel branches of one graph (eager steps run them in turn).  Results
 * are identical for every part count.  Takes effect at the next step call. */
int tenso_batch_set_parts(tenso_batch* b, int n_parts);

/* Bytes of a buffer that holds every instance's state (each 256-byte aligned). */
int tenso_batch_state_bytes(const tenso_batch* b, size_t* bytes);

/* Autotuner: times trial_steps batched steps (programs built and graph
 * captured first, then timed on the stream with HIP events) for each apply
 * tile size in {4e6, 8e6, 16e6, 32e6, 64e6} flops and keeps the fastest on
 * every plan of the batch; *tile_work_out receives it.  The instance states
 * are saved to d_backup (caller-owned device buffer of at least
 * tenso_batch_state_bytes bytes; ENOMEM if smaller) and restored after every
 * trial, so on return they are bit-identical to those on entry.  dt and
 * d_drive_tabs are as for tenso_batch_step with n_steps = trial_steps.
 * Synchronises the stream. */
int tenso_batch_autotune(tenso_batch* b, const double* dt, int trial_steps,
                         const double* const* d_drive_tabs, void* d_backup, size_t backup_bytes,
                         double* tile_work_out, hipStream_t s);

/* ---- learned surrogate (a project addition; not in the paper) ------------
 * Building blocks of a SiLU multilayer perceptron trained on trajectories of
 * the batched solver.  Device FP32 buffers; GEMM operands are rounded to BF16
 * and multiplied on BF16 MFMA with FP32 accumulation.
 * tenso_mlp_gemm: C = beta*C + A*B with A(m,k) = A[m*sam + k*sak], B(k,n) =
 *   B[k*sbk + n*sbn], C row-major (ldc); optional bias[n] added and, with
 *   act = 1, SiLU(C) written to H (H = C copy when act = 0; H nullable).
 * tenso_mlp_silu_bwd: dZ = dH * SiLU'(Z).   tenso_mlp_col_sum: column sums.
 * tenso_mlp_mse: dY = 2(Y-T)/n and loss[0] += mean squared error (device).
 * tenso_mlp_adam: one Adam update of n FP32 parameters (step count t >= 1).
 * All are asynchronous on `s`; they return 0, -1 on bad sizes, -3 on a HIP
 * launch error. */
int tenso_mlp_gemm(int M, int N, int K, const float* A, long sam, long sak, const float* B, long sbk,
                   long sbn, float* C, long ldc, float beta, const float* bias, int act, float* H,
                   hipStream_t s);
int tenso_mlp_silu_bwd(const float* dH, const float* Z, float* dZ, long n, hipStream_t s);
int tenso_mlp_col_sum(const float* X, int rows, int cols, float* out, hipStream_t s);
int tenso_mlp_mse(const float* Y, const float* T, long n, float* dY, float* loss, hipStream_t s);
int tenso_mlp_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1,
                   float b2, float eps, int t, hipStream_t s);

#ifdef __cplusplus
}
#endif
#endif
