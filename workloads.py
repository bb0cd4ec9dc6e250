"""Seeded synthetic workloads (inputs only; no HEOM arithmetic lives here).

Both the GPU path and the CPU oracle draw their problem parameters from this
module: system Hamiltonians, coupling operators, bath parameters, hierarchy
depths, tree shapes, ranks, initial states and drive pulses.  Everything that
turns these parameters into features, generators or trees is implemented
separately on each side.

Units: every workload is dimensionless (hbar = k_B = 1) except the 7-site
exciton model, which is given in cm^-1 / fs / K and converted here to hbar = 1
with energies in cm^-1:
a time t [fs] becomes t * FS_TO_CM and a temperature T [K] becomes T * KB_CM.
"""
import numpy as np

FS_TO_CM = 2.0 * np.pi * 2.99792458e-5   # 2 pi c * 1 cm^-1, in rad/fs
KB_CM = 0.6950348                        # Boltzmann constant in cm^-1 / K

SZ = np.diag([1.0, -1.0]).astype(np.complex128)
SX = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)


class Bath:
    """One bath: coupling operator Q, temperature T, Drude terms (lam, wc),
    Brownian terms (lam, w0, eta), the number of low-temperature corrections
    and how they are taken ("matsubara" or "pade")."""

    def __init__(self, Q, T, dl=(), bo=(), n_ltc=0, decomposition="matsubara"):
        self.Q = np.asarray(Q, dtype=np.complex128)
        self.T = float(T)
        self.dl = [tuple(map(float, x)) for x in dl]
        self.bo = [tuple(map(float, x)) for x in bo]
        self.n_ltc = int(n_ltc)
        self.decomposition = decomposition

    def n_features(self):
        return len(self.dl) + 2 * len(self.bo) + self.n_ltc


class Instance:
    """One TTN-HEOM problem."""

    def __init__(self, name, H, baths, depth, tree, rank, rho0, dt, n_steps,
                 method="ps1", eps=0.0, drive=None, metric="abs"):
        self.name = name
        self.H = np.asarray(H, dtype=np.complex128)
        self.baths = baths
        self.depth = depth
        self.tree = tree          # "train" | "tree2" | "tree3"
        self.rank = rank
        self.rho0 = np.asarray(rho0, dtype=np.complex128)
        self.dt = dt
        self.n_steps = n_steps
        self.method = method
        self.eps = eps
        self.drive = drive        # None or (H_d, A, w, s, t0)
        self.metric = metric      # HEOM metric: "abs", "re" or a complex constant

    @property
    def M(self):
        return self.H.shape[0]

    @property
    def K(self):
        return sum(b.n_features() for b in self.baths)

    def drive_value(self, t):
        """f(t) = A exp(-(t - t0)^2 / (2 s^2)) cos(w t)."""
        if self.drive is None:
            return 0.0
        _, A, w, s, t0 = self.drive
        return A * np.exp(-0.5 * ((t - t0) / s) ** 2) * np.cos(w * t)


def ground(M):
    r = np.zeros((M, M), dtype=np.complex128)
    r[0, 0] = 1.0
    return r


def spin_boson_train(n_steps=2000, rank=8):
    """Spin-boson, Drude bath with 2 Matsubara terms (3 features), depth 10,
    tensor train of rank 8, RK4 dt = 0.01."""
    bath = Bath(SZ, 1.0, dl=[(0.1, 1.0)], n_ltc=2)
    return Instance("spin-boson K=3 N=10 train R=8", 0.5 * SZ + SX, [bath], 10,
                    "train", rank, ground(2), 0.01, n_steps)


def exciton_7site(n_steps=1000, seed=1):
    """7-site exciton model (cm^-1, fs, K) with one Drude bath per site (3
    Matsubara terms each: 28 features), depth 8, binary tree of rank 16,
    dt = 0.1 fs."""
    rng = np.random.default_rng(seed)
    M = 7
    eps = rng.uniform(0.0, 500.0, size=M)
    H = np.diag(eps).astype(np.complex128)
    for i in range(M):
        for j in range(i + 1, M):
            v = rng.normal(0.0, 50.0)
            H[i, j] = H[j, i] = v
    baths = []
    for b in range(M):
        Q = np.zeros((M, M), dtype=np.complex128)
        Q[b, b] = 1.0
        baths.append(Bath(Q, 300.0 * KB_CM, dl=[(35.0, 106.18)], n_ltc=3))
    return Instance("7-site exciton K=28 N=8 binary R=16", H, baths, 8, "tree2", 16,
                    ground(M), 0.1 * FS_TO_CM, n_steps)


def structured_spin_boson_pade(n_steps=50, depth=25, rank=16, dt_fs=0.1):
    """The paper's complete-input-file example (Sec. III A 1, its Table and
    listing): a two-level system H_S = [[-750, 300], [300, 750]] cm^-1 coupled
    through Q = diag(-0.5, 0.5) to a Drude bath (lambda 540, cut-off 70 cm^-1)
    plus one Brownian mode (lambda 161.6, damped frequency w0' = 1243 and width
    10 cm^-1) at 300 K, Pade decomposition with one low-temperature term
    (4 features), depth 25, rho_S(0) = |1><1|.  Here on a tensor train of rank
    16 with RK4 steps of 0.1 fs (the listing's 1 fs suits an adaptive
    integrator; a fixed RK4 step needs dt below 0.15 fs at this hierarchy)."""
    eta, w0p = 10.0, 1243.0
    bath = Bath(np.diag([-0.5, 0.5]).astype(np.complex128), 300.0 * KB_CM,
                dl=[(540.0, 70.0)], bo=[(161.6, float(np.sqrt(w0p ** 2 + eta ** 2)), eta)],
                n_ltc=1, decomposition="pade")
    H = np.array([[-750.0, 300.0], [300.0, 750.0]], dtype=np.complex128)
    rho0 = np.zeros((2, 2), dtype=np.complex128)
    rho0[1, 1] = 1.0
    return Instance("structured spin-boson, Pade, K=4 N=25 train R=16", H, [bath], depth,
                    "train", rank, rho0, dt_fs * FS_TO_CM, n_steps)


def spin_boson_train_mix(n_steps=100, eps=1e-8, max_aux_rank=8):
    """The spin-boson train under the mixed strategy (Sec. VI, Sec. VII E):
    ps2 from rank 2 with eps 1e-8 until a bond reaches rank 8, then direct
    integration at the ranks reached (dopri5, ode_rtol 1e-5, ode_atol 1e-7,
    vmf_atol 1e-7), output every dt = 0.01."""
    base = spin_boson_train(n_steps)
    return Instance("spin-boson K=3 N=10 train, ps2 (eps 1e-8) then vmf at rank 8", base.H,
                    base.baths, base.depth, base.tree, max_aux_rank, base.rho0, base.dt, n_steps,
                    method="ps2", eps=eps)


class TfdInstance:
    """A thermofield ML-MCTDH problem: system H_S, coupling Q, one Brownian
    bath (lam, w0, eta) at T discretised into n_modes star modes on
    [-cutoff, cutoff], Fock dimension dim per mode, n-ary tree, rank, psi(0)."""

    def __init__(self, name, H, Q, lam, w0, eta, T, cutoff, n_modes, dim, n_ary, rank, psi0,
                 dt, n_steps):
        self.name = name
        self.H = np.asarray(H, dtype=np.complex128)
        self.Q = np.asarray(Q, dtype=np.complex128)
        self.lam, self.w0, self.eta, self.T = float(lam), float(w0), float(eta), float(T)
        self.cutoff = float(cutoff)
        self.n_modes, self.dim, self.n_ary, self.rank = int(n_modes), int(dim), int(n_ary), int(rank)
        self.psi0 = np.asarray(psi0, dtype=np.complex128)
        self.dt, self.n_steps = float(dt), int(n_steps)


def tfd_spin_boson(n_modes=50, dim=8, rank=16, n_steps=200, dt_fs=1.0):
    """The paper's MCTDH listing (Sec. III A 5): H_S = [[-750, 300], [300, 750]]
    cm^-1, Q = diag(-0.5, 0.5), one Brownian mode (reorganisation 200, width 10,
    damped frequency 50 cm^-1) at 300 K, cut-off 200 cm^-1, 50 modes of Fock
    dimension 8, psi(0) = |1>, 1 fs steps over 200 fs.  The listing gives no
    rank; a binary tree of rank 16 here."""
    eta, w0p = 10.0, 50.0
    return TfdInstance(f"thermofield spin-boson {n_modes} modes dim {dim} binary R={rank}",
                       [[-750.0, 300.0], [300.0, 750.0]], np.diag([-0.5, 0.5]), 200.0,
                       float(np.sqrt(w0p ** 2 + eta ** 2)), eta, 300.0 * KB_CM, 200.0, n_modes,
                       dim, 2, rank, [0.0, 1.0], dt_fs * FS_TO_CM, n_steps)


def stable_dt(dt_max, T, n_ltc, N, H, wc=1.0):
    """Time step of a batch instance: dt_max unless a half-step RK4 sub-flow
    would leave half of RK4's real stability interval (|z| < 2.785).

    The rate bound uses input parameters only.  Every feature's level is
    truncated on its own, so all of them can be excited at once and the
    hierarchy's decay rates add up: (N - 1) * sum_k |gamma_k|, with
    |gamma| = wc for the Drude feature and 2 pi m T for Matsubara feature m.
    The commutator with H_S adds at most 2 ||H_S||_2."""
    sum_gamma = wc + sum(2.0 * np.pi * m * T for m in range(1, n_ltc + 1))
    rate = (N - 1) * sum_gamma + 2.0 * float(np.linalg.norm(H, 2))
    return min(dt_max, 0.5 * 2.0 * 2.785 / rate)


def uneven_batch(n_inst=512, seed=2, n_steps=200):
    """Batch of uneven spin-boson-type instances (time step 0.01, lowered per
    instance where RK4 would be unstable, see stable_dt)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_inst):
        M = int(rng.integers(2, 9))
        K = int(rng.integers(2, 9))
        N = int(rng.integers(6, 13))
        R = int(rng.integers(8, 33))
        H = np.diag(rng.normal(size=M)).astype(np.complex128)
        for a in range(M):
            for b in range(a + 1, M):
                z = rng.normal() + 1j * rng.normal()
                H[a, b], H[b, a] = z, np.conj(z)
        q = rng.uniform(-1.0, 1.0, size=M)
        lam = float(np.exp(rng.uniform(np.log(0.01), np.log(1.0))))
        T = float(np.exp(rng.uniform(np.log(0.1), np.log(10.0))))
        bath = Bath(np.diag(q).astype(np.complex128), T, dl=[(lam, 1.0)], n_ltc=K - 1)
        out.append(Instance(f"batch[{i}] M={M} K={K} N={N} R={R}", H, [bath], N, "tree2",
                            R, ground(M), stable_dt(0.01, T, K - 1, N, H), n_steps))
    return out


def structured_bath_ternary(n_steps=100, seed=3, eps=1e-6, max_rank=64):
    """Two-level system, Drude + 10 Brownian modes + 3 Matsubara terms (24
    features), depth 10, ternary tree, adaptive rank (ps2)."""
    rng = np.random.default_rng(seed)
    bo = [(0.01, float(rng.uniform(0.5, 5.0)), float(rng.uniform(0.05, 0.5)))
          for _ in range(10)]
    bath = Bath(SZ, 1.0, dl=[(0.1, 1.0)], bo=bo, n_ltc=3)
    return Instance("structured bath K=24 N=10 ternary ps2", 0.5 * SZ + SX, [bath], 10,
                    "tree3", max_rank, ground(2), 0.01, n_steps, method="ps2", eps=eps)


def pulse_drives(seeds):
    """Gaussian pulses A exp(-(t-t0)^2/2s^2) cos(w t) sigma_x, one per seed."""
    out = []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        A = rng.uniform(0.0, 2.0)
        w = rng.uniform(0.5, 3.0)
        s = rng.uniform(1.0, 5.0)
        t0 = rng.uniform(5.0, 15.0)
        out.append((SX, A, w, s, t0))
    return out


def driven_spin_boson(seeds, n_steps=2000):
    """Driven spin-boson trajectories on the bath of spin_boson_train."""
    base = spin_boson_train(n_steps)
    return [Instance(f"driven seed {sd}", base.H, base.baths, base.depth, base.tree,
                     base.rank, base.rho0, base.dt, n_steps, drive=d)
            for sd, d in zip(seeds, pulse_drives(seeds))]


TRAIN_SEEDS = list(range(1000, 1000 + 3584))
VAL_SEEDS = list(range(4584, 5096))
HELDOUT_SEEDS = list(range(9000, 9256))
