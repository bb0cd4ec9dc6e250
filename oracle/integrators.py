"""Local integrator and the projector-splitting sweeps ps1 / ps2.

Paper Sec. II C (last two paragraphs): in both projector-splitting methods the
root tensor travels through a full traversal of the tree, moved to an adjacent
core by a factorisation at every sub-step, so that every core is propagated
while it is the root; ps1 keeps the ranks, ps2 merges neighbouring cores,
propagates the merged tensor and splits it by SVD (adaptive rank).  The paper
defers the detailed algorithm to its companion article; the readings below
follow the published projector-splitting integrators for tree tensor networks
(recursive subflows: QR into a child, integrate the child subtree, QR back,
evolve the bond matrix backward, absorb; then evolve the node forward) and
two-site TDVP generalised to trees.

Readings (documented):
* Local solver: one classical RK4 step per sub-flow over its whole interval;
  forward flows use +L_eff, backward (bond / ps2 node) flows use -L_eff.
* Second order: a first-order sweep over [t0, t0+dt/2] followed by its adjoint
  (the same sub-flows in reverse order) over [t0+dt/2, t0+dt].
* Gauge moves: Householder QR (LAPACK reflector convention) with the phases
  of diag(R) made non-negative; residual columns below 1e-10 of the matrix
  norm are treated as exact zeros, which fixes the orthonormal completion of
  rank-deficient cores (the truncated-rank result depends on it).  When a matricisation has fewer rows than the bond
  dimension the QR move lowers the bond dimension to the row count (exact).
* ps2 truncation: r_eps = the smallest r with sqrt(sum_{i>=r} s_i^2) <=
  eps * sqrt(sum s_i^2); keep r' = min(max_rank, available, r_eps + 1)
  directions (the extra direction is room for the rank to grow, in the
  spirit of TENSO's ps2_ratio that reincorporates part of the discarded
  spectrum).  ps2 starts from the padded initial state at rank 2: with
  rank-1 bonds every two-site tensor of a tree whose inner nodes carry no
  physical leg has a side of dimension 1 and no bond could ever grow.
  Alternative rule (Sec. VII E, ps2_atol and ps2_ratio): r_atol = the number
  of singular values above ps2_atol (at least 1), keep r' = min(max_rank,
  available, ceil(ps2_ratio * r_atol)): of the discarded spectrum, the
  directions just below the threshold are taken back in proportion to what
  was kept (reading: the paper says only that a fraction set by the ratio is
  reincorporated).
  Directions beyond the singular vectors with s_i > 1e-10 s_1 are completed
  by projecting e_0, e_1, ... onto the orthogonal complement of the kept
  singular subspace (deterministic, independent of the vectors' phases).

Pins (tests): at full rank both sweeps equal exact dense propagation up to the
RK4 error; results do not depend on the tree shape at full rank; ps2 with
eps = 0 and a large rank cap equals dense propagation.  At truncated rank,
a generator whose terms each act on one end keeps the exact solution
(x)_e exp(t A_e) Omega(0) at the ranks of Omega(0), and both sweeps
reproduce that closed form up to the RK4 error.  Truncated-rank
trajectories of coupled generators (the HEOM workloads) have no independent
pin ("parity unpinned" beyond the trend tests in rank and depth).
"""
import numpy as np

from .ttn import (Envs, apply_bond, apply_node, apply_two_site, merge,
                  mode_product, two_site_legs)


def rk4(F, y, t0, tau):
    """One classical RK4 step of dy/dt = F(t, y) over [t0, t0 + tau]."""
    k1 = F(t0, y)
    k2 = F(t0 + 0.5 * tau, y + 0.5 * tau * k1)
    k3 = F(t0 + 0.5 * tau, y + 0.5 * tau * k2)
    k4 = F(t0 + tau, y + tau * k3)
    return y + (tau / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)


QR_RANK_TOL = 1e-10
SVD_ZERO_TOL = 1e-10   # singular values below this fraction of the largest are zero
PS2_GROW = 1           # directions kept beyond the rank needed for eps (room to grow)
PS2_INIT_RANK = 2      # ps2 starts from the padded initial state at this rank


def householder_qr(A, tol=None):
    """Householder QR A = Q R (Q: m x k, R: k x n, k = min(m, n)) with LAPACK's
    reflector convention (zgeqr2 / zung2r: beta = -sign(Re alpha) * norm,
    tau = 0 when nothing is left to reflect).

    Rank-deficiency rule (reading): a column whose residual after the previous
    reflections has norm <= tol * ||A||_F is set to exactly zero and gets the
    identity reflector, so the orthonormal completion of a rank-deficient
    matrix is fixed by the well-determined columns alone rather than by
    rounding noise (projector splitting at truncated rank depends on it)."""
    if tol is None:
        tol = QR_RANK_TOL
    A = np.array(A, dtype=np.complex128)
    m, n = A.shape
    k = min(m, n)
    thr2 = (tol * np.linalg.norm(A)) ** 2
    taus = np.zeros(k, dtype=np.complex128)
    vs = []
    for j in range(k):
        x = A[j:, j]
        alpha = x[0]
        xn2 = float(np.sum(np.abs(x[1:]) ** 2))
        if abs(alpha) ** 2 + xn2 <= thr2:
            A[j:, j] = 0.0
            vs.append(np.zeros(m - j, dtype=np.complex128))
            continue
        if xn2 == 0.0 and alpha.imag == 0.0:
            vs.append(np.zeros(m - j, dtype=np.complex128))
            continue
        nrm = np.sqrt(abs(alpha) ** 2 + xn2)
        beta = -nrm if alpha.real >= 0.0 else nrm
        tau = complex((beta - alpha.real) / beta, -alpha.imag / beta)
        v = np.empty(m - j, dtype=np.complex128)
        v[0] = 1.0
        v[1:] = x[1:] / (alpha - beta)
        taus[j] = tau
        vs.append(v)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
        if j + 1 < n:
            w = v.conj() @ A[j:, j + 1:]
            A[j:, j + 1:] -= np.conj(tau) * np.outer(v, w)
    R = np.triu(A[:k, :])
    Q = np.zeros((m, k), dtype=np.complex128)
    Q[np.arange(k), np.arange(k)] = 1.0
    for j in reversed(range(k)):
        if taus[j] != 0:
            v = vs[j]
            w = v.conj() @ Q[j:, :]
            Q[j:, :] -= taus[j] * np.outer(v, w)
    return Q, R


def qr_toward(C, leg):
    """Factor C = Q x_leg R: C[.., a, ..] = sum_b Q[.., b, ..] R[b, a].

    Q is an isometry in `leg` (its rows along `leg` are orthonormal over the
    other legs).  Rows of the matricisation are the other legs in leg order;
    the phases of diag(R) are made non-negative (zero diagonals keep theirs)."""
    Cm = np.moveaxis(C, leg, -1)
    shp = Cm.shape
    mat = Cm.reshape(-1, shp[-1])
    Q, R = householder_qr(mat)
    d = np.diag(R).copy()
    ph = np.ones_like(d)
    nz = np.abs(d) > 0
    ph[nz] = d[nz] / np.abs(d[nz])
    Q = Q * ph[None, :]
    R = np.conj(ph)[:, None] * R
    k = Q.shape[1]
    Qc = np.moveaxis(Q.reshape(shp[:-1] + (k,)), -1, leg)
    return Qc, R


class Propagator:
    """ps1 / ps2 propagation of a TTN state (the paper's SparsePropagator)."""

    def __init__(self, tree, terms, cores, drive_fn=None, trunc=None):
        self.tree = tree
        self.terms = terms
        self.trunc = trunc        # None: the eps rule; (ps2_atol, ps2_ratio): the atol rule
        self.C = [c.copy() for c in cores]
        self.drive_fn = drive_fn
        self.envs = Envs(tree, terms)
        for s in reversed(range(tree.n)):  # canonical toward the root
            if s > 0:
                self.envs.update_down(s, self.C[s])

    def drive(self, t):
        return None if self.drive_fn is None else self.drive_fn(t)

    # -- flows ------------------------------------------------------------
    def _node(self, s, t0, tau, sign):
        self.C[s] = rk4(lambda t, y: sign * apply_node(self.envs, s, y, self.drive(t)),
                        self.C[s], t0, tau)

    def _bond_bwd(self, c, B, t0, tau):
        return rk4(lambda t, y: -apply_bond(self.envs, c, y, self.drive(t)), B, t0, tau)

    def _set_rank(self, c, r):
        self.tree.rank[c] = r

    # -- ps1 ----------------------------------------------------------------
    def _V(self, s, t0, tau):
        tr, C = self.tree, self.C
        for c in tr.children[s]:
            i = tr.leg_of_child(s, c)
            Q, R = qr_toward(C[s], i)          # move the center s -> c
            C[s], C[c] = Q, mode_product(C[c], R, 0)
            self._set_rank(c, Q.shape[i])
            self.envs.update_up(c, C[s])
            self._V(c, t0, tau)
            Q, R = qr_toward(C[c], 0)          # split the bond matrix off c
            C[c], B = Q, R.T
            self.envs.update_down(c, C[c])
            B = self._bond_bwd(c, B, t0, tau)
            C[s] = mode_product(C[s], B.T, i)  # absorb into s
        self._node(s, t0, tau, +1.0)

    def _Vstar(self, s, t0, tau):
        tr, C = self.tree, self.C
        self._node(s, t0, tau, +1.0)
        for c in reversed(tr.children[s]):
            i = tr.leg_of_child(s, c)
            Q, R = qr_toward(C[s], i)          # split the bond matrix off s
            C[s], B = Q, R
            self.envs.update_up(c, C[s])
            B = self._bond_bwd(c, B, t0, tau)
            C[c] = mode_product(C[c], B, 0)    # absorb into c
            self._Vstar(c, t0, tau)
            Q, R = qr_toward(C[c], 0)          # move the center c -> s
            C[c], C[s] = Q, mode_product(C[s], R, i)
            self.envs.update_down(c, C[c])

    def step_ps1(self, t0, dt):
        h = 0.5 * dt
        self._V(0, t0, h)
        self._Vstar(0, t0 + h, h)

    # -- ps2 ----------------------------------------------------------------
    @staticmethod
    def truncation_rank(s, eps, max_rank, avail, grow=PS2_GROW):
        """r_eps = smallest r with sqrt(sum_{i>=r} s_i^2) <= eps * sqrt(sum s_i^2);
        keep r' = min(max_rank, avail, r_eps + grow)."""
        s = np.asarray(s, dtype=np.float64)
        tot2 = float(np.sum(s * s))
        n = len(s)
        r_eps = n
        tail2 = tot2
        for k in range(0, n + 1):
            tail2 = float(np.sum(s[k:] * s[k:]))
            if tail2 <= eps * eps * tot2:
                r_eps = k
                break
        r_eps = max(1, r_eps)
        return max(1, min(max_rank, avail, r_eps + grow))

    @staticmethod
    def truncation_rank_atol(s, atol, ratio, max_rank, avail):
        """r_atol = #(s_i > atol), at least 1; keep r' = min(max_rank, avail,
        ceil(ratio * r_atol))."""
        r_atol = max(1, int(np.sum(np.asarray(s) > atol)))
        return max(1, min(max_rank, avail, int(np.ceil(ratio * r_atol))))

    @staticmethod
    def complete_isometry(U, r):
        """Columns U (n x k, orthonormal) completed to n x r: the unit vectors
        e_0, e_1, ... are projected onto the orthogonal complement of span(U)
        and orthonormalised in order (twice-repeated Gram-Schmidt), skipping
        residuals with norm below 0.5.  Depends on span(U) only."""
        n, k = U.shape
        Q = [U[:, j] for j in range(k)]
        j = 0
        while len(Q) < r and j < n:
            v = np.zeros(n, dtype=np.complex128)
            v[j] = 1.0
            for _ in range(2):
                for q in Q:
                    v = v - q * np.vdot(q, v)
            nv = np.linalg.norm(v)
            if nv > 0.5:
                Q.append(v / nv)
            j += 1
        return np.stack(Q, axis=1)

    def _edge(self, s, c, t0, tau, eps, max_rank, center_to_child):
        tr, C = self.tree, self.C
        i = tr.leg_of_child(s, c)
        Th = merge(tr, C, s, c)
        Th = rk4(lambda t, y: apply_two_site(self.envs, s, c, y, self.drive(t)),
                 Th, t0, tau)
        ns = len(tr.legs[s]) - 1
        shp = Th.shape
        rows = int(np.prod(shp[:ns]))
        mat = Th.reshape(rows, -1)
        U, S, Vh = np.linalg.svd(mat, full_matrices=False)
        if self.trunc is not None:
            r = self.truncation_rank_atol(S, self.trunc[0], self.trunc[1], max_rank, min(mat.shape))
        else:
            r = self.truncation_rank(S, eps, max_rank, min(mat.shape))
        k = int(np.sum(S > SVD_ZERO_TOL * S[0])) if S[0] > 0 else 0
        k = min(k, r)
        if center_to_child:
            Cs = self.complete_isometry(U[:, :k], r)      # rows x r isometry
            Cc = Cs.conj().T @ mat                          # projection
        else:
            W = self.complete_isometry(Vh[:k].conj().T, r)  # cols x r isometry
            Cc = W.conj().T
            Cs = mat @ W
        C[s] = np.moveaxis(Cs.reshape(shp[:ns] + (r,)), -1, i)
        C[c] = Cc.reshape((r,) + shp[ns:])
        self._set_rank(c, r)
        self.rank_log.append(r)

    def _W(self, s, t0, tau, eps, max_rank):
        tr, C = self.tree, self.C
        kids = tr.children[s]
        for idx, c in enumerate(kids):
            i = tr.leg_of_child(s, c)
            self._edge(s, c, t0, tau, eps, max_rank, center_to_child=True)
            self.envs.update_up(c, C[s])
            if tr.children[c]:
                self._node(c, t0, tau, -1.0)
                self._W(c, t0, tau, eps, max_rank)
            Q, R = qr_toward(C[c], 0)
            C[c], C[s] = Q, mode_product(C[s], R, i)
            self._set_rank(c, Q.shape[0])
            self.envs.update_down(c, C[c])
            if idx < len(kids) - 1:
                self._node(s, t0, tau, -1.0)

    def _Wstar(self, s, t0, tau, eps, max_rank):
        tr, C = self.tree, self.C
        kids = tr.children[s]
        for idx in reversed(range(len(kids))):
            c = kids[idx]
            i = tr.leg_of_child(s, c)
            if idx < len(kids) - 1:
                self._node(s, t0, tau, -1.0)
            Q, R = qr_toward(C[s], i)
            C[s], C[c] = Q, mode_product(C[c], R, 0)
            self._set_rank(c, Q.shape[i])
            self.envs.update_up(c, C[s])
            if tr.children[c]:
                self._Wstar(c, t0, tau, eps, max_rank)
                self._node(c, t0, tau, -1.0)
            self._edge(s, c, t0, tau, eps, max_rank, center_to_child=False)
            self.envs.update_down(c, C[c])

    def step_ps2(self, t0, dt, eps, max_rank):
        self.rank_log = []
        h = 0.5 * dt
        self._W(0, t0, h, eps, max_rank)
        self._Wstar(0, t0 + h, h, eps, max_rank)
        return list(self.rank_log)

    def rho(self):
        from .ttn import reduced_rho
        return reduced_rho(self.tree, self.C)
