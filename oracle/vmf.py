"""Direct integration (the paper's vmf), its ODE solver and the mixed strategy.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline call this module; the product path never does.

Paper Sec. II C: the direct strategy integrates the coupled equations of
motion of every core at once with a standard ODE solver at fixed rank; the
equations of the non-root cores contain the inverse of a matrix that is
singular early on, so it is regularised.  Sec. VII E: the solver is dopri5
with relative and absolute tolerances (ode_rtol, ode_atol), and the
regularisation (vmf_atol) is a constant added to the diagonal of that matrix.
Sec. VI and VII E: the mixed strategy runs an auxiliary method (ps2 by default)
until a bond rank reaches max_auxiliary_rank and then the main method (vmf) at
the ranks ps2 left.

The paper defers the equations themselves to its companion article; they are
the time-dependent variational principle for dOmega/dt = L Omega on the tree
(Sec. II C), written here from the McLachlan form of that principle: the time
derivative of the network is the orthogonal projection of L Omega onto the
tangent space at the current cores, in the gauge where every non-root core U_s
stays an isometry toward its parent and its derivative is orthogonal to it
(U_s^H dU_s = 0).  With B_s the rest of the network seen through the bond above
s (Omega = U_s B_s over that bond):

* root:      dA_0/dt = sum_m c_m(t) (x)_l X_{m,l} A_0, the down environments of
             its children and the end factors on its legs (as in ps1);
* non-root:  dU_s/dt = (1 - P_s) [ sum_m c_m(t) (x)_l X_{m,l} U_s ] on the
             parent leg followed by (rho_s + vmf_atol I)^-1, with
             P_s the projector onto the span of U_s (over its non-parent legs),
             rho_s[a', a] = sum_y conj(B_s[a', y]) B_s[a, y] (the density
             matrix on the bond, operand convention: it acts on the parent
             leg like every other leg operator), and on the parent leg the
             mean field of term m, G_{m,s}[a', a] = sum_y conj(B_s[a', y])
             (L_m^out B_s)[a, y] of the part of term m outside the subtree of
             s; a term with no factor outside the subtree has G = rho_s.

Readings (documented):
* Regularisation: the diagonal shift rho_s + vmf_atol I (the paper names the
  shift; TENSO's other regularisation types are not described and not built).
  Default vmf_atol 1e-7 is a reading: the paper's listings do not print it.
* dopri5: the Dormand-Prince 5(4) pair, advancing with the fifth-order
  solution (local extrapolation) and reusing the last stage as the next step's
  first (FSAL).  Error norm: the root mean square over every complex core
  entry of |err| / (ode_atol + ode_rtol max(|y_old|, |y_new|)).  A step is
  accepted when that norm is at most 1; the next step size is h times
  0.9 norm^(-1/5) clipped to [0.2, 10] (10 when the norm is zero).  Each
  output interval dt is covered by substeps, the last shortened to end on it
  (after which the proposed size stays as it was unless that substep's own
  proposal is larger); the first substep of a run tries dt.  With fixed_substeps = n the interval
  is covered by n equal dopri5 steps without error control instead.
* Mixed: after every ps2 step the largest bond rank is compared with
  max_auxiliary_rank; once it is reached, every later step is vmf at the
  current ranks.  The ps2 truncation is the eps rule of the ps2 oracle.

Pins (tests, oracle/ against the mathematics): the dopri5 tableau satisfies the
order conditions up to order 5 (4 for the embedded pair), integrates
quadrature problems with quartic integrands exactly and shows fifth-order
convergence on a linear system against its matrix exponential; at full rank
the vmf tangent vector (every derivative contracted back into the network)
equals L Omega exactly, for random states on every tree shape; at truncated
rank the residual L Omega - dOmega is orthogonal to every tangent direction
and the gauge condition holds; vmf at full rank reproduces dense propagation.
"""
import numpy as np

from .ttn import Envs, apply_node, mode_product

VMF_ATOL = 1e-7
ODE_RTOL = 1e-5
ODE_ATOL = 1e-7

# Dormand-Prince 5(4): nodes, stage weights, fifth- and fourth-order weights
DP_C = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])
DP_A = [
    [],
    [1 / 5],
    [3 / 40, 9 / 40],
    [44 / 45, -56 / 15, 32 / 9],
    [19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729],
    [9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656],
    [35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84],
]
DP_B = np.array([35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0])
DP_BS = np.array([5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100,
                  1 / 40])


def _sandwich(C, open_leg, ops):
    """sum over every leg of C but open_leg of conj(C) ((x) ops C): the
    operand-convention matrix S[a', a] on the open leg."""
    T = C
    for leg, X in ops:
        T = mode_product(T, X, leg)
    Cm = np.moveaxis(C, open_leg, 0).reshape(C.shape[open_leg], -1)
    Tm = np.moveaxis(T, open_leg, 0).reshape(T.shape[open_leg], -1)
    return Cm.conj() @ Tm.T


def mean_fields(tree, terms, cores):
    """Down environments (children first), then top-down the bond densities
    rho_s and the mean fields G_{m,s} (parents first).  Returns (envs, rho)
    where envs.up[s][m] holds G_{m,s} (rho_s for terms with no factor outside
    the subtree of s)."""
    envs = Envs(tree, terms)
    for x in reversed(range(1, tree.n)):
        envs.update_down(x, cores[x])
    rho = [None] * tree.n
    for x in range(1, tree.n):
        p = tree.parent[x]
        open_leg = tree.leg_of_child(p, x)
        rho[x] = _sandwich(cores[p], open_leg, [] if p == 0 else [(0, rho[p])])
        for m, term in enumerate(terms):
            if set(term['factors']) <= tree.sub_ends[x]:
                envs.up[x][m] = rho[x]
                continue
            ops = []
            for i, leg in enumerate(tree.legs[p]):
                if i == open_leg:
                    continue
                X = envs.leg_op(p, leg, m)   # parent leg: G_{m,p} (never None below the root)
                if X is not None:
                    ops.append((i, X))
            envs.up[x][m] = _sandwich(cores[p], open_leg, ops)
    return envs, rho


def vmf_derivative(tree, terms, cores, drive, reg=VMF_ATOL):
    """Time derivative of every core (list in node order)."""
    envs, rho = mean_fields(tree, terms, cores)
    out = [apply_node(envs, 0, cores[0], drive)]
    for s in range(1, tree.n):
        T = apply_node(envs, s, cores[s], drive)
        r = rho[s].shape[0]
        T = mode_product(T, np.linalg.inv(rho[s] + reg * np.eye(r)), 0)
        U = cores[s]
        Um = U.reshape(r, -1)
        Tm = T.reshape(r, -1)
        S = Um.conj() @ Tm.T                 # S[a', a] = sum_beta conj(U[a', beta]) T[a, beta]
        Tm = Tm - S.T @ Um                   # T[a, beta] -= sum_a' S[a', a] U[a', beta]
        out.append(Tm.reshape(U.shape))
    return out


def tangent_dense(tree, cores, derivs):
    """d/dt of the contracted network for the given core derivatives
    (product rule: one core replaced at a time)."""
    from .ttn import contract_dense
    total = None
    for s in range(tree.n):
        cs = list(cores)
        cs[s] = derivs[s]
        d = contract_dense(tree, cs)
        total = d if total is None else total + d
    return total


# --------------------------------------------------------------------------
# dopri5
# --------------------------------------------------------------------------

def _lin(y, h, ks, coefs):
    out = [c.copy() for c in y]
    for k, a in zip(ks, coefs):
        if a != 0.0:
            for i in range(len(out)):
                out[i] = out[i] + (h * a) * k[i]
    return out


def error_norm(err, y0, y1, rtol, atol):
    """RMS over every complex entry of |err| / (atol + rtol max(|y0|, |y1|))."""
    num, cnt = 0.0, 0
    for e, a, b in zip(err, y0, y1):
        sc = atol + rtol * np.maximum(np.abs(a), np.abs(b))
        num += float(np.sum((np.abs(e) / sc) ** 2))
        cnt += e.size
    return np.sqrt(num / max(cnt, 1))


def dopri5_step(f, t, y, h, k1):
    """One Dormand-Prince step: (y_new, err, k7) with err = y5 - y4."""
    ks = [k1]
    for i in range(1, 7):
        yi = _lin(y, h, ks, DP_A[i])
        ks.append(f(t + DP_C[i] * h, yi))
    y1 = _lin(y, h, ks, DP_B)
    err = _lin([np.zeros_like(c) for c in y], h, ks, DP_B - DP_BS)
    return y1, err, ks[6]


class Dopri5:
    """dopri5 over a list of arrays, with the step control of the readings."""

    def __init__(self, f, rtol=ODE_RTOL, atol=ODE_ATOL, fixed_substeps=0):
        self.f = f
        self.rtol, self.atol = rtol, atol
        self.fixed = int(fixed_substeps)
        self.h = None
        self.k1 = None        # FSAL stage at the current point (None: recompute)
        self.accepted = 0
        self.rejected = 0

    def advance(self, t0, y, dt):
        t_end = t0 + dt
        if self.fixed > 0:
            h = dt / self.fixed
            t = t0
            for j in range(self.fixed):
                k1 = self.f(t, y) if self.k1 is None else self.k1
                y, _, self.k1 = dopri5_step(self.f, t, y, h, k1)
                t = t0 + (j + 1) * h
                self.accepted += 1
            return y
        if self.h is None:
            self.h = dt
        t = t0
        while t < t_end:
            h = min(self.h, t_end - t)
            if h <= 1e-14 * abs(dt):
                raise FloatingPointError("dopri5 step size underflow")
            last = t + h >= t_end
            k1 = self.f(t, y) if self.k1 is None else self.k1
            y1, err, k7 = dopri5_step(self.f, t, y, h, k1)
            en = error_norm(err, y, y1, self.rtol, self.atol)
            fac = 10.0 if en == 0.0 else min(10.0, max(0.2, 0.9 * en ** (-0.2)))
            if en <= 1.0:
                t = t_end if last else t + h
                y, self.k1 = y1, k7
                self.accepted += 1
                # a substep shortened to end on the output time keeps the
                # proposed size unless its own proposal is larger
                self.h = h * fac if h >= self.h else max(self.h, h * fac)
            else:
                self.rejected += 1
                self.k1 = k1
                self.h = h * fac
        return y


class VmfPropagator:
    """Fixed-rank direct integration of a root-canonical TTN state."""

    def __init__(self, tree, terms, cores, drive_fn=None, reg=VMF_ATOL, rtol=ODE_RTOL,
                 atol=ODE_ATOL, fixed_substeps=0):
        self.tree, self.terms = tree, terms
        self.C = [c.copy() for c in cores]
        self.drive_fn = drive_fn
        self.reg = reg
        self.ode = Dopri5(self._f, rtol, atol, fixed_substeps)

    def _f(self, t, y):
        drive = None if self.drive_fn is None else self.drive_fn(t)
        return vmf_derivative(self.tree, self.terms, y, drive, self.reg)

    def step(self, t0, dt):
        self.C = self.ode.advance(t0, self.C, dt)

    def rho(self):
        from .ttn import reduced_rho
        return reduced_rho(self.tree, self.C)


def propagate_mix(tree, terms, cores, dt, n_steps, eps, max_aux_rank, drive_fn=None,
                  reg=VMF_ATOL, rtol=ODE_RTOL, atol=ODE_ATOL, fixed_substeps=0, every=1,
                  trunc=None):
    """Mixed strategy: ps2 (eps rule, rank cap max_aux_rank) until a bond rank
    reaches max_aux_rank, then vmf at the ranks reached.  Returns (steps,
    rho records, index of the first vmf step or n_steps, propagator).  trunc:
    (ps2_atol, ps2_ratio) for the atol truncation rule of ps2, None for eps."""
    from .integrators import Propagator
    from .ttn import reduced_rho
    P = Propagator(tree, terms, cores, drive_fn=drive_fn, trunc=trunc)
    V = None
    switch = n_steps
    rhos, steps = [P.rho()], [0]
    for s in range(n_steps):
        t0 = s * dt
        if V is None:
            P.step_ps2(t0, dt, eps, max_aux_rank)
            if max(tree.rank[1:], default=0) >= max_aux_rank:
                switch = s + 1
                V = VmfPropagator(tree, terms, P.C, drive_fn, reg, rtol, atol, fixed_substeps)
        else:
            V.step(t0, dt)
        if (s + 1) % every == 0 or s + 1 == n_steps:
            rhos.append(reduced_rho(tree, P.C if V is None else V.C))
            steps.append(s + 1)
    return np.array(steps), np.array(rhos), switch, (P if V is None else V)
