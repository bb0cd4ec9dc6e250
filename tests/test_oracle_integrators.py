"""Pins of the oracle's ps1 / ps2 sweeps (Sec. II C, projector splitting).

* full rank: both sweeps reproduce exact dense propagation up to RK4 error,
  for a train, a binary and a ternary tree (the tree shape does not matter);
* ps2 with eps = 0 and a large rank cap equals dense propagation;
* truncated rank converges to the dense result as the rank grows;
* gauge covariance: random unitaries inserted on saturated bonds leave the
  trajectory unchanged;
* a time-dependent drive with zero bath coupling matches the 2x2 von Neumann
  equation integrated to tight tolerance."""
import copy

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle.bath import bath_features
from oracle.integrators import Propagator
from oracle.sop import dense_propagate, heom_terms
from oracle.ttn import Tree, initial_state, mode_product, nary_tree, trace_distance, train_tree

SZ = np.diag([1.0, -1.0]).astype(complex)
SX = np.array([[0, 1], [1, 0]], complex)
RHO0 = np.array([[1, 0], [0, 0]], complex)


def spin_boson(N, n_ltc=2, lam=0.1):
    c, cb, g = bath_features(1.0, dl=[(lam, 1.0)], n_ltc=n_ltc)
    return heom_terms(0.5 * SZ + SX, [(SZ, (c, cb, g))], N)


def run_ps1(tree, terms, n, dt=0.01):
    P = Propagator(tree, terms, initial_state(tree, RHO0))
    for s in range(n):
        P.step_ps1(s * dt, dt)
    return P


@pytest.mark.parametrize("mk", [lambda: train_tree(2, [5] * 3, 100),
                                lambda: nary_tree(2, [5] * 3, 2, 100),
                                lambda: nary_tree(2, [3] * 4, 3, 100)])
def test_ps1_full_rank_equals_dense(mk):
    tree = mk()
    terms, dims = spin_boson(tree.end_dims[2], n_ltc=len(tree.end_dims) - 3)
    n = 60
    ref = dense_propagate(terms, dims, RHO0, 0.01, n, every=n)[-1]
    P = run_ps1(tree, terms, n)
    assert trace_distance(P.rho(), ref) < 1e-8


def test_ps2_eps0_equals_dense():
    terms, dims = spin_boson(5)
    n = 50
    ref = dense_propagate(terms, dims, RHO0, 0.01, n, every=n)[-1]
    base = nary_tree(2, [5] * 3, 2, 1)
    tree = Tree(base.parent, base.end_node, base.end_dims, max_rank=2)
    P = Propagator(tree, terms, initial_state(tree, RHO0))
    for s in range(n):
        ranks = P.step_ps2(s * 0.01, 0.01, 0.0, 1000)
    assert trace_distance(P.rho(), ref) < 1e-8
    assert max(ranks) > 1


def test_rank_convergence_trend():
    terms, dims = spin_boson(6)
    n = 60
    ref = dense_propagate(terms, dims, RHO0, 0.01, n, every=n)[-1]
    errs = [trace_distance(run_ps1(train_tree(2, [6] * 3, R), terms, n).rho(), ref)
            for R in (2, 4, 8)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-6


def test_gauge_covariance_at_saturated_rank():
    terms, dims = spin_boson(6)
    tr = train_tree(2, [6] * 3, 3)
    P = run_ps1(tr, terms, 30)
    P2 = Propagator(copy.deepcopy(tr), terms, P.C)
    rng = np.random.default_rng(1)
    for c in range(1, tr.n):
        r = tr.rank[c]
        W, _ = np.linalg.qr(rng.normal(size=(r, r)) + 1j * rng.normal(size=(r, r)))
        p, i = tr.parent[c], tr.leg_of_child(tr.parent[c], c)
        P2.C[p] = mode_product(P2.C[p], W.T, i)
        P2.C[c] = mode_product(P2.C[c], W.conj().T, 0)
    P2 = Propagator(P2.tree, terms, P2.C)
    for s in range(30, 50):
        P.step_ps1(s * 0.01, 0.01)
        P2.step_ps1(s * 0.01, 0.01)
    assert trace_distance(P.rho(), P2.rho()) < 1e-12


def test_drive_zero_coupling_matches_von_neumann():
    """With a time-dependent generator the backward sub-flows (time running
    forward with -L_eff) do not invert the forward ones exactly, so the sweep
    is second order in dt rather than exact at full rank: check the error is
    small and falls ~4x when dt halves."""
    c, cb, g = bath_features(1.0, dl=[(0.0, 1.0)], n_ltc=1)
    H = 0.5 * SZ
    f = lambda t: 1.5 * np.exp(-0.5 * ((t - 0.5) / 0.3) ** 2) * np.cos(1.0 * t)
    terms, dims = heom_terms(H, [(SZ, (c, cb, g))], 2, drives=[(0, SX)])

    def rhs(t, y):
        r = y.reshape(2, 2)
        Ht = H + f(t) * SX
        return (-1j * (Ht @ r - r @ Ht)).reshape(-1)
    sol = solve_ivp(rhs, (0, 1.0), RHO0.reshape(-1).astype(complex), method="DOP853",
                    rtol=1e-12, atol=1e-14)
    ref = sol.y[:, -1].reshape(2, 2)
    errs = []
    for n in (50, 100):
        dt = 1.0 / n
        tree = train_tree(2, [2, 2], 4)
        P = Propagator(tree, terms, initial_state(tree, RHO0),
                       drive_fn=lambda t: np.array([f(t)]))
        for s in range(n):
            P.step_ps1(s * dt, dt)
        errs.append(trace_distance(P.rho(), ref))
    assert errs[1] < 1e-5
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_depth_convergence_trend():
    """A too-shallow hierarchy misses bath memory: with the dense generator
    (no tree truncation) the distance to a deep reference falls with depth."""
    n = 150
    ref_terms, ref_dims = spin_boson(12)
    ref = dense_propagate(ref_terms, ref_dims, RHO0, 0.02, n, every=n)[-1]
    errs = []
    for depth in (2, 4, 7):
        terms, dims = spin_boson(depth)
        errs.append(trace_distance(dense_propagate(terms, dims, RHO0, 0.02, n, every=n)[-1], ref))
    assert errs[0] > errs[1] > errs[2]

