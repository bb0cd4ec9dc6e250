"""Pins of the oracle's ps1 / ps2 sweeps (Sec. II C, projector splitting).

* full rank: both sweeps reproduce exact dense propagation up to RK4 error,
  for a train, a binary and a ternary tree (the tree shape does not matter);
* ps2 with eps = 0 and a large rank cap equals dense propagation;
* truncated rank converges to the dense result as the rank grows;
* gauge covariance: random unitaries inserted on saturated bonds leave the
  trajectory unchanged;
* a time-dependent drive with zero bath coupling matches the 2x2 von Neumann
  equation integrated to tight tolerance;
* truncated rank, exactness on the manifold: a generator whose terms each act
  on one end only keeps the exact solution (x)_e exp(t A_e) Omega(0) at the
  TTN ranks of Omega(0), so the tangent projection drops nothing and both
  sweeps reproduce it at truncated rank up to RK4 error (a two-end term
  breaks this, which shows the ranks really truncate).  A wrong sign of the
  backward bond flow, or a skipped one, fails it by O(1)."""
import copy

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.linalg import expm

from oracle.bath import bath_features
from oracle.integrators import Propagator
from oracle.sop import dense_generator, dense_propagate, heom_terms
from oracle.ttn import (Tree, contract_dense, initial_state, mode_product, nary_tree, trace_distance,
                        train_tree)
from tests.oracle_helpers import canonicalize_root, rand_cores

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



def single_leg_terms(end_dims, rng, per_end=2):
    """Random terms, each with one non-identity factor."""
    terms = []
    for e, d in enumerate(end_dims):
        for _ in range(per_end):
            X = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / np.sqrt(d)
            terms.append({'coef': 0.5 * (rng.normal() + 1j * rng.normal()), 'slot': -1,
                          'factors': {e: X}})
    return terms


def closed_form_single_leg(end_dims, terms, om0, t):
    """Omega(t) = (x)_e exp(t A_e) Omega(0), A_e the sum of the terms on end e."""
    om = om0.copy()
    for e, d in enumerate(end_dims):
        A = np.zeros((d, d), complex)
        for term in terms:
            if e in term['factors']:
                A += term['coef'] * term['factors'][e]
        om = np.moveaxis(np.tensordot(expm(t * A), om, axes=([1], [e])), 0, e)
    return om


def random_canonical_state(tree, rng):
    C = rand_cores(tree, rng)
    canonicalize_root(tree, C)
    C[0] = C[0] / np.linalg.norm(contract_dense(tree, C))
    return C


TRUNC_TREES = [("train", lambda: train_tree(2, [3, 3, 3], 2)),
               ("binary", lambda: nary_tree(2, [3, 3, 3, 3], 2, 2)),
               ("ternary", lambda: nary_tree(2, [3, 3, 3, 3], 3, 2))]


@pytest.mark.parametrize("method", ["ps1", "ps2"])
@pytest.mark.parametrize("name,mk", TRUNC_TREES)
def test_truncated_rank_exact_for_single_leg_generators(name, mk, method):
    rng = np.random.default_rng(21)
    tree = mk()
    full = nary_tree(2, [3] * (len(tree.end_dims) - 2), 2, 10 ** 6)
    assert max(tree.rank) == 2 and max(full.rank) > 2
    C = random_canonical_state(tree, rng)
    terms = single_leg_terms(tree.end_dims, rng)
    dt, n = 0.005, 40
    ref = closed_form_single_leg(tree.end_dims, terms, contract_dense(tree, C), n * dt)
    P = Propagator(tree, terms, C)
    for s in range(n):
        if method == "ps1":
            P.step_ps1(s * dt, dt)
        else:
            P.step_ps2(s * dt, dt, 1e-12, 2)
    assert max(tree.rank) == 2
    err = np.linalg.norm(contract_dense(tree, P.C) - ref) / np.linalg.norm(ref)
    assert err < 1e-8, err


def test_truncated_rank_two_end_term_leaves_the_manifold():
    """The control for the test above: one term coupling two ends makes the
    rank-2 trajectory depart from the dense one by O(0.1)."""
    rng = np.random.default_rng(21)
    tree = nary_tree(2, [3, 3, 3, 3], 2, 2)
    C = random_canonical_state(tree, rng)
    terms = single_leg_terms(tree.end_dims, rng)
    d0, d5 = tree.end_dims[0], tree.end_dims[5]
    terms.append({'coef': 0.3, 'slot': -1,
                  'factors': {0: rng.normal(size=(d0, d0)) + 0j, 5: rng.normal(size=(d5, d5)) + 0j}})
    dt, n = 0.005, 40
    om0 = contract_dense(tree, C)
    ref = expm(n * dt * dense_generator(terms, tree.end_dims).toarray()) @ om0.reshape(-1)
    P = Propagator(tree, terms, C)
    for s in range(n):
        P.step_ps1(s * dt, dt)
    err = np.linalg.norm(contract_dense(tree, P.C).reshape(-1) - ref) / np.linalg.norm(ref)
    assert err > 1e-3, err


def test_ps2_atol_rule_counts():
    """The absolute-threshold ps2 rule (Sec. VII E: ps2_atol, ps2_ratio) on
    spectra with a known count above the threshold."""
    tr = Propagator.truncation_rank_atol
    s = [1.0, 0.1, 1e-3, 1e-8, 1e-9]
    assert tr(s, 1e-7, 1.0, 64, 5) == 3
    assert tr(s, 1e-7, 2.0, 64, 5) == 5          # 6 wanted, 5 available
    assert tr(s, 1e-7, 2.0, 4, 5) == 4           # rank cap
    assert tr(s, 1e-7, 1.5, 64, 5) == 5          # ceil(4.5)
    assert tr(s, 1e-2, 2.0, 64, 5) == 4
    assert tr(s, 10.0, 2.0, 64, 5) == 2          # nothing above: r_atol counts as 1
    assert tr([0.0, 0.0], 0.0, 1.0, 64, 2) == 1


def test_ps2_atol_rule_limits():
    """atol = 0 with ratio 1 keeps every non-zero direction (dense result);
    raising atol lowers the ranks and moves the result away from it."""
    terms, dims = spin_boson(5)
    n = 40
    ref = dense_propagate(terms, dims, RHO0, 0.01, n, every=n)[-1]
    base = nary_tree(2, [5] * 3, 2, 1)
    errs, top = [], []
    for atol in (0.0, 1e-6, 1e-3):
        tree = Tree(base.parent, base.end_node, base.end_dims, max_rank=2)
        P = Propagator(tree, terms, initial_state(tree, RHO0), trunc=(atol, 1.0))
        for s in range(n):
            ranks = P.step_ps2(s * 0.01, 0.01, 0.0, 1000)
        errs.append(trace_distance(P.rho(), ref))
        top.append(max(ranks))
    assert errs[0] < 1e-8
    assert top[0] >= top[1] >= top[2] and top[0] > top[2]
    assert errs[2] > errs[0]
