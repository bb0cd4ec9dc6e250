"""Pins of the direct-integration oracle (Sec. II C: vmf; Sec. VII E: dopri5,
the diagonal regularisation; Sec. VI: the mixed strategy).

* dopri5 tableau: consistency (row sums = nodes), the quadrature order
  conditions (order 5 for the propagating weights, 4 for the embedded ones) and
  the two-stage ones; a nonlinear problem with a closed-form solution shows
  fifth-order convergence of the propagating solution and fourth-order of the
  embedded one (a wrong coefficient anywhere drops an order);
* adaptive control: a linear system integrated with tolerances 1e-9 lands
  within a few tolerances of its matrix exponential;
* vmf tangent vector at full rank (random well-conditioned states, no
  regularisation): sum over cores of the contracted derivatives = L Omega
  exactly, for a train, a binary and a ternary tree;
* at truncated rank: the gauge condition U^H dU = 0 holds and the residual
  L Omega - dOmega is orthogonal to every tangent direction (McLachlan);
* vmf at full rank with dopri5 reproduces dense propagation;
* mixed strategy: it switches at the first ps2 step whose largest rank reaches
  the cap, the ranks are frozen afterwards, and the pre-switch steps equal
  plain ps2."""
import copy

import numpy as np
import pytest
from scipy.linalg import expm

from oracle.bath import bath_features
from oracle.integrators import Propagator
from oracle.sop import dense_generator, dense_rho, heom_terms
from oracle.ttn import contract_dense, initial_state, nary_tree, reduced_rho, train_tree
from oracle.ttn import trace_distance
from oracle.vmf import (DP_A, DP_B, DP_BS, DP_C, Dopri5, VmfPropagator, dopri5_step,
                        propagate_mix, tangent_dense, vmf_derivative)
from tests.oracle_helpers import canonicalize_root, rand_cores

SZ = np.diag([1.0, -1.0]).astype(complex)
SX = np.array([[0, 1], [1, 0]], complex)
RHO0 = np.array([[1, 0], [0, 0]], complex)


def spin_boson(N, n_ltc=2, lam=0.1):
    c, cb, g = bath_features(1.0, dl=[(lam, 1.0)], n_ltc=n_ltc)
    return heom_terms(0.5 * SZ + SX, [(SZ, (c, cb, g))], N)


def _A():
    A = np.zeros((7, 7))
    for i in range(7):
        A[i, :len(DP_A[i])] = DP_A[i]
    return A


def test_tableau_order_conditions():
    A, c = _A(), DP_C
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)
    for k in range(5):
        assert abs(DP_B @ c ** k - 1.0 / (k + 1)) < 1e-14, k
    for k in range(4):
        assert abs(DP_BS @ c ** k - 1.0 / (k + 1)) < 1e-14, k
    assert abs(DP_BS @ c ** 4 - 1.0 / 5) > 1e-6        # the embedded pair is only fourth order
    for b, top in ((DP_B, 5), (DP_BS, 4)):
        assert abs(b @ (A @ c) - 1 / 6) < 1e-14
        assert abs(b @ (A @ (A @ c)) - 1 / 24) < 1e-14
        assert abs(b @ (c * (A @ c)) - 1 / 8) < 1e-14
        assert abs(b @ (A @ c ** 2) - 1 / 12) < 1e-14
    # FSAL: the last stage is taken at the fifth-order solution
    assert np.allclose(A[6], DP_B, atol=0)


def test_tableau_matches_scipy_rk45():
    """scipy's RK45 is the same Dormand-Prince pair (its error weights are
    ours with the opposite sign)."""
    from scipy.integrate._ivp.rk import RK45
    A = _A()
    assert np.array_equal(RK45.C, DP_C[:6])
    assert np.array_equal(RK45.A, A[:6, :5])
    assert np.array_equal(RK45.B, DP_B[:6])
    assert np.allclose(RK45.E, -(DP_B - DP_BS), atol=1e-16)


def test_regularised_derivative_at_the_singular_initial_state():
    """The product initial state has rank-1 bond densities: the shift keeps
    the derivative finite and the gauge condition exact."""
    tree = nary_tree(2, [4] * 4, 2, 3)
    terms, _ = spin_boson(4, n_ltc=3)
    C = initial_state(tree, RHO0)
    d = vmf_derivative(tree, terms, C, None, reg=1e-7)
    assert all(np.all(np.isfinite(x)) for x in d)
    for s in range(1, tree.n):
        r = tree.rank[s]
        Um, dm = C[s].reshape(r, -1), d[s].reshape(r, -1)
        assert np.abs(Um.conj() @ dm.T).max() < 1e-8 * max(1.0, np.abs(dm).max())


def _solve(f, y0, t1, n):
    """n fixed dopri5 steps of size t1 / n from t = 0."""
    y, t, h = [np.array(y0[0], dtype=complex)], 0.0, t1 / n
    for _ in range(n):
        y, _, _ = dopri5_step(f, t, y, h, f(t, y))
        t += h
    return y[0]


def test_fifth_order_convergence_nonlinear():
    # y' = cos(t) y, y(0) = 1: y(t) = exp(sin t)
    f = lambda t, y: [np.cos(t) * y[0]]
    exact = np.exp(np.sin(2.0))
    e = [abs(_solve(f, [1.0], 2.0, n) - exact) for n in (16, 32, 64)]
    r1, r2 = e[0] / e[1], e[1] / e[2]
    assert 28 < r1 < 40 and 28 < r2 < 40, (e, r1, r2)
    # one step: the fifth-order solution's local error falls as h^6, the
    # embedded fourth-order one's as h^5
    loc5, loc4 = [], []
    for hh in (0.2, 0.1, 0.05):
        y1, err, _ = dopri5_step(f, 0.3, [np.array(np.exp(np.sin(0.3)) + 0j)], hh,
                                 f(0.3, [np.array(np.exp(np.sin(0.3)) + 0j)]))
        want = np.exp(np.sin(0.3 + hh))
        loc5.append(abs(y1[0] - want))
        loc4.append(abs(y1[0] - err[0] - want))
    for a, b in zip(loc5, loc5[1:]):
        assert 50 < a / b < 80, loc5
    for a, b in zip(loc4, loc4[1:]):
        assert 25 < a / b < 40, loc4


def test_quartic_quadrature_exact():
    f = lambda t, y: [np.array(3 * t ** 4 - 2 * t ** 3 + t - 5, dtype=complex)]
    F = lambda t: 0.6 * t ** 5 - 0.5 * t ** 4 + 0.5 * t ** 2 - 5 * t
    y1, _, _ = dopri5_step(f, 0.3, [np.array(0j)], 0.7, f(0.3, None))
    assert abs(y1[0] - (F(1.0) - F(0.3))) < 1e-13


def test_adaptive_linear_system_against_expm():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(6, 6)) + 1j * rng.normal(size=(6, 6)) - 3 * np.eye(6)
    y0 = rng.normal(size=6) + 1j * rng.normal(size=6)
    ode = Dopri5(lambda t, y: [A @ y[0]], rtol=1e-9, atol=1e-12)
    y = [y0]
    for s in range(10):
        y = ode.advance(0.1 * s, y, 0.1)
    ref = expm(A) @ y0
    assert np.abs(y[0] - ref).max() < 1e-7 * np.abs(ref).max()
    assert ode.accepted > 10 and ode.rejected >= 0


def _random_state(tree, rng):
    C = rand_cores(tree, rng)
    canonicalize_root(tree, C)
    return C


@pytest.mark.parametrize("mk", [lambda: train_tree(2, [3] * 3, 100),
                                lambda: nary_tree(2, [3] * 4, 2, 100),
                                lambda: nary_tree(2, [3] * 4, 3, 100)])
def test_tangent_equals_generator_at_full_rank(mk):
    tree = mk()
    terms, dims = spin_boson(3, n_ltc=len(tree.end_dims) - 3)
    rng = np.random.default_rng(7)
    C = _random_state(tree, rng)
    d = vmf_derivative(tree, terms, C, None, reg=0.0)
    om = contract_dense(tree, C)
    L = dense_generator(terms, dims)
    want = (L @ om.reshape(-1)).reshape(om.shape)
    got = tangent_dense(tree, C, d)
    assert np.abs(got - want).max() < 1e-9 * np.abs(want).max()


def test_projection_at_truncated_rank():
    tree = nary_tree(2, [4] * 4, 2, 3)
    assert max(tree.rank[1:]) == 3
    terms, dims = spin_boson(4, n_ltc=3)
    rng = np.random.default_rng(11)
    C = _random_state(tree, rng)
    d = vmf_derivative(tree, terms, C, None, reg=0.0)
    om = contract_dense(tree, C)
    L = dense_generator(terms, dims)
    res = (L @ om.reshape(-1)) - tangent_dense(tree, C, d).reshape(-1)
    assert np.linalg.norm(res) > 1e-3 * np.linalg.norm(L @ om.reshape(-1))  # truly truncated
    for s in range(tree.n):
        if s > 0:
            r = tree.rank[s]
            Um, dm = C[s].reshape(r, -1), d[s].reshape(r, -1)
            assert np.abs(Um.conj() @ dm.T).max() < 1e-10 * np.abs(dm).max()
        for _ in range(3):
            X = rng.normal(size=C[s].shape) + 1j * rng.normal(size=C[s].shape)
            if s > 0:
                r = tree.rank[s]
                Um, Xm = C[s].reshape(r, -1), X.reshape(r, -1)
                Xm = Xm - (Um.conj() @ Xm.T).T @ Um
                X = Xm.reshape(X.shape)
            cs = list(C)
            cs[s] = X
            D = contract_dense(tree, cs).reshape(-1)
            assert abs(np.vdot(D, res)) < 1e-9 * np.linalg.norm(D) * np.linalg.norm(res), s


def test_vmf_full_rank_equals_dense():
    tree = nary_tree(2, [3] * 4, 2, 100)
    terms, dims = spin_boson(3, n_ltc=3)
    rng = np.random.default_rng(5)
    C = _random_state(tree, rng)
    nrm = np.linalg.norm(contract_dense(tree, C))
    C[0] = C[0] / nrm
    om0 = contract_dense(tree, C)
    V = VmfPropagator(tree, terms, C, reg=0.0, rtol=1e-10, atol=1e-12)
    for s in range(5):
        V.step(0.05 * s, 0.05)
    L = dense_generator(terms, dims)
    ref = (expm(0.25 * L.toarray() if hasattr(L, "toarray") else 0.25 * L)
           @ om0.reshape(-1)).reshape(om0.shape)
    got = contract_dense(tree, V.C)
    assert np.abs(got - ref).max() < 1e-8 * np.abs(ref).max()
    assert np.abs(reduced_rho(tree, V.C) - dense_rho(ref, dims)).max() < 1e-8


def test_mix_switches_at_the_cap_and_freezes_ranks():
    terms, dims = spin_boson(5)
    base = nary_tree(2, [5] * 3, 2, 100)
    n, dt, eps, cap = 12, 0.01, 1e-8, 4
    t1 = copy.deepcopy(base)
    t1.rank = [0] + [2] * (t1.n - 1)
    t1._clamp()
    steps, rhos, switch, prop = propagate_mix(t1, terms, initial_state(t1, RHO0), dt, n, eps, cap,
                                              fixed_substeps=2)
    # the same ps2 steps alone: the switch comes right after the first step
    # whose largest rank reaches the cap
    t2 = copy.deepcopy(base)
    t2.rank = [0] + [2] * (t2.n - 1)
    t2._clamp()
    P = Propagator(t2, terms, initial_state(t2, RHO0))
    first = None
    for s in range(n):
        P.step_ps2(s * dt, dt, eps, cap)
        if s + 1 < switch:
            assert trace_distance(P.rho(), rhos[s + 1]) < 1e-14
        if first is None and max(t2.rank[1:]) >= cap:
            first = s + 1
    assert first is not None and switch == first < n
    assert isinstance(prop, VmfPropagator)
    assert max(t1.rank[1:]) == cap
    ranks_at_switch = list(t1.rank)
    assert [c.shape for c in prop.C] == [t1.shape(s) for s in range(t1.n)]
    assert list(t1.rank) == ranks_at_switch
    assert np.all(np.isfinite(rhos))
