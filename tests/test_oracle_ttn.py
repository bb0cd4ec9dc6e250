"""Pins of the oracle's tree tensor network (Sec. II C).

The environment-based effective generators (node, bond, two-site) are checked
against the plain definition d<Omega, L Omega>/d conj(X), computed by dense
brute force, on random tiny trees of each shape and every center."""
import json
import os

import numpy as np
import pytest

from oracle.integrators import qr_toward
from oracle.sop import dense_generator, dense_initial
from oracle.ttn import (Tree, apply_bond, apply_node, apply_two_site, contract_dense,
                        initial_state, is_isometry_toward, merge, nary_tree,
                        reduced_rho, train_tree)
from tests.oracle_helpers import (brute_gradient, canonical_envs, rand_cores,
                                  rand_terms)

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")

SHAPES = [
    ("train", lambda: train_tree(2, [3, 2, 3], 5)),
    ("binary", lambda: nary_tree(3, [2, 3, 2, 2], 2, 4)),
    ("ternary", lambda: nary_tree(2, [2, 2, 3, 2, 2], 3, 3)),
]


def test_binary_core_count_printed():
    gold = json.load(open(GOLD))["binary_tree_cores"]
    for K in gold["K_values"]:
        tr = nary_tree(2, [3] * K, 2, 4)
        assert tr.n == K and len(tr.rank) - 1 == K - 1
        inner = [s for s in range(tr.n) if len(tr.legs[s]) == 3]
        assert len(inner) == K  # all cores order three


def test_train_layout_and_clamp():
    tr = train_tree(2, [10, 10, 10], 8)
    assert tr.parent == [-1, 0, 1]
    assert [tr.shape(s) for s in range(3)] == [(2, 2, 4), (4, 10, 8), (8, 10, 10)]
    tr = train_tree(2, [10, 10, 10], 40)
    assert [tr.shape(s) for s in range(3)] == [(2, 2, 4), (4, 10, 40), (40, 10, 10)]


def test_rank_clamp_is_local():
    tr = nary_tree(3, [4, 5, 2, 6, 3, 2, 2], 3, 64)
    for c in range(1, tr.n):
        p = tr.parent[c]
        lo = np.prod(tr.shape(c)[1:])
        hi = np.prod([d for d, l in zip(tr.shape(p), tr.legs[p]) if l != ('c', c)])
        assert tr.rank[c] <= lo and tr.rank[c] <= hi


@pytest.mark.parametrize("name,mk", SHAPES)
def test_initial_state_is_rho_times_vacuum(name, mk):
    tr = mk()
    rho0 = np.array([[0.6, 0.1j], [-0.1j, 0.4]]) if tr.end_dims[0] == 2 else np.eye(3) / 3
    C = initial_state(tr, rho0)
    om = contract_dense(tr, C).reshape(-1)
    assert np.abs(om - dense_initial(rho0, tr.end_dims)).max() == 0.0
    for s in range(1, tr.n):
        assert is_isometry_toward(C[s], 0)
    assert np.abs(reduced_rho(tr, C) - rho0).max() == 0.0


@pytest.mark.parametrize("name,mk", SHAPES)
def test_effective_generators_match_brute_force(name, mk):
    rng = np.random.default_rng(7)
    tr = mk()
    terms = rand_terms(tr.end_dims, 9, rng)
    L = dense_generator(terms, tr.end_dims)
    for c in range(tr.n):
        C = rand_cores(tr, rng)
        env = canonical_envs(tr, terms, C, c)
        LOm = L @ contract_dense(tr, C).reshape(-1)
        Y = apply_node(env, c, C[c], None)
        Yb = brute_gradient(tr, C, c, LOm)
        assert np.abs(Y - Yb).max() <= 1e-12 * np.abs(Yb).max()
        if c == 0:
            continue
        # bond between parent(c) and c: C_c = B x_0 Q
        Q, R = qr_toward(C[c], 0)
        saved = env.down[c]
        env.update_down(c, Q)
        K = apply_bond(env, c, R.T, None)
        Kb = brute_gradient_bond(tr, C, c, Q, LOm)
        assert np.abs(K - Kb).max() <= 1e-12 * np.abs(Kb).max()
        env.down[c] = saved
        # two-site tensor of (parent(c), c)
        s = tr.parent[c]
        Th = merge(tr, C, s, c)
        Y2 = apply_two_site(env, s, c, Th, None)
        Tb = brute_gradient_two_site(tr, C, s, c, Th.shape, LOm)
        assert np.abs(Y2 - Tb).max() <= 1e-12 * np.abs(Tb).max()


def brute_gradient_bond(tr, C, c, Q, LOm):
    from oracle.ttn import mode_product
    r = Q.shape[0]
    out = np.zeros((r, r), dtype=np.complex128)
    for idx in np.ndindex(r, r):
        U = np.zeros((r, r), dtype=np.complex128)
        U[idx] = 1.0
        E = list(C)
        E[c] = mode_product(Q, U, 0)
        out[idx] = np.vdot(contract_dense(tr, E).reshape(-1), LOm)
    return out


def brute_gradient_two_site(tr, C, s, c, shape, LOm):
    i = tr.leg_of_child(s, c)
    ns = len(tr.legs[s]) - 1
    rows = int(np.prod(shape[:ns]))
    out = np.zeros(shape, dtype=np.complex128)
    for idx in np.ndindex(shape):
        U = np.zeros(shape, dtype=np.complex128)
        U[idx] = 1.0
        # a rank-`rows` exact factorisation U = I_rows * U (identity on s-side)
        E = list(C)
        E[s] = np.moveaxis(np.eye(rows).reshape(shape[:ns] + (rows,)), -1, i)
        E[c] = U.reshape((rows,) + shape[ns:])
        out[idx] = np.vdot(contract_dense(tr, E).reshape(-1), LOm)
    return out


def test_qr_toward_convention():
    rng = np.random.default_rng(3)
    C = rng.normal(size=(3, 4, 5)) + 1j * rng.normal(size=(3, 4, 5))
    for leg in range(3):
        Q, R = qr_toward(C, leg)
        assert is_isometry_toward(Q, leg)
        from oracle.ttn import mode_product
        assert np.abs(mode_product(Q, R.T, leg) - C).max() < 1e-13
        d = np.diag(R)
        assert np.all(np.abs(d.imag) < 1e-14) and np.all(d.real >= 0)
    # zero columns keep the Householder identity (exact zeros stay zero)
    Z = np.zeros((4, 3), complex)
    Z[:, 0] = [1, 2j, 0, 1]
    Q, R = qr_toward(Z, 1)
    assert np.all(R[1:, :] == 0)
    assert np.abs(Q.conj().T @ Q - np.eye(3)).max() < 1e-14


def test_householder_matches_lapack_on_full_rank():
    from oracle.integrators import householder_qr
    rng = np.random.default_rng(4)
    for m, n in [(6, 6), (12, 5), (40, 8)]:
        A = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
        Q, R = householder_qr(A)
        Ql, Rl = np.linalg.qr(A)
        assert np.abs(Q @ R - A).max() < 1e-13
        assert np.abs(Q.conj().T @ Q - np.eye(n)).max() < 1e-13
        # same reflectors as LAPACK: identical factors up to rounding
        assert np.abs(Q - Ql).max() < 1e-12 and np.abs(R - Rl).max() < 1e-12


def test_householder_rank_threshold_is_deterministic():
    from oracle.integrators import householder_qr
    rng = np.random.default_rng(5)
    B = rng.normal(size=(10, 2)) + 1j * rng.normal(size=(10, 2))
    A = np.concatenate([B, B @ np.array([[1.0, 2.0], [0.5, -1.0]])], axis=1)  # rank 2
    Q1, R1 = householder_qr(A)
    noise = 1e-14 * (rng.normal(size=A.shape) + 1j * rng.normal(size=A.shape))
    Q2, R2 = householder_qr(A + noise)
    assert np.abs(Q1 - Q2).max() < 1e-10  # completion does not follow the noise
    assert R1[2, 2] == 0 and R1[3, 3] == 0 and np.abs(R1[2:, 2:]).max() < 1e-13
