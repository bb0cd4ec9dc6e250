"""GPU ps1 / ps2 at truncated rank against a closed form (Sec. II C, projector
splitting), through the C-ABI with no oracle integrator involved.

A generator whose terms each act on one end only evolves Omega(0) into
(x)_e exp(t A_e) Omega(0), which keeps the TTN ranks of Omega(0): the
tangent projection drops nothing and the splitting reproduces the exact
solution at truncated rank up to the RK4 error.  The initial state is a
random TTN made canonical toward the root with numpy's QR; the dense tensors
are contracted by the oracle's plain `contract_dense` (test infrastructure)."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle.ttn import contract_dense, nary_tree, train_tree
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

TREES = [
    ("binary", lambda: nary_tree(2, [3, 3, 3, 3], 2, 2)),
    ("ternary", lambda: nary_tree(2, [3, 3, 3, 3], 3, 2)),
    ("binary-wide", lambda: nary_tree(3, [5, 6, 5, 6, 5, 6], 2, 6)),
    ("train", lambda: train_tree(4, [6, 5, 6, 5], 5)),
]


def single_leg_terms(end_dims, rng, per_end=2):
    terms = []
    for e, d in enumerate(end_dims):
        for _ in range(per_end):
            X = (rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))) / np.sqrt(d)
            terms.append({'coef': 0.5 * (rng.normal() + 1j * rng.normal()), 'slot': -1,
                          'factors': {e: X}})
    return terms


def closed_form(end_dims, terms, om0, t):
    om = om0.copy()
    for e, d in enumerate(end_dims):
        A = np.zeros((d, d), complex)
        for term in terms:
            if e in term['factors']:
                A += term['coef'] * term['factors'][e]
        om = np.moveaxis(np.tensordot(expm(t * A), om, axes=([1], [e])), 0, e)
    return om


def canonical_random_state(tree, rng):
    """Random cores; every non-root core made an isometry toward its parent by
    numpy's reduced QR, the R factor absorbed into the parent; unit norm."""
    C = [rng.normal(size=tree.shape(s)) + 1j * rng.normal(size=tree.shape(s))
         for s in range(tree.n)]
    for s in reversed(range(1, tree.n)):
        sh = C[s].shape
        A = np.moveaxis(C[s], 0, -1).reshape(-1, sh[0])
        Q, R = np.linalg.qr(A)
        assert Q.shape[1] == sh[0]
        C[s] = np.moveaxis(Q.reshape(sh[1:] + (sh[0],)), -1, 0)
        p = tree.parent[s]
        i = tree.legs[p].index(('c', s))
        C[p] = np.moveaxis(np.tensordot(R, C[p], axes=([1], [i])), 0, i)
    C[0] = C[0] / np.linalg.norm(contract_dense(tree, C))
    return C


def gpu_plan(tree, terms, precision, method, cap):
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd.heom import TermTable
    t = api.Tree.from_parents(tree.parent, tree.end_node, tree.end_dims, 10 ** 6,
                              bond_rank=[0] + list(tree.rank[1:]))
    tab = TermTable()
    for term in terms:
        tab.add(term['coef'], sorted(term['factors'].items()), slot=term['slot'])
    g = api.Generator(t, tab)
    return api.Plan(t, g, precision=precision, method=method, max_rank=cap)


@pytest.mark.parametrize("precision,tol", [(0, 1e-8), (1, 1e-6)])
@pytest.mark.parametrize("name,mk", TREES)
def test_ps1_truncated_rank_exact_for_single_leg_generator(name, mk, precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[exactness ps1] tree={name} precision={precision}", flush=True)
    rng = np.random.default_rng(31)
    tree = mk()
    C = canonical_random_state(tree, rng)
    terms = single_leg_terms(tree.end_dims, rng)
    dt, n = 0.005, 40
    ref = closed_form(tree.end_dims, terms, contract_dense(tree, C), n * dt)
    plan = gpu_plan(tree, terms, precision, api.PS1, 0)
    assert plan.shapes() == [tree.shape(s) for s in range(tree.n)]
    plan.import_state(C)
    plan.step(n, dt)
    out = plan.export_state()
    err = np.linalg.norm(contract_dense(tree, out) - ref) / np.linalg.norm(ref)
    print(f"  ranks {tree.rank[1:]}, relative error {err:.2e}", flush=True)
    assert err < tol, err


@pytest.mark.parametrize("precision,tol", [(0, 1e-8), (1, 1e-6)])
@pytest.mark.parametrize("name,mk", TREES[:2])
def test_ps2_truncated_rank_exact_for_single_leg_generator(name, mk, precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[exactness ps2] tree={name} precision={precision}", flush=True)
    rng = np.random.default_rng(37)
    tree = mk()
    assert max(tree.rank) == 2
    C = canonical_random_state(tree, rng)
    terms = single_leg_terms(tree.end_dims, rng)
    dt, n = 0.005, 40
    ref = closed_form(tree.end_dims, terms, contract_dense(tree, C), n * dt)
    plan = gpu_plan(tree, terms, precision, api.PS2, 2)
    assert plan.shapes() == [tree.shape(s) for s in range(tree.n)]
    plan.import_state(C)
    plan.step_adaptive(n, dt, 1e-12, 2)
    assert list(plan.ranks()[1:]) == list(tree.rank[1:])
    out = plan.export_state()
    err = np.linalg.norm(contract_dense(tree, out) - ref) / np.linalg.norm(ref)
    print(f"  ranks {tree.rank[1:]}, relative error {err:.2e}", flush=True)
    assert err < tol, err
