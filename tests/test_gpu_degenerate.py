"""Degenerate cases of the ps1 path on the GPU, through the C-ABI, against
closed forms (Sec. II C):

* a one-node tree (every end on the root, no bond): the sweep is the node
  flow alone, so n RK4 steps of the full tensor must equal exp(n dt L)
  Omega(0) up to the RK4 error, L built here by Kronecker products;
* rank-1 bonds (a product state) under a generator of single-end terms: the
  solution stays a product, exp(t A_e) applied end by end;
* zero steps: the state comes back unchanged, bit for bit."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle.ttn import Tree, contract_dense, nary_tree
from tests.gpu_util import require_gpu
from tests.test_gpu_exactness import (canonical_random_state, closed_form, gpu_plan,
                                      single_leg_terms)

pytestmark = pytest.mark.gpu


def dense_L(terms, end_dims):
    D = int(np.prod(end_dims))
    L = np.zeros((D, D), complex)
    for term in terms:
        op = np.ones((1, 1), complex)
        for e, d in enumerate(end_dims):
            op = np.kron(op, term['factors'].get(e, np.eye(d)))
        L += term['coef'] * op
    return L


def mixed_terms(end_dims, rng, n=8):
    """Terms with one or two non-identity factors."""
    terms = []
    for _ in range(n):
        k = int(rng.integers(1, 3))
        es = rng.choice(len(end_dims), size=k, replace=False)
        f = {int(e): (rng.normal(size=(end_dims[e],) * 2) + 1j * rng.normal(size=(end_dims[e],) * 2))
             / end_dims[e] for e in es}
        terms.append({'coef': 0.5 * (rng.normal() + 1j * rng.normal()), 'slot': -1, 'factors': f})
    return terms


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)])
def test_one_node_tree_equals_dense_exponential(precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[degenerate] one-node tree precision={precision}", flush=True)
    rng = np.random.default_rng(41)
    tree = Tree([-1], [0, 0, 0], [3, 3, 5], max_rank=4)
    terms = mixed_terms(tree.end_dims, rng)
    C = canonical_random_state(tree, rng)
    dt, n = 0.005, 40
    ref = expm(n * dt * dense_L(terms, tree.end_dims)) @ C[0].reshape(-1)
    plan = gpu_plan(tree, terms, precision, api.PS1, 0)
    assert plan.shapes() == [(3, 3, 5)]
    plan.import_state(C)
    plan.step(n, dt)
    out = plan.export_state()[0].reshape(-1)
    err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
    print(f"  relative error {err:.2e}", flush=True)
    assert err < tol, err


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)])
def test_rank_one_product_state_stays_exact(precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[degenerate] rank-1 bonds precision={precision}", flush=True)
    rng = np.random.default_rng(43)
    tree = nary_tree(2, [3, 4, 3, 4], 2, 1)
    assert max(tree.rank) == 1
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
    print(f"  relative error {err:.2e}", flush=True)
    assert err < tol, err


@pytest.mark.parametrize("precision", [0, 1])
def test_zero_steps_leave_the_state_unchanged(precision):
    require_gpu()
    from paper_2603_17711_amd import api
    print(f"[degenerate] zero steps precision={precision}", flush=True)
    rng = np.random.default_rng(47)
    tree = nary_tree(2, [3, 3, 3, 3], 2, 3)
    C = canonical_random_state(tree, rng)
    terms = mixed_terms(tree.end_dims, rng)
    plan = gpu_plan(tree, terms, precision, api.PS1, 0)
    plan.import_state(C)
    plan.step(0, 0.01)
    out = plan.export_state()
    for a, b in zip(out, C):
        assert np.array_equal(a, b)
