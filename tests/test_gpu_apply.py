"""GPU parity of the effective generator (tenso_apply_generator) against the
oracle's environment-based apply, on random tiny trees of each shape, every
center, FP64 and FP32 contraction paths."""
import numpy as np
import pytest

import workloads
from oracle.ttn import apply_node, nary_tree, train_tree
from tests.gpu_util import require_gpu
from tests.oracle_helpers import canonical_envs, rand_cores, rand_terms

pytestmark = pytest.mark.gpu

SHAPES = [
    ("train", lambda: train_tree(2, [3, 2, 3], 5)),
    ("binary", lambda: nary_tree(3, [2, 3, 2, 2], 2, 4)),
    ("ternary", lambda: nary_tree(2, [2, 2, 3, 2, 2], 3, 3)),
    ("binary-wide", lambda: nary_tree(5, [7, 9, 6, 8, 5], 2, 20)),
]


def gpu_plan(tree, terms, precision):
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd.heom import TermTable
    t = api.Tree.from_parents(tree.parent, tree.end_node, tree.end_dims, 10 ** 6,
                              bond_rank=[0] + list(tree.rank[1:]))
    tab = TermTable()
    for term in terms:
        tab.add(term['coef'], sorted(term['factors'].items()), slot=term['slot'])
    g = api.Generator(t, tab)
    return api.Plan(t, g, precision=precision)


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-6)])
@pytest.mark.parametrize("name,mk", SHAPES)
def test_apply_generator_matches_oracle(name, mk, precision, tol):
    require_gpu()
    print(f"[apply parity] tree={name} precision={precision}", flush=True)
    rng = np.random.default_rng(11)
    tree = mk()
    terms = rand_terms(tree.end_dims, 12, rng)
    plan = gpu_plan(tree, terms, precision)
    assert plan.shapes() == [tree.shape(s) for s in range(tree.n)]
    worst = 0.0
    for c in range(tree.n):
        C = rand_cores(tree, rng)
        env = canonical_envs(tree, terms, C, c)
        plan.import_state(C)
        Y = plan.apply(c)
        Yo = apply_node(env, c, C[c], None)
        err = np.abs(Y - Yo).max() / np.abs(Yo).max()
        worst = max(worst, err)
        assert err < tol, (name, c, err)
    print(f"  max relative error over centers: {worst:.2e} (bar {tol:.0e})")


def test_apply_generator_rejects_a_non_canonical_center():
    """The state must be canonical toward the center (every other core an
    isometry toward it); the library checks this on the device and returns
    EINVAL otherwise.  The initial state is canonical toward the root only."""
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    print("[apply] non-canonical center -> EINVAL", flush=True)
    inst = workloads.exciton_7site(n_steps=1)
    plan = api.build_instance(inst, precision=api.FP32)
    assert np.isfinite(plan.apply(0)).all()
    with pytest.raises(TensoError) as e:
        plan.apply(3)
    assert e.value.code == "EINVAL" and "canonical" in str(e.value)
    import ctypes as C
    import torch
    from paper_2603_17711_amd._lib import lib
    out = torch.zeros(2 * 7 * 7 * 16, dtype=torch.float64, device="cuda")
    rc = lib().tenso_apply_generator(plan.h, C.c_void_p(plan.state.data_ptr()), plan.n_nodes,
                                     None, C.c_void_p(out.data_ptr()),
                                     C.c_void_p(plan.ws.data_ptr()),
                                     C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1  # EINVAL: no such node
