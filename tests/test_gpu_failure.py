"""Failure handling forced from the host: a NaN planted in a state makes the
next step call return TENSO_ENUMERIC, for a single plan and for the one
poisoned instance of a batch (the others stay unflagged).  NaNs only
propagate through the arithmetic; nothing faults.

Norm growth: a term +g * identity added to a generator multiplies the state
by about exp(g t); over a call that spans g t = 20 (growth ~5e8, finite) the
call returns TENSO_ENUMERIC, for ps1, ps2 and the grown instance of a batch,
while g t = 5 (growth ~150) passes."""
import numpy as np
import pytest

import workloads
from oracle.ttn import nary_tree
from tests.gpu_util import require_gpu
from tests.test_gpu_exactness import canonical_random_state, gpu_plan, single_leg_terms

pytestmark = pytest.mark.gpu


def _poison(plan, index=7):
    st = plan.state.view(dtype=__import__("torch").float64)
    st[index] = float("nan")


def test_plan_step_reports_nonfinite_state():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    inst = workloads.spin_boson_train(n_steps=10)
    print("[failure] NaN planted in a spin-boson state", flush=True)
    p = api.build_instance(inst, precision=api.FP32)
    p.step(2, inst.dt)  # healthy
    _poison(p)
    with pytest.raises(TensoError) as e:
        p.step(2, inst.dt)
    assert "ENUMERIC" in str(e.value)


def test_batch_flags_the_poisoned_instance():
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    insts = workloads.uneven_batch(n_inst=5, seed=9, n_steps=10)
    for inst in insts:
        inst.depth, inst.rank = 4, 4
    print("[failure] NaN planted in instance 2 of a batch of 5", flush=True)
    b = api.Batch([api.build_instance(i, precision=api.FP32) for i in insts])
    dts = [i.dt for i in insts]
    b.step(2, dts)
    assert not b.status().any()
    _poison(b.plans[2])
    torch.cuda.synchronize()
    with pytest.raises(TensoError) as e:
        b.step(2, dts)
    assert "ENUMERIC" in str(e.value)
    assert b.status().tolist() == [False, False, True, False, False]


def _growth_plan(g, method, rng):
    from paper_2603_17711_amd import api
    tree = nary_tree(2, [3, 3, 3, 3], 2, 2)
    terms = single_leg_terms(tree.end_dims, rng)
    d0 = tree.end_dims[0]
    terms.append({'coef': g, 'slot': -1, 'factors': {0: np.eye(d0, dtype=complex)}})
    plan = gpu_plan(tree, terms, api.FP32, method, 2 if method == api.PS2 else 0)
    plan.import_state(canonical_random_state(tree, rng))
    return plan


@pytest.mark.parametrize("method", [0, 1])
def test_norm_growth_is_reported(method):
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    print(f"[failure] norm growth, method {'ps2' if method else 'ps1'}", flush=True)
    rng = np.random.default_rng(53)

    def advance(plan, n, dt):
        if method == api.PS2:
            plan.step_adaptive(n, dt, 1e-12, 2)
        else:
            plan.step(n, dt)

    advance(_growth_plan(5.0, method, rng), 20, 0.05)  # growth ~150: no error
    grown = _growth_plan(20.0, method, rng)
    with pytest.raises(TensoError) as e:
        advance(grown, 20, 0.05)
    assert e.value.code == "ENUMERIC" and "norm" in str(e.value)
    assert all(np.isfinite(c).all() for c in grown.export_state())


def test_batch_flags_the_grown_instance():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    print("[failure] norm growth in instance 1 of a batch of 3", flush=True)
    rng = np.random.default_rng(59)
    plans = [_growth_plan(g, api.PS1, rng) for g in (5.0, 20.0, 0.0)]
    b = api.Batch(plans)
    with pytest.raises(TensoError) as e:
        b.step(20, [0.05] * 3)
    assert e.value.code == "ENUMERIC"
    assert b.status().tolist() == [False, True, False]
