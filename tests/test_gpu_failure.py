"""Failure handling forced from the host: a NaN planted in a state makes the
next step call return TENSO_ENUMERIC, for a single plan and for the one
poisoned instance of a batch (the others stay unflagged).  NaNs only
propagate through the arithmetic; nothing faults."""
import numpy as np
import pytest

import workloads
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _poison(plan, index=7):
    st = plan.state.view(dtype=__import__("torch").float64)
    st[index] = float("nan")


def test_plan_step_reports_nonfinite_state():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    inst = workloads.config0(n_steps=10)
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
    insts = workloads.config2(n_inst=5, seed=9, n_steps=10)
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
