"""Graph replay of steps and the tile-size autotuner.

A captured step replays the same kernels on the same buffers in the same
order as eager launching, so the FP64 master states must agree bit for bit;
each comparison follows unrelated eager device work and a synchronisation,
and every replayed round is checked.  Calls with different step counts reuse
the captured step when no drive is bound (and rebuild it when one is); either
way they must reproduce one call over all the steps bit for bit.  The
autotuner must hand the states back exactly as it found them."""
import numpy as np
import pytest

import workloads
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _instances(n, seed=11):
    rng = np.random.default_rng(seed)
    insts = workloads.uneven_batch(n_inst=n, seed=seed, n_steps=20)
    for inst in insts:
        inst.depth = int(rng.integers(3, 7))
        inst.rank = int(rng.integers(3, 9))
    return insts


def _other_work():
    import torch
    x = torch.randn(1 << 16, device="cuda")
    y = (x * x).sum()
    torch.cuda.synchronize()
    return float(y)


@pytest.mark.parametrize("precision,parts", [(0, 4), (1, 4), (1, 1)])
def test_batch_graph_replay_matches_eager(precision, parts):
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    insts = _instances(7)
    print(f"[graph batch] 7 instances precision={precision} parts={parts}", flush=True)
    ga = api.Batch([api.build_instance(i, precision=precision) for i in insts])
    ga.set_parts(parts)
    eb = api.Batch([api.build_instance(i, precision=precision) for i in insts])
    eb.set_graph(False)
    eb.set_parts(1)
    dts = [i.dt for i in insts]
    for rnd in range(4):
        ga.step(3, dts)
        _other_work()
        eb.step(3, dts)
        torch.cuda.synchronize()
        for k, (pa, pb) in enumerate(zip(ga.plans, eb.plans)):
            assert torch.equal(pa.state, pb.state), f"round {rnd} instance {k}"
        _other_work()


@pytest.mark.parametrize("precision", [0, 1])
def test_plan_graph_replay_matches_eager(precision):
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    inst = workloads.spin_boson_train(n_steps=30)
    print(f"[graph plan] spin-boson train precision={precision}", flush=True)
    a = api.build_instance(inst, precision=precision)
    b = api.build_instance(inst, precision=precision)
    b.set_graph(False)
    for rnd in range(4):
        a.step(5, inst.dt)
        _other_work()
        b.step(5, inst.dt)
        torch.cuda.synchronize()
        assert torch.equal(a.state, b.state), f"round {rnd}"


def test_autotune_restores_states_and_keeps_results():
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    insts = _instances(6, seed=5)
    print("[autotune] 6 instances FP32", flush=True)
    dts = [i.dt for i in insts]
    tuned = api.Batch([api.build_instance(i, precision=1) for i in insts])
    ref = api.Batch([api.build_instance(i, precision=1) for i in insts])
    tuned.step(2, dts)
    ref.step(2, dts)
    torch.cuda.synchronize()
    before = [p.state.clone() for p in tuned.plans]
    w = tuned.autotune(dts, trial_steps=2)
    print(f"  chosen tile work {w:.0e}")
    assert w in (4e6, 8e6, 16e6, 32e6, 64e6)
    for k, (p, s0) in enumerate(zip(tuned.plans, before)):
        assert torch.equal(p.state, s0), f"instance {k} changed by the autotuner"
    tuned.step(10, dts)
    ref.step(10, dts)
    for k, (ra, rb) in enumerate(zip(tuned.rho(), ref.rho())):
        d = trace_distance(ra, rb)
        print(f"  instance {k}: tuned vs default tiles {d:.2e}")
        assert d < 1e-6


@pytest.mark.parametrize("driven", [False, True])
def test_calls_of_different_lengths_match_one_call(driven):
    require_gpu()
    import torch
    from paper_2603_17711_amd import api
    from tests.test_gpu_ps1 import pulsed
    print(f"[graph] step counts 3 + 5 + 2 against 10, driven={driven}", flush=True)
    if driven:
        insts = [pulsed(A, w, n_steps=10) for A, w in [(2.0, 3.0), (1.0, 1.5)]]
    else:
        insts = _instances(5)
    dts = [i.dt for i in insts]
    one = api.Batch([api.build_instance(i, precision=api.FP32) for i in insts])
    parts = api.Batch([api.build_instance(i, precision=api.FP32) for i in insts])
    tabs = [api.drive_table(i, 10) for i in insts] if driven else None
    one.step(10, dts, drive_tabs=tabs)
    done = 0
    for n in (3, 5, 2):
        sub = None
        if driven:
            sub = [t[:, 4 * done:4 * (done + n) + 1].contiguous() for t in tabs]
        parts.step(n, dts, t0s=[done * d for d in dts], drive_tabs=sub)
        done += n
        _other_work()
    torch.cuda.synchronize()
    for k, (pa, pb) in enumerate(zip(one.plans, parts.plans)):
        assert torch.equal(pa.state, pb.state), f"instance {k}"
