"""GPU parity of ps2 (adaptive rank) against the oracle: rho_S trace distance
and the rank decisions, on a train and on the structured-bath ternary tree at
a small rank cap."""
import numpy as np
import pytest

import workloads
from oracle.run import propagate
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def run_ps2(inst, n_steps, precision, cap, every=5):
    from paper_2603_17711_amd import api
    plan = api.build_instance(inst, precision=precision, rank=cap)
    rhos, ranks = [plan.rho()], []
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        plan.step_adaptive(k, inst.dt, inst.eps, cap, t0=done * inst.dt)
        ranks.extend(plan.rank_log())
        done += k
        rhos.append(plan.rho())
    return np.array(rhos), ranks


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-5)])
def test_ps2_train(precision, tol):
    require_gpu()
    inst = workloads.spin_boson_train(n_steps=20)
    inst.method, inst.eps, inst.depth = "ps2", 1e-6, 6
    cap, n = 8, 20
    print(f"[ps2 parity] train K=3 N=6 cap={cap} steps={n} precision={precision}", flush=True)
    _, ro, rlog, _ = propagate(inst, n_steps=n, every=5, max_rank=cap)
    rg, rl_gpu = run_ps2(inst, n, precision, cap)
    d = max(trace_distance(a, b) for a, b in zip(rg, ro))
    flat_o = [r for step in rlog for r in step]
    print(f"  max trace distance {d:.3e}; ranks oracle {flat_o[-6:]} gpu {rl_gpu[-6:]}")
    assert d < tol
    assert flat_o == rl_gpu


def test_ps2_structured_bath_ternary_small_cap():
    require_gpu()
    inst = workloads.structured_bath_ternary(n_steps=6)
    cap, n = 4, 6
    print(f"[ps2 parity] structured bath K=24 ternary cap={cap} steps={n} FP32", flush=True)
    _, ro, rlog, _ = propagate(inst, n_steps=n, every=5, max_rank=cap)
    rg, rl_gpu = run_ps2(inst, n, 1, cap)
    d = max(trace_distance(a, b) for a, b in zip(rg, ro))
    flat_o = [r for step in rlog for r in step]
    print(f"  max trace distance {d:.3e}; ranks match: {flat_o == rl_gpu}")
    assert d < 1e-5
