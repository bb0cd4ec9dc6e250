"""The paper's complete-input-file example (Sec. III A 1, its Table and
listing) as a GPU parity smoke test: a two-level system coupled to a Drude
bath plus one Brownian mode at 300 K, with the Pade decomposition of the Bose
function (one low-temperature term: 4 features), depth 25, on a tensor train
of rank 16, 500 RK4 steps of 0.1 fs.  rho_S is compared every 50 steps with
the stored FP64 oracle trajectory (tests/golden/pade_structured_500.npz)."""
import numpy as np
import pytest

import workloads
from oracle.ttn import trace_distance
from tests.golden.make_golden import load
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)])
def test_structured_spin_boson_pade_against_oracle(precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    n, every = 500, 50
    inst = workloads.structured_spin_boson_pade(n_steps=n)
    g = load("pade_structured_500.npz", [inst])
    print(f"[pade] structured spin-boson (Sec. III A 1 parameters), {n} steps, "
          f"precision {precision}", flush=True)
    plan = api.build_instance(inst, precision=precision)
    ds = [trace_distance(plan.rho(), g["rho"][0])]
    for j in range(1, n // every + 1):
        plan.step(every, inst.dt, t0=(j - 1) * every * inst.dt)
        ds.append(trace_distance(plan.rho(), g["rho"][j]))
    moved = trace_distance(g["rho"][-1], g["rho"][0])
    print(f"  trace distance per record {['%.1e' % d for d in ds]}; rho_S moved by "
          f"{moved:.2f} over 50 fs", flush=True)
    assert moved > 0.05
    assert max(ds) < tol
