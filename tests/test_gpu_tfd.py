"""The thermofield ML-MCTDH workload (Sec. III A 5) on the GPU: a wavefunction
TTN under -iH, ps1, against the oracle on the same tree and rank: a reduced
bath (8 modes, Fock dimension 4, rank 8) over 50 steps, and the paper's
listing (50 modes, dimension 8, rank 16) over 100 steps against the stored
oracle trajectory."""
import numpy as np
import pytest

import workloads
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def run(inst, n, precision, every=10):
    from paper_2603_17711_amd.mctdh import build_tfd
    plan = build_tfd(inst, precision=precision)
    out = [plan.rho_pure()]
    done = 0
    while done < n:
        k = min(every, n - done)
        plan.step(k, inst.dt, t0=done * inst.dt)
        done += k
        out.append(plan.rho_pure())
    return np.array(out)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_tfd_reduced_bath_matches_oracle(precision, tol):
    require_gpu()
    from oracle.tfd import propagate_tfd
    inst = workloads.tfd_spin_boson(n_modes=8, dim=4, rank=8, n_steps=50)
    print(f"[tfd] 8 modes dim 4 rank 8, 50 steps, precision={precision}", flush=True)
    _, rho_o = propagate_tfd(inst, n_steps=50, every=10)
    rg = run(inst, 50, precision)
    d = max(trace_distance(a, b) for a, b in zip(rg, rho_o))
    print(f"  max trace distance {d:.3e}; trace {np.trace(rg[-1]).real:.12f}")
    assert d < tol


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)])
def test_tfd_listing_size_against_stored_oracle(precision, tol):
    require_gpu()
    from tests.golden.make_golden import load
    inst = workloads.tfd_spin_boson()
    g = load("tfd_spin_boson_100.npz", [inst])
    print(f"[tfd] 50 modes dim 8 rank 16, 100 steps, precision={precision}", flush=True)
    rg = run(inst, 100, precision)
    assert list(g["steps"]) == list(range(0, 101, 10))
    ds = [trace_distance(a, b) for a, b in zip(rg, g["rho"])]
    print(f"  max trace distance {max(ds):.3e} (step {10 * int(np.argmax(ds))})")
    assert max(ds) < tol


def test_tfd_rejects_density_trees_for_the_pure_state_density():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    plan = api.build_instance(workloads.spin_boson_train(n_steps=1), precision=0)
    with pytest.raises(TensoError) as e:
        plan.rho_pure()
    assert e.value.code == "EINVAL"
