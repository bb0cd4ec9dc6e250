"""Parity at the benchmark sizes, in the launch configuration bench.py times.

The 512-instance batch runs with its defaults (tile size, four parts replayed
as branches of one HIP graph); every instance must stay finite with a trace
within 1e-5 of one (the projected dynamics conserve it up to the projection
error), and sampled instances are compared with the FP64 oracle one by one:
fixed ones, the largest states, and the instances with the largest trace and
Hermiticity deviations (Hermiticity of rho_S is not exact under the fixed-rank
projection: the oracle itself departs from it, by up to 2e-8 after 3 steps).
The 7-site exciton model (K = 28, rank 16) runs as a single FP32 plan against
the oracle.
The bar is the fixed-rank one: trace distance of rho_S at most 1e-6."""
import numpy as np
import pytest

import workloads
from oracle.run import build, propagate
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu

TOL = 1e-6


def state_sizes(insts):
    out = []
    for inst in insts:
        _, tree = build(inst)
        tot = 0
        for s in range(tree.n):
            tot += int(np.prod(tree.shape(s)))
        out.append(tot)
    return out


def test_full_batch_sampled_against_oracle():
    require_gpu()
    from paper_2603_17711_amd import api
    n = 3
    insts = workloads.uneven_batch(n_inst=512, n_steps=n)
    sizes = state_sizes(insts)
    largest = [int(i) for i in np.argsort(sizes)[::-1][:2]]
    print(f"[full batch] 512 instances, {n} steps, FP32, default tiles and parts", flush=True)
    plans = [api.build_instance(i, precision=api.FP32) for i in insts]
    batch = api.Batch(plans)
    batch.step(n, [i.dt for i in insts])
    assert not batch.status().any()
    rho = batch.rho()
    tr = np.array([np.trace(r).real for r in rho])
    herm = np.array([np.abs(r - r.conj().T).max() for r in rho])
    k_tr, k_herm = int(np.argmax(np.abs(tr - 1))), int(np.argmax(herm))
    print(f"  max |Tr - 1| = {np.abs(tr - 1).max():.2e} (instance {k_tr}), "
          f"max |rho - rho^H| = {herm.max():.2e} (instance {k_herm})", flush=True)
    assert all(np.isfinite(r).all() for r in rho)
    assert np.abs(tr - 1).max() < 1e-5
    sample = sorted(set([0, 1, 128, 255, 384, 511, k_tr, k_herm] + largest))
    print(f"  oracle sample {sample}", flush=True)
    worst = 0.0
    for k in sample:
        _, ro, _, _ = propagate(insts[k], n_steps=n, every=n)
        d = trace_distance(rho[k], ro[-1])
        ho = np.abs(ro[-1] - ro[-1].conj().T).max()
        print(f"  instance {k} (state {sizes[k]} elements): trace distance {d:.3e}, "
              f"|rho - rho^H| GPU {herm[k]:.2e} oracle {ho:.2e}", flush=True)
        worst = max(worst, d)
    assert worst < TOL, worst


def test_full_exciton_7site_against_oracle():
    require_gpu()
    from paper_2603_17711_amd import api
    n = 5
    inst = workloads.exciton_7site(n_steps=n)
    print(f"[full size] 7-site exciton model, K = 28, R = 16, {n} FP32 steps", flush=True)
    plan = api.build_instance(inst, precision=api.FP32)
    plan.step(n, inst.dt)
    _, ro, _, _ = propagate(inst, n_steps=n, every=n)
    d = trace_distance(plan.rho(), ro[-1])
    print(f"  trace distance {d:.3e}", flush=True)
    assert d < TOL, d
