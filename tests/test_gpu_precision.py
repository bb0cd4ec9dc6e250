"""Precision study of the contraction (the precision policy): the spin-boson
train over its 2000 steps in complex FP64, complex FP32 with four real MFMA
products per complex product, and FP32 with three (Gauss), each against the
stored FP64 oracle trajectory; the trace distance is printed at several
horizons and bounded at the end.  BF16 operands (8-bit mantissa) are run for
the record only: they miss the fixed-rank 1e-6 bar by orders of magnitude."""
import numpy as np
import pytest

import workloads
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision,tol", [("fp64", 0, 1e-9), ("fp32", 1, 1e-6),
                                                 ("fp32-3m", 2, 1e-6), ("bf16", 3, 1.0)])
def test_precision_study_spin_boson_train(name, precision, tol):
    require_gpu()
    from paper_2603_17711_amd import api
    from tests.golden.make_golden import load
    n = 2000
    inst = workloads.spin_boson_train(n_steps=n)
    g = load("spin_boson_train_2000.npz", [inst])
    print(f"[precision] spin-boson train, {name}, {n} steps", flush=True)
    plan = api.build_instance(inst, precision=precision)
    ds = [trace_distance(plan.rho(), g["rho"][0])]
    for k in range(1, n // 10 + 1):
        plan.step(10, inst.dt, t0=10 * (k - 1) * inst.dt)
        ds.append(trace_distance(plan.rho(), g["rho"][k]))
    ds = np.array(ds)
    marks = {s: float(ds[: s // 10 + 1].max()) for s in (10, 100, 500, 1000, 2000)}
    print("  max trace distance up to step " +
          ", ".join(f"{s}: {v:.2e}" for s, v in marks.items()), flush=True)
    assert ds.max() < tol
