"""tenso_apply_generator_noalloc, the variant of tenso_apply_generator that
allocates nothing (workspace and launch descriptors in the library's static
device scratch), against tenso_apply_generator on the same states: two calls
in a row, the second on a smaller plan, both through the C ABI.  The two run
the same kernels on the same inputs, so the results agree bit for bit; the
bar is the apply parity bar (FP64 1e-12 relative, FP32 2e-5).  A plan whose
workspace exceeds the scratch is refused with ENOMEM, and the next call works.
"""
import numpy as np
import pytest

import workloads
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def test_noalloc_matches_apply_generator_twice_then_smaller():
    require_gpu()
    from paper_2603_17711_amd import api
    cases = [("7-site exciton K=28 R=16, FP32, 2 steps", workloads.exciton_7site(n_steps=2),
              api.FP32, 2e-5),
             ("spin-boson train K=3 R=8, FP64, 3 steps", workloads.spin_boson_train(n_steps=3),
              api.FP64, 1e-12)]
    sizes = []
    for name, inst, prec, tol in cases:
        print(f"[noalloc] {name}", flush=True)
        plan = api.build_instance(inst, precision=prec)
        plan.step(inst.n_steps, inst.dt)
        ref = plan.apply(0)
        got = plan.apply(0, noalloc=True)
        again = plan.apply(0, noalloc=True)
        err = _rel(got, ref)
        print(f"  |noalloc - apply| / |apply| = {err:.2e} (repeat {_rel(again, ref):.2e}), "
              f"center core {ref.shape}", flush=True)
        assert np.isfinite(got).all() and np.abs(ref).max() > 0
        assert err <= tol and _rel(again, ref) <= tol
        sizes.append(ref.size)
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    print("[noalloc] plan with a 118 MiB workspace (binary tree, M=8, K=8, N=12, R=64)",
          flush=True)
    big = workloads.Instance("big", np.diag(np.arange(8.0)),
                             [workloads.Bath(np.eye(8), 1.0, dl=[(0.1, 1.0)], n_ltc=7)], 12,
                             "tree2", 64, workloads.ground(8), 0.01, 1)
    plan = api.build_instance(big, precision=api.FP32)
    with pytest.raises(TensoError) as e:
        plan.apply(0, noalloc=True)
    assert e.value.code == "ENOMEM" and "scratch" in str(e.value)
    small = api.build_instance(workloads.spin_boson_train(n_steps=1), precision=api.FP32)
    np.testing.assert_array_equal(small.apply(0, noalloc=True), small.apply(0))
