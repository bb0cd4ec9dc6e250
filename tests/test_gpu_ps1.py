"""GPU parity of ps1 propagation against the oracle (trace distance of rho_S,
max over every 10th step and the final step), undriven and with a
time-dependent drive (a Gaussian pulse centred inside the propagated window,
through the drive table), for single plans and for a batch."""
import numpy as np
import pytest

import workloads
from oracle.run import propagate
from oracle.ttn import trace_distance
from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def run_gpu(inst, n_steps, precision, every=10):
    from paper_2603_17711_amd import api
    plan = api.build_instance(inst, precision=precision)
    tab = api.drive_table(inst, n_steps)
    rhos = [plan.rho()]
    done = 0
    while done < n_steps:
        k = min(every, n_steps - done)
        sub = None
        if tab is not None:
            sub = tab[:, 4 * done:4 * (done + k) + 1].contiguous()
        plan.step(k, inst.dt, t0=done * inst.dt, drive_tab=sub)
        done += k
        rhos.append(plan.rho())
    return np.array(rhos)


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-6)])
def test_ps1_spin_boson_train_full_horizon(precision, tol):
    """The spin-boson train at its whole configured horizon (2000 steps),
    rho_S compared at every 10th step with the stored oracle trajectory."""
    require_gpu()
    from tests.golden.make_golden import load
    n = 2000
    inst = workloads.spin_boson_train(n_steps=n)
    g = load("spin_boson_train_2000.npz", [inst])
    print(f"[ps1 parity] spin-boson train steps={n} precision={precision}", flush=True)
    rg = run_gpu(inst, n, precision)
    assert list(g["steps"]) == list(range(0, n + 1, 10))
    ds = [trace_distance(a, b) for a, b in zip(rg, g["rho"])]
    d = max(ds)
    print(f"  max trace distance over {len(ds)} records = {d:.3e} "
          f"(at step {10 * int(np.argmax(ds))}); final {ds[-1]:.3e}")
    assert d < tol


def test_ps1_binary_multi_bath_short():
    require_gpu()
    rng = np.random.default_rng(5)
    M = 3
    H = np.diag(rng.normal(size=M)).astype(complex)
    H[0, 1] = H[1, 0] = 0.3
    H[1, 2] = H[2, 1] = 0.2
    baths = []
    for b in range(M):
        Q = np.zeros((M, M), complex)
        Q[b, b] = 1.0
        baths.append(workloads.Bath(Q, 1.0, dl=[(0.2, 1.0)], n_ltc=1))
    inst = workloads.Instance("3-site", H, baths, 5, "tree2", 6, workloads.ground(M), 0.01, 40)
    print("[ps1 parity] 3-site binary K=6 steps=40 FP64", flush=True)
    _, ro, _, _ = propagate(inst, n_steps=40, every=10)
    rg = run_gpu(inst, 40, 0)
    d = max(trace_distance(a, b) for a, b in zip(rg, ro))
    print(f"  max trace distance = {d:.3e}")
    assert d < 1e-10


def pulsed(A, w, s=0.15, t0=0.3, n_steps=60):
    """The spin-boson model with a sigma_x pulse A exp(-(t-t0)^2/2s^2) cos(w t)
    centred inside the first n_steps * dt."""
    base = workloads.spin_boson_train(n_steps=n_steps)
    return workloads.Instance(f"pulse A={A} w={w}", base.H, base.baths, base.depth, base.tree,
                              base.rank, base.rho0, 0.01, n_steps,
                              drive=(workloads.SX, A, w, s, t0))


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-6)])
def test_ps1_driven_against_oracle(precision, tol):
    require_gpu()
    n = 60
    inst = pulsed(2.0, 3.0, n_steps=n)
    print(f"[ps1 parity] driven spin-boson steps={n} precision={precision}", flush=True)
    _, ro, _, _ = propagate(inst, n_steps=n, every=10)
    _, ru, _, _ = propagate(pulsed(0.0, 3.0, n_steps=n), n_steps=n, every=n)
    assert trace_distance(ro[-1], ru[-1]) > 1e-3  # the pulse matters
    rg = run_gpu(inst, n, precision)
    d = max(trace_distance(a, b) for a, b in zip(rg, ro))
    print(f"  max trace distance = {d:.3e}")
    assert d < tol


def test_batch_driven_against_oracle():
    require_gpu()
    from paper_2603_17711_amd import api
    n = 60
    insts = [pulsed(A, w, n_steps=n) for A, w in [(2.0, 3.0), (1.0, 1.5), (0.5, 0.7)]]
    print(f"[ps1 parity] batch of 3 driven instances steps={n} FP32", flush=True)
    b = api.Batch([api.build_instance(i, precision=api.FP32) for i in insts])
    b.step(n, [i.dt for i in insts], drive_tabs=[api.drive_table(i, n) for i in insts])
    rb = b.rho()
    for k, inst in enumerate(insts):
        _, ro, _, _ = propagate(inst, n_steps=n, every=n)
        d = trace_distance(rb[k], ro[-1])
        print(f"  {inst.name}: trace distance {d:.3e}", flush=True)
        assert d < 1e-6
