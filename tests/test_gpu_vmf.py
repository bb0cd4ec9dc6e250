"""GPU parity of direct (vmf) integration and the mixed strategy against the
oracle (Sec. II C; Sec. VI and VII E: dopri5, the diagonal regularisation,
ps2 then vmf), all in FP64.

* the derivative of every core, element by element, on random root-canonical
  states of a train, a binary and a ternary tree (with and without the
  shift), and at the product initial state whose bond densities are singular;
* trajectories with fixed dopri5 substeps, undriven and with a pulse;
* adaptive steps: the same accepted / rejected substep counts as the oracle
  and rho_S at every step;
* the mixed strategy: the same switch step and rho_S at every step;
* error paths (FP32 plan, wrong plan kind, bad options)."""
import copy

import numpy as np
import pytest

import workloads
from oracle.run import build
from oracle.ttn import initial_state, trace_distance
from oracle.vmf import VmfPropagator, propagate_mix, vmf_derivative
from tests.gpu_util import require_gpu
from tests.oracle_helpers import canonicalize_root, rand_cores

pytestmark = pytest.mark.gpu

SZ, SX = workloads.SZ, workloads.SX


def small(tree="tree2", rank=3, depth=4, n_ltc=3, drive=None, method="ps1", dt=0.01):
    bath = workloads.Bath(SZ, 1.0, dl=[(0.1, 1.0)], n_ltc=n_ltc)
    return workloads.Instance(f"vmf {tree} R={rank}", 0.5 * SZ + SX, [bath], depth, tree, rank,
                              workloads.ground(2), dt, 20, method=method, drive=drive)


def random_state(tree, seed):
    C = rand_cores(tree, np.random.default_rng(seed))
    canonicalize_root(tree, C)
    nrm = np.sqrt(sum(float(np.sum(np.abs(c) ** 2)) for c in C[:1]))
    C[0] = C[0] / nrm
    return C


def plan_for(inst, cores=None):
    from paper_2603_17711_amd import api
    plan = api.build_instance(inst, precision=api.FP64, method=api.VMF)
    if cores is not None:
        plan.import_state(cores)
    return plan


@pytest.mark.parametrize("kind,reg", [("train", 0.0), ("tree2", 0.0), ("tree3", 0.0),
                                      ("tree2", 1e-7)])
def test_vmf_derivative_matches_oracle(kind, reg):
    require_gpu()
    inst = small(kind)
    terms, tree = build(inst)
    C = random_state(tree, 3)
    print(f"[vmf] derivative {kind} reg={reg} ranks={tree.rank[1:]}", flush=True)
    plan = plan_for(inst, C)
    assert plan.shapes() == [tree.shape(s) for s in range(tree.n)]
    want = vmf_derivative(tree, terms, C, None, reg=reg)
    got = plan.vmf_derivative(reg=reg)
    scale = max(np.abs(w).max() for w in want)
    err = max(np.abs(g - w).max() for g, w in zip(got, want))
    print(f"  max |d_gpu - d_oracle| / max|d| = {err / scale:.2e}")
    assert err <= 1e-11 * scale


def test_vmf_derivative_at_the_singular_initial_state():
    """Rank-one bond densities, shift 1e-7: the inverse amplifies rounding by
    up to 1/shift relative to the density's scale."""
    require_gpu()
    inst = small("tree2")
    terms, tree = build(inst)
    C = initial_state(tree, inst.rho0)
    print("[vmf] derivative at the product initial state", flush=True)
    plan = plan_for(inst)
    want = vmf_derivative(tree, terms, C, None, reg=1e-7)
    got = plan.vmf_derivative(reg=1e-7)
    scale = max(np.abs(w).max() for w in want)
    err = max(np.abs(g - w).max() for g, w in zip(got, want))
    print(f"  max |d_gpu - d_oracle| / max|d| = {err / scale:.2e}")
    assert err <= 1e-7 * scale


def _trajectory(inst, C0, n, reg, fixed, rtol=1e-5, atol=1e-7, drive=None):
    terms, tree = build(inst)
    V = VmfPropagator(tree, terms, C0, drive_fn=drive, reg=reg, rtol=rtol, atol=atol,
                      fixed_substeps=fixed)
    plan = plan_for(inst, C0)
    plan.M = 2
    ro, rg = [V.rho()], [plan.rho()]
    for s in range(n):
        V.step(s * inst.dt, inst.dt)
        plan.step_vmf(1, inst.dt, t0=s * inst.dt, rtol=rtol, atol=atol, reg=reg,
                      fixed_substeps=fixed, drive=drive)
        ro.append(V.rho())
        rg.append(plan.rho())
    return ro, rg, V, plan


def test_vmf_fixed_substeps_random_state():
    require_gpu()
    inst = small("tree2")
    _, tree = build(inst)
    C0 = random_state(tree, 5)
    print("[vmf] 30 steps, 2 fixed substeps, random state", flush=True)
    ro, rg, _, _ = _trajectory(inst, C0, 30, 0.0, 2)
    d = max(np.abs(a - b).max() for a, b in zip(ro, rg))
    print(f"  max |rho_gpu - rho_oracle| = {d:.2e}")
    assert d < 1e-11


def test_vmf_fixed_substeps_from_the_initial_state():
    """The physical start (singular densities, shift 1e-7)."""
    require_gpu()
    inst = small("tree2")
    _, tree = build(inst)
    C0 = initial_state(tree, inst.rho0)
    print("[vmf] 30 steps, 2 fixed substeps, product initial state, shift 1e-7", flush=True)
    ro, rg, _, _ = _trajectory(inst, C0, 30, 1e-7, 2)
    d = max(trace_distance(a, b) for a, b in zip(ro, rg))
    print(f"  max trace distance = {d:.2e}")
    assert d < 1e-8


def test_vmf_adaptive_matches_oracle():
    require_gpu()
    inst = small("tree2")
    _, tree = build(inst)
    C0 = random_state(tree, 9)
    print("[vmf] 20 adaptive steps (rtol 1e-6, atol 1e-9)", flush=True)
    ro, rg, V, plan = _trajectory(inst, C0, 20, 0.0, 0, rtol=1e-6, atol=1e-9)
    acc, rej, h = plan.vmf_stats()
    print(f"  gpu accepted {acc} rejected {rej} next h {h:.3e}; oracle {V.ode.accepted} "
          f"{V.ode.rejected} {V.ode.h:.3e}")
    assert (acc, rej) == (V.ode.accepted, V.ode.rejected)
    # the error estimate is a difference of stage sums that cancels to about
    # 1e-8 of the state, so its rounding (and the proposal's) is ~1e-8 relative
    assert abs(h - V.ode.h) <= 1e-6 * V.ode.h
    d = max(np.abs(a - b).max() for a, b in zip(ro, rg))
    print(f"  max |rho_gpu - rho_oracle| = {d:.2e}")
    assert d < 1e-11


def test_vmf_driven_pulse():
    require_gpu()
    drive = (SX, 1.5, 2.0, 0.05, 0.1)
    inst = small("tree2", drive=drive)
    _, tree = build(inst)
    C0 = random_state(tree, 13)
    f = lambda t: np.array([inst.drive_value(t)])
    print("[vmf] driven, 20 steps, 3 fixed substeps", flush=True)
    ro, rg, _, _ = _trajectory(inst, C0, 20, 0.0, 3, drive=f)
    d = max(np.abs(a - b).max() for a, b in zip(ro, rg))
    print(f"  max |rho_gpu - rho_oracle| = {d:.2e}")
    assert d < 1e-11


def test_mix_matches_oracle():
    require_gpu()
    from paper_2603_17711_amd import api
    n, eps, cap = 12, 3e-7, 5
    inst = small("tree2", rank=cap, method="ps2", n_ltc=2, depth=5)
    terms, tree = build(inst)
    print(f"[mix] ps2 (eps {eps}, cap {cap}) then vmf, {n} steps, 2 fixed substeps", flush=True)
    steps, ro, switch, _ = propagate_mix(copy.deepcopy(tree), terms, initial_state(tree, inst.rho0),
                                         inst.dt, n, eps, cap, fixed_substeps=2)
    plan = api.build_instance(inst, precision=api.FP64)
    rg, sw = [plan.rho()], -1
    for s in range(n):
        sw = plan.step_mix(1, inst.dt, eps, cap, t0=s * inst.dt, fixed_substeps=2)
        rg.append(plan.rho())
    print(f"  switch after {sw} ps2 steps (oracle {switch})")
    assert sw == switch and 0 < sw < n
    d = max(trace_distance(a, b) for a, b in zip(ro, rg))
    print(f"  max trace distance = {d:.2e}")
    assert d < 1e-9


def test_vmf_error_paths():
    require_gpu()
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd._lib import TensoError
    inst = small("tree2")
    p32 = api.build_instance(inst, precision=api.FP32)
    with pytest.raises(TensoError, match="EUNSUPPORTED"):
        p32.step_vmf(1, 0.01)
    p64 = api.build_instance(inst, precision=api.FP64)
    with pytest.raises(TensoError, match="EINVAL"):
        p64.step_mix(1, 0.01, 1e-6, 4)          # not a ps2 plan
    with pytest.raises(TensoError, match="EINVAL"):
        p64.step_vmf(1, 0.01, reg=-1.0)
    with pytest.raises(TensoError, match="EINVAL"):
        p64.step_vmf(1, 0.01, rtol=0.0, atol=0.0)
    with pytest.raises(TensoError, match="EUNSUPPORTED"):
        api.build_instance(inst, precision=api.FP32, method=api.VMF)


def test_mix_spin_boson_train_against_stored_oracle():
    """The spin-boson train under the mixed strategy with the default
    tolerances over 100 steps: the same switch, the same accepted and
    rejected substeps, rho_S at every 10th step."""
    require_gpu()
    from paper_2603_17711_amd import api
    from tests.golden.make_golden import load
    inst = workloads.spin_boson_train_mix()
    g = load("mix_spin_boson_train_100.npz", [inst])
    print("[mix] spin-boson train, 100 steps, against the stored oracle", flush=True)
    plan = api.build_instance(inst, precision=api.FP64)
    ds = [trace_distance(plan.rho(), g["rho"][0])]
    sw = -1
    for k in range(1, 11):
        sw = plan.step_mix(10, inst.dt, inst.eps, inst.rank, t0=10 * (k - 1) * inst.dt)
        ds.append(trace_distance(plan.rho(), g["rho"][k]))
    acc, rej, _ = plan.vmf_stats()
    print(f"  switch {sw} (oracle {int(g['switch'])}), substeps {acc}/{rej} "
          f"(oracle {int(g['accepted'])}/{int(g['rejected'])}), max trace distance {max(ds):.2e}")
    assert sw == int(g["switch"])
    assert (acc, rej) == (int(g["accepted"]), int(g["rejected"]))
    assert max(ds) < 1e-9


@pytest.mark.parametrize("atol,ratio", [(1e-7, 2.0), (1e-5, 1.0)])
def test_ps2_atol_rule_matches_oracle(atol, ratio):
    """ps2 with the absolute-threshold rule (ps2_atol, ps2_ratio): the same
    rank at every split as the oracle and the same rho_S."""
    require_gpu()
    from oracle.integrators import Propagator
    from paper_2603_17711_amd import api
    n, cap = 8, 8
    inst = small("tree2", rank=cap, method="ps2", n_ltc=2, depth=5)
    terms, tree = build(inst)
    print(f"[ps2 atol] atol {atol} ratio {ratio}, {n} steps, cap {cap}", flush=True)
    P = Propagator(copy.deepcopy(tree), terms, initial_state(tree, inst.rho0), trunc=(atol, ratio))
    plan = api.build_instance(inst, precision=api.FP64)
    plan.set_ps2_truncation(atol, ratio)
    d = 0.0
    for s in range(n):
        ro = P.step_ps2(s * inst.dt, inst.dt, 0.0, cap)
        plan.step_adaptive(1, inst.dt, 0.0, cap, t0=s * inst.dt)
        assert plan.rank_log() == ro, (s, plan.rank_log(), ro)
        d = max(d, trace_distance(plan.rho(), P.rho()))
    print(f"  ranks of the last step {ro}; max trace distance {d:.2e}")
    assert d < 1e-10


def test_mix_with_the_atol_rule():
    require_gpu()
    from paper_2603_17711_amd import api
    n, cap, trunc = 12, 8, (1e-6, 2.0)
    inst = small("tree2", rank=cap, method="ps2", n_ltc=2, depth=5)
    terms, tree = build(inst)
    print(f"[mix] atol rule {trunc}, cap {cap}, {n} steps", flush=True)
    steps, ro, switch, _ = propagate_mix(copy.deepcopy(tree), terms, initial_state(tree, inst.rho0),
                                         inst.dt, n, 0.0, cap, fixed_substeps=2, trunc=trunc)
    plan = api.build_instance(inst, precision=api.FP64)
    plan.set_ps2_truncation(*trunc)
    rg, sw = [plan.rho()], -1
    for s in range(n):
        sw = plan.step_mix(1, inst.dt, 0.0, cap, t0=s * inst.dt, fixed_substeps=2)
        rg.append(plan.rho())
    print(f"  switch after {sw} ps2 steps (oracle {switch})")
    assert sw == switch and 0 < sw < n
    d = max(trace_distance(a, b) for a, b in zip(ro, rg))
    print(f"  max trace distance = {d:.2e}")
    assert d < 1e-9


def test_vmf_graph_replay_equals_eager():
    """The derivative program replayed from a captured graph gives the same
    bits as eager launches (adaptive steps: the same decisions too)."""
    require_gpu()
    inst = small("tree2")
    _, tree = build(inst)
    C0 = random_state(tree, 21)
    print("[vmf] graph replay against eager launches, 10 adaptive steps", flush=True)
    out = []
    for graph in (True, False):
        plan = plan_for(inst, C0)
        plan.set_graph(graph)
        plan.step_vmf(10, inst.dt, rtol=1e-6, atol=1e-9, reg=0.0)
        out.append((plan.export_state(), plan.vmf_stats()))
    assert out[0][1] == out[1][1]
    for a, b in zip(out[0][0], out[1][0]):
        assert np.array_equal(a, b)
