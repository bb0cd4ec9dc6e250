"""End-to-end learned surrogate at reduced scale: trajectories from the batched
solver, training with the library kernels, monitored rollout with TTN fallback
on held-out seeds, judged against TTN-HEOM.  Reports the error and the gain."""
import numpy as np
import pytest

from tests.gpu_util import require_gpu

pytestmark = pytest.mark.gpu


def test_surrogate_pipeline_small():
    require_gpu()
    from paper_2603_17711_amd import surrogate as S
    print("[surrogate] 384 training + 32 held-out trajectories x 2000 steps", flush=True)
    r = S.experiment(n_train=384, n_held=32, epochs=8)
    print("  ", {k: (round(v, 5) if isinstance(v, float) else v) for k, v in r.items()})
    print(f"  gain {r['gain']:.3f} (TTN-HEOM {r['ttn_heldout_s']:.3f} s against the surrogate's "
          f"{r['surrogate_s']:.3f} s, spot checks {r['spot_s']:.3f} s); median feature error "
          f"{r['median_feature_error']:.2e}, monitor bar 1e-3, trips {r['monitor_trips']}")
    assert r["train_mse_first_last"][1] < r["train_mse_first_last"][0]
    assert np.isfinite(r["max_feature_error"])
    # the gain charges the rollout, the TTN warm-up windows, the spot checks and
    # the fallback runs; tripped spot-checked trajectories reuse their TTN run
    expect = r["rollout_s"] + r["ttn_heldout_s"] * 16 / (r["steps"] // 10 + 1) + r["spot_s"]
    assert r["surrogate_s"] >= expect - 1e-9
    assert abs(r["gain"] - r["ttn_heldout_s"] / r["surrogate_s"]) < 1e-12


def test_forced_monitor_trip_runs_the_ttn_fallback():
    """A monitor that accepts nothing trips every trajectory at its first
    prediction; the fallback must then hand back exactly the TTN-HEOM
    trajectory from that point (same batched solver, same inputs)."""
    require_gpu()
    import workloads
    from paper_2603_17711_amd import surrogate as S
    print("[surrogate] forced trips on 4 trajectories x 400 steps", flush=True)
    n_steps = 400
    held = workloads.driven_spin_boson(workloads.HELDOUT_SEEDS[:4], n_steps)
    rho, _ = S.generate(held, n_steps)
    judge = S.features(rho)
    n_rec = rho.shape[1]
    model = S.MLP(seed=1)  # untrained: its output does not matter here
    f, trip, _ = S.rollout(model, held, judge[:, :S.WINDOW], n_rec, tol=-1.0)
    assert (trip == S.WINDOW).all(), trip
    f, t_fb = S.fallback(held, trip, f, n_steps)
    assert t_fb > 0
    assert np.abs(f[:, S.WINDOW:] - judge[:, S.WINDOW:]).max() < 1e-12
