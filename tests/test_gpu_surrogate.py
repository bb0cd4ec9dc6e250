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
    assert r["train_mse_first_last"][1] < r["train_mse_first_last"][0]
    assert np.isfinite(r["max_feature_error"])
