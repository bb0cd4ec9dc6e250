"""Pin of the FP64 reference MLP: gradients vs central finite differences."""
import numpy as np

from oracle.mlp import init_params, loss_and_grads


def test_mlp_gradients_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [7, 9, 8, 3]
    params = init_params(sizes, rng)
    x = rng.normal(size=(5, 7))
    y = rng.normal(size=(5, 3))
    loss, grads = loss_and_grads(params, x, y)
    h = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + h
                lp, _ = loss_and_grads(params, x, y)
                arr[idx] = old - h
                lm, _ = loss_and_grads(params, x, y)
                arr[idx] = old
                assert abs((lp - lm) / (2 * h) - g[idx]) < 1e-8 * max(1.0, abs(g[idx]))
