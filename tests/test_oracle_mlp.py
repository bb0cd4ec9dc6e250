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


def test_adam_closed_forms():
    """Adam (Kingma & Ba 2015, Algorithm 1) in closed form: with bias
    correction the first step moves each parameter by lr * g / (|g| + eps);
    under a constant gradient every later step does the same (m_hat = g,
    v_hat = g^2 exactly); and the second step with gradients g1, g2 moves by
    lr * m_hat / (sqrt(v_hat) + eps) with
    m_hat = (b1 (1-b1) g1 + (1-b1) g2) / (1 - b1^2),
    v_hat = (b2 (1-b2) g1^2 + (1-b2) g2^2) / (1 - b2^2)."""
    from oracle.mlp import adam_init, adam_step
    rng = np.random.default_rng(1)
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    params = [(rng.normal(size=(3, 4)), rng.normal(size=3))]
    g1 = [(rng.normal(size=(3, 4)), rng.normal(size=3))]
    g2 = [(rng.normal(size=(3, 4)), rng.normal(size=3))]
    st = adam_init(params)
    p1, st = adam_step(params, g1, st, lr, b1, b2, eps)
    for (p0, q1, ga) in zip(params[0], p1[0], g1[0]):
        np.testing.assert_allclose(p0 - q1, lr * ga / (np.abs(ga) + eps), rtol=1e-12, atol=0)
    p2, st = adam_step(p1, g2, st, lr, b1, b2, eps)
    for (q1, q2, ga, gb) in zip(p1[0], p2[0], g1[0], g2[0]):
        mh = (b1 * (1 - b1) * ga + (1 - b1) * gb) / (1 - b1 ** 2)
        vh = (b2 * (1 - b2) * ga ** 2 + (1 - b2) * gb ** 2) / (1 - b2 ** 2)
        np.testing.assert_allclose(q1 - q2, lr * mh / (np.sqrt(vh) + eps), rtol=1e-10, atol=0)
    # constant gradient: five steps, each of lr * g / (|g| + eps)
    st = adam_init(params)
    p = params
    for _ in range(5):
        q, st = adam_step(p, g1, st, lr, b1, b2, eps)
        for (a, b, ga) in zip(p[0], q[0], g1[0]):
            np.testing.assert_allclose(a - b, lr * ga / (np.abs(ga) + eps), rtol=1e-9, atol=0)
        p = q
