"""FP64 reference multilayer perceptron for the learned surrogate.

The surrogate is not part of the paper; it is this project's addition: a
3-layer MLP (in -> W -> W -> out, SiLU activations, mean-squared-error loss)
that maps a window of reduced density matrices and drive samples to the
reduced density matrix a coarse step ahead.  This module is the plain FP64
forward / backward pass that the GPU training kernels are checked against.

Layout: x is (batch, n_in); W_l is (n_out_l, n_in_l) and b_l is (n_out_l,);
y = x W^T + b.  Loss = mean over batch and outputs of (pred - target)^2.

Pin (tests): gradients agree with central finite differences of the loss.
"""
import numpy as np


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(sizes, rng):
    params = []
    for n_in, n_out in zip(sizes[:-1], sizes[1:]):
        W = rng.normal(size=(n_out, n_in)) * np.sqrt(2.0 / n_in)
        b = np.zeros(n_out)
        params.append((W, b))
    return params


def forward(params, x):
    """Returns (prediction, cache of pre-activations and inputs)."""
    cache = []
    h = x
    for l, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = silu(z) if l < len(params) - 1 else z
    return h, cache


def loss_and_grads(params, x, target):
    pred, cache = forward(params, x)
    diff = pred - target
    loss = np.mean(diff * diff)
    g = 2.0 * diff / diff.size
    grads = [None] * len(params)
    for l in reversed(range(len(params))):
        h, z = cache[l]
        if l < len(params) - 1:
            g = g * silu_grad(z)
        W, b = params[l]
        grads[l] = (g.T @ h, g.sum(axis=0))
        g = g @ W
    return loss, grads


def adam_step(params, grads, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015); state = (t, m, v) lists."""
    t, m, v = state
    t += 1
    out = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, gp) in enumerate(((W, gW), (b, gb))):
            m[l][j] = beta1 * m[l][j] + (1 - beta1) * gp
            v[l][j] = beta2 * v[l][j] + (1 - beta2) * gp * gp
            mh = m[l][j] / (1 - beta1 ** t)
            vh = v[l][j] / (1 - beta2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
        out.append(tuple(new))
    return out, (t, m, v)


def adam_init(params):
    m = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    v = [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
    return (0, m, v)
