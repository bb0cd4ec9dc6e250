"""Helpers shared by the oracle tests (canonicalisation and brute force)."""
import numpy as np

from oracle.integrators import qr_toward
from oracle.ttn import Envs, contract_dense, mode_product


def rand_terms(dims, nt, rng, max_factors=2):
    terms = []
    for _ in range(nt):
        k = int(rng.integers(1, max_factors + 1))
        es = rng.choice(len(dims), size=k, replace=False)
        f = {int(e): rng.normal(size=(dims[e], dims[e])) + 1j * rng.normal(size=(dims[e], dims[e]))
             for e in es}
        terms.append({'coef': rng.normal() + 1j * rng.normal(), 'slot': -1, 'factors': f})
    return terms


def rand_cores(tree, rng):
    return [rng.normal(size=tree.shape(s)) + 1j * rng.normal(size=tree.shape(s))
            for s in range(tree.n)]


def canonicalize_root(tree, C):
    for s in reversed(range(1, tree.n)):
        Q, R = qr_toward(C[s], 0)
        C[s] = Q
        p = tree.parent[s]
        C[p] = mode_product(C[p], R, tree.leg_of_child(p, s))


def path_to(tree, c):
    p = [c]
    while p[-1] != 0:
        p.append(tree.parent[p[-1]])
    return p[::-1]


def canonical_envs(tree, terms, C, center):
    """Make C canonical toward `center` in place and return its environments."""
    canonicalize_root(tree, C)
    env = Envs(tree, terms)
    for s in reversed(range(1, tree.n)):
        env.update_down(s, C[s])
    pth = path_to(tree, center)
    for a, b in zip(pth[:-1], pth[1:]):
        i = tree.leg_of_child(a, b)
        Q, R = qr_toward(C[a], i)
        C[a], C[b] = Q, mode_product(C[b], R, 0)
        env.update_up(b, C[a])
    return env


def brute_gradient(tree, C, node, LOm, substitute=None):
    """d<Omega, L Omega>/d conj(X) by enumerating unit tensors X.
    substitute(E, U) puts the unit tensor U into the core list E."""
    shape = C[node].shape if substitute is None else substitute.shape
    out = np.zeros(shape, dtype=np.complex128)
    for idx in np.ndindex(shape):
        U = np.zeros(shape, dtype=np.complex128)
        U[idx] = 1.0
        E = list(C)
        if substitute is None:
            E[node] = U
        else:
            E = substitute(E, U)
        out[idx] = np.vdot(contract_dense(tree, E).reshape(-1), LOm)
    return out
