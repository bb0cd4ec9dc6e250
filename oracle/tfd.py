"""Thermofield ML-MCTDH workload (paper Sec. III A 5, "Adaptability of the
Framework to Other Equations of Motion"): the TTN propagates a wavefunction
under d psi/dt = -i H psi, H = H_S + sum_j w_j b_j^dag b_j
+ Q (x) sum_j g_j (b_j + b_j^dag), with a discretised bath.  Test
infrastructure: only tests, smoke() and bench.py's CPU baseline use it.

Readings (the paper names the method and its inputs, not the formulas):
* Thermofield (Tamascelli et al. 2019, T-TEDOPA): a harmonic bath at
  temperature T acts on the system like a zero-temperature bath with the
  thermal spectral density J_T(w) = J(w) f_BE(w / T) on the whole real axis
  (J odd, so J_T >= 0 for every w); its zero-temperature correlation
  integral(J_T(w) exp(-i w t) dw) is the thermal bath correlation function of
  Sec. II A.  The bath starts in its vacuum.
* Discretisation ("TEDOPA", n modes, cut-off L): the n-point Gauss quadrature
  of the measure J_T(w) dw on [-L, L]: modes w_j are its nodes and g_j^2 its
  weights.  This star bath is unitarily equivalent to the n-site TEDOPA chain
  of the same measure; it reproduces the first 2n moments of the measure.
* Spectral density: the factored Brownian form of Sec. II A (oracle.bath.j_bo)
  with the listing's re_b = lambda, width_b = eta and freq_b = the damped
  frequency w0' (so w0 = sqrt(w0'^2 + eta^2)).
* Tree: the system end (dim M) and a bra end of dimension 1 on the root, the
  mode ends (dim `dim`) below it as in the HEOM trees.  rho_S = Tr_bath
  |psi><psi|.

Pins (tests): the quadrature reproduces the moments of the measure; its bath
correlation function equals the direct integral over [-L, L]; J_T vanishes
for w < 0 as T -> 0; the TTN at full rank equals exact dense Schrodinger
propagation up to the RK4 error; Tr rho_S = 1.
"""
import numpy as np

from .bath import j_bo
from .ttn import Tree, initial_state, nary_tree


def thermal_sd(w, lam, w0, eta, T):
    """J_T(w) = J(w) f_BE(w / T), with f_BE(x) = 1 / (1 - exp(-x)) evaluated as
    -1 / expm1(-x) (no cancellation near w = 0) and the limit T J'(0) at w = 0
    (J is odd, so J(h) / h is J'(0) to O(h^2))."""
    scalar = np.ndim(w) == 0
    w = np.atleast_1d(np.asarray(w, dtype=float))
    out = np.empty_like(w)
    zero = w == 0.0
    nz = ~zero
    out[nz] = np.real(j_bo(w[nz], lam, w0, eta)) / (-np.expm1(-w[nz] / T))
    h = 1e-8
    out[zero] = T * np.real(j_bo(h, lam, w0, eta)) / h
    return out[0] if scalar else out


def gauss_bath(lam, w0, eta, T, cutoff, n, panels=4000, order=16):
    """Nodes and couplings (w_j, g_j) of the n-point Gauss quadrature of the
    measure J_T(w) dw on [-cutoff, cutoff]: the measure is first resolved by a
    composite Gauss-Legendre rule (`panels` panels of `order` points, exact to
    rounding for this smooth density), the Stieltjes procedure on that discrete
    measure gives the three-term recurrence of its orthonormal polynomials, and
    the recurrence's Jacobi matrix has the nodes as eigenvalues and
    mu_0 (first eigenvector component)^2 as weights (Golub-Welsch)."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(-cutoff, cutoff, panels + 1)
    x = np.concatenate([0.5 * (lo + hi) + 0.5 * (hi - lo) * xg
                        for lo, hi in zip(edges[:-1], edges[1:])])
    h = np.concatenate([0.5 * (hi - lo) * wg for lo, hi in zip(edges[:-1], edges[1:])])
    m = thermal_sd(x, lam, w0, eta, T) * h
    mu0 = m.sum()
    a = np.zeros(n)
    b = np.zeros(n)          # b[k] = sqrt(beta_k), k >= 1
    p_prev = np.zeros_like(x)
    p = np.ones_like(x) / np.sqrt(mu0)
    for k in range(n):
        a[k] = np.sum(m * x * p * p)
        q = (x - a[k]) * p - (b[k] if k > 0 else 0.0) * p_prev
        if k + 1 < n:
            b[k + 1] = np.sqrt(np.sum(m * q * q))
            p_prev, p = p, q / b[k + 1]
    J = np.diag(a) + np.diag(b[1:], 1) + np.diag(b[1:], -1)
    nodes, vecs = np.linalg.eigh(J)
    weights = mu0 * vecs[0, :] ** 2
    return nodes, np.sqrt(weights)


def tfd_terms(H, Q, omega, g, dim):
    """SOP terms of L = -i H on ends 0 (system), 1 (bra, dimension 1, identity)
    and 2 + j (mode j)."""
    H = np.asarray(H, dtype=np.complex128)
    Q = np.asarray(Q, dtype=np.complex128)
    n = np.arange(dim, dtype=float)
    num = np.diag(n).astype(np.complex128)
    x = (np.diag(np.sqrt(n[1:]), 1) + np.diag(np.sqrt(n[1:]), -1)).astype(np.complex128)
    terms = [{'coef': -1j, 'slot': -1, 'factors': {0: H}}]
    for j, (w, gj) in enumerate(zip(omega, g)):
        e = 2 + j
        terms.append({'coef': -1j * w, 'slot': -1, 'factors': {e: num}})
        terms.append({'coef': -1j * gj, 'slot': -1, 'factors': {0: Q, e: x}})
    return terms, [H.shape[0], 1] + [dim] * len(omega)


def tfd_tree(M, n_modes, dim, rank, n_ary=2):
    """The HEOM tree shape with a bra end of dimension 1."""
    t = nary_tree(M, [dim] * n_modes, n_ary, rank)
    return Tree(t.parent, t.end_node, [M, 1] + [dim] * n_modes, max_rank=rank)


def initial_wavefunction(tree, psi0):
    """psi0 (x) vacuum, padded to the tree's ranks."""
    return initial_state(tree, np.asarray(psi0, dtype=np.complex128).reshape(-1, 1))


def reduced_rho_pure(tree, cores):
    """rho_S[i, j] = sum over the bath of psi[i, ...] conj(psi[j, ...]) for a
    TTN wavefunction (any gauge): each subtree's Gram matrix
    G_s[a, b] = <subtree_b | subtree_a> bottom-up, then the root."""
    def gram(s):
        T = cores[s]
        Tc = T.conj()
        # contract children Grams into T on their legs, keep the parent leg
        for i in reversed(range(len(tree.legs[s]))):
            kind, x = tree.legs[s][i]
            if kind == 'c':
                T = np.moveaxis(np.tensordot(T, gram(x), axes=([i], [0])), -1, i)
        T = T.reshape(T.shape[0], -1)
        return T @ Tc.reshape(Tc.shape[0], -1).T
    A = cores[0]
    legs = tree.legs[0]
    Ag = A
    for i in reversed(range(len(legs))):
        kind, x = legs[i]
        if kind == 'c':
            Ag = np.moveaxis(np.tensordot(Ag, gram(x), axes=([i], [0])), -1, i)
    M = A.shape[0]
    return Ag.reshape(M, -1) @ A.conj().reshape(M, -1).T


def propagate_tfd(inst, n_steps=None, every=10):
    """ps1 propagation of a workloads.TfdInstance; rho_S at every `every`-th
    step and the last.  Returns (steps, rhos)."""
    from .integrators import Propagator
    w, g = gauss_bath(inst.lam, inst.w0, inst.eta, inst.T, inst.cutoff, inst.n_modes)
    terms, _ = tfd_terms(inst.H, inst.Q, w, g, inst.dim)
    tree = tfd_tree(inst.H.shape[0], inst.n_modes, inst.dim, inst.rank, inst.n_ary)
    P = Propagator(tree, terms, initial_wavefunction(tree, inst.psi0))
    n = inst.n_steps if n_steps is None else n_steps
    steps, rhos = [0], [reduced_rho_pure(P.tree, P.C)]
    for s in range(n):
        P.step_ps1(s * inst.dt, inst.dt)
        if (s + 1) % every == 0 or s + 1 == n:
            steps.append(s + 1)
            rhos.append(reduced_rho_pure(P.tree, P.C))
    return np.array(steps), np.array(rhos)
