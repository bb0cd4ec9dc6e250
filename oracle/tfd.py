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

from .bath import f_be, j_bo
from .ttn import Tree, initial_state, nary_tree


def thermal_sd(w, lam, w0, eta, T):
    """J_T(w) = J(w) f_BE(w / T) (its limit J'(0) T at w = 0)."""
    w = np.asarray(w, dtype=float)
    small = np.abs(w) < 1e-12
    ws = np.where(small, 1e-12, w)
    out = np.real(j_bo(ws, lam, w0, eta) * f_be(ws / T))
    return out


def gauss_bath(lam, w0, eta, T, cutoff, n, n_fine=400001):
    """Nodes and couplings (w_j, g_j) of the n-point Gauss quadrature of the
    measure J_T(w) dw on [-cutoff, cutoff]: the Stieltjes procedure on a fine
    midpoint rule of the measure gives the three-term recurrence of its
    orthonormal polynomials, whose Jacobi matrix has the nodes as eigenvalues
    and mu_0 (first eigenvector component)^2 as weights (Golub-Welsch)."""
    h = 2.0 * cutoff / n_fine
    x = -cutoff + h * (np.arange(n_fine) + 0.5)
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
