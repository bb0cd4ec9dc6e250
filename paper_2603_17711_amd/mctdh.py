"""Thermofield ML-MCTDH on the same tree and kernels (paper Sec. III A 5):
a wavefunction TTN propagated by d psi/dt = -i H psi with
H = H_S + sum_j w_j b_j^dag b_j + Q (x) sum_j g_j (b_j + b_j^dag).

The finite-temperature harmonic bath enters as a zero-temperature star bath
whose modes are the n-point Gauss quadrature of the thermal spectral density
J_T(w) = J(w) / (1 - exp(-w / T)) on [-cutoff, cutoff] (thermofield / T-TEDOPA:
nodes w_j, couplings g_j = sqrt(weights); the star is equivalent to the
n-site TEDOPA chain).  J is the factored Brownian density of Sec. II A.
The tree is the HEOM tree with a bra end of dimension 1; the state starts as
psi_0 (x) vacuum; rho_S = Tr_bath |psi><psi| comes from the root core on the
device (tenso_reduced_rho_pure).
"""
import numpy as np

from .api import FP32, PS1, Generator, Plan, Tree
from .heom import TermTable


def brownian_sd(w, lam, w0, eta):
    """Factored Brownian spectral density (odd in w)."""
    wp2 = w0 * w0 - eta * eta
    return (4.0 * lam * eta / np.pi) * w0 * w0 * w / (
        ((w + np.sqrt(wp2)) ** 2 + eta * eta) * ((w - np.sqrt(wp2)) ** 2 + eta * eta))


def thermal_density(w, lam, w0, eta, T):
    """J(w) / (1 - exp(-w / T)); its limit T J'(0) = T 4 lam eta / (pi w0^2) at w = 0."""
    w = np.atleast_1d(np.asarray(w, dtype=float))
    out = np.empty_like(w)
    small = np.abs(w) < 1e-8 * T
    big = ~small
    out[big] = brownian_sd(w[big], lam, w0, eta) / (-np.expm1(-w[big] / T))
    out[small] = 4.0 * lam * eta / (np.pi * w0 * w0) * T
    return out


def star_bath(lam, w0, eta, T, cutoff, n, panels=2000, order=20):
    """(w_j, g_j): Gauss quadrature of the measure J_T(w) dw on [-cutoff,
    cutoff], by the Lanczos process on a composite Gauss-Legendre
    discretisation of the measure (full reorthogonalisation): the Jacobi
    matrix's eigenvalues are the nodes, mu_0 times the squared first
    components of its eigenvectors the weights."""
    xg, wg = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(-cutoff, cutoff, panels + 1)
    half = 0.5 * (edges[1:] - edges[:-1])
    mid = 0.5 * (edges[1:] + edges[:-1])
    x = (mid[:, None] + half[:, None] * xg[None, :]).reshape(-1)
    m = (half[:, None] * wg[None, :]).reshape(-1) * thermal_density(x, lam, w0, eta, T)
    mu0 = m.sum()
    s = np.sqrt(m / mu0)
    V = np.zeros((x.size, n))
    alpha, beta = np.zeros(n), np.zeros(n)
    v = s.copy()
    for k in range(n):
        V[:, k] = v
        u = x * v
        alpha[k] = v @ u
        u = u - alpha[k] * v - (beta[k] * V[:, k - 1] if k > 0 else 0.0)
        u = u - V[:, :k + 1] @ (V[:, :k + 1].T @ u)  # reorthogonalise
        if k + 1 < n:
            beta[k + 1] = np.linalg.norm(u)
            v = u / beta[k + 1]
    Jm = np.diag(alpha) + np.diag(beta[1:], 1) + np.diag(beta[1:], -1)
    nodes, vec = np.linalg.eigh(Jm)
    return nodes, np.sqrt(mu0 * vec[0] ** 2)


def tfd_table(H, Q, w, g, dim):
    """SOP table of L = -i H: ends 0 (system), 1 (dimension 1), 2 + j modes."""
    H = np.asarray(H, dtype=np.complex128)
    Q = np.asarray(Q, dtype=np.complex128)
    tab = TermTable()
    tab.add(-1j, [(0, H)])
    k = np.arange(dim, dtype=float)
    num = np.diag(k).astype(np.complex128)
    xop = (np.diag(np.sqrt(k[1:]), 1) + np.diag(np.sqrt(k[1:]), -1)).astype(np.complex128)
    for j in range(len(w)):
        tab.add(-1j * w[j], [(2 + j, num)])
        tab.add(-1j * g[j], [(0, Q), (2 + j, xop)])
    return tab


def nary_topology(n_modes, n_ary):
    """(parent, end_node) of the balanced n-ary tree over the mode ends, with
    ends 0 and 1 on the root: a list of modes becomes an end if it has one
    element, a node holding them if it has at most n_ary, else a node over
    n_ary contiguous near-equal chunks (larger first); preorder numbering."""
    parent = [-1]
    end_node = [0, 0] + [0] * n_modes

    def place(modes, holder):
        if len(modes) == 1:
            end_node[2 + modes[0]] = holder
            return
        me = len(parent)
        parent.append(holder)
        if len(modes) <= n_ary:
            for f in modes:
                end_node[2 + f] = me
            return
        q, r = divmod(len(modes), n_ary)
        i = 0
        for c in range(n_ary):
            sz = q + (1 if c < r else 0)
            place(modes[i:i + sz], me)
            i += sz

    if n_modes:
        place(list(range(n_modes)), 0)
    return parent, end_node


def build_tfd(inst, precision=FP32):
    """Plan and initial state for a workloads.TfdInstance."""
    lam, w0, eta = inst.lam, inst.w0, inst.eta
    w, g = star_bath(lam, w0, eta, inst.T, inst.cutoff, inst.n_modes)
    tab = tfd_table(inst.H, inst.Q, w, g, inst.dim)
    parent, end_node = nary_topology(inst.n_modes, inst.n_ary)
    M = inst.H.shape[0]
    tree = Tree.from_parents(parent, end_node, [M, 1] + [inst.dim] * inst.n_modes, inst.rank)
    plan = Plan(tree, Generator(tree, tab), precision=precision, method=PS1, max_rank=inst.rank)
    plan.init_state(np.asarray(inst.psi0, dtype=np.complex128).reshape(M, 1))
    plan.M = M
    return plan
