"""Sum-of-products generator of the bexcitonic HEOM and the dense reference.

Paper Sec. II B: the EDO Omega[i, j, n_1..n_K] obeys dOmega/dt = L(t) Omega
(Eqs. heom-std, EDO-eom) with the dissipator of Eq. (dissipator) and the
sum-of-products form of Eq. (master_lvn): 5 terms per feature plus 2 for the
unitary part.

Conventions (Sec. II B): A^> B = A B acts on the ket leg with matrix A;
A^< B = B A^dagger acts on the bra leg with matrix conj(A).

Ends (open legs) are numbered 0 = ket (dim M), 1 = bra (dim M), 2 + k = feature k
(dim N_k, number basis n = 0..N_k - 1).

Metric (Sec. VII D, reading): z_k = f_k * identity on feature k, with
* 'abs' (the default here): f_k = sqrt((|c_k| + |cbar_k|) / 2);
* 're': f_k = sqrt(|Re c_k + Re cbar_k| / 2), with its sign flipped when
  Im c_k + Im cbar_k exceeds METRIC_EPS (the listing's threshold is not
  printed; a round-off level is taken);
* a complex constant: f_k equal to it for every feature.
Then <n+1| z^-1 a^dag |n> = sqrt(n+1) / f_k and <n| a z |n+1> = f_k sqrt(n+1).
A feature whose factor comes out zero takes f_k = 1.  Every choice is a
similarity transform of the hierarchy that leaves the n = 0 component, and so
rho_S, unchanged, also at finite depth (the transform maps the truncated
subspace onto itself).

A term is a dict {'coef': complex, 'slot': int, 'factors': {end: matrix}}; a
term with slot >= 0 is multiplied by the drive value f_slot(t).  Ends missing
from 'factors' carry the identity (the paper's SparseSPO stores no identities).

Pins (tests): the dense generator reproduces (1) the pure-dephasing closed form,
(2) unitary evolution for lambda = 0 (with a non-real H_S), (3) the exact
reduced dynamics of a qubit coupled to one undamped harmonic mode, computed by
brute force in the joint Hilbert space, and (4) metric invariance of rho_S.
"""
import numpy as np
import scipy.sparse as sp


METRIC_EPS = 1e-14


def metric_abs(c, cbar):
    """TENSO 'abs' metric factor f_k = sqrt((|c_k| + |cbar_k|)/2); a feature
    with c_k = cbar_k = 0 (no coupling) takes f_k = 1, any metric being valid."""
    f = np.sqrt((np.abs(c) + np.abs(cbar)) / 2.0)
    return np.where(f > 0.0, f, 1.0)


def metric_re(c, cbar):
    """TENSO 're' metric factor f_k = sqrt(|Re c_k + Re cbar_k| / 2), negated when
    Im c_k + Im cbar_k > METRIC_EPS; zero becomes 1."""
    c, cbar = np.asarray(c), np.asarray(cbar)
    f = np.sqrt(np.abs(c.real + cbar.real) / 2.0)
    f = np.where(c.imag + cbar.imag > METRIC_EPS, -f, f)
    return np.where(f != 0.0, f, 1.0)


def metric_factors(metric, c, cbar):
    """Per-feature factors for a metric choice: 'abs', 're', a complex constant,
    or an explicit array of factors."""
    if metric is None or (isinstance(metric, str) and metric == 'abs'):
        return metric_abs(c, cbar)
    if isinstance(metric, str) and metric == 're':
        return metric_re(c, cbar)
    if np.isscalar(metric):
        if metric == 0:
            raise ValueError("a metric factor must be nonzero")
        return np.full(len(np.atleast_1d(c)), complex(metric))
    return np.asarray(metric)


def raising(N, f):
    """Matrix of z^-1 a^dagger on the truncated number basis."""
    m = np.zeros((N, N), dtype=np.complex128)
    for n in range(N - 1):
        m[n + 1, n] = np.sqrt(n + 1.0) / f
    return m


def lowering(N, f):
    """Matrix of a z on the truncated number basis."""
    m = np.zeros((N, N), dtype=np.complex128)
    for n in range(N - 1):
        m[n, n + 1] = f * np.sqrt(n + 1.0)
    return m


def number(N):
    return np.diag(np.arange(N, dtype=np.float64)).astype(np.complex128)


def heom_terms(H, baths, depth, drives=(), metric=None):
    """SOP term list of Eq. (master_lvn).

    H      : (M, M) system Hamiltonian
    baths  : list of (Q, (c, cbar, gamma)) -- one coupling operator per bath
    depth  : int or per-feature list, N_k = dimension of feature k
    drives : list of (slot, H_d) time-dependent Hamiltonian terms f_slot(t) H_d
    metric : None or 'abs', 're', a complex constant, or an array of
             per-feature factors f_k
    Returns (terms, end_dims).
    """
    H = np.asarray(H, dtype=np.complex128)
    M = H.shape[0]
    feats = []
    for Q, (c, cb, g) in baths:
        for k in range(len(c)):
            feats.append((np.asarray(Q, dtype=np.complex128), c[k], cb[k], g[k]))
    K = len(feats)
    dims = [depth] * K if np.isscalar(depth) else list(depth)
    if metric is None or isinstance(metric, str) or np.isscalar(metric):
        fk = [metric_factors(metric, np.array([c]), np.array([cb]))[0] for (_, c, cb, _) in feats]
    else:
        fk = list(metric)
    terms = []
    terms.append({'coef': -1j, 'slot': -1, 'factors': {0: H}})
    terms.append({'coef': +1j, 'slot': -1, 'factors': {1: np.conj(H)}})
    for k, (Q, c, cb, g) in enumerate(feats):
        e = 2 + k
        N = dims[k]
        up, dn = raising(N, fk[k]), lowering(N, fk[k])
        terms.append({'coef': g, 'slot': -1, 'factors': {e: number(N)}})
        terms.append({'coef': c, 'slot': -1, 'factors': {0: Q, e: up}})
        terms.append({'coef': -cb, 'slot': -1, 'factors': {1: np.conj(Q), e: up}})
        terms.append({'coef': -1.0, 'slot': -1, 'factors': {0: Q, e: dn}})
        terms.append({'coef': +1.0, 'slot': -1, 'factors': {1: np.conj(Q), e: dn}})
    for slot, Hd in drives:
        Hd = np.asarray(Hd, dtype=np.complex128)
        terms.append({'coef': -1j, 'slot': slot, 'factors': {0: Hd}})
        terms.append({'coef': +1j, 'slot': slot, 'factors': {1: np.conj(Hd)}})
    end_dims = [M, M] + dims
    return terms, end_dims


def term_coef(term, drive_values):
    """coef_m(t): the base coefficient times the drive value of its slot."""
    if term['slot'] >= 0:
        return term['coef'] * drive_values[term['slot']]
    return term['coef']


def dense_generator(terms, end_dims, drive_values=None):
    """Sparse matrix of L = sum_m coef_m kron(factors) on the row-major
    flattening of Omega[e_0, e_1, ...] (Eq. master_lvn written out)."""
    D = int(np.prod(end_dims))
    L = sp.csr_matrix((D, D), dtype=np.complex128)
    for t in terms:
        op = sp.identity(1, dtype=np.complex128, format='csr')
        for e, d in enumerate(end_dims):
            f = t['factors'].get(e)
            op = sp.kron(op, sp.csr_matrix(f) if f is not None
                         else sp.identity(d, dtype=np.complex128), format='csr')
        L = L + term_coef(t, drive_values) * op
    return L.tocsr()


def dense_initial(rho0, end_dims):
    """Omega(0) = rho_S(0) (x) |0...0> (all bexciton numbers zero)."""
    om = np.zeros(end_dims, dtype=np.complex128)
    om[(slice(None), slice(None)) + (0,) * (len(end_dims) - 2)] = rho0
    return om.reshape(-1)


def dense_rho(omega, end_dims):
    """rho_S = <0|Omega> (Sec. II B)."""
    om = omega.reshape(end_dims)
    return om[(slice(None), slice(None)) + (0,) * (len(end_dims) - 2)].copy()


def dense_propagate(terms, end_dims, rho0, dt, n_steps, every=1):
    """Exact propagation of the dense EDO with a time-independent generator
    (scipy expm_multiply).  Returns rho_S at steps 0, every, 2*every, ..."""
    from scipy.sparse.linalg import expm_multiply
    L = dense_generator(terms, end_dims)
    om = dense_initial(rho0, end_dims)
    out = [dense_rho(om, end_dims)]
    for s in range(0, n_steps, every):
        om = expm_multiply(L * (dt * every), om)
        out.append(dense_rho(om, end_dims))
    return np.array(out)
