"""Bath correlation function features (paper Sec. II A, Eq. bcfdecores).

The BCF C(t) = int J(w) f_BE(beta w) exp(-i w t) dw is written as a sum of
exponentials C(t) = sum_k c_k exp(gamma_k t) and C*(t) = sum_k cbar_k exp(gamma_k t)
by the residue theorem: poles of the spectral density in the lower half plane
plus the poles of the Bose function, either its exact Matsubara poles or
those of its Pade approximant (both named in Sec. II A).

Units: hbar = k_B = 1, beta = 1/T.

Readings (the paper is garbled or silent here):
* The Matsubara residue of f_BE(beta w) in the variable w is 1/beta; the printed
  Eq. bcfdecores takes the residue in beta*w and so omits this factor.
* cbar_k is the conjugate of the coefficient of the feature whose exponent is
  conj(gamma_k) (the "conjugate partner" rule), so that C*(t) = conj(C(t)).
* Feature order per bath: DL features, BO pairs in input order, then the
  n_ltc low-temperature corrections (Matsubara m = 1..n_ltc, or the n_ltc Pade
  poles in increasing order).
* Pade decomposition (reading; the paper names it and cites Hu, Xu & Yan,
  J. Chem. Phys. 133, 101106 (2010) without formulas): the Bose function is
  f_BE(x) = 1/x + 1/2 + x g(x^2) with g regular at 0; g is replaced by its
  [N-1/N] Pade approximant in w = x^2, so that
  f_BE(x) ~ 1/x + 1/2 + sum_j 2 eta_j x / (x^2 + xi_j^2), N = n_ltc.  Only the
  Bose-function poles change: the spectral-density features keep the exact
  f_BE at their poles, as Eq. bcfdecores writes them.  Pole j contributes
  gamma = -xi_j / beta and c = -(2 pi i / beta) eta_j J(-i xi_j / beta)
  (xi_j = 2 pi j, eta_j = 1 is the Matsubara case).

Pins: tests compare sum_k c_k exp(gamma_k t) with direct numerical quadrature
of the defining integral (scipy QAWF), for DL and BO spectral densities; the
Pade approximant is pinned by its N = 1 closed form (xi^2 = 60, eta = 5/2), by
the Bose function on the real axis, and by its BCF converging to the
quadrature faster than Matsubara's.
"""
from fractions import Fraction
from math import factorial
import numpy as np


def f_be(x):
    """Bose factor f_BE(x) = 1 / (1 - exp(-x)) for complex x (Sec. II A)."""
    return 1.0 / (1.0 - np.exp(-x))


def j_dl(w, lam, wc):
    """Drude-Lorentz spectral density, Eq. (DL)."""
    return (2.0 * lam / np.pi) * wc * w / (w * w + wc * wc)


def bo_poles(w0, eta):
    """The four poles of the factored Brownian SD (Sec. II A): +-w0' +- i eta,
    with w0' = sqrt(w0^2 - eta^2)."""
    w0p = np.sqrt(w0 * w0 - eta * eta)
    return w0p, np.array([w0p - 1j * eta, -w0p - 1j * eta,
                          w0p + 1j * eta, -w0p + 1j * eta])


def j_bo(w, lam, w0, eta):
    """Factored Brownian-oscillator SD (Sec. II A, the form TENSO uses)."""
    w0p = np.sqrt(w0 * w0 - eta * eta)
    num = (4.0 * lam * eta / np.pi) * (w0p ** 2 + eta ** 2) * w
    den = ((w + w0p) ** 2 + eta ** 2) * ((w - w0p) ** 2 + eta ** 2)
    return num / den


def _bo_residue(pole, lam, w0, eta):
    """Residue of the factored BO SD at one of its simple poles:
    numerator / product of (pole - other poles)."""
    w0p, poles = bo_poles(w0, eta)
    num = (4.0 * lam * eta / np.pi) * (w0p ** 2 + eta ** 2) * pole
    den = 1.0 + 0j
    for p in poles:
        if abs(p - pole) > 1e-300:
            den *= (pole - p)
    return num / den


def bernoulli(n):
    """Exact Bernoulli numbers B_0..B_n (B_1 = -1/2) from
    sum_{k=0}^{m} binom(m+1, k) B_k = 0."""
    B = [Fraction(1)]
    for m in range(1, n + 1):
        s = Fraction(0)
        for k in range(m):
            s += Fraction(factorial(m + 1), factorial(k) * factorial(m + 1 - k)) * B[k]
        B.append(-s / (m + 1))
    return B


def _solve_exact(A, b):
    """Gaussian elimination over the rationals (A: list of rows of Fractions)."""
    n = len(b)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def pade_bose(N):
    """Poles and weights of the [N-1/N] Pade approximant of the Bose function.

    g(w) = (f_BE(x) - 1/x - 1/2) / x, w = x^2, has the Taylor series
    g(w) = sum_k g_k w^k, g_k = B_{2k+2} / (2k+2)!.  The approximant P/Q
    (deg P = N-1, deg Q = N, Q(0) = 1) matches its first 2N coefficients:
    sum_i q_i g_{k-i} = 0 for k = N..2N-1, and p_k = sum_{i<=k} q_i g_{k-i}.
    The conditions are solved exactly over the rationals; the zeros of Q
    (w = -xi_j^2) and the residues of P/Q there (2 eta_j) in floating point.
    Returns (xi, eta), xi ascending: g(w) ~ sum_j 2 eta_j / (w + xi_j^2)."""
    B = bernoulli(4 * N + 2)
    g = [B[2 * k + 2] / factorial(2 * k + 2) for k in range(2 * N)]
    A = [[g[k - i] for i in range(1, N + 1)] for k in range(N, 2 * N)]
    q = [Fraction(1)] + _solve_exact(A, [-g[k] for k in range(N, 2 * N)])
    pc = [sum(q[i] * g[k - i] for i in range(k + 1)) for k in range(N)]
    # in u = w / (2 pi)^2 the coefficients are O(1) for the root finder
    scale = (2.0 * np.pi) ** 2
    qu = np.array([float(q[i]) * scale ** i for i in range(N + 1)])
    pu = np.array([float(pc[i]) * scale ** i for i in range(N)])
    roots = np.roots(qu[::-1])
    dq = np.polyder(qu[::-1])
    xi, eta = [], []
    for u in roots:
        assert abs(u.imag) <= 1e-9 * abs(u) and u.real < 0, "Pade poles must lie on -w > 0"
        u = float(u.real)
        r = np.polyval(pu[::-1], u) / np.polyval(dq, u)   # residue of P/Q in u
        xi.append(np.sqrt(-u * scale))
        eta.append(0.5 * r * scale)
    order = np.argsort(xi)
    return np.array(xi)[order], np.array(eta)[order]


def f_be_pade(x, N):
    """The Pade form of the Bose factor at real x: 1/x + 1/2 + sum 2 eta x/(x^2+xi^2)."""
    xi, eta = pade_bose(N)
    x = np.asarray(x, dtype=float)
    return 1.0 / x + 0.5 + sum(2.0 * e * x / (x * x + z * z) for z, e in zip(xi, eta))


def bath_features(T, dl=(), bo=(), n_ltc=0, method="matsubara"):
    """Features of one bath: lists (c, cbar, gamma) as complex arrays.

    dl : sequence of (lambda, omega_c) Drude-Lorentz terms
    bo : sequence of (lambda, omega_0, eta) Brownian terms (eta < omega_0)
    n_ltc : number of low-temperature corrections
    method : "matsubara" (poles 2 pi m / beta) or "pade" (the n_ltc poles of
             the [n_ltc-1/n_ltc] Pade approximant)
    """
    beta = 1.0 / T
    c, g = [], []
    partner = []  # index of the feature with exponent conj(gamma)
    # Drude-Lorentz: pole of J at w = -i wc; residue lam*wc/pi.
    for lam, wc in dl:
        res = lam * wc / np.pi
        zeta = -1j * wc
        c.append(-2j * np.pi * res * f_be(beta * zeta))
        g.append(-1j * zeta)
        partner.append(len(c) - 1)
    # Brownian: the two lower-half-plane poles +-w0' - i eta.
    for lam, w0, eta in bo:
        w0p, poles = bo_poles(w0, eta)
        i0 = len(c)
        for zeta in poles[:2]:
            res = _bo_residue(zeta, lam, w0, eta)
            c.append(-2j * np.pi * res * f_be(beta * zeta))
            g.append(-1j * zeta)
        partner.extend([i0 + 1, i0])
    # Bose-function poles at w = -i nu: Matsubara nu_m = 2 pi m / beta with
    # residue 1/beta; Pade nu_j = xi_j / beta with residue eta_j / beta.
    if method == "matsubara":
        poles = [(2.0 * np.pi * m, 1.0) for m in range(1, n_ltc + 1)]
    elif method == "pade":
        poles = list(zip(*pade_bose(n_ltc))) if n_ltc > 0 else []
    else:
        raise ValueError(method)
    for xi, wgt in poles:
        nu = xi / beta
        jv = 0j
        for lam, wc in dl:
            jv += j_dl(-1j * nu, lam, wc)
        for lam, w0, eta in bo:
            jv += j_bo(-1j * nu, lam, w0, eta)
        c.append(-2j * np.pi / beta * wgt * jv)
        g.append(-nu + 0j)
        partner.append(len(c) - 1)
    c = np.array(c, dtype=np.complex128)
    g = np.array(g, dtype=np.complex128)
    cbar = np.conj(c[np.array(partner, dtype=int)]) if len(c) else c.copy()
    return c, cbar, g


def bcf_from_features(t, c, g):
    """sum_k c_k exp(gamma_k t) on an array of times."""
    t = np.asarray(t, dtype=float)
    return (c[None, :] * np.exp(np.outer(t, g))).sum(axis=1)


def bcf_quadrature(t, jfun, T):
    """Direct quadrature of C(t) = int J(w) f_BE(beta w) e^{-iwt} dw, t > 0.

    Uses the oddness of J to fold onto w > 0:
    C(t) = int_0^inf J(w) [coth(beta w/2) cos(wt) - i sin(wt)] dw,
    evaluated with the Fourier-weighted QUADPACK routine (QAWF)."""
    from scipy.integrate import quad
    beta = 1.0 / T

    def re_int(w):
        if w == 0.0:
            return 0.0
        return jfun(w) / np.tanh(0.5 * beta * w)

    out = []
    for ti in np.atleast_1d(t):
        # split off [0, a] where the coth factor varies, QAWF on the tail
        a = 50.0
        r1 = quad(lambda w: re_int(w) * np.cos(w * ti), 0.0, a, limit=800,
                  epsabs=1e-14, epsrel=1e-13)[0]
        r2 = quad(lambda w: re_int(w + a), 0.0, np.inf, weight='cos', wvar=ti,
                  limlst=200, epsabs=1e-14)[0] * np.cos(a * ti) - \
            quad(lambda w: re_int(w + a), 0.0, np.inf, weight='sin', wvar=ti,
                 limlst=200, epsabs=1e-14)[0] * np.sin(a * ti)
        i1 = quad(lambda w: jfun(w) * np.sin(w * ti), 0.0, a, limit=800,
                  epsabs=1e-14, epsrel=1e-13)[0]
        i2 = quad(lambda w: jfun(w + a), 0.0, np.inf, weight='sin', wvar=ti,
                  limlst=200, epsabs=1e-14)[0] * np.cos(a * ti) + \
            quad(lambda w: jfun(w + a), 0.0, np.inf, weight='cos', wvar=ti,
                 limlst=200, epsabs=1e-14)[0] * np.sin(a * ti)
        out.append((r1 + r2) - 1j * (i1 + i2))
    return np.array(out)
