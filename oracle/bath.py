"""Bath correlation function features (paper Sec. II A, Eq. bcfdecores).

The BCF C(t) = int J(w) f_BE(beta w) exp(-i w t) dw is written as a sum of
exponentials C(t) = sum_k c_k exp(gamma_k t) and C*(t) = sum_k cbar_k exp(gamma_k t)
by the residue theorem: poles of the spectral density in the lower half plane
plus the Matsubara poles of the Bose function.

Units: hbar = k_B = 1, beta = 1/T.

Readings (the paper is garbled or silent here):
* The Matsubara residue of f_BE(beta w) in the variable w is 1/beta; the printed
  Eq. bcfdecores takes the residue in beta*w and so omits this factor.
* cbar_k is the conjugate of the coefficient of the feature whose exponent is
  conj(gamma_k) (the "conjugate partner" rule), so that C*(t) = conj(C(t)).
* Feature order per bath: DL features, BO pairs in input order, Matsubara
  m = 1..n_ltc.

Pins: tests compare sum_k c_k exp(gamma_k t) with direct numerical quadrature
of the defining integral (scipy QAWF), for DL and BO spectral densities.
"""
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


def bath_features(T, dl=(), bo=(), n_ltc=0):
    """Features of one bath: lists (c, cbar, gamma) as complex arrays.

    dl : sequence of (lambda, omega_c) Drude-Lorentz terms
    bo : sequence of (lambda, omega_0, eta) Brownian terms (eta < omega_0)
    n_ltc : number of Matsubara low-temperature corrections
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
    # Matsubara: poles of f_BE(beta w) at w = -i nu_m, residue 1/beta.
    for m in range(1, n_ltc + 1):
        nu = 2.0 * np.pi * m / beta
        jv = 0j
        for lam, wc in dl:
            jv += j_dl(-1j * nu, lam, wc)
        for lam, w0, eta in bo:
            jv += j_bo(-1j * nu, lam, w0, eta)
        c.append(-2j * np.pi / beta * jv)
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
