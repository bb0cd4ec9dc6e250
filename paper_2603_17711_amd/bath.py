"""Bath-correlation features for the GPU path (paper Sec. II A, Eq. bcfdecores).

C(t) = sum_k c_k exp(gamma_k t) from the residues of the spectral density in the
lower half plane (Drude-Lorentz Eq. DL: one pole; factored Brownian form: two
poles at +-w0' - i eta) and of the Bose factor: its Matsubara poles
(nu_m = 2 pi m / beta, residue 1/beta in the frequency variable), or the poles
of its Pade approximant (Hu, Xu & Yan, J. Chem. Phys. 133, 101106 (2010)),
where only those low-temperature poles change.
cbar_k is the conjugate of the coefficient whose exponent is conj(gamma_k).
"""
import numpy as np


def pade_poles(N):
    """Poles xi_j and weights eta_j of the [N-1/N] Pade form of the Bose
    factor, f(x) ~ 1/x + 1/2 + sum_j 2 eta_j x / (x^2 + xi_j^2).

    From Lambert's continued fraction, f(x) - 1/x - 1/2 = coth(x/2)/2 - 1/x =
    x (1/4) / (3 + (x^2/4) / (5 + (x^2/4) / (7 + ...))); its convergent after
    2N levels is the [N-1/N] approximant in w = x^2.  The convergent's
    denominator is det(D + s S) with D = diag(3, 5, .., 4N+1), S the unit
    off-diagonals and s^2 = -w/4, so its zeros are w = -4 / mu^2 for the
    eigenvalues mu of D^-1/2 S D^-1/2 (entries 1/sqrt((2k+1)(2k+3))): xi = 2/mu,
    mu > 0.  The weights are the residues of the convergent A/B at w = -xi^2
    (A, B and B' from the three-term recurrences), halved."""
    if N <= 0:
        return np.zeros(0), np.zeros(0)
    M = 2 * N
    k = np.arange(1, M)
    off = 1.0 / np.sqrt((2 * k + 1) * (2 * k + 3))
    mu = np.linalg.eigvalsh(np.diag(off, 1) + np.diag(off, -1))
    xi = np.sort(2.0 / mu[mu > 0])
    eta = np.empty(N)
    for j, x in enumerate(xi):
        w = -x * x
        a_prev, a_cur = 1.0, 0.0        # A_{-1}, A_0
        b_prev, b_cur = 0.0, 1.0        # B_{-1}, B_0
        db_prev, db_cur = 0.0, 0.0      # dB/dw
        for lvl in range(1, M + 1):
            bk = 2.0 * lvl + 1.0
            ak, dak = (0.25, 0.0) if lvl == 1 else (0.25 * w, 0.25)
            a_prev, a_cur = a_cur, bk * a_cur + ak * a_prev
            db_prev, db_cur = db_cur, bk * db_cur + ak * db_prev + dak * b_prev
            b_prev, b_cur = b_cur, bk * b_cur + ak * b_prev
        eta[j] = 0.5 * a_cur / db_cur
    return xi, eta


def _fbe(z, beta):
    return 1.0 / (1.0 - np.exp(-beta * z))


def _j_at(z, dl, bo):
    """Spectral density (sum of DL and factored BO terms) at complex z."""
    out = 0j
    for lam, wc in dl:
        out += (2.0 * lam / np.pi) * wc * z / (z * z + wc * wc)
    for lam, w0, eta in bo:
        wp = np.sqrt(w0 * w0 - eta * eta)
        out += (4.0 * lam * eta / np.pi) * (wp * wp + eta * eta) * z / (
            ((z + wp) ** 2 + eta * eta) * ((z - wp) ** 2 + eta * eta))
    return out


def features(T, dl=(), bo=(), n_ltc=0, method="matsubara"):
    """(c, cbar, gamma) complex arrays for one bath, ordered DL, BO pairs, then
    the n_ltc low-temperature poles (method "matsubara" or "pade")."""
    beta = 1.0 / T
    cs, gs, part = [], [], []
    for lam, wc in dl:
        # residue lam*wc/pi at -i wc: c = lam wc (cot(beta wc / 2) - i)
        cs.append(lam * wc * (1.0 / np.tan(0.5 * beta * wc) - 1j))
        gs.append(-wc + 0j)
        part.append(len(cs) - 1)
    for lam, w0, eta in bo:
        wp = np.sqrt(w0 * w0 - eta * eta)
        amp = lam * (wp * wp + eta * eta) / wp
        z1, z2 = wp - 1j * eta, -wp - 1j * eta
        i0 = len(cs)
        cs.append(amp * _fbe(z1, beta))
        gs.append(-1j * z1)
        cs.append(-amp * _fbe(z2, beta))
        gs.append(-1j * z2)
        part += [i0 + 1, i0]
    if method == "matsubara":
        low = [(2.0 * np.pi * m, 1.0) for m in range(1, n_ltc + 1)]
    elif method == "pade":
        low = list(zip(*pade_poles(n_ltc)))
    else:
        raise ValueError(f"unknown decomposition {method!r}")
    for xi, wgt in low:
        nu = xi * T
        cs.append(-2j * np.pi * T * wgt * _j_at(-1j * nu, dl, bo))
        gs.append(-nu + 0j)
        part.append(len(cs) - 1)
    c = np.asarray(cs, dtype=np.complex128)
    g = np.asarray(gs, dtype=np.complex128)
    cb = np.conj(c[np.asarray(part, dtype=int)]) if len(c) else c
    return c, cb, g
