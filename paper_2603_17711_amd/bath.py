"""Bath-correlation features for the GPU path (paper Sec. II A, Eq. bcfdecores).

C(t) = sum_k c_k exp(gamma_k t) from the residues of the spectral density in the
lower half plane (Drude-Lorentz Eq. DL: one pole; factored Brownian form: two
poles at +-w0' - i eta) and of the Bose factor (Matsubara frequencies
nu_m = 2 pi m / beta, residue 1/beta in the frequency variable).
cbar_k is the conjugate of the coefficient whose exponent is conj(gamma_k).
"""
import numpy as np


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


def features(T, dl=(), bo=(), n_ltc=0):
    """(c, cbar, gamma) complex arrays for one bath, ordered DL, BO pairs, Matsubara."""
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
    for m in range(1, n_ltc + 1):
        nu = 2.0 * np.pi * m * T
        cs.append(-2j * np.pi * T * _j_at(-1j * nu, dl, bo))
        gs.append(-nu + 0j)
        part.append(len(cs) - 1)
    c = np.asarray(cs, dtype=np.complex128)
    g = np.asarray(gs, dtype=np.complex128)
    cb = np.conj(c[np.asarray(part, dtype=int)]) if len(c) else c
    return c, cb, g
