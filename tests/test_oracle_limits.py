"""Weak-coupling and high-temperature limits of the oracle's HEOM generator.

For a system weakly coupled to its bath, the long-time reduced state is fixed
by detailed balance between golden-rule rates in the eigenbasis of H_S (the
secular Pauli master equation; Breuer & Petruccione, Sec. 3.3): for a
two-level system with splitting Omega the populations obey
p_1 / p_0 = S(-Omega) / S(Omega), coherences vanish, and corrections are O(lambda).
S(w) is the bath spectrum, the Fourier transform of the correlation function;
for the exponential decomposition C(t) = sum_k c_k e^{gamma_k t} (t >= 0, paper
Sec. II A, Eq. bcfdecores) it is S(w) = 2 Re sum_k c_k / (-gamma_k - i w).

* With the truncated (finite Matsubara) features, the HEOM steady state must
  approach that golden-rule state linearly in lambda.  Nothing here is taken
  from the oracle's generator: a dropped coupling term, a swapped c / c-bar or
  a wrong sign in the up/down couplings (Sec. II B, Eq. heom-std) breaks
  detailed balance and fails it at O(1).
* The exact bath obeys S(-w) = e^{-beta w} S(w), so as the Matsubara sum
  converges the golden-rule state becomes the Gibbs state e^{-beta H_S}/Z, and
  at high temperature and weak coupling the HEOM steady state is within the
  remaining truncation error of Gibbs.
The steady state is the null vector of the dense generator (the eigenvalue
closest to zero, by shift-invert), normalised to unit trace.
"""
import numpy as np
import pytest
import scipy.linalg as la
import scipy.sparse.linalg as sla

from oracle.bath import bath_features
from oracle.sop import dense_generator, dense_rho, heom_terms
from oracle.ttn import trace_distance

SZ = np.diag([1.0, -1.0]).astype(complex)
SX = np.array([[0, 1], [1, 0]], complex)
H = 0.5 * SZ + SX


def spectrum(c, g, w):
    return 2.0 * np.real(np.sum(c / (-g - 1j * w)))


def golden_rule_state(c, g):
    E, V = la.eigh(H)
    om = E[1] - E[0]
    r = spectrum(c, g, -om) / spectrum(c, g, om)
    p1 = r / (1.0 + r)
    return V @ np.diag([1.0 - p1, p1]) @ V.conj().T


def steady_state(T, lam, n_ltc, N):
    c, cb, g = bath_features(T, dl=[(lam, 1.0)], n_ltc=n_ltc)
    terms, dims = heom_terms(H, [(SZ, (c, cb, g))], N)
    L = dense_generator(terms, dims).tocsc()
    w, v = sla.eigs(L, k=1, sigma=1e-9)
    assert abs(w[0]) < 1e-10
    rho = dense_rho(v[:, 0], dims)
    return rho / np.trace(rho), c, g


@pytest.mark.parametrize("T,n_ltc", [(1.0, 2), (3.0, 2)])
def test_weak_coupling_steady_state_is_golden_rule_state(T, n_ltc):
    d = {}
    for lam in (1e-3, 3e-3, 1e-2):
        rho, c, g = steady_state(T, lam, n_ltc, 3)
        pred = golden_rule_state(c, g)
        d[lam] = trace_distance(rho, pred)
        print(f"T={T} n_ltc={n_ltc} lambda={lam}: D(steady, golden rule) = {d[lam]:.3e}")
        assert d[lam] < 0.25 * lam
    # first order in lambda: tenfold coupling, tenfold deviation
    assert 7.0 < d[1e-2] / d[1e-3] < 13.0


def test_golden_rule_ratio_tends_to_boltzmann_as_matsubara_sum_converges():
    E = la.eigvalsh(H)
    om = E[1] - E[0]
    T = 1.0
    errs = []
    for n in (2, 20, 200):
        c, cb, g = bath_features(T, dl=[(0.1, 1.0)], n_ltc=n)
        r = spectrum(c, g, -om) / spectrum(c, g, om)
        errs.append(abs(r - np.exp(-om / T)))
    print("ratio error vs Boltzmann factor for 2, 20, 200 Matsubara terms:", errs)
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-3


def test_high_temperature_weak_coupling_steady_state_is_gibbs():
    T = 3.0
    rho, _, _ = steady_state(T, 1e-3, 10, 2)
    gibbs = la.expm(-H / T)
    gibbs /= np.trace(gibbs)
    d = trace_distance(rho, gibbs)
    print(f"T=3, lambda=1e-3, 10 Matsubara terms: D(steady, Gibbs) = {d:.3e}")
    assert d < 1e-3
    assert abs(np.trace(rho) - 1) < 1e-12 and np.abs(rho - rho.conj().T).max() < 1e-10
