"""Pins of the oracle's bath features (Sec. II A, Eq. bcfdecores).

The feature sum sum_k c_k exp(gamma_k t) is checked against direct numerical
quadrature of C(t) = int J(w) f_BE(beta w) exp(-iwt) dw; C*(t) against the
complex conjugate; the per-site feature count against the paper's FMO value."""
import json
import os

import numpy as np
import pytest

from oracle.bath import bath_features, bcf_from_features, bcf_quadrature, j_bo, j_dl

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")


@pytest.mark.parametrize("lam,wc,T", [(0.1, 1.0, 1.0), (0.5, 2.0, 0.3)])
def test_dl_features_match_quadrature(lam, wc, T):
    c, cb, g = bath_features(T, dl=[(lam, wc)], n_ltc=600)
    ts = np.array([0.4, 1.0, 2.5])
    ref = bcf_quadrature(ts, lambda w: j_dl(w, lam, wc), T)
    assert np.abs(bcf_from_features(ts, c, g) - ref).max() < 1e-9


def test_bo_and_mixed_features_match_quadrature():
    T = 0.7
    dl, bo = [(0.2, 1.5)], [(0.3, 2.0, 0.4), (0.1, 4.0, 0.2)]
    c, cb, g = bath_features(T, dl=dl, bo=bo, n_ltc=600)
    ts = np.array([0.5, 1.7])
    jf = lambda w: j_dl(w, *dl[0]) + j_bo(w, *bo[0]) + j_bo(w, *bo[1])
    assert np.abs(bcf_from_features(ts, c, g) - bcf_quadrature(ts, jf, T)).max() < 1e-9


def test_conjugate_coefficients():
    c, cb, g = bath_features(0.7, dl=[(0.2, 1.5)], bo=[(0.3, 2.0, 0.4)], n_ltc=3)
    ts = np.linspace(0.0, 3.0, 7)
    assert np.abs(np.conj(bcf_from_features(ts, c, g)) - bcf_from_features(ts, cb, g)).max() < 1e-14


def test_dl_closed_form_high_temperature():
    # For beta*wc -> 0, Re c -> 2 lambda T (classical limit of cot)
    lam, wc, T = 0.1, 1.0, 200.0
    c, cb, g = bath_features(T, dl=[(lam, wc)])
    assert abs(c[0].real / (2 * lam * T) - 1.0) < 1e-5
    assert abs(c[0].imag + lam * wc) < 1e-12
    assert g[0] == -wc


def test_feature_count_fmo_printed():
    gold = json.load(open(GOLD))["fmo_77K_features_per_site"]
    bo = [(l, w0, eta) for (l, w0, eta) in gold["bo_terms"]]
    c, cb, g = bath_features(77.0 * 0.6950348, bo=bo, n_ltc=gold["n_ltc"])
    assert len(c) == gold["features_per_site"]
    assert gold["sites"] * len(c) == gold["features_total"]


# --- Pade decomposition of the Bose function (Sec. II A names it next to
# Matsubara's; the [N-1/N] approximant of Hu, Xu & Yan 2010) ---------------

def test_pade_one_pole_closed_form():
    """N = 1: g(w) = (f_BE(x) - 1/x - 1/2)/x = 1/12 - w/720 + ..., whose
    [0/1] approximant a / (1 + b w) matches a = 1/12 and a b = 1/720: poles at
    w = -60, weight 2 eta = 5."""
    from oracle.bath import pade_bose
    xi, eta = pade_bose(1)
    assert abs(xi[0] - np.sqrt(60.0)) < 1e-13 and abs(eta[0] - 2.5) < 1e-13


def test_pade_bose_factor_on_the_real_axis():
    """On |x| <= 5 the approximant reproduces f_BE(x) far better than the
    Matsubara sum with the same number of poles (a Pade approximant matches 2N
    Taylor coefficients), and its error falls by orders of magnitude per pole."""
    from oracle.bath import f_be, f_be_pade
    x = np.linspace(0.05, 5.0, 400)
    exact = f_be(x)
    mats = lambda N: 1.0 / x + 0.5 + sum(2.0 * x / (x * x + (2 * np.pi * m) ** 2)
                                         for m in range(1, N + 1))
    errs = []
    for N in (1, 2, 3, 4):
        e_p = np.abs(f_be_pade(x, N) - exact).max()
        e_m = np.abs(mats(N) - exact).max()
        print(f"N={N}: Pade {e_p:.2e}, Matsubara {e_m:.2e}")
        assert e_p < 0.1 * e_m
        errs.append(e_p)
    assert all(b < 1e-2 * a for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-10


def test_pade_poles_tend_to_matsubara_frequencies():
    """With many poles the lowest ones approach 2 pi j with unit weight."""
    from oracle.bath import pade_bose
    xi, eta = pade_bose(12)
    j = np.arange(1, 5)
    assert np.abs(xi[:4] - 2 * np.pi * j).max() < 1e-6 and np.abs(eta[:4] - 1).max() < 1e-5


@pytest.mark.parametrize("lam,wc,T", [(0.1, 1.0, 0.3), (0.5, 2.0, 0.2)])
def test_pade_features_converge_to_quadrature_faster(lam, wc, T):
    """The Pade BCF converges to the quadrature of the defining integral as the
    number of low-temperature features grows, and from two features on it is
    closer than Matsubara's with as many (at eight, by more than 10x).  (With a
    single feature at low temperature it need not be: one pole then carries
    the whole Matsubara tail.)"""
    ts = np.array([0.2, 0.7, 2.0])
    ref = bcf_quadrature(ts, lambda w: j_dl(w, lam, wc), T)
    err = {}
    for method in ("matsubara", "pade"):
        for N in (2, 4, 8):
            c, cb, g = bath_features(T, dl=[(lam, wc)], n_ltc=N, method=method)
            err[method, N] = np.abs(bcf_from_features(ts, c, g) - ref).max()
            np.testing.assert_allclose(cb, np.conj(c), atol=0)  # real exponents
    print({k: f"{v:.1e}" for k, v in err.items()})
    for N in (2, 4, 8):
        assert err["pade", N] < err["matsubara", N]
    assert err["pade", 2] > err["pade", 4] > err["pade", 8]
    assert err["pade", 8] < 0.1 * err["matsubara", 8]
