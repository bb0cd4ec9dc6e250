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
