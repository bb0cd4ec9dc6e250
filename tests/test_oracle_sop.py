"""Pins of the oracle's SOP generator and dense HEOM (Sec. II B).

* pure dephasing ([H_S, Q] = 0): closed form of the reduced dynamics;
* lambda = 0: unitary evolution with a non-real H_S (pins the bra conjugation);
* a qubit coupled to ONE undamped harmonic mode: HEOM with two features
  gamma = -+ i w reproduces the exact reduced dynamics obtained by brute force
  in the joint qubit (x) oscillator Hilbert space (pins c vs cbar, ket vs bra
  and a non-commuting coupling operator);
* metric invariance of rho_S, trace preservation and Hermiticity."""
import json
import os

import numpy as np
from scipy.linalg import expm

from oracle.bath import bath_features
from oracle.sop import dense_propagate, heom_terms, metric_abs

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.json")
SZ = np.diag([1.0, -1.0]).astype(complex)
SX = np.array([[0, 1], [1, 0]], complex)
SY = np.array([[0, -1j], [1j, 0]])


def test_term_count_printed():
    gold = json.load(open(GOLD))["sop_term_count"]
    c, cb, g = bath_features(1.0, dl=[(0.1, 1.0)], n_ltc=4)
    terms, dims = heom_terms(0.5 * SZ, [(SZ, (c, cb, g))], 5)
    assert len(terms) == gold["per_feature"] * len(c) + gold["unitary"]
    assert dims == [2, 2] + [5] * len(c)


def test_pure_dephasing_closed_form():
    H, Q = 0.5 * SZ, SZ
    c, cb, g = bath_features(1.0, dl=[(0.1, 1.0)], n_ltc=2)
    terms, dims = heom_terms(H, [(Q, (c, cb, g))], 12)
    rho0 = np.full((2, 2), 0.5, complex)
    dt, n = 0.05, 40
    r = dense_propagate(terms, dims, rho0, dt, n, every=n)[-1]
    t = dt * n
    G = np.sum(c * ((np.exp(g * t) - 1) / g ** 2 - t / g))
    Gs = np.sum(cb * ((np.exp(g * t) - 1) / g ** 2 - t / g))
    q, E = np.array([1.0, -1.0]), np.array([0.5, -0.5])
    ex = np.array([[rho0[a, b] * np.exp(-1j * (E[a] - E[b]) * t
                                       - (q[a] - q[b]) * (q[a] * G - q[b] * Gs))
                    for b in range(2)] for a in range(2)])
    assert np.abs(r - ex).max() < 1e-10


def test_zero_coupling_is_unitary():
    H = 0.5 * SZ + 0.4 * SX + 0.3 * SY
    c, cb, g = bath_features(1.0, dl=[(0.0, 1.0)], n_ltc=1)
    terms, dims = heom_terms(H, [(SX, (c, cb, g))], 4)
    rho0 = np.array([[0.7, 0.2 - 0.1j], [0.2 + 0.1j, 0.3]])
    r = dense_propagate(terms, dims, rho0, 0.1, 30, every=30)[-1]
    U = expm(-1j * H * 3.0)
    assert np.abs(r - U @ rho0 @ U.conj().T).max() < 1e-12


def test_single_harmonic_mode_brute_force():
    w, gg, T = 1.3, 0.25, 1.0
    nb = 1.0 / (np.exp(w / T) - 1.0)
    c = np.array([gg ** 2 * (nb + 1) / (2 * w), gg ** 2 * nb / (2 * w)], complex)
    g = np.array([-1j * w, 1j * w])
    cb = np.conj(c[[1, 0]])
    H = 0.5 * SZ + 0.4 * SX + 0.2 * SY
    Q = SX + 0.3 * SZ
    terms, dims = heom_terms(H, [(Q, (c, cb, g))], [14, 14])
    rho0 = np.array([[1, 0], [0, 0]], complex)
    r = dense_propagate(terms, dims, rho0, 0.1, 50, every=50)[-1]
    nmax = 40
    a = np.diag(np.sqrt(np.arange(1, nmax)), 1)
    x = (a + a.T) / np.sqrt(2 * w)
    Hf = np.kron(H, np.eye(nmax)) + gg * np.kron(Q, x) + np.kron(np.eye(2), w * (a.T @ a))
    rb = np.diag(np.exp(-w * np.arange(nmax) / T))
    rb /= np.trace(rb)
    U = expm(-1j * Hf * 5.0)
    R = U @ np.kron(rho0, rb) @ U.conj().T
    rs = R.reshape(2, nmax, 2, nmax).trace(axis1=1, axis2=3)
    assert np.abs(r - rs).max() < 1e-10


def test_metric_invariance_trace_hermiticity():
    H, Q = 0.5 * SZ + SX, SZ + 0.2 * SX
    c, cb, g = bath_features(1.0, dl=[(0.3, 1.0)], bo=[(0.1, 2.0, 0.3)], n_ltc=1)
    rho0 = np.array([[1, 0], [0, 0]], complex)
    t1, d1 = heom_terms(H, [(Q, (c, cb, g))], 5)
    f2 = metric_abs(c, cb) * np.array([0.5, 2.0, 1.7, 0.3])
    t2, d2 = heom_terms(H, [(Q, (c, cb, g))], 5, metric=f2)
    r1 = dense_propagate(t1, d1, rho0, 0.05, 40, every=10)
    r2 = dense_propagate(t2, d2, rho0, 0.05, 40, every=10)
    assert np.abs(r1 - r2).max() < 1e-12
    for r in r1:
        assert abs(np.trace(r) - 1.0) < 1e-13
        assert np.abs(r - r.conj().T).max() < 1e-13
