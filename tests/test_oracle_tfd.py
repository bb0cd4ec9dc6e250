"""Pins of the thermofield ML-MCTDH oracle (oracle/tfd.py): the Gauss
quadrature of the thermal spectral density against adaptive quadrature of its
moments and of its correlation integral, the zero-temperature limit, and the
full-rank TTN wavefunction against exact dense Schrodinger propagation."""
import numpy as np
import scipy.linalg as sla
from scipy.integrate import quad

from oracle.bath import j_bo
from oracle.integrators import Propagator
from oracle.sop import dense_generator
from oracle.tfd import (gauss_bath, initial_wavefunction, reduced_rho_pure, tfd_terms,
                        tfd_tree, thermal_sd)

KB_CM = 0.6950348
LAM, W0P, ETA, CUT = 200.0, 50.0, 10.0, 200.0
W0 = float(np.sqrt(W0P ** 2 + ETA ** 2))
T = 300.0 * KB_CM


def test_gauss_bath_reproduces_the_moments_of_the_measure():
    n = 6
    w, g = gauss_bath(LAM, W0, ETA, T, CUT, n)
    mu0 = quad(lambda x: thermal_sd(x, LAM, W0, ETA, T), -CUT, CUT, limit=400, epsabs=0,
               epsrel=1e-12)[0]
    for k in range(2 * n):
        exact = quad(lambda x: thermal_sd(x, LAM, W0, ETA, T) * x ** k, -CUT, CUT, limit=400,
                     epsabs=0, epsrel=1e-12)[0]
        got = np.sum(g ** 2 * w ** k)
        # the fine midpoint rule of the measure limits the agreement to ~1e-8
        assert abs(got - exact) <= 1e-6 * mu0 * CUT ** k, (k, got, exact)
    assert np.all(np.abs(w) < CUT) and np.all(g > 0)


def test_discrete_bath_correlation_equals_the_integral():
    """sum_j g_j^2 exp(-i w_j t) against integral over [-L, L] of
    J_T(w) exp(-i w t) dw up to 300 fs (t in cm units: fs * 2 pi c)."""
    w, g = gauss_bath(LAM, W0, ETA, T, CUT, 50)
    fs = 2.0 * np.pi * 2.99792458e-5
    for t_fs in (0.0, 20.0, 100.0, 300.0):
        t = t_fs * fs
        re = quad(lambda x: thermal_sd(x, LAM, W0, ETA, T) * np.cos(x * t), -CUT, CUT,
                  limit=800, epsabs=1e-9)[0]
        im = -quad(lambda x: thermal_sd(x, LAM, W0, ETA, T) * np.sin(x * t), -CUT, CUT,
                   limit=800, epsabs=1e-9)[0]
        got = np.sum(g ** 2 * np.exp(-1j * w * t))
        assert abs(got - (re + 1j * im)) < 1e-7 * abs(re + 1j * im) + 1e-8, t_fs


def test_thermal_density_low_temperature_limit():
    x = np.array([-150.0, -30.0, 30.0, 150.0])
    jt = thermal_sd(x, LAM, W0, ETA, 0.5)
    j = np.real(j_bo(x, LAM, W0, ETA))
    assert np.all(np.abs(jt[:2]) < 1e-20)
    assert np.allclose(jt[2:], j[2:], rtol=1e-12)
    # detailed balance J_T(-w) = exp(-w / T) J_T(w)
    jt2 = thermal_sd(np.array([40.0, -40.0]), LAM, W0, ETA, T)
    assert np.isclose(jt2[1], np.exp(-40.0 / T) * jt2[0], rtol=1e-12)


def test_full_rank_ttn_wavefunction_equals_dense_schrodinger():
    H = np.array([[-0.7, 0.3], [0.3, 0.7]], complex)
    Q = np.diag([-0.5, 0.5]).astype(complex)
    w = np.array([-0.8, 0.4, 1.1])
    g = np.array([0.3, 0.5, 0.2])
    terms, dims = tfd_terms(H, Q, w, g, 3)
    tree = tfd_tree(2, 3, 3, rank=64)
    psi0 = np.array([0.0, 1.0], complex)
    P = Propagator(tree, terms, initial_wavefunction(tree, psi0))
    L = dense_generator(terms, dims).toarray()
    v0 = np.zeros(int(np.prod(dims)), complex)
    v0[1 * 27] = 1.0   # psi0 (x) bra 0 (x) vacuum, row-major over (2, 1, 3, 3, 3)
    dt, n = 0.02, 50
    for s in range(n):
        P.step_ps1(s * dt, dt)
    v = sla.expm(L * dt * n) @ v0
    psi = v.reshape(2, -1)
    rho_exact = psi @ psi.conj().T
    rho = reduced_rho_pure(P.tree, P.C)
    assert np.abs(rho - rho_exact).max() < 1e-9
    assert abs(np.trace(rho) - 1.0) < 1e-9


def test_product_star_bath_matches_oracle():
    """The product's star bath (Lanczos on its own Gauss-Legendre resolution of
    the measure) against the oracle's (Stieltjes on another)."""
    from paper_2603_17711_amd.mctdh import star_bath, thermal_density
    w1, g1 = gauss_bath(LAM, W0, ETA, T, CUT, 50)
    w2, g2 = star_bath(LAM, W0, ETA, T, CUT, 50)
    assert np.abs(w1 - w2).max() < 1e-9 * CUT
    assert (np.abs(g1 - g2) / g1).max() < 1e-9
    x = np.array([-120.0, -1e-9, 0.0, 3.0, 77.0])
    assert np.allclose(thermal_density(x, LAM, W0, ETA, T), thermal_sd(x, LAM, W0, ETA, T),
                       rtol=1e-6, atol=0)
