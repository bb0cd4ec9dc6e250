"""The HEOM metric choices of Sec. VII D ('abs', 're', a complex constant):
the 're' sign rule on hand-worked coefficients, invariance of rho_S under every
choice for the dense (untruncated-rank) hierarchy at finite depth, and the
product's factors against the oracle's."""
import numpy as np

from oracle.bath import bath_features
from oracle.sop import dense_propagate, heom_terms, metric_factors, metric_re

SX = np.array([[0, 1], [1, 0]], complex)
SZ = np.array([[1, 0], [0, -1]], complex)


def test_metric_re_rule_on_worked_values():
    # Re c + Re cbar = 4 -> sqrt(2); Im sum = -2 (not above the threshold): positive
    assert np.isclose(metric_re(np.array([2 + 1j]), np.array([2 - 3j]))[0], np.sqrt(2.0))
    # Re sum = 2 -> 1; Im sum = 3 > 0: negative
    assert np.isclose(metric_re(np.array([1 + 2j]), np.array([1 + 1j]))[0], -1.0)
    # |Re sum| = |-2| -> 1; Im sum = 0: positive
    assert np.isclose(metric_re(np.array([-3 + 0j]), np.array([1 + 0j]))[0], 1.0)
    # Re sum = 0 gives a zero factor, replaced by 1
    assert metric_re(np.array([1j]), np.array([-1j]))[0] == 1.0
    # a complex constant is taken as given for every feature
    f = metric_factors(0.8 + 0.6j, np.ones(3), np.ones(3))
    assert np.all(f == 0.8 + 0.6j)


def test_every_metric_leaves_rho_s_unchanged_at_finite_depth():
    """A metric is a diagonal similarity transform of the hierarchy that keeps
    the truncated subspace and the n = 0 component, so rho_S(t) is the same for
    every choice (dense propagation, depth 5, two features with complex
    coefficients)."""
    H, Q = 0.5 * SZ + SX, SZ + 0.2 * SX
    c, cb, g = bath_features(1.0, dl=[(0.3, 1.0)], bo=[(0.1, 2.0, 0.3)], n_ltc=1)
    rho0 = np.array([[1, 0], [0, 0]], complex)
    out = []
    for m in ("abs", "re", 0.8 + 0.6j, -1.7 + 0.2j):
        t, d = heom_terms(H, [(Q, (c, cb, g))], 5, metric=m)
        out.append(dense_propagate(t, d, rho0, 0.05, 40, every=10))
    fre = metric_factors("re", c, cb)
    assert np.any(fre < 0) or np.any(fre != metric_factors("abs", c, cb))  # distinct choices
    for r in out[1:]:
        assert np.abs(r - out[0]).max() < 1e-12


def test_product_metric_factors_match_oracle():
    from paper_2603_17711_amd.heom import metric_factor
    rng = np.random.default_rng(3)
    c = rng.normal(size=50) + 1j * rng.normal(size=50)
    cb = rng.normal(size=50) + 1j * rng.normal(size=50)
    c[:3], cb[:3] = [1j, 2.0, -1 + 1e-16j], [-1j, -2.0, 1 + 0j]
    for m in ("abs", "re", 0.3 - 1.1j):
        want = metric_factors(m, c, cb)
        got = np.array([metric_factor(m, complex(a), complex(b)) for a, b in zip(c, cb)])
        assert np.allclose(got, want, rtol=1e-15, atol=0), m
