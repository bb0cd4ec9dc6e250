"""Host-side pieces of the surrogate's monitor: the qubit trace distance on
features equals half the trace norm of the difference (eigenvalues), and the
trace/positivity check accepts states and rejects non-states."""
import numpy as np

from paper_2603_17711_amd.surrogate import feature_trace_distance, monitor_ok


def rho(f):
    return np.array([[f[0], f[2] + 1j * f[3]], [f[2] - 1j * f[3], f[1]]])


def test_feature_trace_distance_is_half_the_trace_norm():
    rng = np.random.default_rng(0)
    for _ in range(50):
        a, b = rng.normal(size=4), rng.normal(size=4)
        ref = 0.5 * np.abs(np.linalg.eigvalsh(rho(a) - rho(b))).sum()
        assert abs(feature_trace_distance(a, b) - ref) < 1e-12
    # orthogonal pure states are at distance 1, a state from itself at 0
    assert abs(feature_trace_distance([1, 0, 0, 0], [0, 1, 0, 0]) - 1) < 1e-15
    assert feature_trace_distance([0.3, 0.7, 0.1, -0.2], [0.3, 0.7, 0.1, -0.2]) == 0


def test_monitor_accepts_states_and_rejects_non_states():
    assert monitor_ok([1.0, 0.0, 0.0, 0.0])            # pure |0><0|
    assert monitor_ok([0.5, 0.5, 0.5, 0.0])            # pure |+><+|
    assert not monitor_ok([0.6, 0.5, 0.0, 0.0])        # trace 1.1
    assert not monitor_ok([0.5, 0.5, 0.6, 0.0])        # eigenvalue -0.1
    assert monitor_ok([0.5, 0.5, 0.5005, 0.0])         # eigenvalue -5e-4, within 1e-3
