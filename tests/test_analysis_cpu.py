"""Host analysis helpers against processes whose answers are known in closed form."""
import math

import numpy as np

from paper_2106_00712_amd import analysis


def _ar1(rho, n_chains, n, seed):
    rng = np.random.default_rng(seed)
    x = np.empty((n_chains, n))
    x[:, 0] = rng.standard_normal(n_chains) / math.sqrt(1 - rho * rho)
    e = rng.standard_normal((n_chains, n))
    for t in range(1, n):
        x[:, t] = rho * x[:, t - 1] + e[:, t]
    return x


def test_autocorrelation_of_ar1_is_geometric():
    """AR(1) x_t = rho x_{t-1} + noise: A(t) = rho^t and tau_int = (1 + rho) / (2 (1 - rho))."""
    rho = 0.8
    a = analysis.autocorrelation(_ar1(rho, 64, 4000, 1), 10)
    assert a[0] == 1.0 or abs(a[0] - 1.0) < 1e-12
    assert np.max(np.abs(a - rho ** np.arange(11))) < 0.02
    tau = analysis.integrated_time(analysis.autocorrelation(_ar1(rho, 64, 4000, 2), 200))
    assert abs(tau - (1 + rho) / (2 * (1 - rho))) < 0.3


def test_white_noise_has_no_autocorrelation():
    a = analysis.autocorrelation(np.random.default_rng(3).standard_normal((32, 5000)), 5)
    assert np.all(np.abs(a[1:]) < 0.01)


def test_percent_overlap_limits():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(10000)
    assert analysis.percent_overlap(x, x) == 1.0 or abs(analysis.percent_overlap(x, x) - 1.0) < 1e-12
    assert analysis.percent_overlap(x, x + 100.0) == 0.0
    # two normals a shift d apart overlap by 2 Phi(-d/2) in the continuum (0.617 at d = 1)
    ov = analysis.percent_overlap(rng.standard_normal(200000), 1.0 + rng.standard_normal(200000), 200,
                                  (-6.0, 7.0))
    assert abs(ov - math.erfc(0.5 / math.sqrt(2.0))) < 0.01


def test_errors_of_independent_samples():
    rng = np.random.default_rng(5)
    m, se = analysis.mean_and_error(rng.standard_normal(10000))
    assert abs(se - 0.01) < 0.001 and abs(m) < 0.05
    m2, se2 = analysis.binned_error(rng.standard_normal(100000), 100)
    assert abs(se2 - 1 / math.sqrt(100000)) < 0.001
    c, ce = analysis.convergence_curve(np.ones((4, 7)))
    assert np.all(c == 1.0) and np.all(ce == 0.0)
