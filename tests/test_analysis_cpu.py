"""Pins of the autocorrelation-time estimator used by the benchmark's multi-hit measurement.

An AR(1) series x_t = rho x_{t-1} + noise has autocorrelation rho^t and
integrated time (1 + rho) / (2 (1 - rho)) exactly; white noise has 1/2; a
series of independent blocks of length b (each value repeated b times) has
rho(t) = 1 - t/b for t < b, so tau_int = b / 2 exactly in the limit.
"""
import numpy as np
import pytest

from paper_1006_3865_amd import analysis


def ar1(rho, n, seed):
    rng = np.random.default_rng(seed)
    e = rng.standard_normal(n)
    x = np.empty(n)
    x[0] = e[0] / np.sqrt(1 - rho * rho)
    for t in range(1, n):
        x[t] = rho * x[t - 1] + e[t]
    return x


@pytest.mark.parametrize("rho", [0.0, 0.5, 0.9, 0.98])
def test_ar1_integrated_time(rho):
    x = ar1(rho, 400_000, 11 + int(100 * rho))
    tau, w, err = analysis.tau_int(x)
    exact = (1 + rho) / (2 * (1 - rho))
    assert abs(tau - exact) < 4 * err + 0.02 * exact, (tau, exact, err, w)


def test_autocorrelation_of_ar1_matches_powers():
    x = ar1(0.8, 400_000, 3)
    r = analysis.autocorrelation(x)
    assert r[0] == pytest.approx(1.0)
    for t in (1, 2, 5, 10):
        assert r[t] == pytest.approx(0.8 ** t, abs=0.01)


def test_repeated_blocks():
    rng = np.random.default_rng(5)
    b = 20
    x = np.repeat(rng.standard_normal(20_000), b)
    tau, w, err = analysis.tau_int(x)
    assert abs(tau - b / 2) < 4 * err + 0.05 * b, (tau, err)


def test_constant_and_short_series():
    tau, w, err = analysis.tau_int(np.ones(100))
    assert tau == 0.5
    with pytest.raises(ValueError):
        analysis.autocorrelation([1.0])


def test_exact_u_c_against_enumeration_and_independent_kaufman():
    import exact_ising as ex
    for beta in (0.3, ex.BETA_C, 0.6):
        u, c = analysis.exact_u_c(4, beta)
        en = ex.enumeration_averages(4, beta)
        assert u == pytest.approx(en["u"], abs=1e-12)
        assert c == pytest.approx(en["c"], abs=1e-10)
    for L in (8, 64):
        u, c = analysis.exact_u_c(L, ex.BETA_C)
        assert u == pytest.approx(ex.kaufman_u(L, ex.BETA_C), abs=1e-12)
        assert c == pytest.approx(ex.kaufman_c(L, ex.BETA_C), abs=1e-10)


def test_exact_u_approaches_onsager():
    import exact_ising as ex
    u, _ = analysis.exact_u_c(256, 0.3)
    assert u == pytest.approx(ex.onsager_u(0.3), abs=1e-9)


def test_energy_stats_on_independent_gaussians():
    rng = np.random.default_rng(9)
    N, beta, mu, sd = 100, 0.5, -150.0, 12.0
    E = rng.normal(mu, sd, 200_000)
    u, du, c, dc = analysis.energy_stats(E, N, beta)
    assert abs(u - mu / N) < 4 * du and du == pytest.approx(sd / N / np.sqrt(E.size), rel=0.3)
    c_true = beta * beta * sd * sd / N
    assert abs(c - c_true) < 4 * dc and dc == pytest.approx(c_true * np.sqrt(2 / E.size), rel=0.3)
