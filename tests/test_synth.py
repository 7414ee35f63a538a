"""Generator checks: family moments, counts and reproducibility (no method arithmetic)."""
import math

import numpy as np
import pytest

from paper_2408_17118_amd import synth


def _excess_kurtosis(x):
    x = x - x.mean()
    return (x ** 4).mean() / (x ** 2).mean() ** 2 - 3.0


@pytest.mark.parametrize("kind", ["laplace", "uniform", "gaussian"])
def test_family_kurtosis_within_standard_errors(kind):
    # these families have finite eighth moments, so the sample kurtosis has a
    # standard error ~ sqrt(var(x^4)) / T; check 5 standard errors
    rng = np.random.default_rng(123)
    T = 400_000
    s = synth.draw_sources(rng, [kind], T, nu=5.0)[0]
    k = _excess_kurtosis(s)
    se = np.std(s ** 4) / math.sqrt(T)
    assert abs(k - synth.family_kurtosis(kind)) < 5 * se + 1e-3
    assert abs(s.var() - 1.0) < 5 * np.std(s ** 2) / math.sqrt(T)


def test_sine_moments():
    rng = np.random.default_rng(5)
    s = synth.draw_sources(rng, ["sine"] * 4, 200_000, nu=5.0)
    for row in s:
        # >= 200 periods at T = 2e5: sample moments within 1e-2 of the population
        assert abs(row.var() - 1.0) < 1e-2
        assert abs(_excess_kurtosis(row) - (-1.5)) < 2e-2


def test_student_t_unit_variance():
    rng = np.random.default_rng(6)
    s = synth.draw_sources(rng, ["student_t"], 1_000_000, nu=6.0)[0]
    assert abs(s.var() - 1.0) < 0.02      # heavy tails: loose bound
    assert 1.5 < _excess_kurtosis(s) < 6.0  # population value 3, slow convergence


def test_largest_remainder_counts():
    assert synth.largest_remainder(64, list(synth.EEG_MIX)) == [24, 16, 12, 8, 4]
    assert synth.largest_remainder(128, list(synth.EEG_MIX)) == [48, 32, 24, 16, 8]
    assert synth.largest_remainder(24, list(synth.EEG_MIX)) == [9, 6, 5, 3, 1]
    for n in range(16, 129, 8):
        assert sum(synth.largest_remainder(n, list(synth.EEG_MIX))) == n


def test_workload_shapes_and_reproducibility():
    p = synth.small_mixture()
    assert p.X.shape == (8, 10_000) and p.W0.shape == (256, 8)
    assert p.kinds.count("laplace") == 4 and p.kinds.count("gaussian") == 1
    q = synth.small_mixture()
    assert np.array_equal(p.X, q.X) and np.array_equal(p.W0, q.W0)
    # W0 holds FP32-exact values
    assert np.array_equal(p.W0.astype(np.float32).astype(np.float64), p.W0)
    assert np.allclose(p.X, p.A @ p.S)


def test_batched_shapes():
    shapes = synth.batched_shapes()
    assert len(shapes) == 64
    Ns = [n for n, t, _ in shapes]
    Ts = [t for n, t, _ in shapes]
    assert all(n % 8 == 0 and 16 <= n <= 128 for n in Ns)
    assert all(20_000 <= t <= 500_000 for t in Ts)
    again = synth.batched_shapes()
    assert [(n, t) for n, t, _ in again] == list(zip(Ns, Ts))


@pytest.mark.parametrize("rho", [2 * 2 ** (-10 / 4), 2 * 2 ** (-3 / 4), 2 * 2 ** (1 / 4), 2 * 2 ** (10 / 4)])
def test_generalized_gaussian_moments(rho):
    # kurtosis of the generalised Gaussian: G(5/rho) G(1/rho) / G(3/rho)^2 - 3
    # (rho = 1: Laplace, 3; rho = 2: Gaussian, 0; rho -> inf: uniform, -1.2),
    # checked within 5 standard errors, and unit variance
    g = math.gamma
    kap = g(5 / rho) * g(1 / rho) / g(3 / rho) ** 2 - 3
    rng = np.random.default_rng(17)
    T = 400_000
    s = synth.draw_gg(rng, rho, T)
    assert abs(s.var() - 1.0) < 5 * np.std(s ** 2) / math.sqrt(T)
    se = np.std(s ** 4) / math.sqrt(T)
    assert abs(_excess_kurtosis(s) - kap) < 5 * se + 1e-3


def test_generalized_gaussian_reference_points():
    g = math.gamma
    kap = lambda r: g(5 / r) * g(1 / r) / g(3 / r) ** 2 - 3   # noqa: E731
    assert kap(1.0) == pytest.approx(3.0)                      # Laplace
    assert kap(2.0) == pytest.approx(0.0, abs=1e-12)           # Gaussian
    assert kap(8.0) == pytest.approx(-1.0766, abs=1e-4)
    rhos = synth.gg_rhos()
    assert len(rhos) == 20 and sum(r < 2 for r in rhos) == 10 and sum(r > 2 for r in rhos) == 10
    p = synth.artificial_gg(0, n_gauss=10)
    assert p.N == 30 and p.T == 10_000 and p.kinds[-10:] == ["gaussian"] * 10
