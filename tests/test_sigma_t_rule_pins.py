"""Pins of the oracle's sigma_t skewness rule (Sec. 3: sigma_t = lambda + 0.5 exp(-mu S^2) with
S the quartile estimator of the skewness, its quartiles as the paper's footnote defines them, and
lambda = 0.1, mu = 12 for EROS-2), against values fixed by the mathematics: hand-computed
quartiles and skewness of small samples, exact zero skewness of symmetric samples, the bounds of S
and sigma_t, the invariances of S, and the population value ln(4/3) / ln 3 of the exponential
distribution."""
import math

import numpy as np
import pytest

import oracle as O


def test_hand_computed_five_and_four_point_cases():
    # [1, 2, 3, 4, 10]: Q2 = 3, halves [1, 2] and [4, 10] -> Q1 = 1.5, Q3 = 7,
    # S = (7 + 1.5 - 6) / (7 - 1.5) = 5/11
    assert O.hinge_quartiles(np.array([10.0, 3.0, 1.0, 4.0, 2.0])) == (1.5, 3.0, 7.0)
    S = O.bowley_skewness(np.array([10.0, 3.0, 1.0, 4.0, 2.0]))
    assert S == pytest.approx(5.0 / 11.0, rel=1e-15)
    st = O.sigma_t_skewness(np.array([10.0, 3.0, 1.0, 4.0, 2.0]))
    assert st == pytest.approx(0.1 + 0.5 * math.exp(-12.0 * 25.0 / 121.0), rel=1e-15)
    assert st == pytest.approx(0.14190, abs=1e-5)
    # [0, 1, 2, 10]: Q2 = 1.5, halves [0, 1] and [2, 10] -> Q1 = 0.5, Q3 = 6, S = 3.5 / 5.5
    assert O.hinge_quartiles(np.array([2.0, 0.0, 10.0, 1.0])) == (0.5, 1.5, 6.0)
    assert O.bowley_skewness(np.array([2.0, 0.0, 10.0, 1.0])) == pytest.approx(7.0 / 11.0)
    # linear-interpolation quartiles would give Q1 = 2, Q3 = 4 and S = 0 for the first sample
    assert O.quantile(np.array([1.0, 2, 3, 4, 10]), 0.25) == 2.0


def test_symmetric_samples_have_zero_skewness_and_the_widest_kernel():
    rng = np.random.default_rng(5)
    for n in (5, 6, 101, 1000):
        h = rng.normal(size=n // 2)
        x = np.concatenate([h, -h] + ([np.zeros(1)] if n % 2 else [])) + 3.25
        assert O.bowley_skewness(x) == pytest.approx(0.0, abs=1e-14)
        assert O.sigma_t_skewness(x) == pytest.approx(0.6, abs=1e-12)


def test_bounds_and_extremes():
    rng = np.random.default_rng(6)
    for k in range(200):
        n = int(rng.integers(2, 300))
        x = rng.lognormal(0.0, rng.uniform(0.1, 2.0), size=n) * rng.choice([-1.0, 1.0])
        S = O.bowley_skewness(x)
        assert -1.0 <= S <= 1.0
        st = O.sigma_t_skewness(x)
        assert 0.1 <= st <= 0.6
        assert st == pytest.approx(0.1 + 0.5 * math.exp(-12.0 * S * S), rel=1e-15)
    # Q2 = Q1 (median in the lower hinge): S = 1, sigma_t = lambda + 0.5 exp(-mu)
    x = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 5.0, 6.0, 7.0, 8.0])
    assert O.bowley_skewness(x) == 1.0
    assert O.sigma_t_skewness(x) == pytest.approx(0.1 + 0.5 * math.exp(-12.0))
    assert O.bowley_skewness(-x) == -1.0
    # no spread between the quartiles: S = 0 by the stated reading
    assert O.bowley_skewness(np.array([1.0, 2.0, 2.0, 2.0, 2.0, 2.0, 9.0, 2.0])) == 0.0
    # other constants
    assert O.sigma_t_skewness(x, lam=0.2, mu=0.0) == pytest.approx(0.7)


def test_invariances():
    rng = np.random.default_rng(7)
    x = rng.gamma(2.0, size=777)
    S = O.bowley_skewness(x)
    assert S > 0.0
    assert O.bowley_skewness(3.5 * x - 12.0) == pytest.approx(S, rel=1e-12)
    assert O.bowley_skewness(-x) == pytest.approx(-S, rel=1e-12)
    assert O.bowley_skewness(rng.permutation(x)) == S


def test_exponential_population_value():
    # Exponential quartiles ln(4/3), ln 2, ln 4: S = ln(4/3) / ln 3 = 0.26186
    x = np.random.default_rng(8).exponential(size=400001)
    assert O.bowley_skewness(x) == pytest.approx(math.log(4.0 / 3.0) / math.log(3.0), abs=5e-3)


def test_rule_selection():
    y = np.array([10.0, 3.0, 1.0, 4.0, 2.0])
    assert O.sigma_t_of(y, 0.3) == 0.3
    assert O.sigma_t_of(y, O.SIGMA_T_SKEWNESS) == O.sigma_t_skewness(y)
    with pytest.raises(ValueError):
        O.sigma_t_of(y, -2.0)
