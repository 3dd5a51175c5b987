"""Pins for the oracle's series coefficients (Sec. III, Sec. IV.A, Appendix A)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import binom

from oracle import zf_oracle as O


def _golden(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "appendix_a_m2.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            vals[k] = Fraction(v)
    return vals


def test_x_form_coefficients_match_appendix_a(golden_dir):
    g = _golden(golden_dir)
    assert O.x_coefficients(2) == [g["a0"], g["a1"], g["a2"]]


def test_error_polynomial_matches_appendix_a(golden_dir):
    g = _golden(golden_dir)
    f = O.error_polynomial(2)
    # X_{n+1} - I has no constant, linear or quadratic term (a = b = 0, Sec. IV.A)
    assert f[:3] == [0, 0, 0]
    assert f[3:] == [g["c"], g["d"], g["e"]]


def test_delta_coefficients_are_binomial_series_of_inverse_sqrt():
    # (1 - d)^(-1/2) = sum_k binom(-1/2, k) (-d)^k, an independent library evaluation
    for m in range(1, 8):
        c = O.delta_coefficients(m)
        for k, ck in enumerate(c):
            assert float(ck) == pytest.approx(binom(-0.5, k) * (-1) ** k, rel=1e-15)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_error_polynomial_order_and_ratio_bound(m):
    f = O.error_polynomial(m)
    # lowest surviving power is m + 1: convergence of order nu_max = m + 1 (Sec. III)
    assert all(x == 0 for x in f[: m + 1])
    assert f[m + 1] != 0
    # the sum of |coefficients| of f / e^(m+1) is exactly 1, so the ratio
    # ||X_{n+1} - I|| / ||X_n - I||^(m+1) < 1 whenever ||X_n - I|| < 1 (Eq. stopL2)
    assert sum(abs(x) for x in f) == 1
    # X = 0 (e = -1) is mapped to 0: f(-1) = -1
    assert sum(x * (-1) ** k for k, x in enumerate(f)) == -1


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_scalar_map_matches_error_polynomial(m):
    # the oracle's scalar map x -> x p(1-x)^2 against the exact polynomial
    f = O.error_polynomial(m)
    for x in np.linspace(0.05, 1.95, 39):
        e = x - 1.0
        expect = 1.0 + sum(float(fk) * e ** k for k, fk in enumerate(f))
        assert O.scalar_map(float(x), m) == pytest.approx(expect, rel=1e-12, abs=1e-14)


def test_stop_rule_algorithm_2():
    # Err[i] > Err[i-1]^3 stops (strict), equality continues, i = 0 never stops
    assert not O.stop_now(0, 5.0, None, 2, "ratio")
    assert O.stop_now(1, 1e-2, 1e-1, 2, "ratio") is True          # 1e-2 > 1e-3
    assert O.stop_now(1, 1e-4, 1e-1, 2, "ratio") is False         # 1e-4 < 1e-3
    assert O.stop_now(1, 0.125, 0.5, 2, "ratio") is False         # tie continues
    assert O.stop_now(2, 2.0, 3.0, 2, "ratio") is False           # large errors keep going
    assert O.stop_now(1, 1e-3, 1e-1, 3, "ratio") is True          # m = 3: 1e-3 > 1e-4
    assert O.stop_now(1, 1e-5, 1e-1, 3, "ratio") is False         # m = 3: 1e-5 < 1e-4
    assert O.stop_now(1, 1.0, 1.0, 2, "monotone") is True
    assert O.stop_now(1, 0.9, 1.0, 2, "monotone") is False
    assert math.isclose(float(Fraction(5, 8) + Fraction(15, 64) + Fraction(9, 64)), 1.0)
