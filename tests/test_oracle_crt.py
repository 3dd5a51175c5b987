"""Pins of the oracle's residue-emulated FP64 products (row truncation to beta-bit
integers, exact integer product; Ozaki, Uchino & Imamura's scheme II), each against
something other than the oracle's own formula: exact rational arithmetic, integer
matrices, hand-derived values of beta, odd symmetry and exact power-of-two scaling."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs


def _exact_product(A, B):
    """A B^T in exact rational arithmetic (every double is a dyadic rational)."""
    Af = [[Fraction(float(x)) for x in row] for row in A]
    Bf = [[Fraction(float(x)) for x in row] for row in B]
    return [[sum(a * b for a, b in zip(ra, rb)) for rb in Bf] for ra in Af]


def test_moduli_pairwise_coprime_and_int8_residues():
    mods = O.CRT_MODULI
    assert all(math.gcd(a, b) == 1 for i, a in enumerate(mods) for b in mods[:i])
    # balanced residues lie in [-(m // 2), (m - 1) // 2], inside int8 for m <= 256
    assert max(mods) <= 256 and min(mods) >= 2


def test_beta_hand_values():
    """log2 of the product of the first 14 moduli is 110.16 (by hand: 8 + 7.994 +
    7.983 + 7.971 + 7.948 + 7.913 + 7.901 + 7.864 + 7.839 + 7.827 + 7.801 + 7.762 +
    7.721 + 7.636), so 4 K 4^beta <= M gives beta = floor((110.16 - 2 - log2 K) / 2):
    48 for K = 4096, 47 for K = 16384, 50 for K = 128; 15 moduli (117.78) give 51 at
    K = 4096, and 52 (the cap) at K = 128; 13 moduli (102.52) give 44."""
    assert O.crt_beta(4096, 14) == 48
    assert O.crt_beta(16384, 14) == 47
    assert O.crt_beta(128, 14) == 50
    assert O.crt_beta(4096, 15) == 51
    assert O.crt_beta(128, 15) == 52
    assert O.crt_beta(4096, 13) == 44


def test_integer_matrices_are_exact():
    """Integer entries whose row maximum has exponent e keep every bit when beta >= e,
    so the product is the exact integer product."""
    rng = np.random.default_rng(2)
    A = rng.integers(-1000, 1001, (8, 50)).astype(float)
    B = rng.integers(-1000, 1001, (5, 50)).astype(float)
    for L in (10, 14):
        np.testing.assert_array_equal(O.crt_product(A, B, L), A @ B.T)


@pytest.mark.parametrize("L", [10, 12, 14])
def test_product_within_bound_of_exact(L):
    rng = np.random.default_rng(L)
    # entries spanning e^(+-5) inside each row, rows spanning 2^(+-20)
    A = rng.standard_normal((7, 33)) * np.exp(rng.uniform(-5, 5, (7, 33))) * \
        np.ldexp(1.0, rng.integers(-20, 21, (7, 1)))
    B = rng.standard_normal((6, 33))
    beta = O.crt_beta(33, L)
    C = O.crt_product(A, B, L)
    exact = _exact_product(A, B)
    ea = np.frexp(np.max(np.abs(A), axis=1))[1]
    eb = np.frexp(np.max(np.abs(B), axis=1))[1]
    for i in range(7):
        for j in range(6):
            # truncation: each operand entry within 2^(e - beta) of its row's value
            bound = Fraction(2) ** (1 - beta) * 33 * Fraction(2) ** int(ea[i] + eb[j]) * \
                (1 + Fraction(2) ** -beta)
            err = abs(Fraction(float(C[i, j])) - exact[i][j])
            assert err <= bound + abs(exact[i][j]) * Fraction(2) ** -52


def test_odd_symmetry_and_row_scaling():
    """Truncation toward zero is odd: negating an operand negates the product exactly.
    A row scaled by a power of two shifts its exponent only: the product row scales
    exactly."""
    rng = np.random.default_rng(5)
    A = rng.standard_normal((6, 40))
    B = rng.standard_normal((5, 40))
    C = O.crt_product(A, B, 14)
    np.testing.assert_array_equal(O.crt_product(-A, B, 14), -C)
    A2 = A.copy()
    A2[2] *= 2.0 ** -37
    C2 = O.crt_product(A2, B, 14)
    np.testing.assert_array_equal(C2[2], C[2] * 2.0 ** -37)
    np.testing.assert_array_equal(np.delete(C2, 2, 0), np.delete(C, 2, 0))


def test_zero_rows():
    A = np.zeros((3, 4))
    A[1] = [1.0, -2.0, 0.5, 0.0]
    B = np.ones((2, 4))
    C = O.crt_product(A, B, 14)
    np.testing.assert_array_equal(C[[0, 2]], 0.0)
    assert C[1, 0] == -0.5


def test_crt_residual_close_to_fp64():
    S = inputs.overlap_gaussian(96, 1.2, 0)
    Z = O.lowdin(S) * (1 + 1e-4)
    d64 = np.eye(96) - O.gram(S, Z)
    d = O.crt_residual(S, Z, 14)
    assert np.array_equal(d, d.T)
    assert np.max(np.abs(d - d64)) <= 1e-12, np.max(np.abs(d - d64))
