"""Pins of the oracle's emulated FP64 products (integer slices, Ozaki scheme), each
against something other than the oracle's own formula: exact rational arithmetic,
integer matrices (where the scheme is exact), and FP64's own representation."""
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


def test_slices_reconstruct_exactly_with_eight_slices():
    """56 bits of slices hold any double's 53-bit significand relative to its row's max
    exponent when the row spans few binades: the reconstruction is then exact."""
    rng = np.random.default_rng(0)
    A = rng.uniform(0.5, 1.0, (6, 9)) * np.sign(rng.standard_normal((6, 9)))
    sl, e = O.int_slices(A, 8)
    rec = sum(np.ldexp(q.astype(float), -7 * (p + 1)) for p, q in enumerate(sl))
    np.testing.assert_array_equal(np.ldexp(rec, e[:, None]), A)
    assert all(np.max(np.abs(q)) <= 127 for q in sl)


def test_slices_remainder_bound():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((5, 40)) * np.exp(rng.uniform(-30, 30, (5, 40)))
    for s in (3, 5, 7):
        sl, e = O.int_slices(A, s)
        for i in range(5):
            for k in range(40):
                rec = sum(Fraction(int(q[i, k]), 128 ** (p + 1)) for p, q in enumerate(sl))
                r = Fraction(float(A[i, k])) / Fraction(2) ** int(e[i]) - rec
                assert abs(r) < Fraction(1, 128 ** s)


@pytest.mark.parametrize("s", [3, 5, 7])
def test_product_within_bound_of_exact(s):
    rng = np.random.default_rng(s)
    A = rng.standard_normal((7, 33)) * np.exp(rng.uniform(-5, 5, (7, 33)))
    B = rng.standard_normal((6, 33))
    C = O.ozaki_product(A, B, s)
    exact = _exact_product(A, B)
    ea = np.frexp(np.max(np.abs(A), axis=1))[1]
    eb = np.frexp(np.max(np.abs(B), axis=1))[1]
    for i in range(7):
        for j in range(6):
            bound = Fraction(s + 1, 128 ** s) * 33 * Fraction(2) ** int(ea[i] + eb[j])
            assert abs(Fraction(float(C[i, j])) - exact[i][j]) <= bound + abs(exact[i][j]) * Fraction(2) ** -52
    # s = 7 keeps the error within a few hundred ulps of |A||B|^T even for rows spanning
    # e^10 (entries far below the row maximum keep fewer bits)
    if s == 7:
        rel = max(abs(float(Fraction(float(C[i, j])) - exact[i][j])) / (abs(A[i]) @ abs(B[j]))
                  for i in range(7) for j in range(6))
        assert rel < 5e-13


def test_integer_matrices_are_exact():
    """Entries that are integers of magnitude <= 127 sit in the first slice exactly, so
    every s gives the exact integer product."""
    rng = np.random.default_rng(2)
    A = rng.integers(-127, 128, (8, 50)).astype(float)
    B = rng.integers(-127, 128, (5, 50)).astype(float)
    A[:, 0] = 127.0       # row maxima 127: exponent 7, slice 1 = the integer itself
    B[:, 0] = -127.0
    for s in (1, 2, 4):
        np.testing.assert_array_equal(O.ozaki_product(A, B, s), A @ B.T)


def test_zero_rows_and_empty_inner_dimension():
    A = np.zeros((3, 4))
    A[1] = [1.0, -2.0, 0.5, 0.0]
    B = np.ones((2, 4))
    C = O.ozaki_product(A, B, 4)
    np.testing.assert_array_equal(C[[0, 2]], 0.0)
    assert C[1, 0] == -0.5


def test_emulated_residual_close_to_fp64():
    S = inputs.overlap_gaussian(96, 1.2, 0)
    Z = O.lowdin(S) * (1 + 1e-4)
    d64 = np.eye(96) - O.gram(S, Z)
    for s, tol in ((5, 1e-7), (7, 1e-10)):
        d = O.emulated_residual(S, Z, s)
        assert np.array_equal(d, d.T)
        assert np.max(np.abs(d - d64)) <= tol, (s, np.max(np.abs(d - d64)))
