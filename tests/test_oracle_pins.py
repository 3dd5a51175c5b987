"""Hand-computed pins of the oracle's small helpers: the Gershgorin bounds behind the
scaled-identity guess (Sec. III: X0 = S/g has its spectrum in (0, 1], so
||X0 - I||_2 < 1), the RMS residual ||Z^T S Z - I||_F / sqrt(N) that every result is
judged by, and the learned guess's polynomial and features.  Every expected value
is derived here from exact arithmetic or a closed form, not from the oracle."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import zf_guess_oracle as G
from oracle import zf_oracle as O

# A symmetric matrix with mixed signs whose Gershgorin data differ from every other
# plausible bound: row sums of |S_ij| are 3, 4.5 and 1.5 (g = 4.5), the lower bounds
# S_ii - sum_{j != i} |S_ij| are 1, 1.5 and 0.5 (g_lo = 0.5).  ||S||_F = sqrt(16.5)
# and n max |S_ij| = 9 both differ from g.
HAND = [[2, -1, 0], [-1, 3, Fraction(1, 2)], [0, Fraction(1, 2), 1]]


def _hand():
    return np.array([[float(x) for x in row] for row in HAND])


def _rotation3():
    """An exactly orthogonal matrix with rational entries (a 3-4-5 rotation in the
    (0, 1) plane followed by one in the (1, 2) plane), as Fractions."""
    a = [[Fraction(3, 5), Fraction(-4, 5), 0], [Fraction(4, 5), Fraction(3, 5), 0], [0, 0, 1]]
    b = [[1, 0, 0], [0, Fraction(5, 13), Fraction(-12, 13)], [0, Fraction(12, 13), Fraction(5, 13)]]
    return _fmat(a, b)


def _fmat(a, b):
    n = len(a)
    return [[sum(Fraction(a[i][k]) * Fraction(b[k][j]) for k in range(n)) for j in range(n)]
            for i in range(n)]


def _f2np(a):
    return np.array([[float(x) for x in row] for row in a])


def test_gershgorin_hand_matrix():
    S = _hand()
    assert O.gershgorin_max_row_sum(S) == 4.5
    g, g_lo, rmean = G.gershgorin(S)
    assert (g, g_lo, rmean) == (4.5, 0.5, 3.0)
    # the bounds enclose the spectrum
    lam = np.linalg.eigvalsh(S)
    assert g_lo <= lam.min() and lam.max() <= g


def test_scaled_identity_hand_matrix():
    """Z0 = I / sqrt(g) with g = 4.5: diagonal entries with z^2 g = 1, zero elsewhere, and
    X0 = Z0^T S Z0 = S / 4.5 satisfies ||X0 - I||_2 < 1 (Sec. III)."""
    S = _hand()
    Z0 = O.scaled_identity_guess(S)
    assert np.all(Z0[~np.eye(3, dtype=bool)] == 0.0)
    np.testing.assert_allclose(np.diag(Z0) ** 2 * 4.5, 1.0, rtol=5e-16)
    X0 = Z0.T @ S @ Z0
    assert np.max(np.abs(np.linalg.eigvalsh(X0 - np.eye(3)))) < 1.0
    # the exact eigenvalues of S / 4.5 lie in (0, 1]: 1 - lambda / 4.5 < 1
    np.testing.assert_allclose(np.linalg.eigvalsh(X0), np.linalg.eigvalsh(S) / 4.5, rtol=1e-15)


@pytest.mark.parametrize("d", [0.19, 0.75, -0.44, 1e-9])
def test_residual_rms_closed_form(d):
    """For Z = sqrt(1 - d) S^(-1/2): Z^T S Z = (1 - d) I, delta = d I, ||delta||_F =
    |d| sqrt(N), RMS = |d|.  S = Q diag(s) Q^T with an exactly orthogonal Q, so
    S^(-1/2) = Q diag(s^(-1/2)) Q^T is known in closed form."""
    Q = _f2np(_rotation3())
    s = np.array([4.0, 9.0, 0.25])
    S = Q @ np.diag(s) @ Q.T
    Z = math.sqrt(1.0 - d) * (Q @ np.diag(1.0 / np.sqrt(s)) @ Q.T)
    assert O.residual_rms(S, Z) == pytest.approx(abs(d), rel=1e-12, abs=1e-15)
    assert O.residual(S, Z) == pytest.approx(abs(d) * math.sqrt(3.0), rel=1e-12, abs=1e-15)


def test_residual_rms_larger_order():
    """The same closed form at N = 64 (a block-diagonal S of rotated 2 x 2 blocks)."""
    n = 64
    c, sn = 0.6, 0.8
    R = np.array([[c, -sn], [sn, c]])
    S = np.zeros((n, n))
    Sih = np.zeros((n, n))
    for b in range(n // 2):
        lam = np.array([1.0 + b, 2.0 + 0.5 * b])
        S[2 * b:2 * b + 2, 2 * b:2 * b + 2] = R @ np.diag(lam) @ R.T
        Sih[2 * b:2 * b + 2, 2 * b:2 * b + 2] = R @ np.diag(lam ** -0.5) @ R.T
    d = 0.3
    assert O.residual_rms(S, math.sqrt(1 - d) * Sih) == pytest.approx(d, rel=1e-12)


def test_guess_matrix_spectral():
    """Z0 = p(S/g)/sqrt(g) shares S's eigenvectors: Q diag((c0 + c1 x + c2 x^2)/sqrt(g)) Q^T
    with x = s / g.  S is not diagonal, so an element-wise square of S/g, a dropped term or
    a missing 1/sqrt(g) all change the result."""
    Q = _f2np(_rotation3())
    s = np.array([0.5, 1.25, 3.0])
    S = Q @ np.diag(s) @ Q.T
    g = float(np.max(np.sum(np.abs(S), axis=1)))  # pinned by test_gershgorin_hand_matrix
    c = np.array([0.9, 0.3, -0.2])
    x = s / g
    want = Q @ np.diag((c[0] + c[1] * x + c[2] * x * x) / math.sqrt(g)) @ Q.T
    np.testing.assert_allclose(G.guess_matrix(S, c), want, rtol=0, atol=1e-15)


def _ftrace_pow(A, k):
    P = A
    for _ in range(k - 1):
        P = _fmat(P, A)
    return sum(P[i][i] for i in range(len(A)))


def test_features_hand_matrix():
    """The 8 features of the hand matrix from exact rational traces: log N, tr((S/g)^k)/N
    for k = 1..4, max(g_lo, 0)/g, g_lo/g, mean row sum / g."""
    A = [[Fraction(x) for x in row] for row in HAND]
    g = Fraction(9, 2)
    want = [math.log(3)]
    for k in range(1, 5):
        want.append(float(_ftrace_pow(A, k) / g ** k / 3))
    want += [float(Fraction(1, 2) / g), float(Fraction(1, 2) / g), float(Fraction(3) / g)]
    np.testing.assert_allclose(G.features(_hand()), want, rtol=1e-14, atol=0)


def test_features_negative_lower_bound():
    """S = [[1, 2], [2, 1]]: g = 3, g_lo = 1 - 2 = -1, so f[5] = max(g_lo, 0)/g = 0 and
    f[6] = g_lo/g = -1/3; the mean row sum is 3 (f[7] = 1)."""
    f = G.features(np.array([[1.0, 2.0], [2.0, 1.0]]))
    assert f[5] == 0.0 and f[6] == pytest.approx(-1.0 / 3.0, rel=1e-15) and f[7] == 1.0
    # tr(S/3) / 2 = 1/3, tr((S/3)^2) / 2 = (1 + 4 + 4 + 1) / 9 / 2 = 5/9
    assert f[1] == pytest.approx(1.0 / 3.0, rel=1e-15) and f[2] == pytest.approx(5.0 / 9.0, rel=1e-15)
