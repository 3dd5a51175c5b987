"""Pins for the oracle's recursion: spectral map, diagonal S, Loewdin limit,
general-guess limit, exact rational arithmetic and convergence order."""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs

# the paper's printed m = 2 polynomial in X (Appendix A): p(X) = 15/8 - 5/4 X + 3/8 X^2
A2 = (15 / 8, -5 / 4, 3 / 8)


def _small_S(n=64, seed=0, sigma=1.2):
    return inputs.overlap_gaussian(n, sigma, seed)


def test_spectral_map_history():
    """Z0 = I/sqrt(g) commutes with S, so X_n has the eigenvalues of S/g pushed
    n times through x -> x p(x)^2 (Sec. III, Eq. np1).  The whole Err history
    follows from eigvalsh(S) alone."""
    S = _small_S()
    g = np.max(np.sum(np.abs(S), axis=1))
    x = np.linalg.eigvalsh(S) / g
    res = O.refine(S, np.eye(S.shape[0]) / math.sqrt(g), order=2, rule="ratio")
    for n, err in enumerate(res.hist):
        expect = math.sqrt(np.sum((1.0 - x) ** 2))
        if expect > 1e-9:
            assert err == pytest.approx(expect, rel=1e-9), n
        else:
            assert err < 1e-9
        p = A2[0] + A2[1] * x + A2[2] * x * x
        x = x * p * p


def test_diagonal_S_scalar_recursion():
    """Diagonal S: Z stays diagonal (off-diagonals exactly 0), each entry follows
    z <- z p(z^2 s) and tends to s^(-1/2)."""
    s = np.array([0.3, 0.7, 1.0, 1.6, 2.2])
    S = np.diag(s)
    z = np.full(5, 1.0 / math.sqrt(s.max()))
    res = O.refine(S, np.diag(z), order=2, rule="none", max_sweeps=6)
    Z = res.Z
    assert np.all(Z[~np.eye(5, dtype=bool)] == 0.0)
    for _ in range(6):
        x = z * z * s
        z = z * (A2[0] + A2[1] * x + A2[2] * x * x)
    np.testing.assert_allclose(np.diag(Z), z, rtol=1e-14)
    np.testing.assert_allclose(np.diag(Z), 1.0 / np.sqrt(s), rtol=1e-13)


@pytest.mark.parametrize("order", [1, 2, 3, 5])
def test_loewdin_limit(order):
    """Z0 = cI converges to S^(-1/2) (Sec. II.B: Z = S^(-1/2) is a factor)."""
    S = _small_S(48, seed=1)
    res = O.refine(S, O.scaled_identity_guess(S), order=order)
    L = O.lowdin(S)
    # the Loewdin factor itself, against an independent library square root
    L2 = np.real(scipy.linalg.sqrtm(np.linalg.inv(S)))
    np.testing.assert_allclose(L, L2, rtol=0, atol=1e-10 * np.abs(L).max())
    assert np.linalg.norm(res.Z - L) / np.linalg.norm(L) < 1e-12
    assert O.residual_rms(S, res.Z) < 1e-13


def test_general_guess_limit():
    """Z0 = S^(-1/2) + alpha U (Sec. V.A) converges to Z0 X0^(-1/2), which is a
    valid factor but not S^(-1/2)."""
    S = _small_S(40, seed=2)
    U = inputs.uniform_noise(40, 7)
    Z0 = O.lowdin(S) + 0.05 * U
    res = O.refine(S, Z0, order=2)
    Zs = O.limit_for_guess(S, Z0)
    assert np.linalg.norm(res.Z - Zs) / np.linalg.norm(Zs) < 1e-12
    assert O.residual_rms(S, res.Z) < 1e-13
    assert np.linalg.norm(res.Z - O.lowdin(S)) > 1e-3


def _frac_matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(k)), Fraction(0)) for j in range(m)]
            for i in range(n)]


def _frac_T(A):
    return [list(r) for r in zip(*A)]


def _exact_sweeps(S, Z, sweeps):
    """The m = 2 recursion Z <- Z (I + delta/2 + 3/8 delta^2), delta = I - Z^T S Z,
    in exact rational arithmetic."""
    n = len(S)
    eye = [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]
    for _ in range(sweeps):
        X = _frac_matmul(_frac_T(Z), _frac_matmul(S, Z))
        d = [[eye[i][j] - X[i][j] for j in range(n)] for i in range(n)]
        d2 = _frac_matmul(d, d)
        P = [[eye[i][j] + d[i][j] / 2 + Fraction(3, 8) * d2[i][j] for j in range(n)]
             for i in range(n)]
        Z = _frac_matmul(Z, P)
    return Z


@pytest.mark.parametrize("case", ["n1", "n2", "n3"])
def test_exact_rational_brute_force(case):
    F = Fraction
    if case == "n1":
        S = [[F(4)]]
        Z0 = [[F(1, 3)]]
    elif case == "n2":
        S = [[F(1), F(1, 4)], [F(1, 4), F(1)]]
        Z0 = [[F(1), F(0)], [F(0), F(1)]]
    else:
        S = [[F(2), F(1, 2), F(0)], [F(1, 2), F(2), F(1, 3)], [F(0), F(1, 3), F(1)]]
        Z0 = [[F(2, 3), F(1, 10), F(0)], [F(0), F(3, 5), F(-1, 20)], [F(1, 7), F(0), F(4, 5)]]
    sweeps = 3
    Zx = _exact_sweeps(S, Z0, sweeps)
    Sf = np.array(S, dtype=float)
    Z0f = np.array(Z0, dtype=float)
    res = O.refine(Sf, Z0f, order=2, rule="none", max_sweeps=sweeps)
    Ze = np.array(Zx, dtype=float)
    np.testing.assert_allclose(res.Z, Ze, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(O.refine_x_form(Sf, Z0f, sweeps), Ze, rtol=1e-14, atol=1e-15)
    if case == "n1":
        # z -> 1/2 for s = 4
        assert abs(O.refine(Sf, Z0f).Z[0, 0] - 0.5) < 1e-16


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_convergence_order(order):
    """Order m + 1 and the ratio bound of Eq. stopL2.

    (a) Along the scaled-identity history every step above the FP64 floor has
        Err_{n+1} <= Err_n^(m+1): with rho(delta) < 1 the Frobenius norm obeys
        the bound of Sec. IV.A.
    (b) From Z0 = sqrt(1 - d) S^(-1/2), delta_0 = d I exactly and one sweep gives
        Err_1 ~ |C_m| d^(m+1) sqrt(N): the measured order between d = 0.03 and
        d = 0.01 is m + 1, and for m = 2 the constant is the paper's c = 5/8."""
    S = _small_S(64, seed=3)
    n = S.shape[0]
    res = O.refine(S, O.scaled_identity_guess(S), order=order, rule="none", max_sweeps=40)
    for a, b in zip(res.hist, res.hist[1:]):
        if b < 1e-12:
            break
        assert b <= a ** (order + 1) * (1 + 1e-9)
    L = O.lowdin(S)
    e1 = {}
    for d in (0.03, 0.01):
        r = O.refine(S, math.sqrt(1.0 - d) * L, order=order, rule="none", max_sweeps=1)
        assert r.hist[0] == pytest.approx(d * math.sqrt(n), rel=1e-10)
        e1[d] = r.hist[1] / math.sqrt(n)
    q = math.log(e1[0.03] / e1[0.01]) / math.log(3.0)
    assert q == pytest.approx(order + 1, rel=0.05)
    lead = abs(float(O.error_polynomial(order)[order + 1]))
    assert e1[0.01] / 0.01 ** (order + 1) == pytest.approx(lead, rel=0.1)
    if order == 2:
        assert e1[0.01] / 0.01 ** 3 == pytest.approx(5 / 8, rel=0.05)


def test_x_form_equals_delta_form():
    S = _small_S(32, seed=4)
    Z0 = O.scaled_identity_guess(S)
    for sweeps in (1, 3, 6):
        a = O.refine(S, Z0, order=2, rule="none", max_sweeps=sweeps).Z
        b = O.refine_x_form(S, Z0, sweeps, order=2)
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


def test_ratio_stop_returns_better_iterate():
    S = _small_S(64, seed=5)
    res = O.refine(S, O.scaled_identity_guess(S), order=2, rule="ratio")
    assert res.stopped_by == "ratio"
    h = res.hist
    assert res.err == min(h[-1], h[-2])
    assert res.iters in (len(h) - 1, len(h) - 2)
    assert O.residual(S, res.Z) == pytest.approx(res.err, rel=1e-6, abs=1e-15)


def test_divergent_guess_is_detected():
    """||X0 - I||_2 >= 1 violates the convergence condition of Sec. III."""
    S = _small_S(16, seed=6)
    Z0 = 2.0 * O.lowdin(S)           # X0 = 4 I, delta = -3 I
    try:
        res = O.refine(S, Z0, order=2, rule="ratio")
        assert res.err >= 1.0
    except FloatingPointError:
        pass


def test_monotone_rule_runs_to_floor():
    S = _small_S(64, seed=0)
    r = O.refine(S, O.scaled_identity_guess(S), order=2, rule="monotone")
    assert r.stopped_by == "monotone"
    assert r.err / 8.0 < 1e-14
