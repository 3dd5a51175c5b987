"""Pins of the oracle's congruence transform H_perp = Z^T H Z (Sec. II.A, Eq.
standard_form), each against something other than its own formula:

* the generalized symmetric-definite eigenproblem H C = S C eps solved by LAPACK
  (scipy.linalg.eigh(H, S), a Cholesky reduction) has the eigenvalues of H_perp for any
  Z with Z^T S Z = I, symmetric (S^(-1/2)) or not (the inverse Cholesky factor);
* C = Z C_perp solves the generalized problem (the back-transform of Sec. II.A);
* a 2 x 2 closed form, and exact rational arithmetic on a 3 x 3 case.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs


def _pair(n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed)
    return S, inputs.huckel_hamiltonian(S, seed + 100)


@pytest.mark.parametrize("n,seed", [(40, 0), (120, 1)])
def test_eigenvalues_match_generalized_problem(n, seed):
    S, H = _pair(n, seed)
    ref = scipy.linalg.eigh(H, S, eigvals_only=True)
    for Z in (O.lowdin(S), np.linalg.inv(np.linalg.cholesky(S)).T):
        assert np.allclose(Z.T @ S @ Z, np.eye(n), atol=1e-10)
        Hp = O.congruence(H, Z)
        w = np.linalg.eigvalsh(0.5 * (Hp + Hp.T))
        np.testing.assert_allclose(w, ref, rtol=0, atol=1e-9 * np.max(np.abs(ref)))


def test_back_transform_solves_generalized_problem():
    """The inverse Cholesky factor is upper triangular, not symmetric: a transform with Z
    on the wrong side gives a matrix whose eigenvectors do not map back."""
    S, H = _pair(60, 3)
    Z = np.linalg.inv(np.linalg.cholesky(S)).T
    Hp = O.congruence(H, Z)
    assert np.max(np.abs(Hp - Hp.T)) <= 1e-11 * np.max(np.abs(Hp))
    eps, Cp = np.linalg.eigh(0.5 * (Hp + Hp.T))
    C = Z @ Cp
    r = H @ C - S @ C * eps
    assert np.max(np.abs(r)) <= 1e-9 * np.max(np.abs(H))


def test_two_by_two_closed_form():
    """S = [[1, s], [s, 1]], H = [[a, b], [b, a]]: eigenvalues (a+b)/(1+s), (a-b)/(1-s)."""
    s, a, b = 0.3, -10.0, -4.0
    S = np.array([[1.0, s], [s, 1.0]])
    H = np.array([[a, b], [b, a]])
    w = np.linalg.eigvalsh(O.congruence(H, O.lowdin(S)))
    np.testing.assert_allclose(np.sort(w), np.sort([(a + b) / (1 + s), (a - b) / (1 - s)]),
                               rtol=1e-14)


def test_exact_rational():
    F = Fraction
    H = [[F(2), F(1, 3), F(0)], [F(1, 3), F(-1), F(1, 5)], [F(0), F(1, 5), F(4)]]
    Z = [[F(1), F(1, 2), F(0)], [F(0), F(3, 4), F(-1, 7)], [F(1, 9), F(0), F(2)]]
    n = 3
    exact = [[sum(Z[k][i] * H[k][l] * Z[l][j] for k in range(n) for l in range(n))
              for j in range(n)] for i in range(n)]
    got = O.congruence(np.array(H, dtype=float), np.array(Z, dtype=float))
    np.testing.assert_allclose(got, np.array(exact, dtype=float), rtol=1e-15, atol=1e-15)


def test_hamiltonian_input_is_symmetric():
    S, H = _pair(50, 4)
    assert np.array_equal(H, H.T)
    assert np.all(np.diag(H) < 0)
