"""The oracle's pins must catch plausible mistakes: each case plants one in the
oracle (CPU only, via monkeypatch) and checks that a pin test then fails."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import zf_guess_oracle as G
from oracle import zf_oracle as O
from tests import test_oracle_coeffs as TC
from tests import test_oracle_crt as TX
from tests import test_oracle_pins as TP
from tests import test_oracle_congruence as TH
from tests import test_oracle_ozaki as TZ
from tests import test_oracle_recursion as TR
from tests import test_oracle_split as TS


def _dropped_term(m):
    c = [Fraction(1), Fraction(1, 2), Fraction(3, 8), Fraction(5, 16), Fraction(35, 128),
         Fraction(63, 256)][: m + 1]
    if m >= 2:
        c[2] = Fraction(1, 4)
    return c


def _flipped_correction(delta, order):
    c = [float(x) for x in O.delta_coefficients(order)]
    q = c[1] * delta + (c[2] * delta @ delta if order >= 2 else 0.0)
    return -q


def _transposed_gram(S, Z):
    return Z @ S @ Z.T


def _mirrored_congruence(H, Z):
    return Z @ H @ Z.T


_true_ozaki = O.ozaki_product


def _ozaki_dropped_weight(A, B, s):
    """Leaves out the products of weight 2^{-7(s+1)} (the p + q = s + 1 diagonal)."""
    sa, ea = O.int_slices(A, s)
    sb, eb = O.int_slices(B, s)
    acc = np.zeros((A.shape[0], B.shape[0]))
    for d in range(s, 1, -1):
        c = sum(sa[p - 1] @ sb[d - p - 1].T for p in range(1, d))
        acc = acc + np.ldexp(c.astype(np.float64), -7 * d)
    return np.ldexp(acc, ea[:, None] + eb[None, :])


def _ozaki_shifted(A, B, s):
    return 2.0 * _true_ozaki(A, B, s)


_true_crt_truncate = O.crt_truncate


def _crt_floor(A, beta):
    """Rounds toward minus infinity instead of toward zero."""
    A = np.asarray(A, dtype=np.float64)
    m = np.max(np.abs(A), axis=1)
    e = np.where(m > 0, np.frexp(m)[1], 0).astype(np.int64)
    return np.floor(np.ldexp(A, (beta - e)[:, None])).astype(np.int64), e


def _crt_global_exponent(A, beta):
    """One exponent for the whole matrix instead of one per row."""
    A = np.asarray(A, dtype=np.float64)
    e = np.full(A.shape[0], np.frexp(np.max(np.abs(A)))[1], dtype=np.int64)
    return np.trunc(np.ldexp(A, (beta - e)[:, None])).astype(np.int64), e


def _crt_beta_one_more(K, L):
    M = 1
    for m in O.CRT_MODULI[:L]:
        M *= m
    return min(int(math.log2(M / (4 * K)) // 2) + 1, 52)


def _truncating_split(a, fmt="bf16"):
    a32 = O.to_fp32(a)
    u = np.ascontiguousarray(a32).view(np.uint32) & np.uint32(0xFFFF0000)
    hi = u.view(np.float32)
    r = (a32 - hi).astype(np.float32)
    lo = (np.ascontiguousarray(r).view(np.uint32) & np.uint32(0xFFFF0000)).view(np.float32)
    return hi, lo


def _nonstrict_stop(it, err, prev, order, rule):
    if it == 0 or prev is None:
        return False
    return err >= prev ** (order + 1)


def _frobenius_bound(S):
    return float(np.linalg.norm(S))


def _max_entry_bound(S):
    return float(S.shape[0] * np.max(np.abs(S)))


def _gershgorin_diag_twice(S):
    r = np.sum(np.abs(S), axis=1)
    d = np.diag(S)
    return float(np.max(r)), float(np.min(d - r)), float(np.mean(r))


def _rms_over_n(S, Z):
    return O.residual(S, Z) / S.shape[0]


def _guess_elementwise_square(S, c):
    g, _, _ = G.gershgorin(S)
    St = S / g
    return (c[0] * np.eye(S.shape[0]) + c[1] * St + c[2] * St * St) / np.sqrt(g)


def _guess_dropped_linear(S, c):
    g, _, _ = G.gershgorin(S)
    St = S / g
    return (c[0] * np.eye(S.shape[0]) + c[2] * St @ St) / np.sqrt(g)


MUTANTS = [
    ("delta_coefficients", _dropped_term, lambda g: TR.test_spectral_map_history()),
    ("delta_coefficients", _dropped_term, lambda g: TC.test_x_form_coefficients_match_appendix_a(g)),
    ("correction", _flipped_correction, lambda g: TR.test_spectral_map_history()),
    ("gram", _transposed_gram, lambda g: TR.test_general_guess_limit()),
    ("congruence", _mirrored_congruence, lambda g: TH.test_back_transform_solves_generalized_problem()),
    ("congruence", _mirrored_congruence, lambda g: TH.test_exact_rational()),
    ("ozaki_product", _ozaki_dropped_weight, lambda g: TZ.test_product_within_bound_of_exact(3)),
    ("ozaki_product", _ozaki_shifted, lambda g: TZ.test_integer_matrices_are_exact()),
    ("crt_truncate", _crt_floor, lambda g: TX.test_odd_symmetry_and_row_scaling()),
    ("crt_truncate", _crt_global_exponent, lambda g: TX.test_odd_symmetry_and_row_scaling()),
    ("crt_truncate", _crt_global_exponent, lambda g: TX.test_product_within_bound_of_exact(14)),
    ("crt_beta", _crt_beta_one_more, lambda g: TX.test_beta_hand_values()),
    ("split", _truncating_split, lambda g: TS.test_bf16_rounding_edge_values()),
    ("stop_now", _nonstrict_stop, lambda g: TC.test_stop_rule_algorithm_2()),
    ("gershgorin_max_row_sum", _frobenius_bound, lambda g: TP.test_gershgorin_hand_matrix()),
    ("gershgorin_max_row_sum", _frobenius_bound, lambda g: TP.test_scaled_identity_hand_matrix()),
    ("gershgorin_max_row_sum", _max_entry_bound, lambda g: TP.test_scaled_identity_hand_matrix()),
    ("residual_rms", _rms_over_n, lambda g: TP.test_residual_rms_closed_form(0.19)),
    ("residual_rms", _rms_over_n, lambda g: TP.test_residual_rms_larger_order()),
]

# mistakes planted in the learned guess's oracle
GUESS_MUTANTS = [
    ("gershgorin", _gershgorin_diag_twice, lambda g: TP.test_gershgorin_hand_matrix()),
    ("gershgorin", _gershgorin_diag_twice, lambda g: TP.test_features_hand_matrix()),
    ("guess_matrix", _guess_elementwise_square, lambda g: TP.test_guess_matrix_spectral()),
    ("guess_matrix", _guess_dropped_linear, lambda g: TP.test_guess_matrix_spectral()),
]


@pytest.mark.parametrize("name,mutant,pin", MUTANTS, ids=[f"{m[0]}-{i}" for i, m in enumerate(MUTANTS)])
def test_pin_catches_mutant(monkeypatch, golden_dir, name, mutant, pin):
    monkeypatch.setattr(O, name, mutant)
    with pytest.raises(AssertionError):
        pin(golden_dir)


@pytest.mark.parametrize("name,mutant,pin", GUESS_MUTANTS,
                         ids=[f"{m[0]}-{i}" for i, m in enumerate(GUESS_MUTANTS)])
def test_guess_pin_catches_mutant(monkeypatch, golden_dir, name, mutant, pin):
    monkeypatch.setattr(G, name, mutant)
    with pytest.raises(AssertionError):
        pin(golden_dir)
