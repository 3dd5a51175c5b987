"""CPU FP64 oracle for the iterative inverse-overlap factorization Z^T S Z = I.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product (the
HIP library and its Python binding) never calls into it, and this module
imports nothing from the product: it takes its inputs as plain arrays.

Everything here is plain NumPy / Python, FP64 unless a function states
otherwise, with no blocking or fusion beyond what the paper writes down.
Paper references are to Habib, Finkelstein & Niklasson, "Efficient
Mixed-Precision Matrix Factorization of the Inverse Overlap Matrix in
Electronic Structure Calculations with AI-Hardware and GPUs" (LA-UR-24-24032).

Conventions (readings of the paper, each listed in the design notes):

* delta = I - Z^T S Z.  Sec. III and Sec. IV.A write the error as X - I; the
  sign only flips odd powers and never changes a norm.  With this sign the
  update is Z <- Z * sum_k c_k delta^k with every c_k > 0, the truncated
  binomial series of (I - delta)^(-1/2) = X^(-1/2) (Sec. III, the delta form
  given after Algorithm 1).
* order m: number of series terms after the identity; the paper uses m = 2
  (third-order convergence, Sec. III).
* Stop rule "ratio" is Algorithm 2 (Sec. IV.A, Eq. stopL2) with the exponent
  generalized from 3 to m + 1; "monotone" stops once the Frobenius norm no
  longer decreases.  Either way the better of the last two iterates is
  returned (Algorithm 2 leaves that choice open).
* Err is the unnormalized Frobenius norm of delta (Sec. IV.A uses it for the
  stop test); the RMS residual reported to users is Err / sqrt(N).

Functions without an independent pin say so in their docstring.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import torch

# ---------------------------------------------------------------------------
# series coefficients (Sec. III, Eq. np1; Appendix A)
# ---------------------------------------------------------------------------


def delta_coefficients(m: int) -> list[Fraction]:
    """c_0..c_m of Z_{n+1} = Z_n sum_k c_k delta_n^k (Sec. III, delta form).

    The update must reproduce X^(-1/2) = (I - delta)^(-1/2) to order m, so the
    c_k are the binomial-series coefficients C(2k, k) / 4^k."""
    return [Fraction(math.comb(2 * k, k), 4 ** k) for k in range(m + 1)]


def x_coefficients(m: int) -> list[Fraction]:
    """a_0..a_m of Z_{n+1} = Z_n sum_k a_k X_n^k (Sec. III, Eq. np1).

    Obtained by expanding sum_k c_k (1 - X)^k in powers of X; for m = 2 the
    paper prints a = (15/8, -5/4, 3/8) (Appendix A)."""
    c = delta_coefficients(m)
    a = [Fraction(0)] * (m + 1)
    for k, ck in enumerate(c):
        # (1 - X)^k = sum_j C(k, j) (-X)^j
        for j in range(k + 1):
            a[j] += ck * math.comb(k, j) * (-1) ** j
    return a


def _poly_mul(p: list[Fraction], q: list[Fraction]) -> list[Fraction]:
    r = [Fraction(0)] * (len(p) + len(q) - 1)
    for i, pi in enumerate(p):
        for j, qj in enumerate(q):
            r[i + j] += pi * qj
    return r


def error_polynomial(m: int) -> list[Fraction]:
    """Coefficients e_0..e_{2m+1} of X_{n+1} - I as a polynomial in e = X_n - I.

    Sec. IV.A, Eq. Xp1: with X_n = I + e and every matrix a polynomial in X_n,
    X_{n+1} = p(X_n) X_n p(X_n) = (1 + e) p(1 + e)^2.  For m = 2 the paper
    finds X_{n+1} = I + 5/8 e^3 - 15/64 e^4 + 9/64 e^5 (Appendix A)."""
    a = x_coefficients(m)
    # p(1 + e) = sum_k a_k (1 + e)^k as a polynomial in e
    p = [Fraction(0)] * (m + 1)
    for k, ak in enumerate(a):
        for j in range(k + 1):
            p[j] += ak * math.comb(k, j)
    full = _poly_mul(_poly_mul([Fraction(1), Fraction(1)], p), p)
    full[0] -= 1
    return full


# ---------------------------------------------------------------------------
# initial guesses
# ---------------------------------------------------------------------------


def gershgorin_max_row_sum(S: np.ndarray) -> float:
    """g = max_i sum_j |S_ij|, an upper bound on the spectrum of S (Gershgorin)."""
    return float(np.max(np.sum(np.abs(S), axis=1)))


def scaled_identity_guess(S: np.ndarray) -> np.ndarray:
    """Z0 = I / sqrt(g): X0 = S / g has its spectrum in (0, 1], so
    ||X0 - I||_2 < 1, the convergence condition of Sec. III."""
    n = S.shape[0]
    return np.eye(n) / math.sqrt(gershgorin_max_row_sum(S))


# ---------------------------------------------------------------------------
# the recursion (Algorithm 2 with the delta form of Sec. III)
# ---------------------------------------------------------------------------


class OracleResult:
    def __init__(self, Z, iters, hist, stopped_by):
        self.Z = Z                  # the returned iterate
        self.iters = iters          # number of updates applied to the returned Z
        self.hist = hist            # Err_0, Err_1, ... (unnormalized Frobenius norms)
        self.stopped_by = stopped_by  # "ratio" | "monotone" | "max_sweeps"

    @property
    def err(self) -> float:
        return self.hist[self.iters]

    def __repr__(self):
        return f"OracleResult(iters={self.iters}, hist={self.hist}, stop={self.stopped_by})"


def frobenius(A: np.ndarray) -> float:
    """||A||_F with a correctly rounded sum of squares (math.fsum)."""
    return math.sqrt(math.fsum((A * A).ravel().tolist()))


def stop_now(it: int, err: float, prev: float | None, order: int, rule: str) -> bool:
    """Parameter-free stop test of Algorithm 2 (Sec. IV.A, Eq. stopL2).

    ratio:    stop at iteration it > 0 if Err_it > Err_{it-1}^(m+1)
    monotone: stop at iteration it > 0 if Err_it >= Err_{it-1}"""
    if it == 0 or prev is None:
        return False
    if rule == "ratio":
        return err > prev ** (order + 1)
    if rule == "monotone":
        return err >= prev
    if rule == "none":
        return False
    raise ValueError(rule)


def correction(delta: np.ndarray, order: int) -> np.ndarray:
    """Q = sum_{k=1..m} c_k delta^k by Horner's rule: delta (c_1 + delta (c_2 + ...))."""
    c = [float(x) for x in delta_coefficients(order)]
    n = delta.shape[0]
    inner = c[order] * np.eye(n)
    for k in range(order - 1, 0, -1):
        inner = c[k] * np.eye(n) + delta @ inner
    return delta @ inner


def gram(S: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """X = Z^T S Z evaluated as Z^T (S Z) (Sec. III.B computes A = S Z first)."""
    return Z.T @ (S @ Z)


def refine(S: np.ndarray, Z0: np.ndarray, order: int = 2, rule: str = "ratio",
           max_sweeps: int = 100) -> OracleResult:
    """Iterate Z_{n+1} = Z_n (I + Q(delta_n)), delta_n = I - Z_n^T S Z_n (Sec. III,
    Eq. np1 in delta form) under the stop test of Algorithm 2 (Sec. IV.A).

    Each pass: X = Z^T (S Z); Err = ||I - X||_F; stop test; Z <- Z + Z Q."""
    S = np.asarray(S, dtype=np.float64)
    Z = np.array(Z0, dtype=np.float64, copy=True)
    n = S.shape[0]
    eye = np.eye(n)
    hist: list[float] = []
    prev_Z = None
    stopped_by = "max_sweeps"
    for it in range(max_sweeps + 1):
        X = gram(S, Z)
        delta = eye - X
        err = frobenius(delta)
        if not math.isfinite(err):
            raise FloatingPointError(f"non-finite residual at iteration {it}")
        hist.append(err)
        if stop_now(it, err, hist[-2] if it else None, order, rule):
            stopped_by = rule
            break
        if it == max_sweeps:
            break
        prev_Z = Z
        Z = Z + Z @ correction(delta, order)
    last = len(hist) - 1
    if last > 0 and hist[last] > hist[last - 1]:
        return OracleResult(prev_Z, last - 1, hist, stopped_by)
    return OracleResult(Z, last, hist, stopped_by)


def refine_x_form(S: np.ndarray, Z0: np.ndarray, sweeps: int, order: int = 2) -> np.ndarray:
    """Algorithm 1/2 literally in the X form, Z <- Z (a_0 I + a_1 X + ... + a_m X^m),
    for a fixed number of sweeps and no stop test.  Used to cross-check the
    delta form (the two are equal in exact arithmetic, Sec. III)."""
    a = [float(x) for x in x_coefficients(order)]
    Z = np.array(Z0, dtype=np.float64, copy=True)
    n = S.shape[0]
    for _ in range(sweeps):
        X = Z.T @ S @ Z
        P = a[order] * np.eye(n)
        for k in range(order - 1, -1, -1):
            P = a[k] * np.eye(n) + X @ P
        Z = Z @ P
    return Z


def residual(S: np.ndarray, Z: np.ndarray) -> float:
    """||Z^T S Z - I||_F (FP64)."""
    return frobenius(Z.T @ (S @ Z) - np.eye(S.shape[0]))


def residual_rms(S: np.ndarray, Z: np.ndarray) -> float:
    """||Z^T S Z - I||_F / sqrt(N)."""
    return residual(S, Z) / math.sqrt(S.shape[0])


def congruence(H: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """H_perp = Z^T H Z (Sec. II.A, Eq. standard_form): with Z^T S Z = I the generalized
    problem H C = S C eps becomes H_perp C_perp = C_perp eps, C_perp = Z^(-1) C.
    Evaluated as Z^T (H Z), the order the two-product GPU path also takes."""
    H = np.asarray(H, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    return Z.T @ (H @ Z)


# ---------------------------------------------------------------------------
# FP64 products emulated with integer slices (the multi-word splitting line that
# Sec. I and Sec. III.A cite, carried to integer matrix cores): the Ozaki scheme
# (Ozaki, Ogita, Oishi & Rump 2012) with 7-bit signed slices as in Ootomo, Ozaki &
# Yokota 2024.  Used for the residual of the refinement phase (Sec. IV.B).
# ---------------------------------------------------------------------------


def int_slices(A: np.ndarray, s: int) -> tuple[list[np.ndarray], np.ndarray]:
    """Row i of A as 2^{e_i} sum_{p=1..s} a_p 2^{-7p} plus a remainder below
    2^{e_i - 7s}: e_i is the frexp exponent of max_k |A_ik| (0 for a zero row), so
    |A_ik 2^{-e_i}| < 1; each slice takes the integer part of 128 times what is left
    (truncation toward zero, |a_p| <= 127).  Every step is exact in FP64."""
    A = np.asarray(A, dtype=np.float64)
    m = np.max(np.abs(A), axis=1) if A.shape[1] else np.zeros(A.shape[0])
    e = np.where(m > 0, np.frexp(m)[1], 0).astype(np.int64)
    t = np.ldexp(A, -e[:, None])
    out = []
    for _ in range(s):
        t = t * 128.0
        q = np.trunc(t)
        t = t - q
        out.append(q.astype(np.int64))
    return out, e


def ozaki_product(A: np.ndarray, B: np.ndarray, s: int) -> np.ndarray:
    """C = A B^T (A: M x K, B: N x K) from s slices per operand row, keeping the slice
    products a_p b_q^T with p + q <= s + 1.  Products of one weight 2^{-7d}, d = p + q,
    are summed exactly in integers; the weights are combined in FP64 from the smallest
    (d = s + 1) to the largest (d = 2), then scaled by 2^{e_i + f_j}.
    Error: |C - A B^T|_ij < (s + 1) 2^{-7s} K 2^{e_i + f_j}."""
    sa, ea = int_slices(A, s)
    sb, eb = int_slices(B, s)
    acc = np.zeros((np.asarray(A).shape[0], np.asarray(B).shape[0]))
    for d in range(s + 1, 1, -1):
        c = sum(sa[p - 1] @ sb[d - p - 1].T for p in range(1, d))
        acc = acc + np.ldexp(c.astype(np.float64), -7 * d)
    return np.ldexp(acc, ea[:, None] + eb[None, :])


def emulated_residual(S: np.ndarray, Z: np.ndarray, s: int) -> np.ndarray:
    """delta = I - Z^T S Z with both products emulated (Sec. III.B order: A^T = Z^T S,
    then Z^T A), the second one taken from its upper triangle and mirrored."""
    S = np.asarray(S, dtype=np.float64)
    Zt = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).T)
    At = ozaki_product(Zt, S, s)             # rows of Z^T against rows of S (= columns)
    X = ozaki_product(Zt, At, s)             # (Z^T S Z)_ij = sum_k Z^T_ik At_jk
    X = np.triu(X) + np.triu(X, 1).T
    return np.eye(S.shape[0]) - X


# ---------------------------------------------------------------------------
# FP64 products emulated through residues (Ozaki, Uchino & Imamura 2025, "Ozaki
# scheme II"): each operand row is scaled by a power of two and truncated to an
# integer of at most beta bits; the integer product is formed exactly (on the GPU
# from its residues modulo L pairwise coprime moduli <= 256, one int8 product per
# modulus, and the Chinese remainder theorem); the result is that exact product
# scaled back and rounded to FP64.  Defined here by the exact product itself.
# ---------------------------------------------------------------------------

# pairwise coprime moduli, largest first; the first L are used
CRT_MODULI = (256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197, 193)
CRT_MAX_BETA = 52


def crt_beta(K: int, L: int) -> int:
    """Largest beta with 4 K 2^(2 beta) <= M = product of the first L moduli: the exact
    integer product of two K-term rows of beta-bit integers then lies inside
    (-M/4, M/4), so it is fixed by its residues and sits a quarter period away from
    the ambiguous +-M/2 (the reconstruction rounds its quotient by M from a
    floating-point estimate).  Capped at 52."""
    M = 1
    for m in CRT_MODULI[:L]:
        M *= m
    b = 0
    while 4 * K * 4 ** (b + 1) <= M:
        b += 1
    return min(b, CRT_MAX_BETA)


def crt_truncate(A: np.ndarray, beta: int) -> tuple[np.ndarray, np.ndarray]:
    """Row i of A as integers trunc(A_ik 2^(beta - e_i)) (toward zero, |.| < 2^beta),
    e_i the frexp exponent of max_k |A_ik| (0 for a zero row).  Exact in FP64 since
    beta <= 52."""
    A = np.asarray(A, dtype=np.float64)
    m = np.max(np.abs(A), axis=1) if A.shape[1] else np.zeros(A.shape[0])
    e = np.where(m > 0, np.frexp(m)[1], 0).astype(np.int64)
    q = np.trunc(np.ldexp(A, (beta - e)[:, None]))
    return q.astype(np.int64), e


def _exact_int_product(P: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """P Q^T of int64 matrices with entries below 2^52 in magnitude, exactly, as an
    object array of Python ints.  Each entry splits as x = x1 2^26 + x0 with
    0 <= x0 < 2^26 and |x1| < 2^26, so each of the four partial products is below
    2^52 in magnitude; summed over blocks of at most 1024 terms in int64 they stay
    below 2^62, and the blocks and the parts are combined in Python integers."""
    P = np.asarray(P, dtype=np.int64)
    Q = np.asarray(Q, dtype=np.int64)
    P0 = P & ((1 << 26) - 1)
    P1 = (P - P0) >> 26
    Q0 = Q & ((1 << 26) - 1)
    Q1 = (Q - Q0) >> 26
    out = np.zeros((P.shape[0], Q.shape[0]), dtype=object)
    for k0 in range(0, P.shape[1], 1024):
        k = slice(k0, k0 + 1024)
        c11 = (P1[:, k] @ Q1[:, k].T).astype(object)
        c10 = (P1[:, k] @ Q0[:, k].T).astype(object)
        c01 = (P0[:, k] @ Q1[:, k].T).astype(object)
        c00 = (P0[:, k] @ Q0[:, k].T).astype(object)
        out = out + c11 * (1 << 52) + (c10 + c01) * (1 << 26) + c00
    return out


def crt_product(A: np.ndarray, B: np.ndarray, L: int) -> np.ndarray:
    """C = A B^T (A: M x K, B: N x K) from beta-bit row truncations of both operands,
    beta = crt_beta(K, L): C_ij = fl(C'_ij 2^(e_i + f_j - 2 beta)) with C' the exact
    integer product of the truncated rows.  Error against A B^T:
    |C - A B^T|_ij <= 2^(1 - beta) K 2^(e_i + f_j) (1 + 2^-beta) + one rounding."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    beta = crt_beta(A.shape[1], L)
    Ai, ea = crt_truncate(A, beta)
    Bi, eb = crt_truncate(B, beta)
    C = _exact_int_product(Ai, Bi)
    out = np.empty(C.shape)
    for i in range(C.shape[0]):
        for j in range(C.shape[1]):
            # float() of a Python int rounds to nearest even; the power of two is exact
            out[i, j] = math.ldexp(float(C[i, j]), int(ea[i] + eb[j]) - 2 * beta)
    return out


def crt_residual(S: np.ndarray, Z: np.ndarray, L: int) -> np.ndarray:
    """delta = I - Z^T S Z with both products emulated through residues, in the order
    of Sec. III.B (A^T = Z^T S, then Z^T A), the second taken from its upper triangle
    and mirrored."""
    S = np.asarray(S, dtype=np.float64)
    Zt = np.ascontiguousarray(np.asarray(Z, dtype=np.float64).T)
    At = crt_product(Zt, S, L)
    X = crt_product(Zt, At, L)
    X = np.triu(X) + np.triu(X, 1).T
    return np.eye(S.shape[0]) - X


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------


def lowdin(S: np.ndarray) -> np.ndarray:
    """S^(-1/2) = V Lambda^(-1/2) V^T from a dense eigendecomposition (Sec. II.B and
    Sec. V.A build it the same way with cuSolver)."""
    w, V = np.linalg.eigh(S)
    return (V * (1.0 / np.sqrt(w))) @ V.T


def limit_for_guess(S: np.ndarray, Z0: np.ndarray) -> np.ndarray:
    """Z* = Z0 X0^(-1/2), X0 = Z0^T S Z0: the fixed point the recursion reaches from Z0.

    Every iterate is Z0 times a polynomial in X0 and X_{n+1} = g(X_n) with
    g(x) = x p(1 - x)^2, so the accumulated factor tends to x^(-1/2)
    eigenvalue by eigenvalue (Sec. III: X_n -> I).  When Z0 commutes with S
    (Z0 = c I, or any polynomial in S) this is the Loewdin factor S^(-1/2)."""
    X0 = Z0.T @ S @ Z0
    X0 = 0.5 * (X0 + X0.T)
    w, V = np.linalg.eigh(X0)
    return Z0 @ ((V * (1.0 / np.sqrt(w))) @ V.T)


def scalar_map(x: float, order: int) -> float:
    """One step of the recursion on an eigenvalue x of X: x -> x p(1 - x)^2."""
    c = [float(v) for v in delta_coefficients(order)]
    d = 1.0 - x
    p = 0.0
    for ck in reversed(c):
        p = p * d + ck
    return x * p * p


# ---------------------------------------------------------------------------
# two-term split (Sec. III.A, Eqs. dualRep and splitStyle)
# ---------------------------------------------------------------------------


def to_fp32(a: np.ndarray) -> np.ndarray:
    """FP32[A]: round-to-nearest-even conversion of FP64 values (IEEE)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def _round_bf16(a32: np.ndarray) -> np.ndarray:
    """BF16 RNE of FP32 values, returned as FP32 numbers (torch CPU conversion)."""
    t = torch.from_numpy(np.ascontiguousarray(a32, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float32).numpy()


def _round_fp16(a32: np.ndarray) -> np.ndarray:
    """FP16 RNE of FP32 values, returned as FP32 numbers (IEEE conversion)."""
    return np.asarray(a32, dtype=np.float32).astype(np.float16).astype(np.float32)


def split(a: np.ndarray, fmt: str = "bf16") -> tuple[np.ndarray, np.ndarray]:
    """A^(h) = LP[A], A^(l) = LP[A - FP32[A^(h)]] with A held in FP32 (Sec. III.A,
    Eq. splitStyle; LP = BF16 or FP16, round to nearest even).

    Returns hi and lo as FP32 arrays holding exactly representable LP values."""
    a32 = to_fp32(a)
    rnd = _round_bf16 if fmt == "bf16" else _round_fp16
    hi = rnd(a32)
    lo = rnd(a32 - hi)           # a32 - hi is exact in FP32
    return hi, lo


def bf16_bits(a32: np.ndarray) -> np.ndarray:
    """Raw 16-bit patterns of FP32 numbers that are exactly BF16-representable."""
    u = np.ascontiguousarray(a32, dtype=np.float32).view(np.uint32)
    if np.any(u & 0xFFFF):
        raise ValueError("value not representable in BF16")
    return (u >> 16).astype(np.uint16)


def fp16_bits(a32: np.ndarray) -> np.ndarray:
    """Raw 16-bit patterns of FP32 numbers that are exactly FP16-representable."""
    h = np.asarray(a32, dtype=np.float32).astype(np.float16)
    if not np.array_equal(h.astype(np.float32), np.asarray(a32, dtype=np.float32), equal_nan=True):
        raise ValueError("value not representable in FP16")
    return h.view(np.uint16)


def split_product(a_hi, a_lo, b_hi, b_lo) -> np.ndarray:
    """(h)(h) + (h)(l) + (l)(h) of Sec. III.B (Eqs. SZn, Xn): the product of two
    split matrices with the (l)(l) term dropped, evaluated in FP64."""
    ah, al, bh, bl = (np.asarray(x, dtype=np.float64) for x in (a_hi, a_lo, b_hi, b_lo))
    return ah @ bh + ah @ bl + al @ bh
