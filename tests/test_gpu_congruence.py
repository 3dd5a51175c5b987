"""Parity of zf_congruence (H_perp = Z^T H Z, Sec. II.A, Eq. standard_form) against the
oracle's FP64 Z^T (H Z), element by element, through the C ABI.

Z is the inverse Cholesky factor of S (upper triangular, Z^T S Z = I, not symmetric), so
a product taken on the wrong side shows.  H is the extended-Hueckel Hamiltonian of S.

Bound, elementwise, built from the oracle's own split of the actual operands (so that
FP16 lo halves in the subnormal range are covered) and carried through both products.
The device forms W = H Z first (as the rows of Z^T H), stores it in the product's input
format, then Z^T W.  For one product P = A^T B (K = padded inner dimension,
u32 = 2^-24, r_X = X - (X_hi + X_lo) the split's representation error):
* three split products: |A_lo|^T |B_lo| + |r_A|^T |B| + |A|^T |r_B|
  + 3 K u32 (|A_hi| + |A_lo|)^T (|B_hi| + |B_lo|)   (every product of halves is exact
  in FP32; 3K additions round into one accumulator);
* (h)(h): |A - A_hi|^T |B| + |A_hi|^T |B - B_hi| + 2 K u32 |A_hi|^T |B_hi|;
* FP32: |A - fl32(A)|^T |B| + |A|^T |B - fl32(B)| + 2 K u32 |A|^T |B|;
and the second product adds its own terms with W's computed value, |W| + E_1, in
place of W: its split error (u^2 (|W| + E_1) + q for a pair, u (|W| + E_1) + q for the
hi half alone, u the half's unit roundoff, q half the FP16 subnormal spacing; zero for
FP32, which keeps W in FP32).  FP32 underflow adds 6 K 2^-126 (1 + sum_k |Z_ki|) (tiny
overlaps put values below the FP32 normal range).  FP64: 4 K u64 |Z|^T |H| |Z|.  The bound is symmetrized (the lower
triangle is the mirror of the upper) and given a 5 % margin for second-order terms.
"""
import numpy as np
import pytest
import torch

from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs

pytestmark = pytest.mark.gpu

U64, U32 = 2.0 ** -53, 2.0 ** -24
FMT = {"bf16x3": "bf16", "bf16": "bf16", "fp16x3": "fp16", "fp16": "fp16", "fp32": None}
THREE = {"bf16x3": True, "fp16x3": True, "bf16": False, "fp16": False}


@pytest.fixture(scope="module")
def zf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_19163_amd import zf as _zf
    _zf.lib()
    return _zf


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _case(n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed)
    H = inputs.huckel_hamiltonian(S, seed + 100)
    Z = np.linalg.inv(np.linalg.cholesky(S)).T
    return S, H, Z


def _kpad(n):
    return -(-n // 256) * 256


def _parts(X, prec):
    """(|hi|, |lo|, |representation error|) of X in the path's input format."""
    if FMT[prec] is None:
        x32 = O.to_fp32(X).astype(np.float64)
        return np.abs(x32), np.zeros_like(X), np.abs(X - x32)
    hi, lo = O.split(X, FMT[prec])
    hi, lo = hi.astype(np.float64), lo.astype(np.float64)
    if THREE[prec]:
        return np.abs(hi), np.abs(lo), np.abs(X - hi - lo)
    return np.abs(hi), np.zeros_like(X), np.abs(X - hi)


def _product_err(prec, K, A, B):
    """Bound on |fl(A^T B) - A^T B| for the path's product of A^T and B."""
    ah, al, ar = _parts(A, prec)
    bh, bl, br = _parts(B, prec)
    aA, aB = np.abs(A), np.abs(B)
    if FMT[prec] is None:
        return ar.T @ aB + aA.T @ br + 2 * K * U32 * aA.T @ aB
    if THREE[prec]:
        return (al.T @ bl + ar.T @ aB + aA.T @ br + 3 * K * U32 * (ah + al).T @ (bh + bl))
    return ar.T @ aB + ah.T @ br + 2 * K * U32 * ah.T @ bh


U_HALF = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}   # unit roundoff of one half
Q_HALF = {"bf16": 0.0, "fp16": 2.0 ** -25}          # half the FP16 subnormal spacing


def _bound(prec, n, H, Z):
    K = _kpad(n)
    aZ = np.abs(Z)
    if prec == "fp64":
        return 4 * K * U64 * (aZ.T @ np.abs(H) @ aZ) + 1e-300
    e1 = _product_err(prec, K, H, Z)            # first product, H symmetric: |H|^T = |H|
    Wb = np.abs(H @ Z) + e1                     # |W_computed| <= |W| + e1
    _, zl, zr = _parts(Z, prec)
    if FMT[prec] is None:                       # W stays in FP32: no second rounding
        b2 = zr.T @ Wb + 2 * K * U32 * aZ.T @ Wb
    else:
        u, q = U_HALF[FMT[prec]], Q_HALF[FMT[prec]]
        if THREE[prec]:                         # W's pair: |W_lo| <= u |W|, error u^2 |W| + q
            rW = u * u * Wb + q
            b2 = zl.T @ (u * Wb) + zr.T @ Wb + aZ.T @ rW + 3 * K * U32 * (1 + u) * aZ.T @ Wb
        else:                                   # (h)(h) reads W's hi half only
            rW = u * Wb + q
            b2 = zr.T @ Wb + aZ.T @ rW + 2 * K * U32 * aZ.T @ Wb
    # FP32 underflow: values below the FP32 normal range (tiny overlaps, and H with
    # them) may round or flush by up to 2^-126 at each of the <= 6K operations of an
    # output; the first product's absolute error reaches the second through |Z|^T
    t = 6 * K * 2.0 ** -126
    b = aZ.T @ e1 + b2 + t * (aZ.sum(axis=0)[:, None] + 1.0)
    return 1.05 * np.maximum(b, b.T) + 1e-300


PRECS = ["fp64", "bf16x3", "fp16x3", "fp32", "bf16", "fp16"]


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,seed", [(1, 0), (64, 1), (129, 2), (300, 3), (1000, 4)])
def test_congruence_parity(zf, prec, n, seed):
    S, H, Z = _case(n, seed)
    ref = O.congruence(H, Z)
    got = zf.congruence(_cuda(H), _cuda(Z), precision=prec).cpu().numpy()
    err = np.abs(got - ref)
    bnd = _bound(prec, n, H, Z)
    ratio = float(np.max(err / bnd))
    rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print(f"{prec} n={n}: max err/bound {ratio:.3f}, rel Frobenius {rel:.2e}", flush=True)
    assert np.array_equal(got, got.T)            # upper triangle computed and mirrored
    assert ratio <= 1.0


def test_congruence_generalized_eigenvalues(zf):
    """With Z from the library's own refinement (mixed path), the spectrum of H_perp is
    the generalized spectrum of (H, S) from LAPACK to the residual's level."""
    import scipy.linalg
    n = 400
    S, H, _ = _case(n, 7)
    r = zf.refine(_cuda(S), None, precision="bf16x3")
    Hp = zf.congruence(_cuda(H), r.Z, precision="fp64").cpu().numpy()
    w = np.linalg.eigvalsh(Hp)
    ref = scipy.linalg.eigh(H, S, eigvals_only=True)
    # Z^T S Z = I + E shifts the eigenvalues by at most ||E||_2 max|eps|
    tol = 2 * r.final_rms * np.sqrt(n) * np.max(np.abs(ref))
    print(f"max eigenvalue deviation {np.max(np.abs(w - ref)):.2e} (tol {tol:.2e})", flush=True)
    assert np.max(np.abs(w - ref)) <= tol


@pytest.mark.parametrize("which", ["H", "Z"])
def test_congruence_output_aliases_input(zf, which):
    S, H, Z = _case(200, 5)
    Hd, Zd = _cuda(H), _cuda(Z)
    out = Hd if which == "H" else Zd
    zf.congruence(Hd, Zd, precision="bf16x3", out=out)
    ref = O.congruence(H, Z)
    got = out.cpu().numpy()
    assert np.max(np.abs(got - ref) / _bound("bf16x3", 200, H, Z)) <= 1.0


def test_congruence_full_size_sampled(zf):
    """N = 4096 Gaussian-kernel overlap and its Hamiltonian, Z from the mixed refinement:
    256 sampled entries Z[:, i]^T H Z[:, j] recomputed one by one by the oracle."""
    S = inputs.workload("gauss4096", 0)
    H = inputs.huckel_hamiltonian(S, 100)
    Sd, Hd = _cuda(S), _cuda(H)
    Z = zf.refine(Sd, None, precision="bf16x3").Z
    Zn = Z.cpu().numpy()
    rng = np.random.default_rng(0)
    idx = rng.integers(0, 4096, size=(256, 2))
    cols = np.unique(idx.ravel())
    pos = {int(c): k for k, c in enumerate(cols)}
    Zs = Zn[:, cols]                       # the sampled columns of Z
    ref = O.congruence(H, Zs)              # entries Z[:, i]^T H Z[:, j] of the sample
    for prec in ("fp64", "bf16x3"):
        Hp = zf.congruence(Hd, Z, precision=prec).cpu().numpy()
        assert np.array_equal(Hp, Hp.T)
        bnd = _bound(prec, 4096, H, Zs)
        worst = 0.0
        for i, j in idx:
            a, b = pos[int(i)], pos[int(j)]
            worst = max(worst, abs(Hp[i, j] - ref[a, b]) / bnd[a, b])
        print(f"{prec}: worst sampled err/bound {worst:.3f}", flush=True)
        assert worst <= 1.0


def test_congruence_rejects_bad_arguments(zf):
    H = _cuda(np.eye(8))
    import ctypes
    assert zf.lib().zf_congruence(H.data_ptr(), None, 8, 0, H.data_ptr(), None) == zf.ERR_ARG
    assert zf.lib().zf_congruence(H.data_ptr(), H.data_ptr(), 0, 0, H.data_ptr(), None) == zf.ERR_ARG
    assert zf.lib().zf_congruence(H.data_ptr(), H.data_ptr(), 8, 9, H.data_ptr(), None) == zf.ERR_ARG
    assert "precision" in zf.last_error()
