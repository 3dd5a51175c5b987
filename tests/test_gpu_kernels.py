"""Kernel-level parity of libzf against the CPU oracle (GPU; runs through the C ABI).

Tolerances:
* split: bit-exact (an integer decision taken in FP32 on both sides).
* FP64 GEMM: |C - C_ref| <= 2 K u64 (|A||B|^T) + 2 u64 |C_ref|, u64 = 2^-53, the
  standard dot-product bound with a margin of 2.
* BF16x3 GEMM: against the oracle's FP64 evaluation of the same three products,
  |C - C_ref| <= 3 K u32 (|A_h| + |A_l|)(|B_h| + |B_l|)^T, u32 = 2^-24: every
  product is exact in FP32 and at most 3K additions round into the accumulator.
  Against the exact product, the two-term representation adds 3 u^2 |A||B|^T
  with u = 2^-8 (Sec. III.A error bound, three neglected or split terms).
"""
import math

import numpy as np
import pytest
import torch

from oracle import zf_oracle as O

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def zf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_19163_amd import zf as _zf
    _zf.lib()
    return _zf


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _edge_values():
    v = [0.0, -0.0, 1.0, -1.0, 2.0 ** -126, 2.0 ** -149, 3.3895313892515355e38, 1e-30, 65504.0,
         6.1e-5, 5.96e-8, 1 + 2.0 ** -8, 1 + 2.0 ** -9, 1 + 3 * 2.0 ** -9, 1 + 2.0 ** -24,
         1 + 2.0 ** -25, float("inf"), -float("inf"), 1e300, 1e-300]
    return np.array(v)


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_split_bit_exact(zf, fmt):
    rng = np.random.default_rng(0)
    a = np.concatenate([_edge_values(),
                        rng.standard_normal(50000) * np.exp(rng.uniform(-20, 20, 50000)),
                        rng.uniform(-1, 1, 3333)])
    if fmt == "fp16":
        a = a[np.abs(a) < 6e4]
    hi, lo = zf.t_split(_cuda(a), fmt)
    ohi, olo = O.split(a, fmt)
    bits = O.bf16_bits if fmt == "bf16" else O.fp16_bits
    for got, want in ((hi, ohi), (lo, olo)):
        g = got.cpu().numpy().view(np.uint16)
        nan = np.isnan(want)
        # NaN (lo of an infinite value: inf - inf) has no canonical payload
        expo = 0x7F80 if fmt == "bf16" else 0x7C00
        assert np.all((g[nan] & expo) == expo) and np.all((g[nan] & ~np.uint16(expo | 0x8000)) != 0)
        np.testing.assert_array_equal(g[~nan], bits(want[~nan]))


def test_split_empty(zf):
    hi, lo = zf.t_split(torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert hi.numel() == 0


SHAPES = [(128, 128, 128), (200, 200, 300), (96, 260, 70), (1, 1, 1), (384, 256, 513), (640, 640, 384),
          (1024, 512, 256)]   # the last: 16 x 8 tile grid walked in groups of 4 rows


@pytest.mark.parametrize("tile", ["64", "128"])
@pytest.mark.parametrize("m,nn,k", SHAPES + [(1536, 1536, 256)])
def test_gemm_f64(zf, m, nn, k, tile, monkeypatch):
    """Both FP64 tile edges (64 is the default; 128 when ZF_F64_TILE asks and divides)."""
    monkeypatch.setenv("ZF_F64_TILE", tile)
    rng = np.random.default_rng(m * 7 + nn + k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((nn, k))
    C, _ = zf.t_gemm("fp64", _cuda(A), _cuda(B))
    ref = A @ B.T
    bound = 2 * k * U64 * (np.abs(A) @ np.abs(B).T) + 2 * U64 * np.abs(ref)
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("tile", ["64", "128", "256"])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_gemm_bf16x3(zf, m, nn, k, tile, monkeypatch):
    monkeypatch.setenv("ZF_X3_TILE", tile)
    rng = np.random.default_rng(m * 5 + nn + 3 * k)
    A = rng.standard_normal((m, k)) * np.exp(rng.uniform(-3, 3, (m, 1)))
    B = rng.standard_normal((nn, k))
    C, _ = zf.t_gemm("bf16x3", _cuda(A), _cuda(B))
    C = C.cpu().numpy()
    ah, al = O.split(A)
    bh, bl = O.split(B)
    ref = O.split_product(ah, al, bh.T, bl.T)
    absx = (np.abs(ah) + np.abs(al)).astype(float) @ (np.abs(bh) + np.abs(bl)).astype(float).T
    assert np.all(np.abs(C - ref) <= 3 * k * U32 * absx)
    exact = A @ B.T
    u = 2.0 ** -8
    assert np.all(np.abs(C - exact) <= (3 * u * u + 3 * k * U32) * (np.abs(A) @ np.abs(B).T) * 1.01)


@pytest.mark.parametrize("tile", ["64", "128", "256"])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_gemm_hh(zf, m, nn, k, tile, monkeypatch):
    """(h)(h): the hi halves' product only, FP32 accumulation of exact products."""
    monkeypatch.setenv("ZF_X3_TILE", tile)
    rng = np.random.default_rng(m * 3 + nn + 7 * k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((nn, k))
    C, _ = zf.t_gemm("bf16", _cuda(A), _cuda(B))
    ah, _ = O.split(A)
    bh, _ = O.split(B)
    ref = ah.astype(float) @ bh.astype(float).T
    bound = 2 * k * U32 * (np.abs(ah).astype(float) @ np.abs(bh).astype(float).T)
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("tile", ["64", "128", "256"])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_gemm_fp32(zf, m, nn, k, tile, monkeypatch):
    """FP32 operands on the FP32 matrix cores (K traversed in a permuted order): within
    the FP32 dot-product bound of the product of the FP32-rounded operands."""
    monkeypatch.setenv("ZF_X3_TILE", tile)
    rng = np.random.default_rng(m * 11 + nn + 5 * k)
    A = rng.standard_normal((m, k)) * np.exp(rng.uniform(-3, 3, (m, 1)))
    B = rng.standard_normal((nn, k))
    C, _ = zf.t_gemm("fp32", _cuda(A), _cuda(B))
    a32 = O.to_fp32(A).astype(float)
    b32 = O.to_fp32(B).astype(float)
    ref = a32 @ b32.T
    bound = 2 * k * U32 * (np.abs(a32) @ np.abs(b32).T)
    assert np.all(np.abs(C.cpu().numpy() - ref) <= bound)


@pytest.mark.parametrize("prec", ["fp16x3", "fp16"])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_gemm_fp16_halves(zf, prec, m, nn, k):
    """FP16 halves (the paper's Eq. splitStyle): each product of halves is exact in
    FP32 (11 + 11 significant bits), so the bound is the FP32 accumulation bound of
    the (h)(h)(+(h)(l)+(l)(h)) sum of the oracle's FP16 split."""
    rng = np.random.default_rng(m * 13 + nn + 3 * k)
    A = rng.standard_normal((m, k))
    B = rng.standard_normal((nn, k))
    C, _ = zf.t_gemm(prec, _cuda(A), _cuda(B))
    C = C.cpu().numpy()
    ah, al = O.split(A, "fp16")
    bh, bl = O.split(B, "fp16")
    if prec == "fp16x3":
        ref = O.split_product(ah, al, bh.T, bl.T)
        absx = (np.abs(ah) + np.abs(al)).astype(float) @ (np.abs(bh) + np.abs(bl)).astype(float).T
        assert np.all(np.abs(C - ref) <= 3 * k * U32 * absx)
        exact = A @ B.T
        u = 2.0 ** -11
        assert np.all(np.abs(C - exact) <= (3 * u * u + 3 * k * U32) * (np.abs(A) @ np.abs(B).T) * 1.01)
    else:
        ref = ah.astype(float) @ bh.astype(float).T
        bound = 2 * k * U32 * (np.abs(ah).astype(float) @ np.abs(bh).astype(float).T)
        assert np.all(np.abs(C - ref) <= bound)


def test_fp16_matrix_cores_keep_subnormal_halves(zf):
    """Operands whose lo halves are FP16 subnormals (2^-24 .. 2^-14): the product
    keeps them (a flushed lo would leave an error of the lo's size, far above the
    accumulation bound)."""
    rng = np.random.default_rng(3)
    A = rng.uniform(0.5, 1.0, (128, 128)) * 2.0 ** -8 * np.sign(rng.standard_normal((128, 128)))
    B = rng.uniform(0.5, 1.0, (128, 128))
    ah, al = O.split(A, "fp16")
    assert np.mean(np.abs(al[al != 0]) < 2.0 ** -14) > 0.5   # mostly subnormal lo halves
    bh, bl = O.split(B, "fp16")
    C, _ = zf.t_gemm("fp16x3", _cuda(A), _cuda(B))
    ref = O.split_product(ah, al, bh.T, bl.T)
    absx = (np.abs(ah) + np.abs(al)).astype(float) @ (np.abs(bh) + np.abs(bl)).astype(float).T
    assert np.all(np.abs(C.cpu().numpy() - ref) <= 3 * 128 * U32 * absx)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("n,k", [(128, 128), (300, 200), (1000, 256)])
def test_gemm_symmetric_fp32_hh(zf, prec, n, k):
    rng = np.random.default_rng(n + 3 * k)
    A = rng.standard_normal((n, k)) / math.sqrt(k)
    M = rng.standard_normal((k, k))
    B = A @ ((M + M.T) / 2)
    C, nsq = zf.t_gemm(prec, _cuda(A), _cuda(B), sym=True, beta=-1.0, gamma=1.0)
    C = C.cpu().numpy()
    assert np.array_equal(C, C.T)
    if prec == "fp32":
        a, b = O.to_fp32(A).astype(float), O.to_fp32(B).astype(float)
        bound = 2 * k * U32 * (np.abs(a) @ np.abs(b).T) + 4 * U32
    else:
        a, _ = O.split(A)
        b, _ = O.split(B)
        a, b = a.astype(float), b.astype(float)
        bound = 2 * k * U32 * (np.abs(a) @ np.abs(b).T) + 4 * U32
    ref = np.eye(n) - a @ b.T
    up = np.triu(np.ones((n, n), dtype=bool))
    assert np.all(np.abs(C - ref)[up] <= bound[up])
    assert nsq == pytest.approx(math.fsum((C * C).ravel().tolist()), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp64-t128", "bf16x3", "bf16x3-t128", "bf16x3-t64"])
@pytest.mark.parametrize("n,k", [(128, 128), (300, 200), (640, 512), (129, 64), (1000, 256),
                                 (2048, 128)])
def test_gemm_symmetric_delta_epilogue(zf, prec, n, k, monkeypatch):
    """delta = I - A M A^T (symmetric product) in symmetric mode: only tiles on or
    above the diagonal are computed; the result is mirrored exactly and the norm
    partials reproduce ||delta||_F."""
    rng = np.random.default_rng(n + k)
    A = rng.standard_normal((n, k)) / math.sqrt(k)
    M = rng.standard_normal((k, k))
    M = (M + M.T) / 2
    B = A @ M                     # A B^T = A M A^T is symmetric
    if "-t" in prec:
        prec, tile = prec.split("-t")
        monkeypatch.setenv("ZF_X3_SYM_TILE" if prec == "bf16x3" else "ZF_F64_SYM_TILE", tile)
    C, nsq = zf.t_gemm(prec, _cuda(A), _cuda(B), sym=True, beta=-1.0, gamma=1.0)
    C = C.cpu().numpy()
    assert np.array_equal(C, C.T)
    if prec == "fp64":
        ref = np.eye(n) - A @ B.T
        tol = 4 * k * U64 * (np.abs(A) @ np.abs(B).T) + 4 * U64
    else:
        ah, al = O.split(A)
        bh, bl = O.split(B)
        ref = np.eye(n) - O.split_product(ah, al, bh.T, bl.T)
        tol = 3 * k * U32 * ((np.abs(ah) + np.abs(al)).astype(float)
                             @ (np.abs(bh) + np.abs(bl)).astype(float).T) + 4 * U32
    # the mirrored half equals the computed half of the (slightly asymmetric) reference
    up = np.triu(np.ones((n, n), dtype=bool))
    assert np.all(np.abs(C - ref)[up] <= tol[up] if np.ndim(tol) else np.abs(C - ref)[up] <= tol)
    assert nsq == pytest.approx(math.fsum((C * C).ravel().tolist()), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp64", "bf16x3"])
def test_gemm_alpha_d_epilogue(zf, prec):
    """out = alpha D + beta (A B^T), the Z + Z Q and c1 delta + c2 delta^2 forms."""
    rng = np.random.default_rng(9)
    n, k = 257, 190
    A = rng.standard_normal((n, k))
    B = rng.standard_normal((n, k))
    D = rng.standard_normal((n, n))
    C, _ = zf.t_gemm(prec, _cuda(A), _cuda(B), alpha=0.5, D=_cuda(D), beta=0.375)
    ref = 0.5 * D + 0.375 * (A @ B.T)
    scale = np.abs(A) @ np.abs(B).T
    tol = (4 * k * U64 if prec == "fp64" else (3 * 2.0 ** -16 + 3 * k * U32)) * scale + 1e-15
    assert np.all(np.abs(C.cpu().numpy() - ref) <= tol)


@pytest.mark.parametrize("n", [1, 5, 256, 1000])
def test_gershgorin(zf, n):
    rng = np.random.default_rng(n)
    S = rng.standard_normal((n, n))
    S = S + S.T
    g = zf.t_gershgorin(_cuda(S))
    assert g == pytest.approx(O.gershgorin_max_row_sum(S), rel=1e-14)



@pytest.mark.parametrize("prec", ["bf16x3", "bf16", "fp16x3"])
@pytest.mark.parametrize("m,nn,k", [(3072, 3072, 3072), (3000, 2900, 3100)])
def test_gemm_large_tile_grid(zf, m, nn, k, prec):
    """256-wide tiles on grids of 144 and 169 tiles (fewer than the CUs), with the
    alpha D + beta A B^T epilogue and a ragged edge."""
    rng = np.random.default_rng(m + nn + k)
    A = rng.standard_normal((m, k)) * np.exp(rng.uniform(-3, 3, (m, 1)))
    B = rng.standard_normal((nn, k))
    D = rng.standard_normal((m, nn))
    C, _ = zf.t_gemm(prec, _cuda(A), _cuda(B), alpha=0.5, D=_cuda(D), beta=0.375)
    C = C.cpu().numpy()
    fmt = "fp16" if prec == "fp16x3" else "bf16"
    ah, al = O.split(A, fmt)
    bh, bl = O.split(B, fmt)
    if prec == "bf16":
        ref = ah.astype(float) @ bh.astype(float).T
        absx = np.abs(ah).astype(float) @ np.abs(bh).astype(float).T
        terms = 2
    else:
        ref = O.split_product(ah, al, bh.T, bl.T)
        absx = (np.abs(ah) + np.abs(al)).astype(float) @ (np.abs(bh) + np.abs(bl)).astype(float).T
        terms = 3
    ref = 0.5 * D + 0.375 * ref
    bound = 0.375 * terms * k * U32 * absx + 1e-15 * np.abs(D)
    assert np.all(np.abs(C - ref) <= bound)


@pytest.mark.parametrize("k", [512, 4096])
def test_gemm_symmetric_delta_n4096(zf, k):
    """The N = 4096 symmetric product (136 tiles of 256) with the symmetric delta
    epilogue, exact mirroring and the norm partials."""
    n = 4096
    rng = np.random.default_rng(k)
    A = rng.standard_normal((n, k)) / math.sqrt(k)
    M = rng.standard_normal((k, k))
    M = (M + M.T) / 2
    B = A @ M
    C, nsq = zf.t_gemm("bf16x3", _cuda(A), _cuda(B), sym=True, beta=-1.0, gamma=1.0)
    C = C.cpu().numpy()
    assert np.array_equal(C, C.T)
    ah, al = O.split(A)
    bh, bl = O.split(B)
    ref = np.eye(n) - O.split_product(ah, al, bh.T, bl.T)
    tol = 3 * k * U32 * ((np.abs(ah) + np.abs(al)).astype(float)
                         @ (np.abs(bh) + np.abs(bl)).astype(float).T) + 4 * U32
    up = np.triu(np.ones((n, n), dtype=bool))
    assert np.all((np.abs(C - ref) <= tol)[up])
    assert nsq == pytest.approx(math.fsum((C * C).ravel().tolist()), rel=1e-12)


@pytest.mark.parametrize("tile", ["64", "128", "256"])
@pytest.mark.parametrize("prec", ["bf16x3", "bf16", "fp16x3"])
@pytest.mark.parametrize("sym", [False, True])
def test_gemm_kblocked_operands_bitwise(zf, prec, sym, tile, monkeypatch):
    """The solver keeps its pairs K-blocked (32-wide K panels): the same products in the
    same order as the row-major operands, so C and the norm agree bit for bit, on every
    tile edge and on a ragged size (padded to 768, three 256-wide K blocks of panels)."""
    monkeypatch.setenv("ZF_X3_TILE", tile)
    monkeypatch.setenv("ZF_X3_SYM_TILE", tile)
    rng = np.random.default_rng(17 + len(prec) + 2 * int(tile) + sym)
    n, k = 700, 700
    A = rng.standard_normal((n, k))
    B = A @ np.diag(rng.uniform(0.5, 2.0, k)) if sym else rng.standard_normal((n, k))
    D = rng.standard_normal((n, n))
    if sym:
        D = D + D.T
    args = dict(sym=sym, alpha=0.5, D=_cuda(D), beta=-1.0, gamma=1.0)
    C_rm, n_rm = zf.t_gemm(prec, _cuda(A), _cuda(B), **args)
    C_kb, n_kb = zf.t_gemm(prec, _cuda(A), _cuda(B), kblocked=True, **args)
    assert torch.equal(C_rm, C_kb)
    assert n_rm == n_kb
