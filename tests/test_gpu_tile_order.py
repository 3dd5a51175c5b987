"""Tile order of symmetric GEMM grids (GPU; through the C ABI).

The order in which blocks take the tiles of an upper triangle (row by row, or in
bands of rows) changes no arithmetic: each output element comes from one tile's dot
products in a fixed K order.  So every band height must give bit-identical outputs
and norms.  That also shows each band walk covers every tile exactly once: the
output buffer starts zeroed, so a tile that no block takes stays zero.
"""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_19163_amd import zf as _zf
    _zf.lib()
    return _zf


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
@pytest.mark.parametrize("n", [1000, 2560, 4096])
def test_band_heights_agree_bitwise(zf, monkeypatch, prec, n):
    rng = np.random.default_rng(n)
    A = torch.from_numpy(rng.standard_normal((n, n))).cuda()
    monkeypatch.setenv("ZF_SYM_TILE_GROUP", "1")  # row by row
    C1, s1 = zf.t_gemm(prec, A, A, sym=True)
    assert torch.count_nonzero(C1).item() == n * n
    for g in ("2", "3", "4", "8"):  # 3 leaves a partial last band on every grid here
        monkeypatch.setenv("ZF_SYM_TILE_GROUP", g)
        C, s = zf.t_gemm(prec, A, A, sym=True)
        assert torch.equal(C, C1), (prec, n, g)
        assert s == s1, (prec, n, g)
