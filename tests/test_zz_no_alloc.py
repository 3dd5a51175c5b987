"""zf_residual_noalloc, the allocation-free variant of zf_residual (GPU; through the C
ABI): the same RMS residual, bit for bit, on two calls in a row (the second with a
smaller matrix and a smaller padded order), written into a device scalar; sizes above
its limit are refused; repeated calls leave the device's free memory unchanged."""
import numpy as np
import pytest
import torch

from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_19163_amd import zf as _zf
    _zf.lib()
    return _zf


def _case(n, seed):
    S = inputs.overlap_gaussian(n, 1.1, seed)
    rng = np.random.default_rng(seed)
    # an approximate factor: the scaled identity plus noise (residual far from zero)
    Z = O.scaled_identity_guess(S) + 1e-3 * rng.standard_normal((n, n))
    return S, Z


def test_noalloc_equals_residual_two_calls(zf):
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda:0")
    for k, (n, seed) in enumerate([(1000, 0), (300, 1)]):
        S, Z = _case(n, seed)
        Sd = torch.from_numpy(S).cuda()
        Zd = torch.from_numpy(Z).cuda()
        ref = zf.residual(Sd, Zd)  # the allocating entry point
        zf.residual_noalloc(Sd, Zd, out[k:])
        torch.cuda.synchronize()
        got = float(out[k])
        print(f"n={n}: residual {ref!r} noalloc {got!r} oracle {O.residual_rms(S, Z)!r}")
        assert got == ref
        assert got == pytest.approx(O.residual_rms(S, Z), rel=1e-12)


def test_noalloc_limits_and_no_allocation(zf):
    S, Z = _case(1024, 2)
    Sd = torch.from_numpy(S).cuda()
    Zd = torch.from_numpy(Z).cuda()
    out = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    zf.residual_noalloc(Sd, Zd, out)  # n = 1024, the largest order it takes
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        zf.residual_noalloc(Sd, Zd, out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert float(out[0]) == zf.residual(Sd, Zd)
    big = torch.zeros((1025, 1025), dtype=torch.float64, device="cuda:0")
    with pytest.raises(zf.ZFError):
        zf.residual_noalloc(big, big, out)
