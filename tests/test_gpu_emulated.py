"""Emulated FP64 products on the int8 matrix cores (7-bit integer slices, Ozaki scheme)
and the refinement mode that uses them for the residual, against the CPU oracle.

The slice products are exact in int32 and the FP64 combination follows the oracle's
order (smallest weight first, then the 2^(e_i + f_j) scale), so the GEMM must match
O.ozaki_product bit for bit, epilogue included.  The refinement path's final
residual must equal the oracle's emulated residual of the returned Z (the norm's
summation order differs: relative 1e-12), and the returned Z must meet the mixed bar
(FP64 RMS <= 1e-6, recomputed by the oracle).
"""
import ctypes

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


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


SHAPES = [(128, 128, 128), (200, 200, 300), (96, 260, 70), (1, 1, 1), (384, 256, 513),
          (1024, 1024, 1024)]


@pytest.mark.parametrize("slices", [1, 3, 7, 8])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_emulated_gemm_bit_exact(zf, m, nn, k, slices):
    rng = np.random.default_rng(m + 7 * nn + 13 * k + slices)
    A = rng.standard_normal((m, k)) * np.exp(rng.uniform(-20, 20, (m, 1)))
    B = rng.standard_normal((nn, k)) * np.exp(rng.uniform(-3, 3, (nn, k)))
    C, nsq = zf.t_gemm("emu", _cuda(A), _cuda(B), slices=slices)
    ref = O.ozaki_product(A, B, slices)
    np.testing.assert_array_equal(C.cpu().numpy(), ref)
    assert nsq == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)


@pytest.mark.parametrize("n", [64, 129, 640])
def test_emulated_symmetric_delta_bit_exact(zf, n):
    """The residual's second product: delta = I - Z^T A from the upper triangle,
    mirrored, with the I restricted to the valid block."""
    S = inputs.overlap_gaussian(n, 1.2, 1)
    Z = O.lowdin(S) * (1 + 3e-5)
    Zt = np.ascontiguousarray(Z.T)
    At = O.ozaki_product(Zt, S, 7)
    C, nsq = zf.t_gemm("emu", _cuda(Zt), _cuda(At), sym=True, beta=-1.0, gamma=1.0, slices=7)
    X = O.ozaki_product(Zt, At, 7)
    ref = np.eye(n) - (np.triu(X) + np.triu(X, 1).T)
    got = C.cpu().numpy()
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(ref, O.emulated_residual(S, Z, 7))
    assert nsq == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)


def test_emulated_integer_and_special_rows(zf):
    rng = np.random.default_rng(5)
    A = rng.integers(-127, 128, (130, 200)).astype(float)
    B = rng.integers(-127, 128, (70, 200)).astype(float)
    A[:, 0], B[:, 0] = 127.0, -127.0
    C, _ = zf.t_gemm("emu", _cuda(A), _cuda(B), slices=2)
    np.testing.assert_array_equal(C.cpu().numpy(), A @ B.T)
    A[3] = 0.0                    # a zero row: exact zeros
    A[7, 11] = np.inf             # a non-finite entry: that row's products are NaN
    B[2, 5] = np.nan
    C = zf.t_gemm("emu", _cuda(A), _cuda(B), slices=4)[0].cpu().numpy()
    assert np.all(C[3][np.arange(70) != 2] == 0.0)
    assert np.all(np.isnan(C[7])) and np.all(np.isnan(C[:, 2]))
    ok = np.ones_like(C, dtype=bool)
    ok[7, :] = False
    ok[:, 2] = False
    assert np.all(np.isfinite(C[ok]))


def test_emulated_bad_arguments(zf):
    A = _cuda(np.ones((8, 8)))
    C = torch.empty_like(A)
    L = zf.lib()
    for slices in (0, 9):
        assert L.zf_t_ozaki(slices, 0, 8, 8, 8, A.data_ptr(), A.data_ptr(), 0.0, None, 1.0, 0.0,
                            C.data_ptr(), None, None) == zf.ERR_ARG
    assert L.zf_t_ozaki(7, 0, 8, 8, 16385, A.data_ptr(), A.data_ptr(), 0.0, None, 1.0, 0.0,
                        C.data_ptr(), None, None) == zf.ERR_ARG


@pytest.mark.parametrize("n,seed", [(1, 0), (129, 2), (300, 3), (640, 4)])
def test_refine_emulated_residual(zf, n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed) if n > 1 else np.array([[4.0]])
    r = zf.refine(_cuda(S), None, precision="bf16x3", refine="emu")
    Z = r.Z.cpu().numpy()
    rms64 = O.residual_rms(S, Z)
    rms_emu = O.frobenius(O.emulated_residual(S, Z, 7)) / np.sqrt(n)
    print(f"n={n}: {r.low_evals}+{r.high_evals} evals, final {r.final_rms:.3e}, oracle emulated "
          f"{rms_emu:.3e}, FP64 {rms64:.3e}", flush=True)
    assert r.status == 0 and r.high_evals >= 1
    assert rms64 <= 1e-6
    assert r.final_rms == pytest.approx(rms_emu, rel=1e-10, abs=1e-300)
    # the emulated residual tracks the FP64 one far below the mixed bar
    assert abs(rms_emu - rms64) <= 1e-9


def test_refine_emulated_slice_override(zf, monkeypatch):
    monkeypatch.setenv("ZF_EMU_SLICES", "5")
    S = inputs.overlap_gaussian(200, 1.2, 6)
    r = zf.refine(_cuda(S), None, precision="bf16x3", refine="emu")
    Z = r.Z.cpu().numpy()
    assert r.final_rms == pytest.approx(O.frobenius(O.emulated_residual(S, Z, 5)) / np.sqrt(200),
                                        rel=1e-10)
    assert O.residual_rms(S, Z) <= 1e-6


def test_refine_emulated_rejects_large_n(zf):
    S = _cuda(np.eye(4))
    o = zf.Opts(2, zf.BF16X3, zf.STOP_RATIO, 100, zf.REFINE_EMU, 10, zf.Z0_SCALED_IDENTITY)
    res = zf.Result()
    rc = zf.lib().zf_refine_ex(S.data_ptr(), None, 16385, ctypes.byref(o), S.data_ptr(),
                               ctypes.byref(res), None, 0, None)
    assert rc == zf.ERR_ARG and "16384" in zf.last_error()


def test_n4096_emulated(zf):
    """The N = 4096 Gaussian-kernel overlap: the emulated refinement meets the mixed bar,
    its reported residual equals the oracle's FP64 one to the emulation's accuracy, and
    it reaches the FP64-residual mode's result."""
    S = inputs.workload("gauss4096", 0)
    Sd = _cuda(S)
    re = zf.refine(Sd, None, precision="bf16x3", refine="emu")
    rd = zf.refine(Sd, None, precision="bf16x3", refine="f64_delta")
    Ze = re.Z.cpu().numpy()
    rms = O.residual_rms(S, Ze)
    print(f"emu: {re.low_evals}+{re.high_evals} evals, final {re.final_rms:.3e}, FP64 {rms:.3e}; "
          f"f64_delta final {rd.final_rms:.3e}", flush=True)
    assert re.status == 0 and rms <= 1e-6
    assert abs(re.final_rms - rms) <= 1e-9
    assert np.linalg.norm(Ze - rd.Z.cpu().numpy()) / np.linalg.norm(Ze) <= 1e-8
