"""FP64 products emulated through residues on the int8 matrix cores (row truncation
to beta-bit integers, one int8 product per modulus, Chinese remainder theorem) and the
refinement modes that use them for the residual, against the CPU oracle.

The oracle defines the product as the exact integer product of the truncated rows,
scaled and rounded once.  The library reconstructs that integer from its residues in
FP64 limbs: the result must lie within two units of the integer product's last place
(2^(e_i + f_j - 2 beta)) plus one rounding of the exact value.  Integer matrices are
exact.  The refinement modes must meet the mixed bar (FP64 RMS <= 1e-6 recomputed by
the oracle, Z within 1e-4 of the oracle's FP64 iterate) and report the residual of the
arithmetic they ran (the emulated one for ZF_REFINE_CRT, FP64 for ZF_REFINE_CRT_FIRST).
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


def _units(A, B, L, k):
    beta = O.crt_beta(k, L)
    ea = np.frexp(np.max(np.abs(A), axis=1))[1]
    eb = np.frexp(np.max(np.abs(B), axis=1))[1]
    return np.ldexp(1.0, ea[:, None] + eb[None, :] - 2 * beta)


def _assert_close(got, ref, units):
    err = np.abs(got - ref)
    bound = 2.0 * units + np.abs(ref) * 2.0 ** -51
    bad = err > bound
    assert not np.any(bad), (np.max(err / bound), np.argwhere(bad)[:5])


SHAPES = [(256, 256, 256), (200, 200, 300), (96, 260, 70), (1, 1, 1), (384, 256, 513),
          (1024, 1024, 1024)]


@pytest.mark.parametrize("L", [8, 12, 14, 15])
@pytest.mark.parametrize("m,nn,k", SHAPES)
def test_crt_gemm_against_exact_product(zf, m, nn, k, L):
    rng = np.random.default_rng(m + 7 * nn + 13 * k + L)
    A = rng.standard_normal((m, k)) * np.exp(rng.uniform(-20, 20, (m, 1)))
    B = rng.standard_normal((nn, k)) * np.exp(rng.uniform(-3, 3, (nn, k)))
    C, nsq = zf.t_gemm("crt", _cuda(A), _cuda(B), slices=L)
    ref = O.crt_product(A, B, L)
    got = C.cpu().numpy()
    _assert_close(got, ref, _units(A, B, L, k))
    assert nsq == pytest.approx(float(np.sum(ref * ref)), rel=1e-12)


@pytest.mark.parametrize("n", [64, 129, 640])
def test_crt_symmetric_delta(zf, n):
    """The residual's second product: delta = I - Z^T A from the upper triangle,
    mirrored exactly, with the I restricted to the valid block."""
    S = inputs.overlap_gaussian(n, 1.2, 1)
    Z = O.lowdin(S) * (1 + 3e-5)
    Zt = np.ascontiguousarray(Z.T)
    At = O.crt_product(Zt, S, 14)
    C, nsq = zf.t_gemm("crt", _cuda(Zt), _cuda(At), sym=True, beta=-1.0, gamma=1.0, slices=14)
    got = C.cpu().numpy()
    ref = O.crt_residual(S, Z, 14)
    assert np.array_equal(got, got.T)
    _assert_close(got, ref, _units(Zt, At, 14, n))
    assert nsq == pytest.approx(float(np.sum(ref * ref)), rel=1e-9)


def test_crt_integer_and_special_rows(zf):
    rng = np.random.default_rng(5)
    A = rng.integers(-1000, 1001, (130, 200)).astype(float)
    B = rng.integers(-1000, 1001, (70, 200)).astype(float)
    C, _ = zf.t_gemm("crt", _cuda(A), _cuda(B), slices=14)
    np.testing.assert_array_equal(C.cpu().numpy(), A @ B.T)
    A[3] = 0.0                    # a zero row: exact zeros
    A[7, 11] = np.inf             # a non-finite entry: that row's products are NaN
    B[2, 5] = np.nan
    C = zf.t_gemm("crt", _cuda(A), _cuda(B), slices=14)[0].cpu().numpy()
    assert np.all(C[3][np.arange(70) != 2] == 0.0)
    assert np.all(np.isnan(C[7])) and np.all(np.isnan(C[:, 2]))
    ok = np.ones_like(C, dtype=bool)
    ok[7, :] = False
    ok[:, 2] = False
    assert np.all(np.isfinite(C[ok]))


def test_crt_bad_arguments(zf):
    A = _cuda(np.ones((8, 8)))
    C = torch.empty_like(A)
    L = zf.lib()
    for moduli in (1, 16):
        assert L.zf_t_crt(moduli, 0, 8, 8, 8, A.data_ptr(), A.data_ptr(), 0.0, None, 1.0, 0.0,
                          C.data_ptr(), None, None) == zf.ERR_ARG
    assert L.zf_t_crt(14, 0, 8, 8, 16385, A.data_ptr(), A.data_ptr(), 0.0, None, 1.0, 0.0,
                      C.data_ptr(), None, None) == zf.ERR_ARG


@pytest.mark.parametrize("n,seed", [(1, 0), (129, 2), (300, 3), (640, 4)])
def test_refine_crt_residual(zf, n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed) if n > 1 else np.array([[4.0]])
    ref = O.refine(S, O.scaled_identity_guess(S), order=2)
    for mode in ("crt", "crt_first"):
        r = zf.refine(_cuda(S), None, precision="bf16x3", refine=mode)
        Z = r.Z.cpu().numpy()
        rms64 = O.residual_rms(S, Z)
        rms_crt = O.frobenius(O.crt_residual(S, Z, 14)) / np.sqrt(n)
        print(f"n={n} {mode}: {r.low_evals}+{r.high_evals} evals, final {r.final_rms:.3e}, "
              f"oracle emulated {rms_crt:.3e}, FP64 {rms64:.3e}", flush=True)
        assert r.status == 0 and r.high_evals >= 1
        assert rms64 <= 1e-6
        assert np.linalg.norm(Z - ref.Z) / np.linalg.norm(ref.Z) <= 1e-4
        if mode == "crt" or r.high_evals == 1:
            # the last evaluation was emulated
            assert r.final_rms == pytest.approx(rms_crt, rel=1e-6, abs=1e-300)
        else:
            assert r.final_rms == pytest.approx(rms64, rel=1e-6, abs=1e-300)
        assert abs(rms_crt - rms64) <= 1e-9


def test_refine_crt_moduli_override(zf, monkeypatch):
    monkeypatch.setenv("ZF_EMU_MODULI", "12")
    S = inputs.overlap_gaussian(200, 1.2, 6)
    r = zf.refine(_cuda(S), None, precision="bf16x3", refine="crt")
    Z = r.Z.cpu().numpy()
    assert r.final_rms == pytest.approx(O.frobenius(O.crt_residual(S, Z, 12)) / np.sqrt(200),
                                        rel=1e-6)
    assert O.residual_rms(S, Z) <= 1e-6


def test_refine_crt_rejects_large_n(zf):
    S = _cuda(np.eye(4))
    for mode in (zf.REFINE_CRT, zf.REFINE_CRT_FIRST):
        o = zf.Opts(2, zf.BF16X3, zf.STOP_RATIO, 100, mode, 10, zf.Z0_SCALED_IDENTITY)
        res = zf.Result()
        rc = zf.lib().zf_refine_ex(S.data_ptr(), None, 16385, ctypes.byref(o), S.data_ptr(),
                                   ctypes.byref(res), None, 0, None)
        assert rc == zf.ERR_ARG and "16384" in zf.last_error()


@pytest.mark.parametrize("wl", ["gauss4096", "cluster5049"])
def test_fullsize_crt(zf, wl):
    """The N = 4096 overlap and the ill-conditioned N = 5049 cluster: both residue modes
    meet the mixed bar and land on the FP64-residual mode's Z."""
    S = inputs.workload(wl, 0)
    Sd = _cuda(S)
    rd = zf.refine(Sd, None, precision="bf16x3", refine="f64_delta")
    Zd = rd.Z.cpu().numpy()
    for mode in ("crt_first", "crt"):
        r = zf.refine(Sd, None, precision="bf16x3", refine=mode)
        Z = r.Z.cpu().numpy()
        rms = O.residual_rms(S, Z)
        print(f"{wl} {mode}: {r.low_evals}+{r.high_evals} evals, final {r.final_rms:.3e}, FP64 "
              f"{rms:.3e}; f64_delta {rd.final_rms:.3e}", flush=True)
        assert r.status == 0 and rms <= 1e-6
        assert rms <= 2.0 * O.residual_rms(S, Zd) + 1e-12
        assert np.linalg.norm(Z - Zd) / np.linalg.norm(Zd) <= 1e-6


def test_warm_start_crt_first(zf):
    """An MD-like warm start at N = 3000 (two frames of the random-walk trajectory; the
    second refined from the first's Z) with the residue-emulated first refinement
    residual: the FP64 final residual meets the FP64 bar by the oracle, and Z, the
    update count and the evaluation counts match the FP64-residual refinement's."""
    f0, f1 = list(inputs.md_trajectory(3000, 2, 0))
    S0, S1 = _cuda(f0), _cuda(f1)
    prev = zf.refine(S0, None, precision="bf16x3", refine="crt_first").Z.clone()
    runs = {}
    for mode in ("crt_first", "f64_delta"):
        r = zf.refine(S1, prev, precision="bf16x3", refine=mode)
        Z = r.Z.cpu().numpy()
        rms = O.residual_rms(f1, Z)
        print(f"warm {mode}: {r.iters} updates, {r.low_evals}+{r.high_evals} evals, final "
              f"{r.final_rms:.3e}, oracle {rms:.3e}", flush=True)
        assert r.status == 0 and r.z0_used == zf.Z0_GIVEN
        assert rms <= 1e-10 and r.final_rms == pytest.approx(rms, rel=1e-6)
        runs[mode] = (r, Z)
    (rc, Zc), (rd, Zd) = runs["crt_first"], runs["f64_delta"]
    assert (rc.iters, rc.low_evals, rc.high_evals) == (rd.iters, rd.low_evals, rd.high_evals)
    assert np.linalg.norm(Zc - Zd) / np.linalg.norm(Zd) <= 1e-9
