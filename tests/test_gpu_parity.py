"""End-to-end parity of zf_refine against the CPU oracle (GPU; through the C ABI).

Bars:
* FP64 path (Table I "double"): the same number of updates as the oracle under
  the ratio rule, the residual history equal to 1e-9 relative while it is above
  the FP64 floor, ||Z - Z_oracle||_F / ||Z_oracle||_F <= 1e-11, and
  ||Z^T S Z - I||_F / sqrt(N) <= 1e-10.
* Mixed path (BF16x3 with an FP64 refinement phase): ||Z^T S Z - I||_F / sqrt(N)
  <= 1e-6 measured by the oracle, and ||Z - Z_oracle|| / ||Z_oracle|| <= 1e-4
  (the low-precision sweeps perturb Z by about 2^-16 ||Z Q|| per sweep, a
  component the residual cannot see; the bound allows a few such sweeps).
"""
import math

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


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


_S_CACHE = {}


def _S(n, seed=0, sigma=1.2):
    key = (n, seed, sigma)
    if key not in _S_CACHE:
        _S_CACHE[key] = inputs.overlap_gaussian(n, sigma, seed)
    return _S_CACHE[key]


@pytest.mark.parametrize("n,seed", [(256, 0), (256, 1), (300, 2), (129, 3), (64, 4)])
def test_fp64_path_matches_oracle(zf, n, seed):
    S = _S(n, seed)
    ref = O.refine(S, O.scaled_identity_guess(S), order=2, rule="ratio")
    r = zf.refine(_cuda(S), None, order=2, precision="fp64", stop="ratio")
    Z = r.Z.cpu().numpy()
    print(f"n={n} seed={seed} oracle iters={ref.iters} hist={ref.hist}")
    print(f"gpu iters={r.iters} hist={r.hist}")
    assert r.iters == ref.iters
    assert len(r.hist) == len(ref.hist)
    for a, b in zip(r.hist, ref.hist):
        if b > 1e-10:
            assert a == pytest.approx(b, rel=1e-9)
    assert _rel(Z, ref.Z) <= 1e-11
    assert O.residual_rms(S, Z) <= 1e-10
    assert r.final_rms <= 1e-10


def test_fp64_monotone_rule(zf):
    """The N = 256 workload as literally stated: stop once ||delta||_F stops
    decreasing.  Near the floor the decision rides on rounding noise, so the
    update count may differ by a few sweeps; the result may not."""
    S = _S(256, 0)
    ref = O.refine(S, O.scaled_identity_guess(S), order=2, rule="monotone")
    r = zf.refine(_cuda(S), None, order=2, precision="fp64", stop="monotone")
    Z = r.Z.cpu().numpy()
    assert abs(r.iters - ref.iters) <= 3
    assert O.residual_rms(S, Z) <= 1e-10
    assert _rel(Z, ref.Z) <= 1e-11


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_fp64_orders(zf, order):
    S = _S(200, 5)
    ref = O.refine(S, O.scaled_identity_guess(S), order=order)
    r = zf.refine(_cuda(S), None, order=order, precision="fp64")
    assert r.iters == ref.iters
    assert _rel(r.Z.cpu().numpy(), ref.Z) <= 1e-11
    assert r.final_rms <= 1e-10


@pytest.mark.parametrize("n,seed", [(256, 0), (300, 2), (129, 3), (512, 6)])
def test_mixed_path(zf, n, seed):
    S = _S(n, seed)
    ref = O.refine(S, O.scaled_identity_guess(S), order=2)
    r = zf.refine(_cuda(S), None, order=2, precision="bf16x3", refine="f64_delta")
    Z = r.Z.cpu().numpy()
    rms = O.residual_rms(S, Z)
    print(f"n={n}: iters={r.iters} low={r.low_evals} high={r.high_evals} hist={r.hist} "
          f"rms={rms:.3e} vs_oracle={_rel(Z, ref.Z):.3e}")
    assert rms <= 1e-6
    assert r.final_rms == pytest.approx(rms, rel=1e-3, abs=1e-15)
    assert _rel(Z, ref.Z) <= 1e-4
    assert r.high_evals >= 1


@pytest.mark.parametrize("order", [1, 3, 5])
def test_mixed_orders(zf, order):
    S = _S(256, 1)
    r = zf.refine(_cuda(S), None, order=order, precision="bf16x3")
    assert O.residual_rms(S, r.Z.cpu().numpy()) <= 1e-6


def test_mixed_full_fp64_refinement(zf):
    S = _S(300, 7)
    r = zf.refine(_cuda(S), None, precision="bf16x3", refine="f64_full")
    assert O.residual_rms(S, r.Z.cpu().numpy()) <= 1e-10


def test_mixed_without_refinement_stalls_above_fp64(zf):
    """(h)(h)+(h)(l)+(l)(h) alone stops at its own floor (Sec. V.C): far better
    than the guess, far worse than FP64."""
    S = _S(256, 0)
    r = zf.refine(_cuda(S), None, precision="bf16x3", refine="off")
    rms = O.residual_rms(S, r.Z.cpu().numpy())
    assert 1e-9 < rms < 1e-3
    assert r.high_evals == 0


def test_general_guess(zf):
    """Z0 = S^(-1/2) + alpha U (Sec. V.A) converges to Z0 X0^(-1/2), not S^(-1/2)."""
    n = 256
    S = _S(n, 8)
    Z0 = O.lowdin(S) + 0.005 * inputs.uniform_noise(n, 1)
    ref = O.refine(S, Z0)
    lim = O.limit_for_guess(S, Z0)
    r = zf.refine(_cuda(S), _cuda(Z0), precision="fp64")
    Z = r.Z.cpu().numpy()
    assert r.iters == ref.iters
    assert _rel(Z, ref.Z) <= 1e-11
    assert _rel(Z, lim) <= 1e-10
    rm = zf.refine(_cuda(S), _cuda(Z0), precision="bf16x3")
    assert O.residual_rms(S, rm.Z.cpu().numpy()) <= 1e-6
    assert _rel(rm.Z.cpu().numpy(), lim) <= 1e-4


def test_output_may_alias_guess(zf):
    S = _S(130, 9)
    Z0 = _cuda(O.scaled_identity_guess(S))
    r = zf.refine(_cuda(S), Z0, precision="fp64", out=Z0)
    assert r.Z.data_ptr() == Z0.data_ptr()
    assert O.residual_rms(S, Z0.cpu().numpy()) <= 1e-10


def test_short_form_entry_point(zf):
    S = _S(256, 0)
    out = torch.empty((256, 256), dtype=torch.float64, device="cuda")
    rc, iters, hist = zf.refine_basic(_cuda(S), None, 2, "fp64", out)
    ref = O.refine(S, O.scaled_identity_guess(S))
    assert rc == 0 and iters == ref.iters and len(hist) == len(ref.hist)


def test_tiny_exact_cases(zf):
    # n = 1: s = 4, z0 = 1/3 -> 1/2
    r = zf.refine(_cuda([[4.0]]), _cuda([[1.0 / 3.0]]), precision="fp64")
    assert abs(r.Z.item() - 0.5) < 1e-15
    S = np.array([[1.0, 0.25], [0.25, 1.0]])
    ref = O.refine(S, np.eye(2))
    r = zf.refine(_cuda(S), _cuda(np.eye(2)), precision="fp64")
    assert r.iters == ref.iters
    np.testing.assert_allclose(r.Z.cpu().numpy(), ref.Z, rtol=1e-14, atol=1e-15)


def test_diagonal_S(zf):
    s = np.linspace(0.2, 3.0, 150)
    S = np.diag(s)
    r = zf.refine(_cuda(S), None, precision="fp64")
    Z = r.Z.cpu().numpy()
    assert np.all(Z[~np.eye(150, dtype=bool)] == 0.0)
    np.testing.assert_allclose(np.diag(Z), 1.0 / np.sqrt(s), rtol=1e-14)


def test_residual_entry_point(zf):
    S = _S(300, 10)
    Z = O.lowdin(S) + 1e-3 * inputs.uniform_noise(300, 2)
    rms = zf.residual(_cuda(S), _cuda(Z))
    assert rms == pytest.approx(O.residual_rms(S, Z), rel=1e-10)


def test_deterministic(zf):
    S = _cuda(_S(384, 11))
    a = zf.refine(S, None, precision="bf16x3")
    b = zf.refine(S, None, precision="bf16x3")
    assert torch.equal(a.Z, b.Z) and a.hist == b.hist


def test_errors(zf):
    S = _S(64, 12)
    with pytest.raises(zf.ZFError) as e:
        zf.refine(_cuda(S), None, order=0)
    assert e.value.code == zf.ERR_ARG
    with pytest.raises(zf.ZFError) as e:
        zf.refine(_cuda(S), None, order=6)
    assert e.value.code == zf.ERR_ARG
    bad = S.copy()
    bad[3, 5] = bad[5, 3] = np.nan
    with pytest.raises(zf.ZFError) as e:
        zf.refine(_cuda(bad), None, precision="fp64")
    assert e.value.code == zf.ERR_NONFINITE
    with pytest.raises(zf.ZFError) as e:
        zf.refine(_cuda(S), _cuda(2.0 * O.lowdin(S)), precision="fp64")
    assert e.value.code in (zf.ERR_NOT_CONVERGED, zf.ERR_NONFINITE)
    # the library still works after errors
    r = zf.refine(_cuda(S), None, precision="fp64")
    assert r.final_rms <= 1e-10


def test_hist_truncation_flag(zf):
    S = _S(128, 13)
    r = zf.refine(_cuda(S), None, precision="fp64", hist_cap=2)
    assert r.flags & zf.WARN_HIST_TRUNC
    assert len(r.hist) == 2


def test_sweep_cap_flag(zf):
    S = _S(128, 13)
    Z0 = O.lowdin(S) + 1e-3 * inputs.uniform_noise(128, 3)   # starts with Err_F < 1
    r = zf.refine(_cuda(S), _cuda(Z0), precision="fp64", max_sweeps=1)
    assert r.flags & zf.WARN_MAXSWEEPS
    assert r.iters == 1
    assert r.final_err < 1.0
