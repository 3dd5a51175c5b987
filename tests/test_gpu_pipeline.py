"""The stop test on the device, with the next sweep queued ahead (GPU; through the C ABI).

The host queues the update of sweep n and the residual of sweep n + 1 before it reads
sweep n's decision; a stop sets a gate that turns those launches into no-ops.  Checked:
* every decision equals the rule of Algorithm 2 (Sec. IV.A) applied on the host to the
  returned history, phase by phase: no stop before the last evaluation of a phase, a
  stop at it (or the sweep cap);
* the timed GEMM launches equal the products the returned counts imply: one full and
  one symmetric product per residual, m - 1 symmetric products and one full product per
  update, the updates being one fewer than the evaluations of each phase (the launches
  the gate turned off are not counted);
* the monotone rule, whose stop can return the iterate before the last one, returns it
  intact (the update queued behind the stop never overwrote its buffer): its residual,
  recomputed, equals the reported one bit for bit.
"""
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


def _check_phase(errs, order, rule):
    """errs: one phase's history; the phase ran until its first stop."""
    def stop(n):
        if rule == "monotone":
            return errs[n] >= errs[n - 1]
        return errs[n] > errs[n - 1] ** (order + 1)

    def borderline(n):  # the device's pow may differ from the host's in the last bit
        t = errs[n - 1] if rule == "monotone" else errs[n - 1] ** (order + 1)
        return abs(errs[n] - t) <= 1e-12 * abs(t)

    for n in range(1, len(errs) - 1):
        assert borderline(n) or not stop(n), f"no stop expected at {n}: {errs}"
    if len(errs) > 1:
        assert borderline(len(errs) - 1) or stop(len(errs) - 1), f"stop expected: {errs}"


@pytest.mark.parametrize("precision,refine,order", [("bf16x3", "f64_delta", 2),
                                                    ("bf16x3", "crt_first", 2),
                                                    ("bf16x3", "f64_delta", 3),
                                                    ("fp64", "f64_delta", 2)])
def test_decisions_follow_the_rule(zf, precision, refine, order):
    S = inputs.overlap_gaussian(700, 1.2, 5)
    r = zf.refine(_cuda(S), None, order=order, precision=precision, refine=refine)
    low, high = r.low_evals, r.high_evals
    assert len(r.hist) == low + high
    if precision == "fp64":
        _check_phase(r.hist, order, "ratio")
    else:
        _check_phase(r.hist[:low], order, "ratio")
        _check_phase(r.hist[low:], order, "ratio")
    assert O.residual_rms(S, r.Z.cpu().numpy()) <= (1e-10 if precision == "fp64" else 1e-6)


@pytest.mark.parametrize("order", [2, 3])
def test_counted_launches_match_the_counts(zf, order):
    S = inputs.overlap_gaussian(640, 1.2, 8)
    zf.profile_enable(True)
    try:
        zf.profile_reset()
        r = zf.refine(_cuda(S), None, order=order, precision="bf16x3", refine="f64_delta")
        prof = zf.profile_read()
    finally:
        zf.profile_enable(False)
    low, high = r.low_evals, r.high_evals
    upd_low, upd_high = low - 1, high - 1
    # BF16x3: the first phase's residuals and updates, and the refinement's corrections
    assert prof["gemm_x3"][0] == low + upd_low + upd_high
    assert prof["gemm_x3_sym"][0] == low + (order - 1) * (upd_low + upd_high)
    # FP64: the refinement phase's residuals
    assert prof["gemm_f64"][0] == high
    assert prof["gemm_f64_sym"][0] == high


def test_monotone_stop_returns_the_earlier_iterate(zf):
    """Near the FP64 floor the monotone rule stops on a rise and returns the iterate
    before the last one.  Its residual, recomputed by the library's own FP64 products
    (the same kernels on the same values), must equal the reported one bit for bit;
    had the update queued behind the stop overwritten that buffer, it would not."""
    S = inputs.overlap_gaussian(256, 1.2, 0)
    ref = O.refine(S, O.scaled_identity_guess(S), order=2, rule="monotone")
    r = zf.refine(_cuda(S), None, order=2, precision="fp64", stop="monotone")
    _check_phase(r.hist, 2, "monotone")
    if r.hist[-1] > r.hist[-2]:
        assert r.iters == len(r.hist) - 2 and r.final_err == r.hist[-2]
    assert zf.residual(_cuda(S), r.Z) == r.final_rms
    Z = r.Z.cpu().numpy()
    assert np.linalg.norm(Z - ref.Z) / np.linalg.norm(ref.Z) <= 1e-11
