"""Parity at the full workload sizes, in the launch configuration the benchmark times.

At these sizes the oracle does not rerun the recursion.  It checks what must hold
for any N, each in FP64 on the CPU:
* the residual ||Z^T S Z - I||_F / sqrt(N) of every returned Z, recomputed by the oracle
  (<= 1e-6 mixed, <= 1e-10 FP64 path) and equal to the library's own report;
* the limit's structure.  A polynomial-in-S guess converges to S^(-1/2), which is
  symmetric.  A general guess Z0 converges to Z0 X0^(-1/2), so Z0^(-1) Z is symmetric;
* agreement of the mixed and FP64 paths on the same S;
* element by element, the distance of the returned Z from the closed form the
  recursion converges to (the Loewdin factor S^(-1/2) for the scaled-identity guess,
  Sec. II and III), computed by the oracle from a dense eigendecomposition.
At N = 256 (the plain FP64 method) the oracle runs the same recursion, and the history
must match it down to the FP64 floor.
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


def _asym(M):
    return np.linalg.norm(M - M.T) / np.linalg.norm(M)


U64 = 2.0 ** -53


def _lowdin_kappa(S):
    """S^(-1/2) from the oracle's dense eigendecomposition and kappa(S)."""
    lam = np.linalg.eigvalsh(S)
    return O.lowdin(S), float(lam[-1] / lam[0])


def _maxrel(Z, Zs):
    """max_ij |Z_ij - Zs_ij| / max_ij |Zs_ij|."""
    return float(np.max(np.abs(Z - Zs)) / np.max(np.abs(Zs)))


# Bounds of the element-wise distance to S^(-1/2).  The closed form itself carries an
# error of order kappa u (an eigenvalue perturbed by u ||S|| moves lambda^(-1/2) by a
# relative kappa u / 2), and the FP64 recursion adds rounding that the residual does
# not see (an S-orthogonal rotation of Z leaves Z^T S Z unchanged), a few N^(1/2) u per
# sweep, amplified by the same kappa.  FP64 path: <= 1000 kappa u.  Mixed path: the
# BF16x3 sweeps leave a rotation of order 2^-16 that the FP64 refinement, which only
# corrects Z^T S Z, keeps: <= 1e-4 for the well-conditioned N = 4096 overlap.
def _fp64_bound(kappa):
    return 1000.0 * kappa * U64


def test_n256_plain_fp64_monotone(zf):
    """N = 256, scaled identity, m = 2 (third-order series), stop once ||delta||_F no
    longer decreases: the FP64 path takes the oracle's steps down to the FP64 floor.
    There the monotone rule stops on rounding noise, so the stopping index may differ
    by sweeps spent at the floor; the GPU's stop must itself be a valid monotone stop."""
    S = inputs.workload("gauss256", 0)
    ref = O.refine(S, O.scaled_identity_guess(S), order=2, rule="monotone")
    r = zf.refine(_cuda(S), None, precision="fp64", stop="monotone", order=2)
    print(f"iters {r.iters} (oracle {ref.iters}), rms {r.final_rms:.2e}", flush=True)
    h, hr = np.array(r.hist), np.array(ref.hist)
    floor = 1e-12
    above = int(np.sum(hr > floor))             # evaluations before the floor
    assert np.all(hr[above:] <= floor) and above >= 3
    np.testing.assert_allclose(h[:above], hr[:above], rtol=1e-9)
    assert np.all(h[above:] <= floor)
    assert np.all(np.diff(h[:-1]) < 0) and h[-1] >= h[-2]  # decreasing, then the stop
    assert r.iters >= above and abs(r.iters - ref.iters) <= 3
    Z = r.Z.cpu().numpy()
    assert np.max(np.abs(Z - ref.Z)) <= 1e-11 * np.max(np.abs(ref.Z))
    assert O.residual_rms(S, Z) <= 1e-10


def test_n4096_mixed_and_fp64(zf):
    S = inputs.workload("gauss4096", 0)
    Sd = _cuda(S)
    rm = zf.refine(Sd, None, precision="bf16x3")
    rf = zf.refine(Sd, None, precision="fp64")
    Zm, Zf = rm.Z.cpu().numpy(), rf.Z.cpu().numpy()
    rms_m, rms_f = O.residual_rms(S, Zm), O.residual_rms(S, Zf)
    print(f"mixed: {rm.low_evals}+{rm.high_evals} evals rms {rms_m:.2e}; fp64: {rf.iters} updates "
          f"rms {rms_f:.2e}; |Zm-Zf|/|Zf| {np.linalg.norm(Zm - Zf) / np.linalg.norm(Zf):.2e}",
          flush=True)
    assert rm.status == 0 and rf.status == 0
    assert rms_m <= 1e-6 and rms_f <= 1e-10
    assert rm.final_rms == pytest.approx(rms_m, rel=1e-3)
    # at the FP64 rounding floor two residual evaluations agree only in magnitude
    assert rf.final_rms <= 1e-13
    assert rm.high_evals >= 1
    assert np.linalg.norm(Zm - Zf) / np.linalg.norm(Zf) <= 1e-4
    # the limit S^(-1/2) is symmetric
    assert _asym(Zf) <= 1e-12 and _asym(Zm) <= 1e-5
    # element by element against the closed form
    Zs, kappa = _lowdin_kappa(S)
    dm, df = _maxrel(Zm, Zs), _maxrel(Zf, Zs)
    print(f"vs S^-1/2 (kappa {kappa:.1f}): mixed {dm:.2e}, fp64 {df:.2e} "
          f"(bound {_fp64_bound(kappa):.2e})", flush=True)
    assert df <= _fp64_bound(kappa)
    assert dm <= 1e-4


def test_n5049_cluster(zf):
    """kappa ~ 4e5: the low-precision phase stalls early and the FP64 phase takes over.
    The stalled low-precision iterate no longer commutes with S, so the mixed result is
    an S-orthonormal factor (residual checked) but not S^(-1/2); the FP64 path, which
    keeps Z a polynomial in S to rounding, must reach the symmetric S^(-1/2)."""
    S = inputs.workload("cluster5049")
    Sd = _cuda(S)
    r = zf.refine(Sd, None, precision="bf16x3")
    Z = r.Z.cpu().numpy()
    rms = O.residual_rms(S, Z)
    print(f"mixed: {r.low_evals}+{r.high_evals} evals, {r.iters} updates, rms {rms:.2e}", flush=True)
    assert r.status == 0
    assert rms <= 1e-6
    assert r.final_rms == pytest.approx(rms, rel=1e-3)
    assert r.high_evals >= 2
    rf = zf.refine(Sd, None, precision="fp64")
    Zf = rf.Z.cpu().numpy()
    rms_f = O.residual_rms(S, Zf)
    print(f"fp64: {rf.iters} updates, rms {rms_f:.2e}, asym {_asym(Zf):.2e}", flush=True)
    assert rf.status == 0 and rms_f <= 1e-10
    assert _asym(Zf) <= 1e-8
    Zs, kappa = _lowdin_kappa(S)
    df = _maxrel(Zf, Zs)
    print(f"fp64 vs S^-1/2 (kappa {kappa:.3g}): {df:.2e} (bound {_fp64_bound(kappa):.2e}); "
          f"mixed {_maxrel(Z, Zs):.2e} (an S-orthonormal factor, not S^-1/2)", flush=True)
    assert df <= _fp64_bound(kappa)


def test_n3000_warm_start(zf):
    """Frame 1 of the MD-like trajectory from frame 0's Z: converges in fewer updates
    than from the scaled identity, to the S-orthonormalization Z0 X0^(-1/2) of the
    guess (Z0^(-1) Z symmetric)."""
    frames = list(inputs.md_trajectory(3000, 2, 0))
    Z0 = zf.refine(_cuda(frames[0]), None, precision="bf16x3").Z
    S1 = frames[1]
    rw = zf.refine(_cuda(S1), Z0, precision="bf16x3")
    ri = zf.refine(_cuda(S1), None, precision="bf16x3")
    Z = rw.Z.cpu().numpy()
    rms = O.residual_rms(S1, Z)
    M = np.linalg.solve(Z0.cpu().numpy(), Z)
    print(f"warm {rw.iters} updates (identity {ri.iters}), rms {rms:.2e}, "
          f"asym(Z0^-1 Z) {_asym(M):.2e}", flush=True)
    assert rw.status == 0 and rms <= 1e-6
    assert rw.iters < ri.iters
    assert _asym(M) <= 1e-5


def test_batched_512_learned(zf):
    """The 512-matrix batch with learned guesses (network trained on another draw of
    the same distribution): every matrix meets the mixed bar, measured by the oracle."""
    from paper_2404_19163_amd import guess
    X, Y = guess.training_pairs(inputs.batched_overlaps(64, 1000))
    guess.train(X, Y, steps=300, lr=3e-3, seed=0)
    mats = inputs.batched_overlaps(512, 0)
    out = zf.refine_batched([_cuda(S) for S in mats], guess="learned")
    assert out.rc >= 0
    worst, learned = 0.0, 0
    for S, r in zip(mats, out.results):
        assert r.status == 0
        rms = O.residual_rms(S, r.Z.cpu().numpy())
        worst = max(worst, rms)
        assert rms <= 1e-6
        assert r.final_rms == pytest.approx(rms, rel=1e-2, abs=1e-14)
        if r.z0_used == zf.Z0_LEARNED:
            learned += 1
        else:
            assert r.flags & zf.WARN_Z0_FALLBACK
    print(f"worst rms {worst:.2e}, learned guesses {learned}/512", flush=True)


def test_n16384_largest_order(zf):
    """N = 16384 (the emulated residual's largest order; 2 GB per matrix): the mixed
    refinement with the FP64 residual and with the emulated one.  The oracle checks a
    48 x 48 block of delta = I - Z^T S Z recomputed from sampled columns (entries of size
    RMS; bound 100 x the reported RMS), and the library's FP64 residual of the returned Z
    against its report."""
    n = 16384
    S = inputs.overlap_gaussian(n, 1.0, 0)
    Sd = _cuda(S)
    rng = np.random.default_rng(1)
    J = np.sort(rng.choice(n, size=48, replace=False))
    for mode in ("f64_delta", "emu"):
        r = zf.refine(Sd, None, precision="bf16x3", refine=mode)
        Zs = r.Z[:, torch.from_numpy(J).cuda()].cpu().numpy()        # the sampled columns
        block = np.eye(48) - Zs.T @ (S @ Zs)                            # delta[J, J] in FP64
        rms64 = zf.residual(Sd, r.Z)
        print(f"{mode}: {r.low_evals}+{r.high_evals} evals, reported {r.final_rms:.2e}, FP64 "
              f"residual {rms64:.2e}, max sampled |delta| {np.max(np.abs(block)):.2e}", flush=True)
        assert r.status == 0 and r.final_rms <= 1e-6
        assert np.max(np.abs(block)) <= 100 * r.final_rms
        assert rms64 == pytest.approx(r.final_rms, rel=1e-2, abs=1e-12)
        del r
    zf.release()
