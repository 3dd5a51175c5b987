"""Batched refinement (grouped GEMMs in one graph) against the CPU oracle.

Bar per matrix: oracle-measured ||Z^T S Z - I||_F / sqrt(N) <= 1e-6 with the FP64
refinement phase, and ||Z - Z_oracle|| / ||Z_oracle|| <= 1e-4 (the mixed-path bar of
test_gpu_parity).  Graph replay and eager launches of the same kernels must agree
bitwise.
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


SIZES = [64, 70, 100, 128, 129, 200, 256, 300, 513, 700]


@pytest.fixture(scope="module")
def batch():
    rng = np.random.default_rng(5)
    mats = []
    for i, n in enumerate(SIZES):
        pos = inputs.rsa_positions(n, 0.1, 0.0, rng)
        K = inputs.gaussian_kernel_overlap(pos, 1.0)
        mats.append(inputs.shift_to_condition(K, float(10 ** rng.uniform(1, 4))))
    refs = [O.refine(S, O.scaled_identity_guess(S), order=2) for S in mats]
    return mats, refs


def test_batched_matches_oracle(zf, batch):
    mats, refs = batch
    out = zf.refine_batched([_cuda(S) for S in mats])
    assert out.rc >= 0
    for S, ref, r in zip(mats, refs, out.results):
        Z = r.Z.cpu().numpy()
        rms = O.residual_rms(S, Z)
        print(f"n={S.shape[0]} iters={r.iters} low={r.low_evals} high={r.high_evals} "
              f"rms={rms:.2e} vs_oracle={_rel(Z, ref.Z):.2e}")
        assert r.status == 0
        assert rms <= 1e-6
        assert _rel(Z, ref.Z) <= 1e-4
        assert r.final_rms == pytest.approx(rms, rel=1e-3, abs=1e-15)
        assert r.high_evals >= 1 and len(r.hist) == r.low_evals + r.high_evals


def test_batched_same_stop_decisions_as_single(zf, batch):
    """Each matrix follows the same stop rule as zf_refine_ex; with different tile
    shapes the low-precision floor may move the stop by a sweep."""
    mats, _ = batch
    out = zf.refine_batched([_cuda(S) for S in mats])
    for S, rb in zip(mats, out.results):
        rs = zf.refine(_cuda(S), None)
        assert abs(rs.iters - rb.iters) <= 2
        assert abs(rs.low_evals - rb.low_evals) <= 2


def test_graph_replay_equals_eager(zf, batch):
    mats, _ = batch
    S = [_cuda(x) for x in mats]
    zf.batched_use_graph(False)
    try:
        eager = zf.refine_batched(S)
    finally:
        zf.batched_use_graph(True)
    for rep in range(3):
        g = zf.refine_batched(S)
        torch.cuda.synchronize()
        for a, b in zip(eager.results, g.results):
            assert torch.equal(a.Z, b.Z), rep
            assert a.hist == b.hist and a.iters == b.iters


def test_graph_lengths_agree(zf, batch):
    """One graph holding every macro-sweep the caps allow (one launch per call; the
    macro-sweeps after every matrix stopped change nothing) and shorter graphs (the
    live count read after each launch; the default holds 8) give bitwise the same
    results and the same number of live macro-sweeps."""
    mats, _ = batch
    S = [_cuda(x) for x in mats]
    zf.batched_set_graph_sweeps(0)
    try:
        one = zf.refine_batched(S)
        sweeps, launches = zf.batched_last_stats()
    finally:
        zf.batched_set_graph_sweeps(8)
    assert launches == 1
    # the FP64 phase starts once every low phase has stopped
    assert sweeps == max(r.low_evals for r in one.results) + max(r.high_evals for r in one.results)
    for k in (1, 3, 5, 8):
        zf.batched_set_graph_sweeps(k)
        try:
            part = zf.refine_batched(S)
            s_k, l_k = zf.batched_last_stats()
        finally:
            zf.batched_set_graph_sweeps(8)
        assert s_k == sweeps
        assert l_k == -(-sweeps // k)  # the launch holding the last live macro-sweep ends it
        for a, b in zip(one.results, part.results):
            assert torch.equal(a.Z, b.Z), k
            assert a.hist == b.hist and a.iters == b.iters
    with pytest.raises(zf.ZFError):
        zf.batched_set_graph_sweeps(-1)


def test_batched_given_guesses_and_refine_off(zf, batch):
    mats, refs = batch
    S = [_cuda(x) for x in mats[:4]]
    z0 = [None if i % 2 else _cuda(O.lowdin(mats[i]) + 1e-3 * inputs.uniform_noise(mats[i].shape[0], i))
          for i in range(4)]
    out = zf.refine_batched(S, z0)
    for i, r in enumerate(out.results):
        Z = r.Z.cpu().numpy()
        assert O.residual_rms(mats[i], Z) <= 1e-6
        if z0[i] is not None:
            lim = O.limit_for_guess(mats[i], z0[i].cpu().numpy())
            assert _rel(Z, lim) <= 1e-4
    off = zf.refine_batched(S, refine="off")
    for i, r in enumerate(off.results):
        rms = O.residual_rms(mats[i], r.Z.cpu().numpy())
        assert rms < 1e-3 and r.high_evals == 0


def test_batched_error_isolated(zf, batch):
    mats, _ = batch
    bad = mats[1].copy()
    bad[2, 3] = bad[3, 2] = np.nan
    S = [_cuda(mats[0]), _cuda(bad), _cuda(mats[2])]
    out = zf.refine_batched(S, raise_on_error=False)
    assert out.rc == zf.ERR_NONFINITE
    assert out.results[1].status == zf.ERR_NONFINITE
    for i in (0, 2):
        assert out.results[i].status == 0
        assert O.residual_rms(mats[i], out.results[i].Z.cpu().numpy()) <= 1e-6


def test_batched_arguments(zf, batch):
    mats, _ = batch
    with pytest.raises(zf.ZFError) as e:
        zf.refine_batched([_cuda(mats[0])], order=3)
    assert e.value.code == zf.ERR_ARG
    with pytest.raises(zf.ZFError):
        zf.batched_set_tiles([100], [96])


def test_autotune_installs_a_working_table(zf, batch):
    mats, _ = batch
    saved = zf.batched_get_tiles()
    try:
        tiles, ms = zf.batched_autotune([128, 256, 512, 1024], batch=8, reps=2)
        assert all(t in (64, 128) for t in tiles)
        assert all(a > 0 and b > 0 for a, b in ms)
        assert zf.batched_get_tiles()[1] == tiles
        out = zf.refine_batched([_cuda(S) for S in mats[:5]])
        for S, r in zip(mats[:5], out.results):
            assert O.residual_rms(S, r.Z.cpu().numpy()) <= 1e-6
        # every tile edge on every bucket gives a valid result
        for edge in (64, 128):
            zf.batched_set_tiles([1 << 20], [edge])
            out = zf.refine_batched([_cuda(S) for S in mats[:5]])
            for S, r in zip(mats[:5], out.results):
                assert O.residual_rms(S, r.Z.cpu().numpy()) <= 1e-6
    finally:
        zf.batched_set_tiles(*saved)


def test_batched_deterministic(zf, batch):
    mats, _ = batch
    S = [_cuda(x) for x in mats[:6]]
    a = zf.refine_batched(S)
    b = zf.refine_batched(S)
    for x, y in zip(a.results, b.results):
        assert torch.equal(x.Z, y.Z)
