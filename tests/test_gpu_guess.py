"""Learned initial guess: library kernels against the CPU oracle, and the gain.

Bars: features within FP32 rounding of the oracle (rel 1e-5), labels within 1e-7
relative (FP64 GEMMs), the FP32 gradient within 1e-3 relative of the FP64 oracle
backprop (largest entries), Adam's first step equal to lr sign(g).  The trained
network must save sweeps on average over the scaled identity on held-out matrices,
with every result still meeting ||Z^T S Z - I||_F / sqrt(N) <= 1e-6.
"""
import numpy as np
import pytest
import torch

from oracle import zf_guess_oracle as G
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


@pytest.mark.parametrize("n,seed", [(64, 0), (150, 1), (300, 2)])
def test_features_match_oracle(zf, n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed)
    f = zf.features(_cuda(S)).cpu().numpy()
    np.testing.assert_allclose(f, G.features(S), rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("n,seed", [(80, 3), (257, 4)])
def test_label_matches_oracle(zf, n, seed):
    S = inputs.overlap_gaussian(n, 1.2, seed)
    Z = O.lowdin(S) + 1e-3 * inputs.uniform_noise(n, seed)
    c = zf.guess_label(_cuda(S), _cuda(Z))
    np.testing.assert_allclose(c, G.label_from_z(S, Z), rtol=1e-7, atol=1e-9)


def _norm_and_data(seed=0, B=37):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 8)).astype(np.float32) * 0.7 + 0.2
    Y = rng.normal(size=(B, 3)).astype(np.float32)
    mu_x, sd_x = rng.normal(size=8).astype(np.float32) * 0.1, (0.5 + rng.random(8)).astype(np.float32)
    mu_y, sd_y = rng.normal(size=3).astype(np.float32), (0.5 + rng.random(3)).astype(np.float32)
    return X, Y, (mu_x, sd_x, mu_y, sd_y)


def test_gradient_matches_oracle(zf):
    from paper_2404_19163_amd import guess
    X, Y, (mu_x, sd_x, mu_y, sd_y) = _norm_and_data()
    theta = guess.init_params(3)
    zf.mlp_set_norm(mu_x, sd_x, mu_y, sd_y)
    zf.mlp_set_params(theta)
    g, loss = zf.mlp_grad(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda())
    Xs = (X.astype(np.float64) - mu_x) / sd_x
    Ys = (Y.astype(np.float64) - mu_y) / sd_y
    g_ref = G.grad(theta.astype(np.float64), Xs, Ys)
    assert loss == pytest.approx(G.loss(theta.astype(np.float64), Xs, Ys), rel=1e-5)
    scale = np.max(np.abs(g_ref))
    assert np.max(np.abs(g - g_ref)) <= 1e-3 * scale
    # the parameters did not move
    np.testing.assert_array_equal(zf.mlp_get_params(), theta)


def test_adam_first_step(zf):
    from paper_2404_19163_amd import guess
    X, Y, norm = _norm_and_data(seed=1)
    theta = guess.init_params(4)
    zf.mlp_set_norm(*norm)
    zf.mlp_set_params(theta)
    Xd, Yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
    g, _ = zf.mlp_grad(Xd, Yd)
    zf.mlp_train_step(Xd, Yd, 1e-2)
    t1 = zf.mlp_get_params()
    big = np.abs(g) > 1e-4
    np.testing.assert_allclose((theta - t1)[big], 1e-2 * np.sign(g[big]), rtol=1e-3, atol=1e-6)


def test_training_reduces_loss(zf):
    from paper_2404_19163_amd import guess
    X, Y, _ = _norm_and_data(seed=2, B=64)
    losses, _ = guess.train(X, Y, steps=60, lr=1e-2, seed=5)
    assert losses[-1] < 0.5 * losses[0]


def test_fallback_without_network(zf):
    lib = zf.lib()
    # a fresh parameter set that makes p negative everywhere forces the fallback too
    from paper_2404_19163_amd import guess
    zf.mlp_set_norm(np.zeros(8), np.ones(8), np.array([-5.0, 0, 0]), np.ones(3))
    zf.mlp_set_params(np.zeros(guess.N_PARAMS, dtype=np.float32))
    S = inputs.overlap_gaussian(128, 1.2, 7)
    r = zf.refine(_cuda(S), None, guess="learned", precision="fp64")
    assert r.flags & zf.WARN_Z0_FALLBACK
    assert r.z0_used == zf.Z0_SCALED_IDENTITY
    assert r.final_rms <= 1e-10
    del lib


def test_learned_guess_saves_sweeps(zf):
    """Train on matrices the method refines, then compare update counts on held-out
    matrices of the same family."""
    from paper_2404_19163_amd import guess
    rng = np.random.default_rng(11)

    def family(count, seed):
        out = []
        r = np.random.default_rng(seed)
        for _ in range(count):
            n = int(r.integers(64, 257))
            sigma = float(r.uniform(0.9, 1.3))
            out.append(inputs.overlap_gaussian(n, sigma, int(r.integers(1 << 30))))
        return out

    train_set = family(48, 1)
    X, Y = guess.training_pairs(train_set)
    losses, _ = guess.train(X, Y, steps=400, lr=3e-3, seed=0)
    assert losses[-1] < losses[0]
    held = family(10, 2)
    gain = []
    for S in held:
        Sd = _cuda(S)
        r_id = zf.refine(Sd, None, precision="bf16x3")
        r_lg = zf.refine(Sd, None, precision="bf16x3", guess="learned")
        assert O.residual_rms(S, r_lg.Z.cpu().numpy()) <= 1e-6
        assert r_lg.z0_used == zf.Z0_LEARNED
        gain.append(r_id.low_evals - r_lg.low_evals)
    print("low-precision sweeps saved per matrix:", gain)
    assert np.mean(gain) > 0.5
    del rng
