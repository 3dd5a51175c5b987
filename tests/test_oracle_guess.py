"""Pins for the learned-guess oracle: backprop against finite differences, Adam's
closed-form first step, features against eigenvalues, labels against a direct
least-squares solve on the spectrum, acceptance against the convergence bound."""
import math

import numpy as np
import pytest

from oracle import zf_guess_oracle as G
from oracle import zf_oracle as O
from paper_2404_19163_amd import inputs


def _theta(seed=0):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.3, G.n_params())


def test_param_count():
    assert G.n_params() == 8 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3 == 4931


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(1)
    th = _theta(1)
    X = rng.normal(size=(7, 8))
    T = rng.normal(size=(7, 3))
    g = G.grad(th, X, T)
    h = 1e-6
    for idx in rng.choice(G.n_params(), 60, replace=False):
        e = np.zeros_like(th)
        e[idx] = h
        fd = (G.loss(th + e, X, T) - G.loss(th - e, X, T)) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-5, abs=1e-9)


def test_forward_by_hand():
    th = np.zeros(G.n_params())
    P = G.unpack(th)
    P["W1"][0, 0] = 1.0          # h1_0 = tanh(x_0)
    P["W2"][0, 0] = 2.0          # h2_0 = tanh(2 tanh(x_0))
    P["W3"][1, 0] = 3.0          # y_1 = 3 h2_0 + b3_1
    P["b3"][1] = 0.5
    X = np.array([[0.7, 0, 0, 0, 0, 0, 0, 0]])
    Y, _ = G.forward(th, X)
    assert Y[0, 1] == pytest.approx(3 * math.tanh(2 * math.tanh(0.7)) + 0.5, rel=1e-15)
    assert Y[0, 0] == 0.0 and Y[0, 2] == 0.0


def test_adam_first_step_is_lr_sign():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t1, m, v = G.adam_step(th, np.zeros(3), np.zeros(3), g, 1, lr=0.01)
    np.testing.assert_allclose(t1, th - 0.01 * np.sign(g), rtol=0, atol=1e-7)


def test_features_against_eigenvalues():
    S = inputs.overlap_gaussian(60, 1.2, 3)
    f = G.features(S)
    lam = np.linalg.eigvalsh(S)
    g, glo, rmean = G.gershgorin(S)
    x = lam / g
    assert f[0] == pytest.approx(math.log(60))
    for k in range(1, 5):
        assert f[k] == pytest.approx(np.mean(x ** k), rel=1e-12)
    assert lam.max() <= g * (1 + 1e-12) and lam.min() >= glo - 1e-12     # Gershgorin
    assert f[5] == max(glo, 0) / g and f[6] == glo / g and f[7] == pytest.approx(rmean / g)


def test_label_is_spectral_least_squares():
    """For Z = S^(-1/2) the fit reduces to min_c sum_i (sqrt(x_i) p(x_i) - 1)^2."""
    S = inputs.overlap_gaussian(50, 1.2, 4)
    Z = O.lowdin(S)
    c = G.label_from_z(S, Z)
    g, _, _ = G.gershgorin(S)
    x = np.linalg.eigvalsh(S) / g
    A = np.sqrt(x)[:, None] * np.stack([np.ones_like(x), x, x * x], 1)
    c2, *_ = np.linalg.lstsq(A, np.ones_like(x), rcond=None)
    np.testing.assert_allclose(c, c2, rtol=1e-7, atol=1e-9)


def test_label_exact_for_scaled_identity_overlap():
    # S = s I: St = I (g = s), and Z = s^(-1/2) I is reached exactly by p = 1 (c0+c1+c2 = 1
    # with the normal equations' minimum-norm... all x_i = 1, so only p(1) = 1 is fixed)
    S = 4.0 * np.eye(5)
    c = G.guess_matrix(S, np.array([1.0, 0.0, 0.0]))
    np.testing.assert_allclose(c, 0.5 * np.eye(5))


def test_acceptance_bounds_phi():
    # p(x) = 3 on [0, 1]: phi(1) = 9 -> rescaled to max 1.9
    c = G.accept(np.array([3.0, 0.0, 0.0]), 0.0)
    x = np.linspace(0, 1, 101)
    phi = x * (c[0] + c[1] * x + c[2] * x * x) ** 2
    assert phi.max() == pytest.approx(1.9)
    # p changes sign inside the interval -> rejected
    assert G.accept(np.array([1.0, -3.0, 0.0]), 0.0) is None
    # an accepted guess converges: ||X0 - I||_2 < 1 on a real overlap matrix
    S = inputs.overlap_gaussian(80, 1.2, 5)
    Zs = O.lowdin(S)
    c = G.accept(G.label_from_z(S, Zs), max(G.gershgorin(S)[1], 0) / G.gershgorin(S)[0])
    Z0 = G.guess_matrix(S, c)
    X0 = Z0.T @ S @ Z0
    assert np.max(np.abs(np.linalg.eigvalsh(np.eye(80) - X0))) < 1.0


def test_learned_form_guess_saves_sweeps():
    """The weighted least-squares quadratic (what the network is trained to output)
    starts closer than the scaled identity and needs fewer updates."""
    gains = []
    for seed in range(4):
        S = inputs.overlap_gaussian(120, 1.0, 10 + seed)
        g, glo, _ = G.gershgorin(S)
        c = G.accept(G.label_from_z(S, O.lowdin(S)), max(glo, 0) / g)
        assert c is not None
        r_id = O.refine(S, O.scaled_identity_guess(S))
        r_lg = O.refine(S, G.guess_matrix(S, c))
        gains.append(r_id.iters - r_lg.iters)
    assert np.mean(gains) >= 1.0
