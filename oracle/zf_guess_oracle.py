"""CPU FP64 oracle of the learned initial guess Z0 = p(S/g)/sqrt(g), p quadratic.

TEST INFRASTRUCTURE ONLY (the same rule as zf_oracle: tests, the smoke check and
the benchmark's CPU leg may use it; the product never does).

The paper refines any Z0 with ||Z0^T S Z0 - I||_2 < 1 (Sec. III) and stresses good
guesses from earlier steps (Sec. VI).  This guess is a small network mapping cheap
spectral features of S to the three coefficients of p:

  features  f = [log N, tr(St^k)/N (k = 1..4), max(g_lo, 0)/g, g_lo/g, mean_i r_i / g]
            with r_i = sum_j |S_ij|, g = max_i r_i (Gershgorin upper bound), g_lo =
            min_i (S_ii - sum_{j != i} |S_ij|) (Gershgorin lower bound), St = S / g;
  network   8 -> 64 -> 64 -> 3, tanh, on standardized features and labels;
  labels    the least-squares fit of Z0 to the converged Z in the S^(1/2)-weighted
            norm, min_c ||S^(1/2) (p(St)/sqrt(g) - Z)||_F (normal equations below);
  accept    phi(x) = x p(x)^2 is the eigenvalue of X0 = Z0^T S Z0 at x = lambda / g;
            convergence needs 0 < phi < 2 on the spectrum (||X0 - I||_2 < 1).  The
            guess is rescaled so that max phi <= 1.9 on the Gershgorin interval
            [max(g_lo, 0)/g, 1] and rejected (scaled identity instead) unless p > 0 there.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT, N_HID, N_OUT = 8, 64, 3
PHI_MAX = 1.9


def gershgorin(S: np.ndarray):
    r = np.sum(np.abs(S), axis=1)
    d = np.diag(S)
    lo = np.min(d - (r - np.abs(d)))
    return float(np.max(r)), float(lo), float(np.mean(r))


def features(S: np.ndarray) -> np.ndarray:
    """The 8 features above, by matrix products (FP64)."""
    n = S.shape[0]
    g, glo, rmean = gershgorin(S)
    St = S / g
    P = np.eye(n)
    tr = []
    for _ in range(4):
        P = P @ St
        tr.append(np.trace(P) / n)
    return np.array([math.log(n), *tr, max(glo, 0.0) / g, glo / g, rmean / g])


def label_from_z(S: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """c = argmin ||S^(1/2)(p(St)/sqrt(g) - Z)||_F, p(x) = c0 + c1 x + c2 x^2.

    With B_j = St^j / sqrt(g): G_jk = <S^(1/2) B_j, S^(1/2) B_k> = tr(St^(j+k+1)) and
    r_j = <S^(1/2) B_j, S^(1/2) Z> = sqrt(g) tr(St^(j+1) Z)."""
    g, _, _ = gershgorin(S)
    St = S / g
    n = S.shape[0]
    pw = [np.eye(n)]
    for _ in range(5):
        pw.append(pw[-1] @ St)
    G = np.array([[np.trace(pw[j + k + 1]) for k in range(3)] for j in range(3)])
    r = np.array([math.sqrt(g) * np.trace(pw[j + 1] @ Z) for j in range(3)])
    return np.linalg.solve(G, r)


def guess_matrix(S: np.ndarray, c: np.ndarray) -> np.ndarray:
    g, _, _ = gershgorin(S)
    St = S / g
    return (c[0] * np.eye(S.shape[0]) + c[1] * St + c[2] * St @ St) / math.sqrt(g)


def accept(c: np.ndarray, x_lo: float, samples: int = 1025):
    """Rescale c so max phi <= PHI_MAX on [x_lo, 1]; None if p <= 0 somewhere there."""
    x = np.linspace(max(x_lo, 0.0), 1.0, samples)
    p = c[0] + c[1] * x + c[2] * x * x
    if np.any(p[1:] <= 0.0) or (x[0] > 0.0 and p[0] <= 0.0):
        return None
    phi = x * p * p
    m = float(np.max(phi))
    if m > PHI_MAX:
        c = c * math.sqrt(PHI_MAX / m)
    return c


# ---------------------------------------------------------------------------
# the network (FP64 reference of the library's FP32 kernels)
# ---------------------------------------------------------------------------
def param_shapes():
    return [("W1", (N_HID, N_FEAT)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
            ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in param_shapes():
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes())


def forward(theta: np.ndarray, X: np.ndarray):
    """X: (B, 8) standardized features -> (Y (B, 3), cache)."""
    P = unpack(theta)
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.tanh(z2)
    Y = h2 @ P["W3"].T + P["b3"]
    return Y, (X, h1, h2)


def loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> float:
    """Mean squared error over every sample and output."""
    Y, _ = forward(theta, X)
    return float(np.mean((Y - T) ** 2))


def grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray) -> np.ndarray:
    """d loss / d theta by backpropagation through the three layers."""
    P = unpack(theta)
    Y, (X, h1, h2) = forward(theta, X)
    dY = 2.0 * (Y - T) / Y.size
    gW3 = dY.T @ h2
    gb3 = dY.sum(0)
    dz2 = (dY @ P["W3"]) * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * (1.0 - h1 * h1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(theta, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) with bias correction; t counts from 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
