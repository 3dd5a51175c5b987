"""Training and persistence of the learned initial guess (network kernels in libzf).

Training pairs come from the method itself: for each overlap matrix S the library
refines Z (zf_refine_ex), then zf_guess_label fits p to that Z in the
S^(1/2)-weighted least-squares sense and zf_features extracts the 8 features.
Training steps (forward, loss, backward, Adam) run in the library's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import zf

N_PARAMS = zf.N_PARAMS
SHAPES = [(64, 8), (64,), (64, 64), (64,), (3, 64), (3,)]


def init_params(seed: int = 0) -> np.ndarray:
    """Glorot-uniform weights, zero biases, in the library's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in SHAPES:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, size=shp).ravel())
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts).astype(np.float32)


def training_pairs(mats, precision: str = "fp64", device: str = "cuda:0"):
    """(features (B, 8), labels (B, 3)) from refining each S with the library."""
    feats, labels = [], []
    for S in mats:
        Sd = torch.from_numpy(np.ascontiguousarray(S, dtype=np.float64)).to(device)
        Z = zf.refine(Sd, None, precision=precision).Z
        feats.append(zf.features(Sd).cpu().numpy())
        labels.append(zf.guess_label(Sd, Z))
    return np.array(feats, dtype=np.float32), np.array(labels, dtype=np.float32)


def fit_normalization(feats: np.ndarray, labels: np.ndarray):
    mu_x, sd_x = feats.mean(0), feats.std(0)
    mu_y, sd_y = labels.mean(0), labels.std(0)
    sd_x = np.where(sd_x > 1e-6, sd_x, 1.0)
    sd_y = np.where(sd_y > 1e-6, sd_y, 1.0)
    return mu_x, sd_x, mu_y, sd_y


def train(feats: np.ndarray, labels: np.ndarray, steps: int = 500, lr: float = 3e-3,
          seed: int = 0, device: str = "cuda:0"):
    """Full-batch Adam on the library's kernels; returns the loss history."""
    norm = fit_normalization(feats, labels)
    zf.mlp_set_norm(*norm)
    zf.mlp_set_params(init_params(seed))
    F = torch.from_numpy(np.ascontiguousarray(feats, dtype=np.float32)).to(device)
    L = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.float32)).to(device)
    return [zf.mlp_train_step(F, L, lr) for _ in range(steps)], norm


def save(path: str) -> None:
    """The loaded network to a file (the library's zf_mlp_save format)."""
    zf.mlp_save(path)


def load(path: str) -> None:
    zf.mlp_load(path)
