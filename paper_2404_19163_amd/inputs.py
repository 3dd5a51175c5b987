"""Seeded synthetic inputs: dense SPD overlap matrices S and initial guesses Z0.

This module only builds inputs.  It holds none of the factorization's
arithmetic (no Z0 rule, no recursion, no split), so the CPU oracle and the
GPU path can both be fed from it without sharing any part of the method.

Workload families (all FP64, row-major, symmetric, unit diagonal):

* ``gaussian_kernel_overlap`` -- one normalized s-type Gaussian per atom at
  random positions in a cube of number density ``density`` (atoms / A^3):
  S_ij = exp(-r_ij^2 / (2 sigma^2)).  Positions come from random sequential
  addition with a minimum pair distance ``d_min`` (A); ``d_min = 0`` gives
  plain uniform positions.  This is the Gram matrix of Gaussian functions,
  hence SPD.  Overlap matrices of atom-centred bases are the paper's
  application (Sec. II.A, Eq. Overlap).
* ``cluster_spd_overlap`` -- a 561-atom fcc cuboctahedral cluster with one
  normalized primitive Gaussian per s, p and d function (9 per atom,
  N = 5049).  A small shared exponent makes S ill-conditioned, standing in
  for the Ag561 nanoparticle overlap matrix of Sec. V.D, which is not
  available.
* ``paper_synthetic`` -- the synthetic family of Sec. V.A: exp(-|i-j|/2)
  sin(i+1) (symmetrized, see the docstring) shifted to a chosen lowest
  eigenvalue, with Z0 = S^{-1/2} + alpha U built by the caller.
* ``md_trajectory`` -- positions perturbed frame by frame (random walk) for
  warm-start workloads (the MD use case named in Sec. VI).
* ``batched_overlaps`` -- many Gaussian-kernel matrices of uneven N with a
  controlled condition number.
* ``huckel_hamiltonian`` -- a symmetric Hamiltonian matching an overlap S
  (extended-Hueckel form), the H of the generalized problem H C = S C eps that
  Z^T S Z = I reduces to standard form (Sec. II.A).
"""
from __future__ import annotations

import math

import numpy as np

BOHR_IN_ANGSTROM = 0.529177210903


# --------------------------------------------------------------------------
# positions
# --------------------------------------------------------------------------
def rsa_positions(n: int, density: float, d_min: float, rng: np.random.Generator,
                  max_rounds: int = 1000) -> np.ndarray:
    """n points, uniform in a cube of side (n/density)^(1/3) (open boundaries).

    With d_min > 0 this is random sequential addition: candidates are drawn in
    batches and taken in draw order; a candidate is kept only if no point kept
    before it lies closer than d_min."""
    from scipy.spatial import cKDTree

    side = (n / density) ** (1.0 / 3.0)
    if d_min <= 0.0:
        return rng.uniform(0.0, side, size=(n, 3))
    kept = np.empty((0, 3))
    for _ in range(max_rounds):
        need = n - kept.shape[0]
        if need == 0:
            return kept
        cand = rng.uniform(0.0, side, size=(max(64, need + need // 4), 3))
        if kept.shape[0]:
            dist, _ = cKDTree(kept).query(cand, k=1)
            cand = cand[dist >= d_min]
        # greedy in draw order among the survivors
        pairs = cKDTree(cand).query_pairs(d_min, output_type="ndarray")
        ok = np.ones(cand.shape[0], dtype=bool)
        if pairs.size:
            later = np.maximum(pairs[:, 0], pairs[:, 1])
            earlier = np.minimum(pairs[:, 0], pairs[:, 1])
            order = np.argsort(later, kind="stable")
            for e, l in zip(earlier[order], later[order]):
                if ok[e]:
                    ok[l] = False
        cand = cand[ok][:need]
        kept = np.concatenate([kept, cand])
    raise RuntimeError("random sequential addition did not place all points")


def _exp_inplace(x: np.ndarray) -> np.ndarray:
    """Elementwise exp in FP64, in place (torch's multithreaded CPU kernel)."""
    import torch

    torch.from_numpy(x).exp_()
    return x


def gaussian_kernel_overlap(pos: np.ndarray, sigma: float) -> np.ndarray:
    """S_ij = exp(-|r_i - r_j|^2 / (2 sigma^2)) in FP64.

    The squared distance is summed per axis from (x_i - x_j)^2, which is
    bitwise symmetric, so S is exactly symmetric with a unit diagonal."""
    n = pos.shape[0]
    r2 = np.zeros((n, n))
    buf = np.empty((n, n))
    for ax in range(3):
        np.subtract.outer(pos[:, ax], pos[:, ax], out=buf)
        np.multiply(buf, buf, out=buf)
        r2 += buf
    del buf
    r2 *= -1.0 / (2.0 * sigma * sigma)
    return _exp_inplace(r2)


def overlap_gaussian(n: int, sigma: float, seed: int, density: float = 0.1,
                     d_min: float = 0.8) -> np.ndarray:
    """Gaussian-kernel overlap of n atoms (seeded)."""
    rng = np.random.default_rng(seed)
    return gaussian_kernel_overlap(rsa_positions(n, density, d_min, rng), sigma)


# --------------------------------------------------------------------------
# s/p/d cluster
# --------------------------------------------------------------------------
def cuboctahedron_positions(shells: int = 5, lattice_a: float = 4.09) -> np.ndarray:
    """fcc cuboctahedron: integer points (i,j,k) with even i+j+k, max|.| <= shells and
    |i|+|j|+|k| <= 2*shells, in units of a/2.  shells = 5 gives 561 atoms."""
    r = np.arange(-2 * shells, 2 * shells + 1)
    i, j, k = np.meshgrid(r, r, r, indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    keep = ((i + j + k) % 2 == 0) & (np.maximum(np.maximum(abs(i), abs(j)), abs(k)) <= shells) \
        & (abs(i) + abs(j) + abs(k) <= 2 * shells)
    return np.stack([i[keep], j[keep], k[keep]], axis=1).astype(np.float64) * (lattice_a / 2.0)


# Cartesian monomials up to l = 2 and the 9 real functions built from them:
# s; p_x, p_y, p_z; d_xy, d_xz, d_yz, d_{x2-y2}, d_{z2}.
_CART = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1),
         (1, 1, 0), (1, 0, 1), (0, 1, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2)]
_SPH = np.zeros((9, 10))
_SPH[0, 0] = 1.0
_SPH[1, 1] = _SPH[2, 2] = _SPH[3, 3] = 1.0
_SPH[4, 4] = _SPH[5, 5] = _SPH[6, 6] = 1.0
_SPH[7, 7], _SPH[7, 8] = 1.0, -1.0
_SPH[8, 7], _SPH[8, 8], _SPH[8, 9] = -1.0, -1.0, 2.0


def _os_1d(xpa: np.ndarray, xpb: np.ndarray, s00: np.ndarray, p: float) -> np.ndarray:
    """1-D Obara-Saika overlap table S[i][j], i, j <= 2, for every pair."""
    t = np.zeros(s00.shape + (3, 3))
    t[..., 0, 0] = s00
    h = 0.5 / p
    t[..., 1, 0] = xpa * t[..., 0, 0]
    t[..., 0, 1] = xpb * t[..., 0, 0]
    t[..., 1, 1] = xpb * t[..., 1, 0] + h * t[..., 0, 0]
    t[..., 2, 0] = xpa * t[..., 1, 0] + h * t[..., 0, 0]
    t[..., 0, 2] = xpb * t[..., 0, 1] + h * t[..., 0, 0]
    t[..., 2, 1] = xpb * t[..., 2, 0] + h * 2 * t[..., 1, 0]
    t[..., 1, 2] = xpa * t[..., 0, 2] + h * 2 * t[..., 0, 1]
    t[..., 2, 2] = xpb * t[..., 2, 1] + h * (2 * t[..., 1, 1] + t[..., 2, 0])
    return t


def spd_gaussian_overlap(pos: np.ndarray, alpha: float) -> np.ndarray:
    """Overlap of 9 unit-normalized primitive Gaussians (s, p, 5 real d) per atom,
    all with exponent alpha (A^-2).  Returns the (9 n) x (9 n) FP64 matrix with
    atom-major ordering."""
    n = pos.shape[0]
    p = 2.0 * alpha
    mu = alpha * alpha / p
    S = np.empty((9 * n, 9 * n))
    blk = 64
    for a0 in range(0, n, blk):
        A = pos[a0:a0 + blk]
        d = A[:, None, :] - pos[None, :, :]            # (bA, n, 3), A - B
        P_minus_A = -0.5 * d                            # P = (A + B)/2
        P_minus_B = 0.5 * d
        tabs = []
        for ax in range(3):
            s00 = np.sqrt(np.pi / p) * np.exp(-mu * d[..., ax] ** 2)
            tabs.append(_os_1d(P_minus_A[..., ax], P_minus_B[..., ax], s00, p))
        cart = np.empty(d.shape[:2] + (10, 10))
        for u, (ax, ay, az) in enumerate(_CART):
            for v, (bx, by, bz) in enumerate(_CART):
                cart[..., u, v] = tabs[0][..., ax, bx] * tabs[1][..., ay, by] * tabs[2][..., az, bz]
        sph = np.einsum("ia,xyab,jb->xyij", _SPH, cart, _SPH, optimize=True)
        bA = A.shape[0]
        S[9 * a0:9 * (a0 + bA)] = sph.transpose(0, 2, 1, 3).reshape(9 * bA, 9 * n)
    dn = np.sqrt(np.diag(S).copy())
    S /= dn[:, None]
    S /= dn[None, :]
    S = 0.5 * (S + S.T)
    np.fill_diagonal(S, 1.0)
    return S


def cluster_spd_overlap(alpha_bohr: float = 0.08, shells: int = 5,
                        lattice_a: float = 4.09) -> np.ndarray:
    """The 561-atom cluster overlap (N = 5049 for shells = 5).  alpha in bohr^-2."""
    alpha = alpha_bohr / (BOHR_IN_ANGSTROM ** 2)
    return spd_gaussian_overlap(cuboctahedron_positions(shells, lattice_a), alpha)


# --------------------------------------------------------------------------
# the synthetic family of Sec. V.A
# --------------------------------------------------------------------------
def paper_synthetic(n: int, gamma: float = 0.5) -> np.ndarray:
    """exp(-|i-j|/2) sin(i+1) for 1 <= i, j <= n, shifted by (gamma - eps_1) I.

    As printed this matrix is not symmetric (the sin factor depends on the row
    only); the symmetric part (A + A^T)/2 is used, then shifted so that its
    lowest eigenvalue becomes gamma."""
    i = np.arange(1, n + 1, dtype=np.float64)
    A = np.exp(-np.abs(i[:, None] - i[None, :]) / 2.0) * np.sin(i + 1.0)[:, None]
    A = 0.5 * (A + A.T)
    eps1 = np.linalg.eigvalsh(A)[0]
    return A + (gamma - eps1) * np.eye(n)


def uniform_noise(n: int, seed: int) -> np.ndarray:
    """U_ij ~ U(-0.5, 0.5), seeded (the perturbation of Sec. V.A)."""
    return np.random.default_rng(seed).uniform(-0.5, 0.5, size=(n, n))


def huckel_hamiltonian(S: np.ndarray, seed: int, k: float = 1.75, e_lo: float = -14.0,
                       e_hi: float = -6.0) -> np.ndarray:
    """H_ii = e_i with on-site energies e_i ~ U(e_lo, e_hi) (eV), H_ij = k S_ij (e_i + e_j)/2
    (Wolfsberg-Helmholz).  Symmetric, indefinite in general."""
    e = np.random.default_rng(seed).uniform(e_lo, e_hi, size=S.shape[0])
    H = k * S * (0.5 * (e[:, None] + e[None, :]))
    np.fill_diagonal(H, e)
    return 0.5 * (H + H.T)


# --------------------------------------------------------------------------
# MD-like trajectory and batches
# --------------------------------------------------------------------------
def md_trajectory(n: int, frames: int, seed: int, sigma: float = 1.0, step: float = 0.01,
                  density: float = 0.1, d_min: float = 0.8):
    """Yield S for each frame: positions random-walk by N(0, step^2) per coordinate."""
    rng = np.random.default_rng(seed)
    pos = rsa_positions(n, density, d_min, rng)
    for f in range(frames):
        if f:
            pos = pos + rng.normal(0.0, step, size=pos.shape)
        yield gaussian_kernel_overlap(pos, sigma)


def shift_to_condition(K: np.ndarray, kappa: float) -> np.ndarray:
    """(K + tau I)/(1 + tau) with tau chosen so that cond = kappa (unit diagonal kept)."""
    w = np.linalg.eigvalsh(K)
    lo, hi = w[0], w[-1]
    tau = (hi - kappa * lo) / (kappa - 1.0)
    if tau <= -lo:
        raise ValueError("requested condition number not reachable")
    S = (K + tau * np.eye(K.shape[0])) / (1.0 + tau)
    S = 0.5 * (S + S.T)
    np.fill_diagonal(S, 1.0)
    return S


def batch_sizes(count: int, seed: int, n_lo: int = 64, n_hi: int = 1024) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)


def batched_overlaps(count: int, seed: int, n_lo: int = 64, n_hi: int = 1024,
                     kappa_lo: float = 10.0, kappa_hi: float = 1e4, sigma: float = 1.0):
    """count Gaussian-kernel overlaps, N log-uniform in [n_lo, n_hi], target
    condition number log-uniform in [kappa_lo, kappa_hi]."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(int)
    kap = 10.0 ** rng.uniform(math.log10(kappa_lo), math.log10(kappa_hi), size=count)
    out = []
    for n, k in zip(ns, kap):
        pos = rsa_positions(int(n), 0.1, 0.0, rng)
        K = gaussian_kernel_overlap(pos, sigma)
        out.append(shift_to_condition(K, float(k)))
    return out


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
WORKLOADS = {
    # name: (N, sigma) for the Gaussian-kernel family
    "gauss256": (256, 1.2),
    "gauss4096": (4096, 1.0),
    "gauss3000": (3000, 1.0),
}


def workload(name: str, seed: int = 0) -> np.ndarray:
    if name == "cluster5049":
        return cluster_spd_overlap()
    n, sigma = WORKLOADS[name]
    return overlap_gaussian(n, sigma, seed)
