"""Seeded synthetic Tucker-sum workloads.

This module only draws inputs: Gaussian cores, orthonormal factors and the
per-term rank tables of the five workloads the hot path is exercised on.  It
holds none of the recompression arithmetic, so both the FP64 oracle and the
GPU path can take their inputs from it without sharing any of the method.

Every array is float64, Fortran ordered (mode 1 fastest), as the paper's
unfolding convention (Section 2.1, eq. for the unfolding index) expects.

A Tucker sum is returned as a dict:
  dims    : tuple of d mode sizes n_k
  ranks   : int array [s, d], ranks[i, k] = r_k^(i)
  cores   : list of s arrays, core i has shape ranks[i]
  factors : list of s lists of d arrays, factors[i][k] has shape (n_k, r_k^(i))
  coeffs  : float array [s] (all ones unless stated)
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "orthonormal", "gaussian_core", "decaying_core", "tucker_sum",
    "config_tiny", "config_structured", "config_precision", "config_batch",
    "config_gradient", "gradient_target", "e1_low_rank_sum", "e2_cancelling_sum",
    "random_sum", "WORKLOADS",
]


def orthonormal(rng: np.random.Generator, n: int, r: int) -> np.ndarray:
    """n x r matrix with orthonormal columns: Q of the QR of a Gaussian matrix."""
    a = rng.standard_normal((n, r))
    q, _ = np.linalg.qr(a)
    return np.asfortranarray(q)


def gaussian_core(rng: np.random.Generator, shape) -> np.ndarray:
    return np.asfortranarray(rng.standard_normal(tuple(int(x) for x in shape)))


def decaying_core(rng: np.random.Generator, shape, rate: float = 0.1) -> np.ndarray:
    """Gaussian entries scaled by 10^(-rate * (i_1 + ... + i_d)), 0-based indices."""
    shape = tuple(int(x) for x in shape)
    g = rng.standard_normal(shape)
    idx = np.zeros(shape)
    for k, n in enumerate(shape):
        sh = [1] * len(shape)
        sh[k] = n
        idx = idx + np.arange(n, dtype=np.float64).reshape(sh)
    return np.asfortranarray(g * 10.0 ** (-rate * idx))


def tucker_sum(dims, ranks, cores, factors, coeffs=None) -> dict:
    ranks = np.asarray(ranks, dtype=np.int64).reshape(len(cores), len(dims))
    if coeffs is None:
        coeffs = np.ones(len(cores))
    return {"dims": tuple(int(x) for x in dims), "ranks": ranks, "cores": list(cores),
            "factors": [list(f) for f in factors], "coeffs": np.asarray(coeffs, dtype=np.float64)}


def random_sum(seed: int, dims, ranks, decay: float | None = None, coeffs=None,
               orthonormal_factors: bool = True) -> dict:
    """Generic seeded sum: ranks is [s, d]; cores Gaussian (optionally decaying)."""
    rng = np.random.default_rng(seed)
    ranks = np.asarray(ranks, dtype=np.int64)
    cores, factors = [], []
    for i in range(ranks.shape[0]):
        r = ranks[i]
        cores.append(decaying_core(rng, r, decay) if decay else gaussian_core(rng, r))
        if orthonormal_factors:
            factors.append([orthonormal(rng, dims[k], int(r[k])) for k in range(len(dims))])
        else:
            factors.append([np.asfortranarray(rng.standard_normal((dims[k], int(r[k]))))
                            for k in range(len(dims))])
    return tucker_sum(dims, ranks, cores, factors, coeffs)


def config_tiny(seed: int = 1) -> dict:
    """d=3, 64^3, s=4 terms, cores 8^3 N(0,1), orthonormal 64x8 factors.
    Sketch: Kronecker, target 16 + oversampling 8 = 24 per mode."""
    s = random_sum(seed, (64, 64, 64), np.full((4, 3), 8))
    s.update(kind="kron", ell=(24, 24, 24), omega_seed=1001)
    return s


def config_structured(seed: int = 2) -> dict:
    """d=3, 512^3, s=16, ranks uniform in [16, 48] per term and mode, cores
    N(0,1) * 10^(-0.1(i+j+k)), orthonormal factors; target 64 + 10."""
    rng = np.random.default_rng(seed)
    ranks = rng.integers(16, 49, size=(16, 3))
    s = random_sum(seed + 100, (512, 512, 512), ranks, decay=0.1)
    s.update(kind="krp", ell=(74, 74, 74), omega_seed=1002)
    return s


def config_precision(seed: int = 3) -> dict:
    """d=4, 256^4, s=8, cores 32^4 Gaussian, orthonormal 256x32; KRP 48 + 8."""
    s = random_sum(seed, (256,) * 4, np.full((8, 4), 32))
    s.update(kind="krp", ell=(56,) * 4, omega_seed=1003)
    return s


def config_batch(seed: int = 4, count: int = 256) -> list[dict]:
    """`count` independent sums, d=3; one mode size per sum from
    {64,128,192,256,384}; s in [2,10]; ranks in [4,40]; decaying Gaussian
    cores; KRP width min(48, n/4) + 8."""
    rng = np.random.default_rng(seed)
    sizes = (64, 128, 192, 256, 384)
    out = []
    for b in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        s = int(rng.integers(2, 11))
        ranks = rng.integers(4, 41, size=(s, 3))
        one = random_sum(int(rng.integers(0, 2**31 - 1)), (n, n, n), ranks, decay=0.1)
        m = min(48, n // 4) + 8
        one.update(kind="krp", ell=(m, m, m), omega_seed=1004 + b)
        out.append(one)
    return out


def config_gradient(seed: int = 5) -> dict:
    """d=3, 256^3, s=6, cores 24^3, orthonormal 256x24; KRP 32 + 8 = 40."""
    s = random_sum(seed, (256,) * 3, np.full((6, 3), 24))
    s.update(kind="krp", ell=(40, 40, 40), omega_seed=1005)
    return s


def gradient_target(seed: int = 55, n: int = 256, r: int = 32) -> dict:
    """Fixed random rank-32 Tucker target for the gradient workload."""
    return random_sum(seed, (n, n, n), np.full((1, 3), r))


def e1_low_rank_sum(seed: int, d: int = 4, n: int = 64, terms: int = 20, r_true: int = 10) -> dict:
    """Rank-1 terms whose factors are random combinations of a fixed
    orthonormal basis Q_k (n x r_true) per mode (Section 5.1.1 construction):
    the sum has multilinear rank at most r_true in every mode."""
    rng = np.random.default_rng(seed)
    bases = [orthonormal(rng, n, r_true) for _ in range(d)]
    cores, factors = [], []
    for _ in range(terms):
        cores.append(gaussian_core(rng, (1,) * d))
        factors.append([np.asfortranarray(bases[k] @ rng.standard_normal((r_true, 1)))
                        for k in range(d)])
    return tucker_sum((n,) * d, np.ones((terms, d), dtype=np.int64), cores, factors)


def e2_cancelling_sum(seed: int, n: int = 200, terms: int = 60, r_noise: int = 12) -> tuple[dict, dict]:
    """Section 5.1.2 construction: a rank-5 target with diagonal core
    {1, .8, .6, 2e-6, 1e-6}, plus terms/2 noise tensors of rank 12 with
    diagonal cores log-spaced from 1e6 to 1e-5, added then subtracted.
    Returns (sum, target).  Target and noise factors are seeded orthonormal
    Gaussians (the paper does not say how they are drawn)."""
    rng = np.random.default_rng(seed)
    d = 3

    def diag_core(vals):
        g = np.zeros((len(vals),) * d, order="F")
        for j, v in enumerate(vals):
            g[(j,) * d] = v
        return g

    tgt_core = diag_core([1.0, 0.8, 0.6, 2e-6, 1e-6])
    tgt_f = [orthonormal(rng, n, 5) for _ in range(d)]
    target = tucker_sum((n,) * d, np.full((1, d), 5), [tgt_core], [tgt_f])
    noise_vals = np.logspace(6, -5, r_noise)
    half = terms // 2
    noises = [([orthonormal(rng, n, r_noise) for _ in range(d)]) for _ in range(half)]
    r = 5 + r_noise
    cores, factors = [], []
    # each summand (1/terms) X_target +/- X_noise^(i) is one Tucker tensor of
    # rank 5 + r_noise: concatenated factors, block-diagonal core
    for sign in (1.0, -1.0):
        for i in range(half):
            g = np.zeros((r,) * d, order="F")
            g[(slice(0, 5),) * d] = tgt_core / terms
            g[(slice(5, r),) * d] = sign * diag_core(noise_vals)
            cores.append(g)
            factors.append([np.asfortranarray(np.concatenate([tgt_f[k], noises[i][k]], axis=1))
                            for k in range(d)])
    return tucker_sum((n,) * d, np.full((terms, d), r), cores, factors), target


WORKLOADS = {
    "tiny": config_tiny,
    "structured": config_structured,
    "precision": config_precision,
    "batch": config_batch,
    "gradient": config_gradient,
}
