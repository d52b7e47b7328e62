"""Seeded Gaussian test matrices Omega_k (Section 3.1: standard Gaussian
n_k x m matrices for the Khatri-Rao sketch, n_k x q_k for the Kronecker
sketch; one matrix per mode, reused for every unfolding it enters).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper fixes only the distribution.  Reading adopted here, and implemented
independently on the GPU:
  * entry e = i + n_k * t (column-major) of Omega_k uses Philox4x32-10 block
    p = e // 2 with counter (lo32(p), hi32(p), k, 0) and key
    (lo32(seed), hi32(seed)), k the 0-based mode;
  * u1 = ((x1 << 32 | x0) >> 11) + 1) * 2^-53  in (0, 1],
    u2 = ((x3 << 32 | x2) >> 11) * 2^-53       in [0, 1);
  * Box-Muller in FP64: rho = sqrt(-2 ln u1), z0 = rho cos(2 pi u2),
    z1 = rho sin(2 pi u2); entry e takes z0 if e is even, z1 if odd;
  * the value is rounded to 8 significant bits, round-to-nearest-even on the
    FP64 bit pattern, so it is exactly representable in BF16, FP32 and FP64
    and every precision form sketches with the identical matrix.
"""
import numpy as np

from .philox import philox4x32_10


def round_to_bf16_f64(x):
    """Round float64 values to the nearest value with an 8-bit significand
    (ties to even), operating on the IEEE-754 binary64 bit pattern: drop the
    low 45 of the 52 stored fraction bits."""
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    b = x.view(np.uint64)
    keep_lsb = (b >> np.uint64(45)) & np.uint64(1)
    b = (b + np.uint64((1 << 44) - 1) + keep_lsb) & ~np.uint64((1 << 45) - 1)
    return b.view(np.float64)


def box_muller_pair(x):
    """Map Philox outputs [..., 4] (uint32) to two FP64 standard normals."""
    x = x.astype(np.uint64)
    w0 = (x[..., 1] << np.uint64(32)) | x[..., 0]
    w1 = (x[..., 3] << np.uint64(32)) | x[..., 2]
    u1 = ((w0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (w1 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    ang = (2.0 * np.pi) * u2
    return rho * np.cos(ang), rho * np.sin(ang)


def omega(seed: int, mode: int, rows: int, cols: int, rounded: bool = True) -> np.ndarray:
    """Omega_k for 0-based mode `mode`: rows x cols, float64, Fortran order."""
    count = rows * cols
    e = np.arange(count, dtype=np.uint64)
    p = e >> np.uint64(1)
    ctr = np.zeros((count, 4), dtype=np.uint64)
    ctr[:, 0] = p & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = p >> np.uint64(32)
    ctr[:, 2] = np.uint64(mode)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    z0, z1 = box_muller_pair(philox4x32_10(ctr, key))
    z = np.where((e & np.uint64(1)) == 0, z0, z1)
    if rounded:
        z = round_to_bf16_f64(z)
    return np.asfortranarray(z.reshape((rows, cols), order="F"))


def omegas(seed: int, dims, widths, rounded: bool = True) -> list:
    """One Omega_k per mode: dims[k] x widths[k]."""
    return [omega(seed, k, int(dims[k]), int(widths[k]), rounded) for k in range(len(dims))]
