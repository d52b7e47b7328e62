"""Philox4x32-10 counter-based generator, written from its published
definition (J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random numbers:
as easy as 1, 2, 3", SC'11, Section 3 and the Philox-4x32 round constants).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One block maps a 128-bit counter (four 32-bit words) and a 64-bit key (two
32-bit words) to four 32-bit outputs through ten rounds.  Each round does two
32x32->64 multiplications by fixed multipliers, swaps and xors the halves
with the other counter words and the round key; the key is bumped by two
Weyl constants between rounds.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ctr: array [..., 4] of uint32 counter words; key: array [..., 2] (or a
    pair broadcastable to it).  Returns uint32 array [..., 4].
    """
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    key = np.asarray(key, dtype=np.uint64)
    k0 = np.broadcast_to(key[..., 0], c[0].shape).astype(np.uint64)
    k1 = np.broadcast_to(key[..., 1], c[0].shape).astype(np.uint64)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    mask = np.uint64(MASK32)
    s32 = np.uint64(32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
        p0 = m0 * c[0]          # exact: both factors < 2^32
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack([x.astype(np.uint32) for x in c], axis=-1)
