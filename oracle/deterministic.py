"""Deterministic sum-and-round baseline: TuckerAxby (Algorithm 1) applied to
all terms, then TuckerRounding (Algorithm 2).  Dense block-superdiagonal core,
so tiny inputs only.  Used as an independent reference for the sketched
result on sums of exactly low multilinear rank (Section 5.1.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
import numpy as np

from .tensor import ttm, unfold


def tucker_axby_all(tsum: dict):
    """Formal sum: W_n = [U_n^(1) ... U_n^(s)], core with c_i G^(i) in
    disjoint blocks along the super-diagonal (Algorithm 1, repeated)."""
    d = len(tsum["dims"])
    ranks = np.asarray(tsum["ranks"])
    tot = ranks.sum(axis=0)
    core = np.zeros(tuple(int(x) for x in tot), order="F")
    off = np.zeros(d, dtype=np.int64)
    for c, g, r in zip(tsum["coeffs"], tsum["cores"], ranks):
        sl = tuple(slice(int(off[k]), int(off[k] + r[k])) for k in range(d))
        core[sl] = c * g
        off += r
    facs = [np.concatenate([us[n] for us in tsum["factors"]], axis=1) for n in range(d)]
    return core, facs


def tucker_rounding(core, facs, tau: float):
    """Algorithm 2: QR of every factor with R absorbed into the core, then
    ST-HOSVD with theta = tau^2 ||G||^2 / d and per-mode rank
    min{r : sum_{j > r} s_j^2 <= theta}."""
    d = core.ndim
    g = core
    us = []
    for n in range(d):
        q, r = np.linalg.qr(facs[n], mode="reduced")
        us.append(q)
        g = ttm(g, r, n)
    theta = tau ** 2 * float(np.sum(g ** 2)) / d
    for n in range(d):
        l, s, _ = np.linalg.svd(unfold(g, n), full_matrices=False)
        tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1][1:], [0.0]])
        rn = int(np.argmax(tail <= theta)) + 1
        p = l[:, :rn]
        us[n] = us[n] @ p
        g = ttm(g, p.T, n)
    return g, us
