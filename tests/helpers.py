"""Shared test utilities: moving seeded synthetic sums to torch tensors in
column-major layout, and relative errors."""
import numpy as np


def to_torch(tsum, device, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    from paper_2603_13532_amd import fortran

    def conv(a):
        t = torch.from_numpy(np.asfortranarray(a)).to(device=device, dtype=dtype)
        return fortran(t)
    cores = [conv(g) for g in tsum["cores"]]
    factors = [[conv(u) for u in us] for us in tsum["factors"]]
    return cores, factors


def np_of(t):
    return np.asfortranarray(t.detach().to("cpu").double().numpy())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    d = np.linalg.norm((a - b).ravel())
    return d / nb if nb > 0 else d


# ---------------------------------------------------------------- precision ladder
# Unit roundoffs of each arithmetic form.  `rep`: relative error of one
# product from representing its operands (the BF16 splits keep 8, 16 or 24
# significant bits of each FP32 operand); `acc`: unit roundoff of the
# accumulation (FP32 for every FP32-class form).
UNIT = {
    "fp64": {"rep": 0.0, "acc": 2.0 ** -53},
    "fp32": {"rep": 0.0, "acc": 2.0 ** -24},
    "bf16x6": {"rep": 2.0 ** -23, "acc": 2.0 ** -24},
    "bf16x3": {"rep": 2.0 ** -16, "acc": 2.0 ** -24},
    "bf16x1": {"rep": 2.0 ** -8, "acc": 2.0 ** -24},
}


def rounded_to_f32(tsum):
    """The same sum with cores and factors rounded to FP32 (the values an FP32
    input buffer holds), still as float64 arrays."""
    out = dict(tsum)
    out["cores"] = [np.asfortranarray(g.astype(np.float32).astype(np.float64)) for g in tsum["cores"]]
    out["factors"] = [[np.asfortranarray(u.astype(np.float32).astype(np.float64)) for u in us]
                      for us in tsum["factors"]]
    return out


def absolute_sum(tsum):
    """|c_i|, |G^(i)|, |U_k^(i)|: evaluating a product chain on these gives the
    sum of the absolute values of its terms, the componentwise scale of its
    rounding error."""
    out = dict(tsum)
    out["cores"] = [np.abs(g) for g in tsum["cores"]]
    out["factors"] = [[np.abs(u) for u in us] for us in tsum["factors"]]
    out["coeffs"] = np.abs(np.asarray(tsum["coeffs"], dtype=np.float64))
    return out


def envelope_tol(form, stages, k_total, lam=4.0):
    """Componentwise error scale of a chain of `stages` products with total
    reduction length k_total: each product's representation error plus the
    probabilistic accumulation bound lam * sqrt(K) * u (Higham and Mary,
    SIAM J. Sci. Comput. 2019)."""
    u = UNIT[form]
    return stages * 2.0 * u["rep"] + lam * np.sqrt(k_total) * u["acc"]


def envelope_ratio(got, want, scale, tol):
    """Largest |got - want| / (tol * scale) over all elements (<= 1 passes)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = tol * np.asarray(scale, dtype=np.float64) + 1e-300
    return float(np.max(np.abs(got - want) / den))


def column_errors(got, want):
    """Per column: max |got - want| / max |want| (the column's own scale)."""
    got = np.asarray(got, dtype=np.float64).reshape(got.shape[0], -1)
    want = np.asarray(want, dtype=np.float64).reshape(want.shape[0], -1)
    num = np.max(np.abs(got - want), axis=0)
    den = np.maximum(np.max(np.abs(want), axis=0), 1e-300)
    return num / den


def slice_errors(got, want):
    """Per mode-1 slice X[i, ...]: max |got - want| / max |want[i, ...]|."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    g = got.reshape(got.shape[0], -1, order="F")
    w = want.reshape(want.shape[0], -1, order="F")
    return np.max(np.abs(g - w), axis=1) / np.maximum(np.max(np.abs(w), axis=1), 1e-300)


def _ttm(x, a, k):
    y = np.tensordot(a, x, axes=([1], [k]))
    return np.moveaxis(y, 0, k)


def tucker_rel_diff(ha, qa, hb, qb, device=None):
    """||[[ha; qa]] - [[hb; qb]]|| / ||[[hb; qb]]|| without forming either
    tensor: both are written in one orthonormal basis Z_k of
    range([qa_k, qb_k]) per mode (Householder QR in FP64) and the two cores
    hx x_k (Z_k^T qx_k) are subtracted, so nothing cancels and neither set of
    factors needs to be orthonormal.  With `device` the contraction runs in
    FP64 PyTorch on that device (the cores have prod_k (w_a + w_b) entries)."""
    d = len(qa)
    if device is None:
        ca = np.asarray(ha, dtype=np.float64)
        cb = np.asarray(hb, dtype=np.float64)
        for k in range(d):
            a = np.asarray(qa[k], dtype=np.float64)
            b = np.asarray(qb[k], dtype=np.float64)
            z, _ = np.linalg.qr(np.concatenate([a, b], axis=1))
            ca = _ttm(ca, z.T @ a, k)
            cb = _ttm(cb, z.T @ b, k)
        return float(np.linalg.norm((ca - cb).ravel()) / np.linalg.norm(cb.ravel()))
    import torch

    def dev(x):
        if isinstance(x, torch.Tensor):
            return x.to(device=device, dtype=torch.float64)
        return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)
    ca, cb = dev(ha), dev(hb)
    for k in range(d):
        a, b = dev(qa[k]), dev(qb[k])
        z, _ = torch.linalg.qr(torch.cat([a, b], dim=1))
        for which in (0, 1):
            m = (z.T @ (a if which == 0 else b)).contiguous()
            c = ca if which == 0 else cb
            c = torch.movedim(torch.tensordot(m, c, dims=([1], [k])), 0, k)
            if which == 0:
                ca = c
            else:
                cb = c
    out = float(torch.linalg.vector_norm(ca - cb) / torch.linalg.vector_norm(cb))
    del ca, cb
    return out


def condition_bound(h, ranks):
    """The GPU factors the mode Grams, whose eigenvectors near the cut are
    determined to about u sigma_1^2 / sigma_r^2 of the kept singular value:
    the reconstructions then differ by about u sigma_1 / sigma_r of ||H||
    (the oracle takes singular vectors of the unfoldings directly)."""
    worst = 1.0
    g = h
    for n, r in enumerate(ranks):
        s = np.linalg.svd(_unfold(g, n), compute_uv=False)
        worst = max(worst, s[0] / s[r - 1])
        l = np.linalg.svd(_unfold(g, n), full_matrices=False)[0][:, :r]
        g = _ttm_o(g, l.T, n)
    return 256 * 2.0 ** -53 * worst




def _unfold(x, n):
    from oracle import tensor as T
    return T.unfold(x, n)


def _ttm_o(x, a, n):
    from oracle import tensor as T
    return T.ttm(x, a, n)
