"""Precision-ladder parity cases shared by the GPU tests and the probe that
prints their measured error levels: every arithmetic form of the library
through its C ABI (tucker_sum_sketch, tucker_sum_project,
tucker_sum_recompress) against the FP64 oracle on the same FP32-stored
inputs."""
import numpy as np

import synth
from helpers import (absolute_sum, column_errors, envelope_ratio, envelope_tol, np_of, rel,
                     rounded_to_f32, slice_errors, to_torch, tucker_rel_diff)
from oracle import recompress as RC
from oracle import sketch as S

DEV = "cuda:0"

# form -> (sketch arithmetic, projection arithmetic)
FORMS = {
    "fp64": ("fp64", "fp64"),
    "fp32": ("fp32", "fp32"),
    "bf16x6": ("bf16x6", "bf16x6"),
    "bf16x3": ("bf16x3", "bf16x6"),
    "bf16x1": ("bf16x1", "bf16x6"),
    # FP64 sketch and QR, mixed projection (FP32 inputs)
    "fp64s_fp32p": ("fp64", "fp32"),
    "fp64s_bf16x6p": ("fp64", "bf16x6"),
}


def _ragged(seed, dims, ranks, coeffs=None, decay=None):
    return synth.random_sum(seed, dims, ranks, decay=decay, orthonormal_factors=False,
                            coeffs=coeffs if coeffs is not None else
                            np.linspace(-1.5, 2.0, len(ranks)))


def case(name):
    """(sum, kind, sizes, seed) of a named case."""
    if name == "ragged3_krp":       # three row tiles, two rank tiles, ragged tails
        return (_ragged(100, (130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]]),
                "krp", [80], 31)
    if name == "ragged3_kron":
        return (_ragged(101, (130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]]),
                "kron", [3, 5, 4], 32)
    if name == "order2_krp":        # Khatri-Rao of one factor sketch (general cursor)
        return _ragged(102, (65, 33), [[17, 9], [65, 3]]), "krp", [20], 33
    if name == "order4_krp":        # fixed cursor over three other modes
        return _ragged(103, (40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]]), "krp", [11], 34
    if name == "order4_kron":
        return _ragged(104, (40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]]), "kron", [2, 3, 2, 2], 35
    if name == "order5_krp":        # general cursor with the factor sketches in LDS
        return (_ragged(105, (12, 10, 9, 8, 7), [[3, 2, 4, 2, 3], [2, 3, 2, 3, 2]]),
                "krp", [9], 36)
    if name == "wide_ranks_krp":    # factor sketches too large for LDS: global-memory cursor
        return (_ragged(106, (100, 90, 80), [[60, 60, 20], [30, 50, 50]]), "krp", [70], 37)
    if name == "structured_krp":    # d=3, 512^3, 16 terms, decaying cores, m = 74
        ts = synth.config_structured()
        return ts, "krp", [74], ts["omega_seed"]
    if name == "structured_kron":   # the same sum, Kronecker q = 9 (S = 81)
        ts = synth.config_structured()
        return ts, "kron", RC.kron_sizes(ts["ell"]), ts["omega_seed"]
    if name == "precision_krp":     # d=4, 256^4, 8 terms, cores 32^4, m = 56
        ts = synth.config_precision()
        return ts, "krp", [56], ts["omega_seed"]
    raise KeyError(name)


SMALL = ["ragged3_krp", "ragged3_kron", "order2_krp", "order4_krp", "order4_kron", "order5_krp",
         "wide_ranks_krp"]
LARGE = ["structured_krp", "structured_kron", "precision_krp"]


def chain_lengths(ts, kind, sizes):
    """Longest total reduction length of the sketch chain (factor sketch,
    core sketch, term expansion) and of the projection chain (Q^T U, the
    multi-TTM, the term sum)."""
    dims = ts["dims"]
    d = len(dims)
    ranks = np.asarray(ts["ranks"])
    ky = 0
    for n in range(d):
        core = np.max(np.prod(np.delete(ranks, n, axis=1), axis=1)) if kind == "krp" else \
            np.max(np.sum(np.delete(ranks, n, axis=1), axis=1))
        ky = max(ky, max(dims) + int(core) + int(np.sum(ranks[:, n])))
    kh = max(dims) + int(np.max(np.sum(ranks, axis=1))) + int(np.max(np.sum(ranks, axis=0)))
    return ky, kh


def measure(tsk, name, form, ref_cache=None):
    """Every error of one (case, form): Y (Frobenius, componentwise envelope,
    worst column), H given the oracle's Q (Frobenius, envelope, worst mode-1
    slice), Q (Frobenius and worst column, full-rank modes only) and the
    recompressed tensor end to end."""
    import torch
    ts, kind, sizes, seed = case(name)
    d = len(ts["dims"])
    sp, pp = FORMS[form]
    f64 = form == "fp64"
    tsx = ts if f64 else rounded_to_f32(ts)
    key = (name, f64)
    if ref_cache is not None and key in ref_cache:
        ref, yabs, habs = ref_cache[key]
    else:
        ref = RC.recompress(tsx, kind, sizes, seed)
        absum = absolute_sum(tsx)
        yabs = S.structured_sketch(absum, [np.abs(o) for o in ref["omegas"]], kind)
        habs = RC.project_structured(absum, [np.abs(q) for q in ref["Q"]])
        if ref_cache is not None:
            ref_cache[key] = (ref, yabs, habs)
    dtype = torch.float64 if f64 else torch.float32
    cores, factors = to_torch(tsx, DEV, dtype)
    ky, kh = chain_lengths(tsx, kind, sizes)
    out = {"case": name, "form": form}
    # sketch stage
    ys = tsk.tucker_sum_sketch(cores, factors, kind, sizes, seed, coeffs=tsx["coeffs"],
                               sketch_prec=sp)
    torch.cuda.synchronize()
    ys = [np_of(y) for y in ys]
    tol_y = envelope_tol(sp, d + 2, ky)
    out["y_rel"] = max(rel(a, b) for a, b in zip(ys, ref["Y"]))
    out["y_env"] = max(envelope_ratio(a, b, s, tol_y) for a, b, s in zip(ys, ref["Y"], yabs))
    out["y_col"] = max(float(np.max(column_errors(a, b))) for a, b in zip(ys, ref["Y"]))
    # projection stage on the oracle's bases
    qref = [torch.from_numpy(np.asfortranarray(q)).to(DEV) for q in ref["Q"]]
    hq = np_of(tsk.tucker_sum_project(cores, factors, qref, coeffs=tsx["coeffs"],
                                      project_prec=pp, out_dtype=torch.float64))
    tol_h = envelope_tol(pp, d + 1, kh)
    out["h_rel"] = rel(hq, ref["H"])
    out["h_env"] = envelope_ratio(hq, ref["H"], habs, tol_h)
    out["h_slice"] = float(np.max(slice_errors(hq, ref["H"])))
    # the whole recompression
    qs, h = tsk.tucker_sum_recompress(cores, factors, kind, sizes, seed, coeffs=tsx["coeffs"],
                                      sketch_prec=sp, project_prec=pp)
    torch.cuda.synchronize()
    qs = [np_of(q) for q in qs]
    h = np_of(h)
    out["x_rel"] = tucker_rel_diff(h, qs, ref["H"], ref["Q"], device=DEV)
    out["orth"] = max(float(np.linalg.norm(q.T @ q - np.eye(q.shape[1]))) for q in qs)
    full = [y.shape[0] >= y.shape[1] and np.linalg.svd(y, compute_uv=False)[-1] >
            1e-9 * np.linalg.norm(y, 2) for y in ref["Y"]]
    out["full_rank"] = all(full)
    qerr = [rel(a, b) for a, b, f in zip(qs, ref["Q"], full) if f]
    out["q_rel"] = max(qerr) if qerr else None
    qcol = [float(np.max(column_errors(a, b))) for a, b, f in zip(qs, ref["Q"], full) if f]
    out["q_col"] = max(qcol) if qcol else None
    return out
