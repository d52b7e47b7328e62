"""Sketching-based recompression of Tucker-tensor sums on MI355X (gfx950).

Thin PyTorch binding over the C ABI in include/tsk.h (libtsk.so).  PyTorch
supplies device memory and the current HIP stream; every step of the method
runs in the library's HIP kernels.  This module only marshals arguments:
tensors are passed by pointer in column-major (Fortran) order, the layout the
paper's unfolding convention uses (Section 2.1).

A Tucker sum is given as `cores` (list of s tensors, core i of shape
(r_1^(i), ..., r_d^(i))) and `factors` (list of s lists of d tensors of shape
(n_k, r_k^(i))), all on the same CUDA/HIP device, all float64 or all float32.
"""
import ctypes
from ctypes import POINTER, byref, c_double, c_int32, c_int64, c_size_t, c_void_p

import torch

from . import _lib
from ._lib import KINDS, PRECISIONS, QR_POLICIES, TSK_F32, TSK_F64, TskError, check, load

__all__ = [
    "fortran", "empty_fortran", "krp_width", "kron_sizes", "sketch_widths", "sketch_omega",
    "tucker_sum_sketch", "tucker_sum_recompress", "qr_fallback_count", "Handle", "TskError",
    "Recompressor", "BatchRecompressor", "tucker_sum_recompress_batched",
    "tucker_sum_recompress_backward", "recompress", "tucker_sum_recompress_noalloc",
    "tucker_sum_project", "tucker_truncate", "round_sum", "effective_subranks", "sketch_sum",
    "round_deterministic", "effective_subranks_batched", "tucker_truncate_batched",
    "sketch_sum_batched", "carve_fortran", "autotune", "autotune_save", "autotune_load",
    "autotune_clear",
]


# ---------------------------------------------------------------- layout helpers
def is_fortran(t: torch.Tensor) -> bool:
    expect = 1
    for size, stride in zip(t.shape, t.stride()):
        if size != 1 and stride != expect:
            return False
        expect *= size
    return True


def fortran(t: torch.Tensor) -> torch.Tensor:
    """Same values, column-major memory (a copy only if needed)."""
    if is_fortran(t):
        return t
    rev = list(reversed(range(t.dim())))
    return t.permute(rev).contiguous().permute(rev)


def empty_fortran(shape, dtype, device) -> torch.Tensor:
    rev = list(reversed(range(len(shape))))
    return torch.empty(tuple(reversed(tuple(shape))), dtype=dtype, device=device).permute(rev)


def carve_fortran(shapes, dtype, device):
    """Column-major tensors of the given shapes as views of ONE allocation
    (each view 256-byte aligned): a batch's many small outputs without a
    caching-allocator call per tensor."""
    es = torch.empty((), dtype=dtype).element_size()
    align = max(1, 256 // es)
    views, total = [], 0
    for sh in shapes:
        sh = tuple(int(x) for x in sh)
        strides, n = [], 1
        for x in sh:
            strides.append(n)
            n *= x
        views.append((sh, tuple(strides), total))
        total += (n + align - 1) // align * align
    buf = torch.empty(max(total, 1), dtype=dtype, device=device)
    view = buf.as_strided
    return [view(sh, st, off) for sh, st, off in views]


def _dtype_code(dt) -> int:
    if dt == torch.float64:
        return TSK_F64
    if dt == torch.float32:
        return TSK_F32
    raise TypeError(f"unsupported dtype {dt}")


def _stream_ptr(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


# ---------------------------------------------------------------- sizes (host only)
def krp_width(ell) -> int:
    arr = (c_int32 * len(ell))(*ell)
    out = c_int32()
    check(load().tsk_krp_width(len(ell), arr, byref(out)))
    return out.value


def kron_sizes(ell) -> list:
    arr = (c_int32 * len(ell))(*ell)
    out = (c_int32 * len(ell))()
    check(load().tsk_kron_sizes(len(ell), arr, out))
    return list(out)


# ---------------------------------------------------------------- handle
class Handle:
    """One library handle per device, plus a growable workspace tensor."""

    _cache = {}

    def __init__(self, device=None):
        device = torch.device("cuda", torch.cuda.current_device() if device is None else
                              torch.device(device).index or 0)
        self.device = device
        self.ptr = c_void_p()
        check(load().tsk_create(byref(self.ptr), device.index))
        self.ws = None

    @classmethod
    def get(cls, device=None) -> "Handle":
        idx = torch.cuda.current_device() if device is None else (torch.device(device).index or 0)
        if idx not in cls._cache:
            cls._cache[idx] = Handle(torch.device("cuda", idx))
        return cls._cache[idx]

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        return self.ws

    def __del__(self):
        try:
            if self.ptr:
                load().tsk_destroy(self.ptr)
        except Exception:
            pass


def _with_workspace(h, call, size):
    """call(ws) -> status through the handle's growable workspace.  A call
    given too small a workspace is refused before anything is enqueued, so
    then size() -> bytes is queried and the call made again on a grown one
    (with some headroom): a sequence of similar calls plans each once
    instead of twice."""
    ws = h.ws if h.ws is not None else h.workspace(1 << 20)
    st = call(ws)
    if st == _WORKSPACE_TOO_SMALL:
        ws = h.workspace(int(size() * 1.25))
        st = call(ws)
    check(st, h.ptr)


_WORKSPACE_TOO_SMALL = 4


# ---------------------------------------------------------------- marshalling
def _tensor_info(t, seen):
    """(tensor, column-major tensor, dtype, device, shape, pointer) of t,
    memoised in `seen` (keyed by id; the entry keeps t alive, so ids stay
    unique while `seen` does)."""
    got = seen.get(id(t)) if seen is not None else None
    if got is None:
        f = fortran(t)
        dv = f.device
        got = (t, f, f.dtype, (dv.type, dv.index), tuple(f.shape), f.data_ptr(), dv)
        if seen is not None:
            seen[id(t)] = got
    return got


class _Marshal:
    """Keeps the ctypes arrays alive for the duration of one call.  Calls
    over many sums that share tensors pass one `seen` dict, so that each
    distinct tensor is laid out and inspected once."""

    def __init__(self, cores, factors, coeffs, kind, sizes, seed, omega, sketch_prec,
                 project_prec, qr_policy, seen=None):
        s = len(cores)
        d = len(factors[0])
        ci = [_tensor_info(g, seen) for g in cores]
        fi = [[_tensor_info(u, seen) for u in us] for us in factors]
        dt, dkey, dev = ci[0][2], ci[0][3], ci[0][6]
        for g, us in zip(ci, fi):
            if len(g[4]) != d or len(us) != d:
                raise ValueError("every core must have one dimension per factor")
            if g[2] is not dt or g[3] != dkey:
                raise ValueError("all cores and factors must share dtype and device")
            for k, u in enumerate(us):
                if u[2] is not dt or u[3] != dkey:
                    raise ValueError("all cores and factors must share dtype and device")
                if len(u[4]) != 2 or u[4][1] != g[4][k]:
                    raise ValueError(f"factor {k} shape {u[4]} does not match core")
        self.cores = [g[1] for g in ci]
        self.factors = [[u[1] for u in us] for us in fi]
        self.dims = [u[4][0] for u in fi[0]]
        for us in fi:
            if [u[4][0] for u in us] != self.dims:
                raise ValueError("all terms must share the mode sizes")
        self.d, self.s, self.dtype, self.device = d, s, dt, dev
        self.c_dims = (c_int64 * d)(*self.dims)
        self.c_ranks = (c_int32 * (s * d))(*[x for g in ci for x in g[4]])
        self.c_cores = (c_void_p * s)(*[g[5] for g in ci])
        self.c_factors = (c_void_p * (s * d))(*[u[5] for us in fi for u in us])
        self.c_coeffs = None if coeffs is None else (c_double * s)(*[float(c) for c in coeffs])
        self.sum = _lib.TuckerSum(d, s, self.c_dims, self.c_ranks, self.c_cores, self.c_factors,
                                  self.c_coeffs, _dtype_code(dt))
        self.omega = None
        self.c_omega = None
        if omega is not None:
            self.omega = [fortran(o.to(dt)) for o in omega]
            self.c_omega = (c_void_p * d)(*[o.data_ptr() for o in self.omega])
        self.set_spec(kind, sizes, seed, sketch_prec, project_prec, qr_policy)

    @classmethod
    def many(cls, sums, sketch_prec="fp64", project_prec="fp64"):
        """One marshal per sum (dicts with cores, factors and optionally
        coeffs; spec "krp", sizes [1], seed 0 until set_spec), with the same
        checks as the constructor but the ctypes arrays of all sums laid out
        flat, one array per field, each sum's TuckerSum pointing at its
        stretch: the per-sum cost of a batch is a few list operations instead
        of five ctypes arrays."""
        seen = {}
        dims_all, ranks_all, cores_all, facs_all, coefs_all, layout = [], [], [], [], [], []
        first = []

        def info(t):
            # a tensor's dtype and device are checked once, when it is first seen
            got = _tensor_info(t, seen)
            if not first:
                first.append(got)
            elif got[2] is not first[0][2] or got[3] != first[0][3]:
                raise ValueError("all cores and factors must share dtype and device")
            return got

        get = seen.get
        add_rank, add_core, add_fac = ranks_all.extend, cores_all.append, facs_all.append
        for x in sums:
            cores, factors, coeffs = x["cores"], x["factors"], x.get("coeffs")
            s, d = len(cores), len(factors[0])
            if len(factors) != s:
                raise ValueError("every term needs one core and one list of factors")
            dims = None
            for g, us in zip(cores, factors):
                gi = get(id(g)) or info(g)
                rk = gi[4]
                if len(rk) != d or len(us) != d:
                    raise ValueError("every core must have one dimension per factor")
                add_rank(rk)
                add_core(gi[5])
                col = []
                for k in range(d):
                    u = us[k]
                    ui = get(id(u)) or info(u)
                    sh = ui[4]
                    if len(sh) != 2 or sh[1] != rk[k]:
                        raise ValueError(f"factor {k} shape {sh} does not match core")
                    col.append(sh[0])
                    add_fac(ui[5])
                if dims is None:
                    dims = col
                elif col != dims:
                    raise ValueError("all terms must share the mode sizes")
            layout.append((d, s, dims, None if coeffs is None else len(coefs_all)))
            dims_all += dims
            if coeffs is not None:
                coefs_all += [float(c) for c in coeffs]
        c_dims = (c_int64 * max(len(dims_all), 1))(*dims_all)
        c_ranks = (c_int32 * max(len(ranks_all), 1))(*ranks_all)
        c_cores = (c_void_p * max(len(cores_all), 1))(*cores_all)
        c_facs = (c_void_p * max(len(facs_all), 1))(*facs_all)
        c_coefs = (c_double * max(len(coefs_all), 1))(*coefs_all)
        a_dims, a_ranks = ctypes.addressof(c_dims), ctypes.addressof(c_ranks)
        a_cores, a_facs = ctypes.addressof(c_cores), ctypes.addressof(c_facs)
        a_coefs = ctypes.addressof(c_coefs)
        P64, P32, PV, PD = POINTER(c_int64), POINTER(c_int32), POINTER(c_void_p), POINTER(c_double)
        shared = (c_dims, c_ranks, c_cores, c_facs, c_coefs, seen)
        dt, dev = (first[0][2], first[0][6]) if first else (None, None)
        code = _dtype_code(dt) if dt is not None else 0
        out, at_d, at_t, at_r = [], 0, 0, 0
        for d, s, dims, at_c in layout:
            m = cls.__new__(cls)
            m.d, m.s, m.dtype, m.device, m.dims = d, s, dt, dev, dims
            m._shared = shared
            m.omega = m.c_omega = None
            m.sum = _lib.TuckerSum(
                d, s, ctypes.cast(a_dims + 8 * at_d, P64), ctypes.cast(a_ranks + 4 * at_r, P32),
                ctypes.cast(a_cores + 8 * at_t, PV), ctypes.cast(a_facs + 8 * at_r, PV),
                None if at_c is None else ctypes.cast(a_coefs + 8 * at_c, PD), code)
            m.set_spec("krp", [1], 0, sketch_prec, project_prec)
            out.append(m)
            at_d += d
            at_t += s
            at_r += s * d
        return out

    def set_spec(self, kind, sizes, seed, sketch_prec="fp64", project_prec="fp64",
                 qr_policy="auto"):
        sizes = [int(x) for x in sizes]
        self.c_sizes = (c_int32 * len(sizes))(*sizes)
        self.spec = _lib.SketchSpec(KINDS[kind.lower()], self.c_sizes, int(seed) & (2 ** 64 - 1),
                                    self.c_omega, PRECISIONS[sketch_prec], PRECISIONS[project_prec],
                                    QR_POLICIES[qr_policy])

    def widths(self):
        sw = (c_int64 * self.d)()
        bw = (c_int64 * self.d)()
        check(load().tsk_sketch_widths(byref(self.sum), byref(self.spec), sw, bw))
        return list(sw), list(bw)


def sketch_widths(cores, factors, kind, sizes, seed=0):
    m = _Marshal(cores, factors, None, kind, sizes, seed, None, "fp64", "fp64", "auto")
    return m.widths()


def sketch_omega(seed: int, mode: int, rows: int, cols: int, dtype=torch.float64, device=None):
    """Omega_k (rows x cols, column-major) generated on the device."""
    h = Handle.get(device)
    out = empty_fortran((rows, cols), dtype, h.device)
    check(load().tsk_sketch_omega(h.ptr, int(seed) & (2 ** 64 - 1), mode, rows, cols,
                                  c_void_p(out.data_ptr()), _dtype_code(dtype),
                                  c_void_p(_stream_ptr(h.device))), h.ptr)
    return out


def _workspace(h, m):
    nbytes = c_size_t()
    check(load().tucker_sum_workspace_size(h.ptr, byref(m.sum), byref(m.spec), byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    return ws, nbytes.value


def tucker_sum_sketch(cores, factors, kind, sizes, seed, coeffs=None, omega=None,
                      sketch_prec="fp64"):
    """Y_n = X_(n) S_n for every mode n (FP64 outputs, shape (n_n, W_n))."""
    m = _Marshal(cores, factors, coeffs, kind, sizes, seed, omega, sketch_prec, "fp64", "auto")
    h = Handle.get(m.device)
    sw, _ = m.widths()
    ys = [empty_fortran((m.dims[n], sw[n]), torch.float64, m.device) for n in range(m.d)]
    c_y = (c_void_p * m.d)(*[y.data_ptr() for y in ys])
    ws, nb = _workspace(h, m)
    check(load().tucker_sum_sketch(h.ptr, byref(m.sum), byref(m.spec), c_y,
                                   c_void_p(ws.data_ptr()), ws.numel(),
                                   c_void_p(_stream_ptr(m.device))), h.ptr)
    return ys


def tucker_sum_recompress(cores, factors, kind, sizes, seed, coeffs=None, omega=None,
                          sketch_prec="fp64", project_prec="fp64", out_dtype=None,
                          qr_policy="auto", return_r=False):
    """Stages 2-3: returns (Q list, H) (and R list if return_r) with
    X ~ [[H; Q_1, ..., Q_d]]."""
    m = _Marshal(cores, factors, coeffs, kind, sizes, seed, omega, sketch_prec, project_prec,
                 qr_policy)
    h = Handle.get(m.device)
    out_dtype = m.dtype if out_dtype is None else out_dtype
    sw, bw = m.widths()
    qs = [empty_fortran((m.dims[n], bw[n]), out_dtype, m.device) for n in range(m.d)]
    hh = empty_fortran(tuple(bw), out_dtype, m.device)
    c_q = (c_void_p * m.d)(*[q.data_ptr() for q in qs])
    rs = None
    c_r = None
    if return_r:
        rs = [empty_fortran((bw[n], sw[n]), torch.float64, m.device) for n in range(m.d)]
        c_r = (c_void_p * m.d)(*[r.data_ptr() for r in rs])
    ws, nb = _workspace(h, m)
    check(load().tucker_sum_recompress(h.ptr, byref(m.sum), byref(m.spec), c_q,
                                       c_void_p(hh.data_ptr()), _dtype_code(out_dtype), c_r,
                                       c_void_p(ws.data_ptr()), ws.numel(),
                                       c_void_p(_stream_ptr(m.device))), h.ptr)
    return (qs, hh, rs) if return_r else (qs, hh)


def tucker_sum_project(cores, factors, bases, coeffs=None, project_prec="fp64", out_dtype=None):
    """Stage 3 alone: H = sum_i c_i G^(i) x_k B_k^T U_k^(i) for the given bases
    (list of d tensors of shape (n_k, w_k), float64 or float32)."""
    m = _Marshal(cores, factors, coeffs, "krp", [1], 0, None, project_prec, project_prec, "auto")
    h = Handle.get(m.device)
    bases = [fortran(b) for b in bases]
    bdt = bases[0].dtype
    if any(b.dtype != bdt or b.dim() != 2 or b.shape[0] != m.dims[k] for k, b in enumerate(bases)):
        raise ValueError("bases must be (n_k, w_k) tensors of one dtype")
    out_dtype = m.dtype if out_dtype is None else out_dtype
    widths = [int(b.shape[1]) for b in bases]
    c_w = (c_int64 * m.d)(*widths)
    c_b = (c_void_p * m.d)(*[b.data_ptr() for b in bases])
    nbytes = c_size_t()
    check(load().tucker_sum_project_workspace_size(h.ptr, byref(m.sum), c_w, _dtype_code(bdt),
                                                   PRECISIONS[project_prec], byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    hh = empty_fortran(tuple(widths), out_dtype, m.device)
    check(load().tucker_sum_project(h.ptr, byref(m.sum), c_b, c_w, _dtype_code(bdt),
                                    PRECISIONS[project_prec], c_void_p(hh.data_ptr()),
                                    _dtype_code(out_dtype), c_void_p(ws.data_ptr()), ws.numel(),
                                    c_void_p(_stream_ptr(m.device))), h.ptr)
    return hh


def tucker_truncate(Q, H, eps):
    """Stage 4: ST-HOSVD of the core H (FP64) with relative tolerance eps
    and U_n = Q_n V_n.  Returns (G, [U_1..U_d], ranks), G of shape ranks and
    U_n of shape (n_n, r_n) (views of the library's outputs)."""
    dev = H.device
    d = H.dim()
    Qf = [fortran(q.to(torch.float64)) for q in Q]
    Hf = fortran(H.to(torch.float64))
    dims = [int(q.shape[0]) for q in Qf]
    widths = [int(x) for x in Hf.shape]
    if [int(q.shape[1]) for q in Qf] != widths:
        raise ValueError("Q_k must have as many columns as H has entries along mode k")
    h = Handle.get(dev)
    c_dims = (c_int64 * d)(*dims)
    c_w = (c_int64 * d)(*widths)
    nbytes = c_size_t()
    check(load().tucker_truncate_workspace_size(h.ptr, d, c_dims, c_w, float(eps),
                                                byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    U = [empty_fortran((n, w), torch.float64, dev) for n, w in zip(dims, widths)]
    total = 1
    for w in widths:
        total *= w
    G = torch.empty(total, dtype=torch.float64, device=dev)
    ranks = (c_int32 * d)()
    check(load().tucker_truncate(h.ptr, d, c_dims, c_w, (c_void_p * d)(*[q.data_ptr() for q in Qf]),
                                 c_void_p(Hf.data_ptr()), float(eps),
                                 (c_void_p * d)(*[u.data_ptr() for u in U]),
                                 c_void_p(G.data_ptr()), ranks, c_void_p(ws.data_ptr()),
                                 ws.numel(), c_void_p(_stream_ptr(dev))), h.ptr)
    r = list(ranks)
    n = 1
    for x in r:
        n *= x
    core = G[:n].reshape(tuple(reversed(r))).permute(tuple(reversed(range(d))))
    return core, [u[:, :rk] for u, rk in zip(U, r)], r


def round_sum(cores, factors, kind, sizes, seed, eps, coeffs=None, sketch_prec="fp64",
              project_prec="fp64"):
    """Sketch-based sum with fixed sketch sizes followed by Stage 4: the
    recompression (Stages 2-3, FP64 outputs) and the ST-HOSVD truncation of
    its core with tolerance eps.  Returns (G, [U_1..U_d], ranks)."""
    qs, hh = tucker_sum_recompress(cores, factors, kind, sizes, seed, coeffs=coeffs,
                                   sketch_prec=sketch_prec, project_prec=project_prec,
                                   out_dtype=torch.float64)
    return tucker_truncate(qs, hh, eps)


def effective_subranks(cores, factors, eps, p, coeffs=None):
    """Stage 1 (phase 1 of Algorithm 3): ell_n = r_n + p_n per mode."""
    m = _Marshal(cores, factors, coeffs, "krp", [1], 0, None, "fp64", "fp64", "auto")
    h = Handle.get(m.device)
    pv = [int(x) for x in (p if hasattr(p, "__len__") else [p] * m.d)]
    nbytes = c_size_t()
    check(load().tucker_sum_subranks_workspace_size(h.ptr, byref(m.sum), byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    out = (c_int32 * m.d)()
    check(load().tucker_sum_subranks(h.ptr, byref(m.sum), float(eps), (c_int32 * m.d)(*pv), out,
                                     c_void_p(ws.data_ptr()), ws.numel(),
                                     c_void_p(_stream_ptr(m.device))), h.ptr)
    return list(out)


def sketch_sum(cores, factors, kind, eps, p, seed, coeffs=None, sketch_prec="fp64",
               project_prec="fp64"):
    """The whole sketch-based sum of Algorithm 5 (kind "krp") or 4 ("kron")
    as a sequence of the library's calls: Stage 1 sizes from eps and p, the
    sketch width (max ell for KRP, the heuristic q_k for Kronecker), Stages
    2-3, and the Stage 4 truncation with eps.  Returns (G, [U..], ranks,
    sizes)."""
    ell = effective_subranks(cores, factors, eps, p, coeffs=coeffs)
    sizes = [krp_width(ell)] if kind == "krp" else kron_sizes(ell)
    g, us, ranks = round_sum(cores, factors, kind, sizes, seed, eps, coeffs=coeffs,
                             sketch_prec=sketch_prec, project_prec=project_prec)
    return g, us, ranks, sizes


def _core_view(G, r):
    n = 1
    for x in r:
        n *= x
    return G[:n].reshape(tuple(reversed(r))).permute(tuple(reversed(range(len(r)))))


def effective_subranks_batched(sums, eps, p):
    """Stage 1 for many sums in one launch sequence (one synchronisation).
    `sums`: list of dicts with keys cores, factors and optionally coeffs; p:
    an int or a per-mode list shared by every sum.  Returns a list of ell
    lists."""
    return _subranks_batched(_Marshal.many(sums), eps, p)


def _subranks_batched(ms, eps, p):
    B = len(ms)
    h = Handle.get(ms[0].device)
    c_sums = (_lib.TuckerSum * B)(*[m.sum for m in ms])
    pv = []
    for m in ms:
        pv += [int(x) for x in (p if hasattr(p, "__len__") else [p] * m.d)]
    total = len(pv)
    out = (c_int32 * total)()
    c_p = (c_int32 * total)(*pv)
    stream = c_void_p(_stream_ptr(ms[0].device))

    def size():
        nbytes = c_size_t()
        check(load().tucker_sum_subranks_batched_workspace_size(h.ptr, B, c_sums, byref(nbytes)),
              h.ptr)
        return nbytes.value
    _with_workspace(h, lambda ws: load().tucker_sum_subranks_batched(
        h.ptr, B, c_sums, float(eps), c_p, out, c_void_p(ws.data_ptr()), ws.numel(), stream), size)
    res, at = [], 0
    for m in ms:
        res.append(list(out[at:at + m.d]))
        at += m.d
    return res


def tucker_truncate_batched(jobs, eps):
    """Stage 4 for many cores at once: `jobs` is a list of (Q list, H) pairs
    (FP64, as tucker_truncate takes them).  Returns a list of (G, [U..],
    ranks).  The outputs of all jobs share one allocation; the ctypes
    arguments are flat arrays with one entry per (job, mode)."""
    dev = jobs[0][1].device
    h = Handle.get(dev)
    Qs, Hs, ds = [], [], []
    for Q, H in jobs:
        Qs.append([fortran(q if q.dtype == torch.float64 else q.to(torch.float64)) for q in Q])
        Hs.append(fortran(H if H.dtype == torch.float64 else H.to(torch.float64)))
        ds.append(H.dim())
    tot = sum(ds)
    dims = [int(q.shape[0]) for qs in Qs for q in qs]
    widths = [int(x) for hh in Hs for x in hh.shape]
    if [int(q.shape[1]) for qs in Qs for q in qs] != widths:
        raise ValueError("Q_k must have as many columns as H has entries along mode k")
    # element offsets of every U_k (n_k x w_k) and G (prod w_k), 256-byte aligned
    offs, top, at = [], 0, 0
    for d in ds:
        o = []
        size = 1
        for k in range(d):
            o.append(top)
            top += (dims[at + k] * widths[at + k] + 31) // 32 * 32
            size *= widths[at + k]
        o.append(top)
        top += (size + 31) // 32 * 32
        offs.append(o)
        at += d
    buf = torch.empty(max(top, 1), dtype=torch.float64, device=dev)
    base = buf.data_ptr()
    c_dims = (c_int64 * tot)(*dims)
    c_w = (c_int64 * tot)(*widths)
    c_q = (c_void_p * tot)(*[q.data_ptr() for qs in Qs for q in qs])
    c_u = (c_void_p * tot)(*[base + 8 * x for o, d in zip(offs, ds) for x in o[:d]])
    c_r = (c_int32 * tot)()
    P64, PV, P32 = POINTER(c_int64), POINTER(c_void_p), POINTER(c_int32)
    a_dims, a_w = ctypes.addressof(c_dims), ctypes.addressof(c_w)
    a_q, a_u, a_r = ctypes.addressof(c_q), ctypes.addressof(c_u), ctypes.addressof(c_r)
    structs, at = [], 0
    for d, hh, o in zip(ds, Hs, offs):
        structs.append(_lib.Truncation(
            d, ctypes.cast(a_dims + 8 * at, P64), ctypes.cast(a_w + 8 * at, P64),
            ctypes.cast(a_q + 8 * at, PV), hh.data_ptr(), float(eps), ctypes.cast(a_u + 8 * at, PV),
            base + 8 * o[d], ctypes.cast(a_r + 4 * at, P32)))
        at += d
    B = len(structs)
    c_jobs = (_lib.Truncation * B)(*structs)
    nbytes = c_size_t()
    check(load().tucker_truncate_batched_workspace_size(h.ptr, B, c_jobs, byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    check(load().tucker_truncate_batched(h.ptr, B, c_jobs, c_void_p(ws.data_ptr()), ws.numel(),
                                         c_void_p(_stream_ptr(dev))), h.ptr)
    ranks = list(c_r)
    res, at = [], 0
    for d, o in zip(ds, offs):
        r = ranks[at:at + d]
        us = [buf.as_strided((dims[at + k], r[k]), (1, dims[at + k]), o[k]) for k in range(d)]
        strides, st = [], 1
        for x in r:
            strides.append(st)
            st *= x
        res.append((buf.as_strided(tuple(r), tuple(strides), o[d]), us, r))
        at += d
    del Qs, Hs  # kept alive until the call above returned
    return res


def sketch_sum_batched(sums, kind, eps, p, seed, sketch_prec="fp64", project_prec="fp64",
                       timings=None):
    """Algorithm 5 (kind "krp") or 4 ("kron") for many independent sums,
    each stage one launch sequence over all of them: Stage 1 sizes from eps
    and p, the sketch widths, Stages 2-3 (tucker_sum_recompress_batched,
    FP64 outputs) and the Stage 4 truncation with eps.  `sums`: list of dicts
    with cores, factors and optionally coeffs; `seed`: an int shared by every
    sum or a list.  Returns a list of (G, [U..], ranks, sizes).

    With `timings` (a dict, for profiling), the device is synchronised after
    every phase and the phase's wall milliseconds are added under "marshal",
    "stage1", "plan" (sketch sizes and the batched plan), "recompress"
    (Stages 2-3) and "truncate" (Stage 4)."""
    mark = _phase_clock(timings, sums[0]["cores"][0].device if sums else None)
    ms = _Marshal.many(sums, sketch_prec, project_prec)
    mark("marshal")
    ells = _subranks_batched(ms, eps, p)
    mark("stage1")
    seeds = seed if hasattr(seed, "__len__") else [seed] * len(sums)
    sizes = []
    for m, ell, sd in zip(ms, ells, seeds):
        sz = [krp_width(ell)] if kind == "krp" else kron_sizes(ell)
        sizes.append(sz)
        m.set_spec(kind, sz, sd, sketch_prec, project_prec)
    br = BatchRecompressor(None, sketch_prec, project_prec, torch.float64, _marshals=ms,
                           _shared_ws=True)
    mark("plan")
    q, h = br()
    mark("recompress")
    tr = tucker_truncate_batched(list(zip(q, h)), eps)
    mark("truncate")
    return [(g, us, r, sz) for (g, us, r), sz in zip(tr, sizes)]


def _phase_clock(timings, device):
    """A marker that adds the wall milliseconds since the previous mark to
    timings[name] after synchronising `device` (a no-op without timings)."""
    if timings is None or device is None:
        return lambda name: None
    import time
    torch.cuda.synchronize(device)
    last = [time.perf_counter()]

    def mark(name):
        torch.cuda.synchronize(device)
        now = time.perf_counter()
        timings[name] = timings.get(name, 0.0) + 1e3 * (now - last[0])
        last[0] = now
    return mark


def round_deterministic(cores, factors, tau, coeffs=None):
    """The paper's deterministic baseline (Algorithm 1 over all terms, then
    Algorithm 2 with tolerance tau) on the GPU.  Returns (G, [U..], ranks)."""
    m = _Marshal(cores, factors, coeffs, "krp", [1], 0, None, "fp64", "fp64", "auto")
    h = Handle.get(m.device)
    nbytes = c_size_t()
    check(load().tucker_sum_round_deterministic_workspace_size(h.ptr, byref(m.sum), float(tau),
                                                               byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    R = [sum(int(g.shape[k]) for g in m.cores) for k in range(m.d)]
    widths = [min(n, r) for n, r in zip(m.dims, R)]
    U = [empty_fortran((n, w), torch.float64, m.device) for n, w in zip(m.dims, widths)]
    total = 1
    for w in widths:
        total *= w
    G = torch.empty(total, dtype=torch.float64, device=m.device)
    ranks = (c_int32 * m.d)()
    check(load().tucker_sum_round_deterministic(h.ptr, byref(m.sum), float(tau),
                                                (c_void_p * m.d)(*[u.data_ptr() for u in U]),
                                                c_void_p(G.data_ptr()), ranks,
                                                c_void_p(ws.data_ptr()), ws.numel(),
                                                c_void_p(_stream_ptr(m.device))), h.ptr)
    r = list(ranks)
    n = 1
    for x in r:
        n *= x
    core = G[:n].reshape(tuple(reversed(r))).permute(tuple(reversed(range(m.d))))
    return core, [u[:, :rk] for u, rk in zip(U, r)], r


def tucker_sum_recompress_noalloc(cores, factors, kind, sizes, seed, Q_out, H_out, coeffs=None,
                                  sketch_prec="fp64", project_prec="fp64", qr_policy="auto",
                                  R_out=None):
    """tucker_sum_recompress into caller-allocated outputs (Q_out list, H_out,
    optional R_out list; column-major, shapes as tucker_sum_recompress
    returns) through the entry point that allocates nothing: intermediates
    live in the library's static per-device scratch array, so calls that
    overlap on one device race."""
    m = _Marshal(cores, factors, coeffs, kind, sizes, seed, None, sketch_prec, project_prec,
                 qr_policy)
    h = Handle.get(m.device)
    out_dtype = H_out.dtype
    for t in list(Q_out) + [H_out] + list(R_out or []):
        if not is_fortran(t):
            raise ValueError("outputs must be column-major (empty_fortran)")
    c_q = (c_void_p * m.d)(*[q.data_ptr() for q in Q_out])
    c_r = None if R_out is None else (c_void_p * m.d)(*[r.data_ptr() for r in R_out])
    check(load().tucker_sum_recompress_noalloc(h.ptr, byref(m.sum), byref(m.spec), c_q,
                                               c_void_p(H_out.data_ptr()), _dtype_code(out_dtype),
                                               c_r, c_void_p(_stream_ptr(m.device))), h.ptr)
    return Q_out, H_out


class Recompressor:
    """Pre-marshalled recompression of one fixed Tucker sum: repeated calls
    reuse the pointer tables, outputs and workspace (used by the benchmark)."""

    def __init__(self, cores, factors, kind, sizes, seed, coeffs=None, sketch_prec="fp64",
                 project_prec="fp64", out_dtype=None, qr_policy="auto"):
        self.m = _Marshal(cores, factors, coeffs, kind, sizes, seed, None, sketch_prec,
                          project_prec, qr_policy)
        m = self.m
        self.h = Handle.get(m.device)
        self.out_dtype = m.dtype if out_dtype is None else out_dtype
        sw, bw = m.widths()
        self.Q = [empty_fortran((m.dims[n], bw[n]), self.out_dtype, m.device) for n in range(m.d)]
        self.H = empty_fortran(tuple(bw), self.out_dtype, m.device)
        self.c_q = (c_void_p * m.d)(*[q.data_ptr() for q in self.Q])
        nbytes = c_size_t()
        check(load().tucker_sum_workspace_size(self.h.ptr, byref(m.sum), byref(m.spec),
                                               byref(nbytes)), self.h.ptr)
        self.ws = torch.empty(max(nbytes.value, 256), dtype=torch.uint8, device=m.device)
        self.ws_bytes = nbytes.value

    def capture(self):
        """Record one recompression into a HIP graph (replayed by replay()).
        The library enqueues only kernels and one descriptor upload, no
        memset, so the graph replays the whole step."""
        self.graph_stream = torch.cuda.Stream(self.m.device)
        self.graph = torch.cuda.CUDAGraph()
        cur = torch.cuda.current_stream(self.m.device)
        self.graph_stream.wait_stream(cur)
        with torch.cuda.graph(self.graph, stream=self.graph_stream, capture_error_mode="relaxed"):
            self(self.graph_stream.cuda_stream)
        cur.wait_stream(self.graph_stream)
        return self

    def replay(self):
        self.graph.replay()
        return self.Q, self.H

    def __call__(self, stream=None):
        st = _stream_ptr(self.m.device) if stream is None else stream
        check(load().tucker_sum_recompress(self.h.ptr, byref(self.m.sum), byref(self.m.spec),
                                           self.c_q, c_void_p(self.H.data_ptr()),
                                           _dtype_code(self.out_dtype), None,
                                           c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                           c_void_p(st)), self.h.ptr)
        return self.Q, self.H


class BatchRecompressor:
    """Many independent Tucker sums recompressed by one launch sequence
    (tucker_sum_recompress_batched): each stage of every sum runs in the same
    grouped kernel launches.  `sums` is a list of dicts with keys cores,
    factors, kind, sizes, seed and optionally coeffs; all share order, sketch
    kind and precisions."""

    def __init__(self, sums, sketch_prec="fp64", project_prec="fp64", out_dtype=None,
                 qr_policy="auto", _marshals=None, _shared_ws=False):
        if _marshals is None:
            _marshals = _Marshal.many(sums, sketch_prec, project_prec)
            for m, x in zip(_marshals, sums):
                m.set_spec(x["kind"], x["sizes"], x["seed"], sketch_prec, project_prec, qr_policy)
        self.ms = _marshals
        m0 = self.ms[0]
        self.h = Handle.get(m0.device)
        self.out_dtype = m0.dtype if out_dtype is None else out_dtype
        B = len(self.ms)
        self.c_sums = (_lib.TuckerSum * B)(*[m.sum for m in self.ms])
        self.c_specs = (_lib.SketchSpec * B)(*[m.spec for m in self.ms])
        self.Q, self.H, self._cq = [], [], []
        bws = [m.widths()[1] for m in self.ms]
        shapes = []
        for m, bw in zip(self.ms, bws):
            shapes += [(m.dims[n], bw[n]) for n in range(m.d)] + [tuple(bw)]
        bufs = carve_fortran(shapes, self.out_dtype, m0.device)
        at = 0
        for m in self.ms:
            qs = bufs[at:at + m.d]
            self.Q.append(qs)
            self.H.append(bufs[at + m.d])
            at += m.d + 1
            self._cq.append((c_void_p * m.d)(*[q.data_ptr() for q in qs]))
        self.c_q = (POINTER(c_void_p) * B)(*[ctypes.cast(a, POINTER(c_void_p)) for a in self._cq])
        self.c_h = (c_void_p * B)(*[h.data_ptr() for h in self.H])
        # a one-shot call (_shared_ws) runs in the handle's workspace and plans
        # once; otherwise the call owns a workspace, which graph capture needs
        self.ws = None if _shared_ws else torch.empty(max(self._size(), 256), dtype=torch.uint8,
                                                      device=m0.device)

    def _size(self):
        nbytes = c_size_t()
        check(load().tucker_sum_batched_workspace_size(self.h.ptr, len(self.ms), self.c_sums,
                                                       self.c_specs, byref(nbytes)), self.h.ptr)
        return nbytes.value

    def __call__(self, stream=None):
        st = _stream_ptr(self.ms[0].device) if stream is None else stream

        def call(ws):
            return load().tucker_sum_recompress_batched(
                self.h.ptr, len(self.ms), self.c_sums, self.c_specs, self.c_q, self.c_h,
                _dtype_code(self.out_dtype), c_void_p(ws.data_ptr()), ws.numel(), c_void_p(st))
        if self.ws is None:
            _with_workspace(self.h, call, self._size)
        else:
            check(call(self.ws), self.h.ptr)
        return self.Q, self.H

    def capture(self):
        if self.ws is None:
            # the handle's workspace may be reallocated by a later call
            raise RuntimeError("a recompressor on the handle's shared workspace cannot be captured")
        dev = self.ms[0].device
        self.graph_stream = torch.cuda.Stream(dev)
        self.graph = torch.cuda.CUDAGraph()
        cur = torch.cuda.current_stream(dev)
        self.graph_stream.wait_stream(cur)
        with torch.cuda.graph(self.graph, stream=self.graph_stream, capture_error_mode="relaxed"):
            self(self.graph_stream.cuda_stream)
        cur.wait_stream(self.graph_stream)
        return self

    def replay(self):
        self.graph.replay()
        return self.Q, self.H


def autotune(sums, sketch_prec="fp64", project_prec="fp64", out_dtype=None, qr_policy="auto",
             reps=5):
    """Measure the planner's launch parameters on this batch (the arguments
    of tucker_sum_recompress_batched) and keep the fastest per launch class
    in the device's handle; later plans use them.  Recompressors built
    before the call keep their workspace size: build them again."""
    br = BatchRecompressor(sums, sketch_prec, project_prec, out_dtype, qr_policy)
    check(load().tsk_autotune(br.h.ptr, len(br.ms), br.c_sums, br.c_specs, br.c_q, br.c_h,
                              _dtype_code(br.out_dtype), int(reps),
                              c_void_p(_stream_ptr(br.ms[0].device))), br.h.ptr)


def autotune_save(path, device=None):
    """Write the handle's tuning table as JSON."""
    h = Handle.get(device)
    check(load().tsk_autotune_save(h.ptr, str(path).encode()), h.ptr)


def autotune_load(path, device=None):
    """Replace the handle's tuning table with a JSON cache's (rejected if it
    was written for another GPU architecture)."""
    h = Handle.get(device)
    check(load().tsk_autotune_load(h.ptr, str(path).encode()), h.ptr)


def autotune_clear(device=None):
    h = Handle.get(device)
    check(load().tsk_autotune_clear(h.ptr), h.ptr)


def tucker_sum_recompress_batched(sums, sketch_prec="fp64", project_prec="fp64", out_dtype=None,
                                  qr_policy="auto"):
    """Recompress a list of independent sums in one launch sequence; returns
    a list of (Q list, H)."""
    br = BatchRecompressor(sums, sketch_prec, project_prec, out_dtype, qr_policy)
    q, h = br()
    return list(zip(q, h))


def tucker_sum_recompress_backward(cores, factors, kind, sizes, seed, Q, R, H_bar, Q_bar=None,
                                   coeffs=None, sketch_prec="fp64"):
    """Gradients of a loss with respect to every core and factor, given the
    forward outputs Q, R and the loss gradients H_bar (and Q_bar, or None).
    Returns (core_bar list, factor_bar list of lists) in the input dtype."""
    m = _Marshal(cores, factors, coeffs, kind, sizes, seed, None, sketch_prec, sketch_prec, "auto")
    h = Handle.get(m.device)
    out_dtype = H_bar.dtype
    Qf = [fortran(q.to(out_dtype)) for q in Q]
    Rf = [fortran(r.to(torch.float64)) for r in R]
    Hf = fortran(H_bar.to(out_dtype))
    Qbf = None if Q_bar is None else [fortran(q.to(out_dtype)) for q in Q_bar]
    core_bar = [empty_fortran(tuple(g.shape), m.dtype, m.device) for g in m.cores]
    factor_bar = [[empty_fortran(tuple(u.shape), m.dtype, m.device) for u in us] for us in m.factors]
    c_q = (c_void_p * m.d)(*[q.data_ptr() for q in Qf])
    c_r = (c_void_p * m.d)(*[r.data_ptr() for r in Rf])
    c_qb = None if Qbf is None else (c_void_p * m.d)(*[q.data_ptr() for q in Qbf])
    c_gb = (c_void_p * m.s)(*[g.data_ptr() for g in core_bar])
    c_ub = (c_void_p * (m.s * m.d))(*[u.data_ptr() for us in factor_bar for u in us])
    nbytes = c_size_t()
    check(load().tucker_sum_backward_workspace_size(h.ptr, byref(m.sum), byref(m.spec),
                                                    byref(nbytes)), h.ptr)
    ws = h.workspace(nbytes.value)
    check(load().tucker_sum_recompress_backward(
        h.ptr, byref(m.sum), byref(m.spec), c_q, c_r, c_void_p(Hf.data_ptr()), c_qb,
        _dtype_code(out_dtype), c_gb, c_ub, c_void_p(ws.data_ptr()), ws.numel(),
        c_void_p(_stream_ptr(m.device))), h.ptr)
    return core_bar, factor_bar


class _RecompressFn(torch.autograd.Function):
    """Differentiable Stages 2-3 (Khatri-Rao sketch): forward and backward are
    both the library's HIP kernels (tucker_sum_recompress with R_out, and
    tucker_sum_recompress_backward)."""

    @staticmethod
    def forward(ctx, meta, *flat):
        s, d = meta["s"], meta["d"]
        cores = list(flat[:s])
        factors = [list(flat[s + i * d: s + (i + 1) * d]) for i in range(s)]
        qs, h, rs = tucker_sum_recompress(cores, factors, meta["kind"], meta["sizes"], meta["seed"],
                                          coeffs=meta["coeffs"], sketch_prec=meta["sketch_prec"],
                                          project_prec=meta["project_prec"], return_r=True)
        ctx.meta = meta
        ctx.save_for_backward(*flat, *qs, *rs)
        return (h, *qs)

    @staticmethod
    def backward(ctx, h_bar, *q_bars):
        meta = ctx.meta
        s, d = meta["s"], meta["d"]
        saved = ctx.saved_tensors
        nin = s + s * d
        flat = saved[:nin]
        qs = list(saved[nin:nin + d])
        rs = list(saved[nin + d:nin + 2 * d])
        cores = list(flat[:s])
        factors = [list(flat[s + i * d: s + (i + 1) * d]) for i in range(s)]
        if h_bar is None:
            h_bar = torch.zeros(tuple(q.shape[1] for q in qs), dtype=qs[0].dtype, device=qs[0].device)
        if all(q is None for q in q_bars):
            q_bar = None
        else:
            q_bar = [torch.zeros_like(q) if g is None else g for q, g in zip(qs, q_bars)]
        gb, ub = tucker_sum_recompress_backward(cores, factors, meta["kind"], meta["sizes"],
                                                meta["seed"], qs, rs, h_bar, q_bar,
                                                coeffs=meta["coeffs"],
                                                sketch_prec=meta["sketch_prec"])
        # raises TskError (TSK_ERR_RANK_DEFICIENT) when some R_n was
        # numerically singular, i.e. the forward's Y_n had deficient rank
        qr_fallback_count(qs[0].device)
        return (None, *gb, *[u for us in ub for u in us])


def recompress(cores, factors, kind, sizes, seed, coeffs=None, sketch_prec="fp64",
               project_prec=None):
    """Differentiable recompression: returns (H, [Q_1..Q_d]) with gradients
    flowing to every core and factor through the hand-written adjoint."""
    meta = {"s": len(cores), "d": len(factors[0]), "kind": kind, "sizes": list(sizes),
            "seed": seed, "coeffs": None if coeffs is None else [float(c) for c in coeffs],
            "sketch_prec": sketch_prec, "project_prec": project_prec or sketch_prec}
    flat = list(cores) + [u for us in factors for u in us]
    out = _RecompressFn.apply(meta, *flat)
    return out[0], list(out[1:])


def qr_fallback_count(device=None) -> int:
    h = Handle.get(device)
    out = c_int64()
    check(load().tsk_qr_fallback_count(h.ptr, c_void_p(_stream_ptr(h.device)), byref(out)), h.ptr)
    return out.value
