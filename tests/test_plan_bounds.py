"""Host-only bounds check of every planned launch: each address a kernel
descriptor can reach must lie in the workspace or in a caller buffer of the
right size.  Runs the library's planner on the CPU (no GPU), for every
workload shape the GPU tests and the benchmark use."""
import ctypes

import numpy as np
import pytest

import synth
from oracle.recompress import kron_sizes

PRECS = ["fp64", "fp32", "bf16x1", "bf16x3", "bf16x6"]


def selfcheck(dims, ranks, kind, sizes, sketch_prec="fp64", project_prec="fp64", in_f64=True,
              out_f64=True, sketch_only=False, with_r=False, with_omega=False):
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(_lib.SketchSpec), ctypes.c_int,
                   ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    c_sizes = (ctypes.c_int32 * len(sizes))(*sizes)
    c_om = (ctypes.c_void_p * d)(*([0x1000] * d)) if with_omega else None
    tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
    spec = _lib.SketchSpec(_lib.KINDS[kind], c_sizes, 5, c_om, _lib.PRECISIONS[sketch_prec],
                           _lib.PRECISIONS[project_prec], 0)
    msg = ctypes.create_string_buffer(512)
    rc = fn(ctypes.byref(tsum), ctypes.byref(spec), 0 if out_f64 else 1, int(sketch_only),
            int(with_r), msg, 512)
    return rc, msg.value.decode()


CASES = [
    ((64, 64, 64), np.full((4, 3), 8), "kron", [5, 5, 5]),
    ((64, 64, 64), np.full((4, 3), 8), "krp", [24]),
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]], "krp", [80]),
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]], "kron", [3, 5, 4]),
    ((65, 33), [[17, 9], [65, 3]], "krp", [20]),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]], "krp", [11]),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]], "kron", [2, 3, 2, 2]),
    ((9, 40, 30), [[3, 4, 5], [4, 3, 2]], "krp", [14]),
    ((24,) * 4, np.ones((20, 4), dtype=int), "krp", [12]),
    ((24,) * 4, np.ones((20, 4), dtype=int), "kron", [3, 3, 3, 3]),
    ((1, 1, 1), [[1, 1, 1]], "krp", [1]),
    ((5, 300, 7), [[5, 200, 7]], "krp", [100]),       # wide Y: Householder-only mode
    ((256,) * 4, np.full((8, 4), 32), "krp", [56]),
    ((256,) * 3, np.full((6, 3), 24), "krp", [40]),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_plan_in_bounds(case):
    dims, ranks, kind, sizes = CASES[case]
    for sp, pp in [("fp64", "fp64"), ("fp32", "fp32"), ("bf16x6", "bf16x3"), ("bf16x1", "fp64")]:
        for in_f64 in (True, False):
            for out_f64 in (True, False):
                for sketch_only in (False, True):
                    rc, msg = selfcheck(dims, ranks, kind, sizes, sp, pp, in_f64, out_f64,
                                        sketch_only, with_r=not sketch_only, with_omega=sketch_only)
                    assert rc == 0, (sp, pp, in_f64, out_f64, sketch_only, msg)


def test_plan_in_bounds_structured_workload():
    ts = synth.config_structured()
    for kind, sizes in (("krp", [74]), ("kron", kron_sizes(ts["ell"]))):
        for sp in PRECS:
            rc, msg = selfcheck(ts["dims"], ts["ranks"], kind, sizes, sp, sp, sp == "fp64", True)
            assert rc == 0, (kind, sp, msg)


def test_plan_in_bounds_batch_shapes():
    for one in synth.config_batch(count=24):
        rc, msg = selfcheck(one["dims"], one["ranks"], "krp", [one["ell"][0]], "fp32", "fp32", False, False)
        assert rc == 0, msg


def test_selfcheck_detects_invalid_problem():
    rc, msg = selfcheck((10, 10), [[0, 2]], "krp", [3])
    assert rc == 1 and "ranks" in msg


@pytest.mark.parametrize("n,prec,ok", [(4_000_000, "fp64", True), (5_000_000, "fp64", False),
                                       (4_000_000, "fp32", True), (5_000_000, "fp32", False)])
def test_long_modes_beyond_31_bit_tile_offsets_are_rejected(n, prec, ok):
    """The contraction kernels reach a 64-row panel through 32-bit byte
    offsets from its origin, and offsets of 2^31 and up read as zero.  The
    Gram product of the QR reads the FP64 Y_n with stride n across a tile
    (in every precision form), so a mode of 5M rows must be refused as
    unsupported instead of silently computing with zeros.  (Rank 4 at width
    4, so that the mode's QR is planned as Cholesky QR.)"""
    rc, msg = selfcheck((n, 6), [[4, 4]], "krp", [4], prec, prec, prec == "fp64", prec == "fp64")
    if ok:
        assert rc == 0, msg
    else:
        assert rc == 2 and "2^31" in msg, (rc, msg)


def test_khatri_rao_core_beyond_31_bit_offsets_is_rejected():
    rc, msg = selfcheck((20, 20), [[2 ** 14, 2 ** 14]], "krp", [4])
    assert rc == 2 and "2^31" in msg, (rc, msg)
    rc, msg = selfcheck((20, 20), [[2 ** 14, 2 ** 14]], "krp", [4], "fp32", "fp32", False, False)
    assert rc == 0, msg


def selfcheck_batched(sums, kind_sizes, prec="fp32", in_f64=False, out_f64=False):
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_batched
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(_lib.SketchSpec),
                   ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    keep = []
    ts = (_lib.TuckerSum * len(sums))()
    sp = (_lib.SketchSpec * len(sums))()
    for b, (one, (kind, sizes)) in enumerate(zip(sums, kind_sizes)):
        ranks = np.asarray(one["ranks"])
        s, d = ranks.shape
        c_dims = (ctypes.c_int64 * d)(*one["dims"])
        c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
        c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
        c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
        c_sizes = (ctypes.c_int32 * len(sizes))(*sizes)
        keep += [c_dims, c_ranks, c_cores, c_fac, c_sizes]
        ts[b] = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
        sp[b] = _lib.SketchSpec(_lib.KINDS[kind], c_sizes, 1004 + b, None, _lib.PRECISIONS[prec],
                                _lib.PRECISIONS[prec], 0)
    msg = ctypes.create_string_buffer(512)
    rc = fn(len(sums), ts, sp, 0 if out_f64 else 1, msg, 512)
    return rc, msg.value.decode()


@pytest.mark.parametrize("prec,in_f64,out_f64", [("fp32", False, False), ("fp64", True, True),
                                                 ("bf16x6", False, True)])
def test_batched_plan_in_bounds(prec, in_f64, out_f64):
    sums = synth.config_batch(count=40)
    rc, msg = selfcheck_batched(sums, [("krp", [one["ell"][0]]) for one in sums], prec, in_f64, out_f64)
    assert rc == 0, msg


def test_batched_plan_kron_mixed_shapes():
    sums = [synth.random_sum(i, (30 + i, 20, 25), [[3, 4, 5], [2, 2, 2]]) for i in range(5)]
    rc, msg = selfcheck_batched(sums, [("kron", [2, 3, 2])] * 5, "fp64", True, True)
    assert rc == 0, msg


def selfcheck_backward(dims, ranks, m, prec="fp32", in_f64=False, out_f64=False, with_qbar=True):
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_backward
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(_lib.SketchSpec), ctypes.c_int,
                   ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    c_sizes = (ctypes.c_int32 * 1)(m)
    tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
    spec = _lib.SketchSpec(0, c_sizes, 5, None, _lib.PRECISIONS[prec], _lib.PRECISIONS[prec], 0)
    msg = ctypes.create_string_buffer(512)
    rc = fn(ctypes.byref(tsum), ctypes.byref(spec), 0 if out_f64 else 1, int(with_qbar), msg, 512)
    return rc, msg.value.decode()


@pytest.mark.parametrize("dims,ranks,m", [((256,) * 3, np.full((6, 3), 24), 40),
                                          ((12, 10, 9), [[3, 2, 4], [2, 3, 2], [4, 4, 3]], 6),
                                          ((8, 7, 6, 7), [[3, 3, 3, 3], [2, 3, 2, 3]], 5),
                                          ((70, 65, 80), [[33, 5, 70], [2, 40, 9]], 64)])
def test_backward_plan_in_bounds(dims, ranks, m):
    for prec, in_f64, out_f64 in (("fp64", True, True), ("fp32", False, False), ("fp32", True, False),
                                  ("bf16x6", False, True)):
        for qb in (True, False):
            rc, msg = selfcheck_backward(dims, ranks, m, prec, in_f64, out_f64, qb)
            assert rc == 0, (prec, in_f64, out_f64, qb, msg)


def test_backward_rejects_kron_and_oversketch():
    rc, msg = selfcheck_backward((10, 40, 40), [[3, 3, 3]], 12)
    assert rc == 2 and "sketch width" in msg


def selfcheck_project(dims, ranks, widths, basis_f64, prec, in_f64, out_f64):
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_project
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(ctypes.c_int64), ctypes.c_int,
                   ctypes.c_int, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
    c_w = (ctypes.c_int64 * d)(*widths)
    msg = ctypes.create_string_buffer(512)
    rc = fn(ctypes.byref(tsum), c_w, 0 if basis_f64 else 1, _lib.PRECISIONS[prec],
            0 if out_f64 else 1, msg, 512)
    return rc, msg.value.decode()


@pytest.mark.parametrize("case", range(len(CASES)))
def test_project_plan_in_bounds(case):
    """Stage 3 alone on the same shapes, with basis widths both the sketch's
    and ragged ones (wider than the mode, narrower, a single column)."""
    dims, ranks, kind, sizes = CASES[case]
    d = len(dims)
    w_sketch = [min(n, sizes[0]) for n in dims] if kind == "krp" else \
        [min(n, int(np.prod([sizes[k] for k in range(d) if k != i]))) for i, n in enumerate(dims)]
    for widths in (w_sketch, [1] * d, [n + 3 for n in dims]):
        for prec in ("fp64", "fp32", "bf16x6"):
            for basis_f64 in (True, False):
                for in_f64 in (True, False):
                    rc, msg = selfcheck_project(dims, ranks, widths, basis_f64, prec, in_f64,
                                                not in_f64)
                    if rc == 2 and widths[0] > dims[0]:
                        # refused, not misplanned: the wide intermediates'
                        # strides pass the kernels' 31-bit tile offsets
                        assert "2^31" in msg
                        continue
                    assert rc == 0, (widths, prec, basis_f64, in_f64, msg)


@pytest.mark.parametrize("dims,widths,ranks", [
    ((64, 64, 64), (25, 25, 25), (25, 25, 25)),
    ((64, 64, 64), (25, 25, 25), (1, 1, 1)),
    ((512, 512, 512), (74, 74, 74), (30, 74, 2)),
    ((512, 512, 512), (81, 81, 81), (81, 40, 81)),
    ((256,) * 4, (56,) * 4, (20, 56, 3, 56)),
    ((40, 30), (11, 11), (5, 11)),
    ((9, 96, 96, 5, 7), (9, 96, 33, 5, 7), (9, 50, 1, 5, 2)),
    ((200, 150, 120), (200, 120, 97), (30, 120, 5)),  # widths past the LDS eigensolver
])
def test_truncate_plan_in_bounds(dims, widths, ranks):
    """Every launch of every mode of the Stage-4 truncation, planned with
    the ranks the device could report, stays inside the workspace and the
    caller's buffers."""
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_truncate
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                   ctypes.POINTER(ctypes.c_int32), ctypes.c_char_p, ctypes.c_size_t]
    d = len(dims)
    msg = ctypes.create_string_buffer(512)
    rc = fn(d, (ctypes.c_int64 * d)(*dims), (ctypes.c_int64 * d)(*widths),
            (ctypes.c_int32 * d)(*ranks), msg, 512)
    assert rc == 0, msg.value.decode()


@pytest.mark.parametrize("dims,ranks", [
    ((64, 64, 64), np.full((4, 3), 8)),
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]]),
    ((512, 512, 512), None),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]]),
])
def test_subranks_plan_in_bounds(dims, ranks):
    from paper_2603_13532_amd import _lib
    if ranks is None:
        ranks = synth.config_structured()["ranks"]
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_subranks
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(_lib.TuckerSum), ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    for in_f64 in (True, False):
        tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
        msg = ctypes.create_string_buffer(512)
        rc = fn(ctypes.byref(tsum), msg, 512)
        assert rc == 0, msg.value.decode()


@pytest.mark.parametrize("dims,ranks", [
    ((64, 64, 64), np.full((4, 3), 8)),                       # tall factors, CholQR2
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]]),  # wide mode 1 (R > n)
    ((24,) * 4, np.ones((20, 4), dtype=int)),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]]),
    ((200, 200, 200), np.full((60, 3), 17)),                   # section 5.1.2 shape, R = 1020
])
def test_deterministic_plan_in_bounds(dims, ranks):
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_deterministic
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(_lib.TuckerSum), ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    for in_f64 in (True, False):
        tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0 if in_f64 else 1)
        msg = ctypes.create_string_buffer(512)
        rc = fn(ctypes.byref(tsum), msg, 512)
        assert rc == 0, msg.value.decode()


def test_truncate_batched_plan_in_bounds():
    """The batched Stage-4 truncation over jobs of different widths (some
    past the LDS eigensolver) and device ranks stays in bounds, including
    the grouped eigensolver launches."""
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_truncate_batched
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                   ctypes.c_char_p, ctypes.c_size_t]
    rng = np.random.default_rng(3)
    for batch in (1, 2, 64):
        dims, widths, ranks = [], [], []
        for j in range(batch):
            n = [int(x) for x in rng.integers(20, 200, 3)]
            w = [int(min(x, rng.integers(1, 130))) for x in n]
            r = [int(rng.integers(1, x + 1)) for x in w]
            dims += n
            widths += w
            ranks += r
        msg = ctypes.create_string_buffer(512)
        rc = fn(batch, 3, (ctypes.c_int64 * len(dims))(*dims),
                (ctypes.c_int64 * len(widths))(*widths), (ctypes.c_int32 * len(ranks))(*ranks),
                msg, 512)
        assert rc == 0, (batch, msg.value.decode())


def test_subranks_batched_plan_in_bounds():
    """Batched Stage 1 over sums of different shapes (one with a mode above
    the LDS eigensolver's width) and both input dtypes."""
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_selfcheck_subranks_batched
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.POINTER(_lib.TuckerSum), ctypes.c_char_p,
                   ctypes.c_size_t]
    shapes = [((64, 64, 64), np.full((4, 3), 8)),
              ((130, 70, 90), np.array([[70, 5, 33], [1, 66, 12], [40, 40, 40]])),
              ((100, 100, 100), np.full((9, 3), 6)),
              ((40, 30, 20, 25), np.array([[6, 5, 4, 7], [3, 8, 2, 5]]))]
    keep = []
    for in_f64 in (True, False):
        sums = []
        for dims, ranks in shapes:
            s, d = ranks.shape
            arrs = ((ctypes.c_int64 * d)(*dims),
                    (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()]),
                    (ctypes.c_void_p * s)(*([0x1000] * s)),
                    (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d))))
            keep.append(arrs)
            sums.append(_lib.TuckerSum(d, s, arrs[0], arrs[1], arrs[2], arrs[3], None,
                                       0 if in_f64 else 1))
        c_sums = (_lib.TuckerSum * len(sums))(*sums)
        msg = ctypes.create_string_buffer(512)
        rc = fn(len(sums), c_sums, msg, 512)
        assert rc == 0, msg.value.decode()


def describe(dims, ranks, kind, sizes):
    """The planner's launch list of one sum (tsk_plan_describe), one kernel
    name per launch."""
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_describe
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(_lib.SketchSpec),
                   ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    ranks = np.asarray(ranks)
    s, d = ranks.shape
    c_dims = (ctypes.c_int64 * d)(*dims)
    c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
    c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
    c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
    c_sizes = (ctypes.c_int32 * len(sizes))(*sizes)
    tsum = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 0)
    spec = _lib.SketchSpec(_lib.KINDS[kind], c_sizes, 5, None, _lib.PRECISIONS["fp64"],
                           _lib.PRECISIONS["fp64"], 0)
    msg = ctypes.create_string_buffer(1 << 14)
    rc = fn(1, ctypes.byref(tsum), ctypes.byref(spec), 0, msg, 1 << 14)
    assert rc == 0, msg.value.decode()
    lines = msg.value.decode().splitlines()[:-1]
    return [ln.split()[0] for ln in lines], lines


def test_rank_deficient_mode_skips_cholesky_and_overlaps_it():
    """A mode whose total rank (sum over terms of r_n) is below its sketch
    width has a rank-deficient Y_n, so its Gram is singular and Cholesky QR
    would break down: the plan sends it to Householder directly, in a launch
    forked onto the second stream before the other modes' Cholesky passes
    and joined before the projection."""
    # mode 0: total rank 6 < 10 (deficient); modes 1, 2: 30 >= 10
    names, lines = describe((200, 100, 100), [[3, 15, 15], [3, 15, 15]], "krp", [10])
    assert names.count("fork") == 1 and names.count("join") == 1
    f, j = names.index("fork"), names.index("join")
    assert names[f + 1] == "householder_kernel"
    assert int(lines[f + 1].split("blocks=")[1].split()[0]) == 1  # the one deficient mode
    chol = [i for i, n in enumerate(names) if n == "chol_kernel"]
    assert len(chol) == 2 and all(f + 1 < i < j for i in chol)
    # the breakdown launch for the Cholesky modes comes after both passes
    hh = [i for i, n in enumerate(names) if n == "householder_kernel"]
    assert len(hh) == 2 and chol[-1] < hh[1] < j
    assert int(lines[hh[1]].split("blocks=")[1].split()[0]) == 2
    assert all(i > j for i, n in enumerate(names) if n.startswith("gemm_kernel")
               and ("proj_w" in lines[i] or "proj_final" in lines[i]))
    # full rank in every mode: no fork, one Householder launch after the passes
    names, _ = describe((200, 100, 100), [[6, 15, 15], [6, 15, 15]], "krp", [10])
    assert "fork" not in names and "join" not in names
    assert names.count("householder_kernel") == 1
    assert names.index("householder_kernel") > max(i for i, n in enumerate(names)
                                                   if n == "chol_kernel")


def describe_batched(sums, m_of, prec="fp64", project="fp32"):
    """tsk_plan_describe of a KRP batch (FP32-stored inputs): one line per launch."""
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_plan_describe
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_int32, ctypes.POINTER(_lib.TuckerSum), ctypes.POINTER(_lib.SketchSpec),
                   ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t]
    keep = []
    ts = (_lib.TuckerSum * len(sums))()
    sp = (_lib.SketchSpec * len(sums))()
    for b, one in enumerate(sums):
        ranks = np.asarray(one["ranks"])
        s, d = ranks.shape
        c_dims = (ctypes.c_int64 * d)(*one["dims"])
        c_ranks = (ctypes.c_int32 * (s * d))(*[int(x) for x in ranks.ravel()])
        c_cores = (ctypes.c_void_p * s)(*([0x1000] * s))
        c_fac = (ctypes.c_void_p * (s * d))(*([0x1000] * (s * d)))
        c_sizes = (ctypes.c_int32 * 1)(m_of(one))
        keep += [c_dims, c_ranks, c_cores, c_fac, c_sizes]
        ts[b] = _lib.TuckerSum(d, s, c_dims, c_ranks, c_cores, c_fac, None, 1)
        sp[b] = _lib.SketchSpec(_lib.KINDS["krp"], c_sizes, 7 + b, None, _lib.PRECISIONS[prec],
                                _lib.PRECISIONS[project], 0)
    msg = ctypes.create_string_buffer(1 << 16)
    rc = fn(len(sums), ts, sp, 1, msg, 1 << 16)
    assert rc == 0, msg.value.decode()
    return msg.value.decode().splitlines()[:-1]


def test_one_tile_batch_elements_are_grouped_per_workgroup():
    """The projection's mode-2 TTM is one 64 x 64 tile per trailing index
    (r_3 of each term).  With 8192 or more such elements in a launch, each
    workgroup takes bpw = min(8, elements // 8192) consecutive ones; fewer,
    and every element keeps its own workgroup.  Every output width here is
    at most 56, so every element is a single tile."""
    def blocks(line):
        return int(line.split("blocks=")[1].split()[0])
    big = synth.config_batch(count=256)
    ttm = [ln for ln in describe_batched(big, lambda one: one["ell"][0]) if "proj_ttm" in ln]
    assert len(ttm) == 2
    r3 = [int(r[2]) for one in big for r in np.asarray(one["ranks"])]
    bpw = min(8, sum(r3) // 8192)
    assert bpw >= 2
    assert blocks(ttm[1]) == sum(-(-x // bpw) for x in r3)
    small = big[:16]
    ttm = [ln for ln in describe_batched(small, lambda one: one["ell"][0]) if "proj_ttm" in ln]
    r3 = [int(r[2]) for one in small for r in np.asarray(one["ranks"])]
    assert sum(r3) < 8192 and blocks(ttm[1]) == sum(r3)
