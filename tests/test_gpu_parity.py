"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle
on the same seeded inputs."""
import numpy as np
import pytest

import synth
from helpers import np_of, rel, to_torch
from oracle import recompress as RC
from oracle import sketch as S
from oracle import tensor as T
from oracle.omega import omega as oracle_omega

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as m
    return m


def sizes_of(kind, ell_or_sizes):
    return list(ell_or_sizes)


def run(tsk, ts, kind, sizes, seed, **kw):
    import torch
    cores, factors = to_torch(ts, DEV, kw.pop("dtype", torch.float64))
    out = tsk.tucker_sum_recompress(cores, factors, kind, sizes, seed, coeffs=ts["coeffs"], **kw)
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("seed,mode,rows,cols", [(1, 0, 64, 5), (2 ** 40 + 3, 2, 513, 74),
                                                  (1002, 1, 512, 74), (7, 3, 1, 1), (9, 0, 3, 7)])
def test_omega_bitwise(tsk, seed, mode, rows, cols):
    import torch
    want = oracle_omega(seed, mode, rows, cols)
    got = np_of(tsk.sketch_omega(seed, mode, rows, cols, torch.float64, DEV))
    mism = int(np.sum(got != want))
    assert mism == 0, f"{mism} of {rows * cols} entries differ"
    got32 = np_of(tsk.sketch_omega(seed, mode, rows, cols, torch.float32, DEV))
    assert np.array_equal(got32, want)


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_sketch_tiny(tsk, kind):
    import torch
    ts = synth.config_tiny()
    sizes = [24] if kind == "krp" else RC.kron_sizes(ts["ell"])
    om = [oracle_omega(ts["omega_seed"], k, 64, w) for k, w in enumerate(RC.omega_widths(3, kind, sizes))]
    want = S.structured_sketch(ts, om, kind)
    cores, factors = to_torch(ts, DEV)
    ys = tsk.tucker_sum_sketch(cores, factors, kind, sizes, ts["omega_seed"], coeffs=ts["coeffs"])
    torch.cuda.synchronize()
    for y, w in zip(ys, want):
        assert y.shape == w.shape
        assert rel(np_of(y), w) < 1e-13


def full_rank(y, tol=1e-9):
    s = np.linalg.svd(y, compute_uv=False)
    return s.size > 0 and s[-1] > tol * s[0] and y.shape[0] >= y.shape[1]


def check_recompress(tsk, ts, kind, sizes, seed, qtol=1e-10, htol=1e-11, **kw):
    """Q_n and H are unique when every Y_n has full column rank (diag R >= 0);
    otherwise the trailing columns of Q_n are arbitrary and only the
    recompressed tensor [[H; Q]] (and orthonormality) can be compared."""
    ref = RC.recompress(ts, kind, sizes, seed)
    qs, h = run(tsk, ts, kind, sizes, seed, **kw)
    assert h.shape == ref["H"].shape
    for q in qs:
        qn = np_of(q)
        assert np.linalg.norm(qn.T @ qn - np.eye(qn.shape[1])) < 1e-11
    if all(full_rank(y) for y in ref["Y"]):
        for q, qr in zip(qs, ref["Q"]):
            assert q.shape == qr.shape
            assert rel(np_of(q), qr) < qtol
        assert rel(np_of(h), ref["H"]) < htol
    else:
        assert int(np.prod(ts["dims"])) <= 4_000_000, "rank-deficient check needs a dense reconstruction"
        xh_ref = RC.reconstruct(ref["H"], ref["Q"])
        xh = RC.reconstruct(np_of(h), [np_of(q) for q in qs])
        assert rel(xh, xh_ref) < htol
    return ref, qs, h


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_recompress_tiny(tsk, kind):
    ts = synth.config_tiny()
    sizes = [24] if kind == "krp" else RC.kron_sizes(ts["ell"])
    ref, qs, h = check_recompress(tsk, ts, kind, sizes, ts["omega_seed"])
    x = T.sum_to_dense(ts)
    e_gpu = T.rel_err(RC.reconstruct(np_of(h), [np_of(q) for q in qs]), x)
    e_ref = T.rel_err(RC.reconstruct(ref["H"], ref["Q"]), x)
    assert abs(e_gpu - e_ref) < 1e-12


RAGGED = [
    # (dims, ranks per term, kind, sizes): several tiles, ragged tails, uneven ranks
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]], "krp", [80]),
    ((130, 70, 90), [[70, 5, 33], [1, 66, 12], [40, 40, 40]], "kron", [3, 5, 4]),
    ((65, 33), [[17, 9], [65, 3]], "krp", [20]),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]], "krp", [11]),
    ((40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]], "kron", [2, 3, 2, 2]),
]


@pytest.mark.parametrize("case", range(len(RAGGED)))
def test_recompress_ragged(tsk, case):
    dims, ranks, kind, sizes = RAGGED[case]
    ts = synth.random_sum(100 + case, dims, ranks, orthonormal_factors=False,
                          coeffs=np.linspace(-1.5, 2.0, len(ranks)))
    ref = RC.recompress(ts, kind, sizes, 31 + case)
    import torch
    cores, factors = to_torch(ts, DEV)
    ys = tsk.tucker_sum_sketch(cores, factors, kind, sizes, 31 + case, coeffs=ts["coeffs"])
    torch.cuda.synchronize()
    for y, w in zip(ys, ref["Y"]):
        assert rel(np_of(y), w) < 1e-13
    check_recompress(tsk, ts, kind, sizes, 31 + case)


def test_linearity_on_device(tsk):
    import torch
    ts = synth.random_sum(5, (70, 50, 60), [[8, 9, 7], [5, 6, 4], [9, 3, 8]], coeffs=[1.0, -2.0, 0.5])
    cores, factors = to_torch(ts, DEV)
    whole = tsk.tucker_sum_sketch(cores, factors, "krp", [12], 5, coeffs=ts["coeffs"])
    acc = None
    for i in range(3):
        part = tsk.tucker_sum_sketch([cores[i]], [factors[i]], "krp", [12], 5, coeffs=[ts["coeffs"][i]])
        acc = part if acc is None else [a + p for a, p in zip(acc, part)]
    torch.cuda.synchronize()
    for a, b in zip(whole, acc):
        assert rel(np_of(a), np_of(b)) < 1e-13


@pytest.mark.parametrize("kind,sizes", [("krp", [12]), ("kron", [3, 3, 3, 3])])
def test_exact_recovery_rank_deficient(tsk, kind, sizes):
    """Rank-10 sum sketched with 12 (or 27) columns: Y_n is rank deficient,
    Cholesky QR breaks down and the device takes the Householder path; the
    recompression is still exact."""
    ts = synth.e1_low_rank_sum(seed=5, d=4, n=24, terms=20, r_true=10)
    before = tsk.qr_fallback_count(DEV)
    qs, h = run(tsk, ts, kind, sizes, 12)
    after = tsk.qr_fallback_count(DEV)
    assert after - before == 4
    x = T.sum_to_dense(ts)
    xh = RC.reconstruct(np_of(h), [np_of(q) for q in qs])
    assert T.rel_err(xh, x) < 1e-12
    for q in qs:
        qn = np_of(q)
        assert np.linalg.norm(qn.T @ qn - np.eye(qn.shape[1])) < 1e-12


def test_householder_policy_matches_cholqr2(tsk):
    ts = synth.random_sum(9, (96, 80, 72), [[10, 12, 9], [11, 7, 13]])
    a_q, a_h = run(tsk, ts, "krp", [16], 3)
    b_q, b_h = run(tsk, ts, "krp", [16], 3, qr_policy="householder")
    for x, y in zip(a_q, b_q):
        assert rel(np_of(x), np_of(y)) < 1e-11
    assert rel(np_of(a_h), np_of(b_h)) < 1e-11
    check_recompress(tsk, ts, "krp", [16], 3, qr_policy="householder")


@pytest.mark.parametrize("dims,ranks,m", [
    # mode 0: 700 x 40 panel, too large for LDS whole -> two-level TSQR
    # (full rank: compared with Cholesky QR2; rank-deficient: through [[H; Q]])
    ((700, 60, 50), [[20, 20, 18], [15, 14, 15], [12, 12, 12]], 40),
    ((700, 60, 50), [[12, 9, 8], [10, 11, 7], [9, 8, 10]], 40),
    # mode 0: 200 x 100 panel (W > 96 and not tall) -> panel in global memory
    ((200, 150, 120), [[40, 30, 35], [38, 36, 30], [30, 34, 33]], 100),
    # every mode <= 384 x 64 -> eight-wave register panel (384 x 56, 64 x 56,
    # 60 x 56), full rank and rank-deficient; large coefficients make the
    # column norms large, where scaling a column through a (scal - 1) multiple
    # of itself would lose digits
    ((384, 64, 60), [[30, 30, 30], [20, 20, 20], [10, 10, 10]], 56),
    ((384, 64, 60), [[12, 9, 8], [10, 11, 7], [9, 8, 10]], 56),
])
def test_householder_panel_paths(tsk, dims, ranks, m):
    """Householder with the panel in registers (eight waves), in LDS, in two
    stacked halves (TSQR) and in global memory, each against the oracle."""
    ts = synth.random_sum(13, dims, ranks, coeffs=[300.0, -150.0, 80.0])
    check_recompress(tsk, ts, "krp", [m], 5, qr_policy="householder")
    if m <= 96:
        a_q, a_h = run(tsk, ts, "krp", [m], 5)
        b_q, b_h = run(tsk, ts, "krp", [m], 5, qr_policy="householder")
        for x, y in zip(a_q, b_q):
            assert rel(np_of(x), np_of(y)) < 1e-11
        assert rel(np_of(a_h), np_of(b_h)) < 1e-11


def test_zero_sum(tsk):
    ts = synth.random_sum(10, (40, 30, 20), [[3, 4, 5], [2, 2, 2]], coeffs=[0.0, 0.0])
    qs, h = run(tsk, ts, "krp", [6], 1)
    assert np.all(np_of(h) == 0)
    for q in qs:
        qn = np_of(q)
        assert np.linalg.norm(qn.T @ qn - np.eye(qn.shape[1])) < 1e-12


def test_oversketch_width(tsk):
    """m > n_k: economy QR keeps min(n_k, m) columns of that mode."""
    ts = synth.random_sum(11, (9, 40, 30), [[3, 4, 5], [4, 3, 2]])
    qs, h = run(tsk, ts, "krp", [14], 2)
    assert [q.shape[1] for q in qs] == [9, 14, 14]
    assert tuple(h.shape) == (9, 14, 14)
    x = T.sum_to_dense(ts)
    ref = RC.recompress(ts, "krp", [14], 2)
    xh = RC.reconstruct(np_of(h), [np_of(q) for q in qs])
    assert T.rel_err(xh, RC.reconstruct(ref["H"], ref["Q"])) < 1e-12


def test_r_factor(tsk):
    ts = synth.random_sum(12, (50, 60, 70), [[5, 6, 7], [7, 6, 5]])
    qs, h, rs = run(tsk, ts, "krp", [10], 4, return_r=True)
    ref = RC.recompress(ts, "krp", [10], 4)
    for r, rr in zip(rs, ref["R"]):
        assert rel(np_of(r), rr) < 1e-11


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_structured_workload_fp64(tsk, kind):
    """d=3, 512^3, 16 terms, ranks in [16, 48], decaying cores: KRP m = 74,
    Kron q = 9 (S = 81)."""
    ts = synth.config_structured()
    sizes = [74] if kind == "krp" else RC.kron_sizes(ts["ell"])
    check_recompress(tsk, ts, kind, sizes, ts["omega_seed"])


@pytest.mark.slow
def test_precision_workload_fp64(tsk):
    """d=4, 256^4, 8 terms, cores 32^4, KRP m = 56, all FP64."""
    ts = synth.config_precision()
    check_recompress(tsk, ts, "krp", [56], ts["omega_seed"])


def test_cholqr2_policy_reports_rank_deficiency(tsk):
    """qr_policy 'cholqr2': a breakdown is reported by the next
    qr_fallback_count call as TSK_ERR_RANK_DEFICIENT; the outputs are the
    Householder result and the recompression is still exact."""
    ts = synth.e1_low_rank_sum(seed=9, d=3, n=40, terms=12, r_true=6)
    try:
        tsk.qr_fallback_count(DEV)
    except tsk.TskError:
        pass
    qs, h = run(tsk, ts, "krp", [9], 3, qr_policy="cholqr2")
    with pytest.raises(tsk.TskError) as ei:
        tsk.qr_fallback_count(DEV)
    assert ei.value.name == "TSK_ERR_RANK_DEFICIENT"
    tsk.qr_fallback_count(DEV)  # cleared after one report
    x = T.sum_to_dense(ts)
    assert T.rel_err(RC.reconstruct(np_of(h), [np_of(q) for q in qs]), x) < 1e-12


def test_breakdown_flags_do_not_outlive_a_call(tsk):
    """The per-mode Cholesky breakdown flags live in the workspace and are
    set by the first Cholesky pass of every call.  On one workspace, a call
    on a rank-deficient sum (every mode falls back to Householder) followed
    by a call on a full-rank sum of the same shapes: the second call takes no
    fallback and matches a call on a fresh workspace bit for bit."""
    import torch
    low = synth.e1_low_rank_sum(seed=9, d=3, n=40, terms=12, r_true=6)
    full = synth.random_sum(11, (40,) * 3, np.ones((12, 3), dtype=np.int64))
    cores, factors = to_torch(low, DEV)
    rc = tsk.Recompressor(cores, factors, "krp", [9], 3, coeffs=low["coeffs"])
    c0 = tsk.qr_fallback_count(DEV)
    qs, h = rc()
    torch.cuda.synchronize()
    c1 = tsk.qr_fallback_count(DEV)
    assert c1 > c0  # total rank 6 < sketch width 9: the modes break down
    x = T.sum_to_dense(low)
    assert T.rel_err(RC.reconstruct(np_of(h), [np_of(q) for q in qs]), x) < 1e-12
    fc, ff = to_torch(full, DEV)
    with torch.no_grad():
        for a, b in zip(cores, fc):
            a.copy_(b)
        for fa, fb in zip(factors, ff):
            for a, b in zip(fa, fb):
                a.copy_(b)
    qs, h = rc()
    torch.cuda.synchronize()
    assert tsk.qr_fallback_count(DEV) == c1
    q_ref, h_ref = run(tsk, full, "krp", [9], 3)
    assert torch.equal(h, h_ref)
    for q, qr in zip(qs, q_ref):
        assert torch.equal(q, qr)
