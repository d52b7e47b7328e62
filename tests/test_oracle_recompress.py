"""Pins for the oracle's recompression (Stages 2-3 of Algorithms 4/5) and
sketch sizes (Section 3.2)."""
import numpy as np
import pytest

import synth
from oracle import recompress as RC
from oracle import tensor as T
from oracle import sketch as S
from oracle.deterministic import tucker_axby_all, tucker_rounding


def test_kron_sizes_golden(golden):
    for row in golden("kron_sketch_sizes.txt"):
        d = int(row[0])
        ell = [int(x) for x in row[1:1 + d]]
        want = [int(x) for x in row[1 + d:1 + 2 * d]]
        q = RC.kron_sizes(ell)
        assert q == want, (ell, q)
        for n in range(d):
            assert int(np.prod([q[j] for j in range(d) if j != n])) >= ell[n]


def test_krp_width_is_max():
    assert RC.krp_width([3, 9, 4]) == 9


def gram_schmidt(y):
    """Classical Gram-Schmidt with reorthogonalisation, column by column."""
    n, m = y.shape
    q = np.zeros((n, m))
    r = np.zeros((m, m))
    for j in range(m):
        v = y[:, j].copy()
        for _ in range(2):
            for i in range(j):
                c = float(q[:, i] @ v)
                r[i, j] += c
                v -= c * q[:, i]
        r[j, j] = float(np.sqrt(v @ v))
        q[:, j] = v / r[j, j]
    return q, r


def test_thin_qr_textbook_properties():
    y = np.random.default_rng(0).standard_normal((40, 9))
    q, r = RC.thin_qr(y)
    assert np.linalg.norm(q.T @ q - np.eye(9)) < 1e-14
    assert np.linalg.norm(q @ r - y) / np.linalg.norm(y) < 1e-14
    assert np.all(np.diag(r) >= 0)
    assert np.allclose(np.tril(r, -1), 0)
    qg, rg = gram_schmidt(y)
    assert np.allclose(q, qg, rtol=1e-12, atol=1e-12)
    assert np.allclose(r, rg, rtol=1e-12, atol=1e-12)


def test_thin_qr_oversketch_width():
    y = np.random.default_rng(1).standard_normal((6, 10))
    q, r = RC.thin_qr(y)
    assert q.shape == (6, 6) and r.shape == (6, 10)
    assert RC.basis_widths((6, 50), "krp", (10,)) == [6, 10]


def tiny_sum(seed):
    return synth.random_sum(seed, (9, 8, 7), [[2, 3, 2], [3, 2, 2], [2, 2, 3]], orthonormal_factors=False,
                            coeffs=[1.0, -0.7, 1.3])


@pytest.mark.parametrize("kind,sizes", [("krp", (4,)), ("kron", (2, 2, 3))])
def test_projection_is_orthogonal_projection(kind, sizes):
    ts = tiny_sum(3)
    out = RC.recompress(ts, kind, sizes, seed=77)
    x = T.sum_to_dense(ts)
    proj = x
    for k, q in enumerate(out["Q"]):
        proj = T.ttm(proj, q @ q.T, k)
    assert T.rel_err(RC.reconstruct(out["H"], out["Q"]), proj) < 1e-13
    dense = RC.recompress(ts, kind, sizes, seed=77, structured=False)
    assert T.rel_err(out["H"], dense["H"]) < 1e-12
    for a, b in zip(out["Y"], dense["Y"]):
        assert T.rel_err(a, b) < 1e-12


def test_projection_linearity():
    ts = tiny_sum(4)
    out = RC.recompress(ts, "krp", (5,), seed=3)
    acc = 0
    for i in range(3):
        one = dict(ts, cores=[ts["cores"][i]], factors=[ts["factors"][i]], coeffs=ts["coeffs"][i:i + 1])
        acc = acc + RC.project_structured(one, out["Q"])
    assert T.rel_err(out["H"], acc) < 1e-13


def test_error_bound_sum_of_mode_residuals():
    """||X - X_hat||^2 <= sum_k ||(I - Q_k Q_k^T) X_(k)||^2 for orthogonal
    projections onto each mode."""
    ts = synth.config_tiny()
    q = RC.kron_sizes(ts["ell"])
    out = RC.recompress(ts, "kron", q, ts["omega_seed"])
    x = T.sum_to_dense(ts)
    lhs = np.sum((x - RC.reconstruct(out["H"], out["Q"])) ** 2)
    rhs = 0.0
    for k, qk in enumerate(out["Q"]):
        xk = T.unfold(x, k)
        rhs += np.sum((xk - qk @ (qk.T @ xk)) ** 2)
    assert lhs <= rhs * (1 + 1e-12)
    assert lhs > 0


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_exact_recovery_tiny_config_three_terms(kind):
    """Tiny workload with s = 3: the sum has multilinear rank <= 24 and the
    sketch keeps 25 columns (Kron q = 5) or m = 25 (KRP), so recovery is exact."""
    ts = synth.config_tiny()
    ts = dict(ts, cores=ts["cores"][:3], factors=ts["factors"][:3], coeffs=ts["coeffs"][:3],
              ranks=ts["ranks"][:3])
    sizes = (5, 5, 5) if kind == "kron" else (25,)
    out = RC.recompress(ts, kind, sizes, seed=11)
    x = T.sum_to_dense(ts)
    assert T.rel_err(RC.reconstruct(out["H"], out["Q"]), x) < 1e-12


@pytest.mark.parametrize("kind,sizes", [("krp", (12,)), ("kron", (3, 3, 3, 3))])
def test_exact_recovery_low_rank_construction(kind, sizes):
    """Rank-1 terms in a shared rank-10 subspace (Section 5.1.1 construction,
    at small scale): sketch width >= 10 recovers the sum exactly, and the
    result agrees with deterministic sum-and-round (Algorithms 1+2)."""
    ts = synth.e1_low_rank_sum(seed=5, d=4, n=24, terms=20, r_true=10)
    out = RC.recompress(ts, kind, sizes, seed=12)
    x = T.sum_to_dense(ts)
    xh = RC.reconstruct(out["H"], out["Q"])
    assert T.rel_err(xh, x) < 1e-12
    core, facs = tucker_axby_all(ts)
    g, us = tucker_rounding(core, facs, 1e-6)
    xdet = T.tucker_to_dense(g, us)
    assert T.rel_err(xdet, x) < 1e-12
    printed = {r[0]: float(r[1]) for r in __import__("conftest").read_golden("paper_error_levels.txt")}
    # same order as the paper's FP64 level for this construction
    assert T.rel_err(xh, xdet) < 100 * printed["e1"]


def test_cancelling_sum_recovers_target_fp64():
    """Section 5.1.2 construction (n = 200, 60 summands, each the target / 60
    plus or minus a rank-12 noise tensor with diagonal core up to 1e6): the
    sketched sum with m = 7 recovers the rank-5 target in FP64, signal
    components down to 1e-6 included.  Eager rounding loses them (the paper
    prints a relative error of 6.72 for it).

    Bound: partial sums of Y_n and H reach about 1e6 times the target, so FP64
    accumulation leaves about u * 1e6 * sqrt(summands) ~ 1e-9 relative per
    entry; 1e-7 leaves room.  The paper prints ~2e-11 for its own (MATLAB)
    run of this construction, whose factor distribution it does not state."""
    ts, target = synth.e2_cancelling_sum(seed=7)
    out = RC.recompress(ts, "krp", (7,), seed=21)
    xt = T.sum_to_dense(target)
    err = T.rel_err(RC.reconstruct(out["H"], out["Q"]), xt)
    assert err < 1e-7, err
    # the two smallest target components (2e-6, 1e-6) are still resolved
    xh = RC.reconstruct(out["H"], out["Q"])
    tf = target["factors"][0]
    for j, want in ((3, 2e-6), (4, 1e-6)):
        coef = xh
        for k in range(3):
            coef = T.ttm(coef, tf[k][:, j:j + 1].T, k)
        assert abs(float(coef.ravel()[0]) - want) < 1e-2 * want


def test_single_orthonormal_term_reproduced():
    ts = synth.random_sum(8, (20, 18, 16), [[4, 3, 5]])
    out = RC.recompress(ts, "krp", (6,), seed=4)
    x = T.sum_to_dense(ts)
    assert T.rel_err(RC.reconstruct(out["H"], out["Q"]), x) < 1e-13


def test_zero_sum():
    ts = tiny_sum(9)
    ts = dict(ts, coeffs=np.zeros(3))
    out = RC.recompress(ts, "krp", (4,), seed=1)
    assert np.all(out["H"] == 0)
    for q in out["Q"]:
        assert np.linalg.norm(q.T @ q - np.eye(q.shape[1])) < 1e-13


def test_tucker_form_error_matches_dense():
    ts = synth.config_tiny()
    out = RC.recompress(ts, "kron", (5, 5, 5), seed=ts["omega_seed"])
    x = T.sum_to_dense(ts)
    dense_err = T.rel_err(RC.reconstruct(out["H"], out["Q"]), x)
    assert abs(RC.rel_err_tucker(out["H"], out["Q"], ts) - dense_err) < 1e-8


def test_stage4_st_hosvd_tolerance():
    ts = synth.e1_low_rank_sum(seed=6, d=3, n=30, terms=15, r_true=6)
    out = RC.recompress(ts, "krp", (10,), seed=2)
    g, vs = RC.st_hosvd(out["H"], 1e-6)
    assert g.shape == (6, 6, 6)
    us = [q @ v for q, v in zip(out["Q"], vs)]
    x = T.sum_to_dense(ts)
    assert T.rel_err(T.tucker_to_dense(g, us), x) < 1e-6


def test_stage1_effective_subranks():
    ts = synth.e1_low_rank_sum(seed=7, d=3, n=30, terms=15, r_true=6)
    assert RC.effective_subranks(ts, 1e-6, 2) == [8, 8, 8]
