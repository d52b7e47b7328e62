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


def _rank_rule(lam, theta):
    """Smallest r >= 1 whose discarded values sum to at most theta (hand
    evaluation of the rule, independent of the oracle's code)."""
    lam = list(lam)
    for r in range(1, len(lam) + 1):
        if sum(lam[r:]) <= theta:
            return r
    return len(lam)


@pytest.mark.parametrize("eps", [1e-6, 1e-3, 0.05, 0.3])
def test_stage4_diagonal_core_closed_form(eps):
    """H = [[C; A_1, A_2, A_3]] with a diagonal core c_iii = s_i and
    orthonormal A_k: every unfolding's singular values are s (the Khatri-Rao
    product of orthonormal columns is orthonormal), the truncated core stays
    diagonal, so the ranks follow the rule on s and its prefixes and the
    result is A_k[:, :r] diag(s[:r]) exactly."""
    rng = np.random.default_rng(3)
    s = 10.0 ** (-0.25 * np.arange(12)) * (1 + 0.1 * rng.random(12))
    n = (15, 13, 14)
    A = [np.linalg.qr(rng.standard_normal((nk, 12)))[0] for nk in n]
    C = np.zeros((12, 12, 12))
    for i in range(12):
        C[i, i, i] = s[i]
    H = T.tucker_to_dense(C, A)
    theta = eps ** 2 * float(np.sum(s ** 2)) / 3
    r1 = _rank_rule(s ** 2, theta)
    r2 = _rank_rule(s[:r1] ** 2, theta)
    r3 = _rank_rule(s[:r2] ** 2, theta)
    g, vs = RC.st_hosvd(H, eps)
    assert g.shape == (r1, r2, r3)
    want = np.zeros(n)
    for i in range(r3):
        want += s[i] * np.einsum("a,b,c->abc", A[0][:, i], A[1][:, i], A[2][:, i])
    assert np.linalg.norm(T.tucker_to_dense(g, vs) - want) < 1e-12 * np.linalg.norm(H)
    err2 = float(np.sum(s[r3:] ** 2))
    assert abs(np.linalg.norm(T.tucker_to_dense(g, vs) - H) ** 2 - err2) < 1e-12 * float(np.sum(s ** 2))


def test_stage4_two_modes_is_truncated_svd():
    """d = 2: ST-HOSVD keeps the leading singular triplets of the matrix
    (Eckart-Young): H = A diag(s) B^T built with known A, B, s."""
    rng = np.random.default_rng(4)
    s = np.array([5.0, 3.0, 2.0, 0.5, 0.1, 0.01, 0.001])
    A = np.linalg.qr(rng.standard_normal((20, 7)))[0]
    B = np.linalg.qr(rng.standard_normal((16, 7)))[0]
    H = A @ np.diag(s) @ B.T
    eps = 0.05
    theta = eps ** 2 * float(np.sum(s ** 2)) / 2
    r = _rank_rule(s ** 2, theta)
    g, vs = RC.st_hosvd(H, eps)
    assert g.shape[0] == r
    want = A[:, :r] @ np.diag(s[:r]) @ B[:, :r].T
    assert np.linalg.norm(vs[0] @ g @ vs[1].T - want) < 1e-12 * np.linalg.norm(H)


def test_stage4_error_bound_and_monotone_ranks():
    """||H - [[G; V]]|| <= eps ||H|| (ST-HOSVD: the squared error is at most
    the discarded sum of every mode, each <= theta = eps^2 ||H||^2 / d), and
    ranks do not grow as eps grows."""
    rng = np.random.default_rng(5)
    H = synth.decaying_core(rng, (14, 12, 10), rate=0.15)
    prev = None
    for eps in (1e-8, 1e-4, 1e-2, 0.1, 0.5):
        g, vs = RC.st_hosvd(H, eps)
        err = np.linalg.norm(T.tucker_to_dense(g, vs) - H)
        assert err <= eps * np.linalg.norm(H) * (1 + 1e-12)
        if prev is not None:
            assert all(a <= b for a, b in zip(g.shape, prev))
        prev = g.shape


def test_stage1_single_orthonormal_term_closed_form():
    """One term with orthonormal U_n: V_n = ||G|| U_n, so V_n^T V_n =
    ||G||^2 I and the kept rank is r - floor(eps^2 r / d) plus p."""
    for eps, p in ((1e-3, 0), (0.5, 1), (0.9, 2)):
        ts = synth.random_sum(8, (30, 25, 20), [[9, 7, 5]])
        want = [r - int(np.floor(eps ** 2 * r / 3 + 1e-12)) + p for r in (9, 7, 5)]
        assert RC.effective_subranks(ts, eps, p) == want


def test_stage1_shared_and_orthogonal_factors():
    """Terms sharing one factor add their weights into one eigenvalue per
    column (rank r, not s r); terms with orthogonal factors keep separate
    eigenvalue groups ||G_i||^2, and the light group is dropped exactly when
    its total is at most eps^2 / d times the whole."""
    rng = np.random.default_rng(9)
    U = [np.linalg.qr(rng.standard_normal((40, 12)))[0] for _ in range(3)]
    g1 = rng.standard_normal((6, 6, 6))
    g2 = 1e-3 * rng.standard_normal((6, 6, 6))
    shared = synth.tucker_sum((40, 40, 40), [[6, 6, 6]] * 3,
                              [g1, 2 * g1, -g1], [[u[:, :6] for u in U]] * 3)
    assert RC.effective_subranks(shared, 1e-6, 0) == [6, 6, 6]
    orth = synth.tucker_sum((40, 40, 40), [[6, 6, 6]] * 2, [g1, g2],
                            [[u[:, :6] for u in U], [u[:, 6:] for u in U]])
    w1, w2 = np.sum(g1 ** 2), np.sum(g2 ** 2)
    for eps in (1e-4, 1e-1):
        tau = eps ** 2 / 3 * 6 * (w1 + w2)
        got = RC.effective_subranks(orth, eps, 0)
        lam = sorted([w1] * 6 + [w2] * 6, reverse=True)
        assert got == [_rank_rule(lam, tau)] * 3
        assert (got[0] == 6) == (6 * w2 <= tau)


def test_stage1_coefficients_scale_the_cores():
    """A coefficient c_i acts as the core c_i G^(i) (and its sign does not
    matter to a Gram matrix)."""
    ts = synth.random_sum(12, (30, 25, 20), [[5, 4, 6], [3, 6, 2], [4, 4, 4]],
                          coeffs=[2.0, -1e-3, 0.5])
    scaled = dict(ts)
    scaled["cores"] = [abs(c) * g for c, g in zip(ts["coeffs"], ts["cores"])]
    scaled["coeffs"] = np.ones(3)
    for eps in (1e-6, 1e-3, 0.2):
        assert RC.effective_subranks(ts, eps, 1) == RC.effective_subranks(scaled, eps, 1)
