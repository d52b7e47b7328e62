"""Pins for the oracle's tensor algebra against definitions written out
element by element (Section 2.1, Definition 1, Proposition 1)."""
import itertools

import numpy as np
import pytest

from oracle import tensor as T
from oracle import sketch as S
from oracle import recompress as RC


def rng(seed=0):
    return np.random.default_rng(seed)


def test_kron_matches_library_and_definition():
    a = rng(1).standard_normal((3, 4))
    b = rng(2).standard_normal((2, 5))
    k = T.kron(a, b)
    assert np.array_equal(k, np.kron(a, b))
    # 1-based definition (A (x) B)_{(i-1)p+k,(j-1)q+l} = a_ij b_kl
    p, q = b.shape
    for i, j, kk, ll in itertools.product(range(1, 4), range(1, 5), range(1, 3), range(1, 6)):
        assert k[(i - 1) * p + kk - 1, (j - 1) * q + ll - 1] == a[i - 1, j - 1] * b[kk - 1, ll - 1]


def test_khatri_rao_is_columnwise_kron():
    a = rng(3).standard_normal((3, 6))
    b = rng(4).standard_normal((4, 6))
    k = T.khatri_rao(a, b)
    full = np.kron(a, b)
    for t in range(6):
        assert np.array_equal(k[:, t], full[:, t * 6 + t])


@pytest.mark.parametrize("shape", [(2, 3, 4), (3, 2, 2, 3), (5, 4)])
def test_unfolding_index_formula(shape):
    x = rng(5).standard_normal(shape)
    d = len(shape)
    for k in range(d):
        u = T.unfold(x, k)
        for idx in itertools.product(*[range(n) for n in shape]):
            # 1-based eq.: j = 1 + sum_{m != k} (i_m - 1) prod_{l < m, l != k} n_l
            j = 1
            for m in range(d):
                if m == k:
                    continue
                stride = 1
                for l in range(m):
                    if l != k:
                        stride *= shape[l]
                j += idx[m] * stride
            assert u[idx[k], j - 1] == x[idx]
        assert np.array_equal(T.fold(u, k, shape), x)


def ttm_elementwise(x, a, k):
    shape = list(x.shape)
    shape[k] = a.shape[0]
    y = np.zeros(shape)
    for idx in itertools.product(*[range(n) for n in shape]):
        tot = 0.0
        for ik in range(x.shape[k]):
            src = list(idx)
            src[k] = ik
            tot += x[tuple(src)] * a[idx[k], ik]
        y[idx] = tot
    return y


def test_ttm_elementwise_definition():
    x = rng(6).standard_normal((3, 4, 2))
    for k in range(3):
        a = rng(7 + k).standard_normal((5, x.shape[k]))
        assert np.allclose(T.ttm(x, a, k), ttm_elementwise(x, a, k), rtol=1e-14, atol=1e-14)


def tucker_elementwise(g, us):
    shape = tuple(u.shape[0] for u in us)
    x = np.zeros(shape)
    for idx in itertools.product(*[range(n) for n in shape]):
        tot = 0.0
        for j in itertools.product(*[range(r) for r in g.shape]):
            p = g[j]
            for k, u in enumerate(us):
                p *= u[idx[k], j[k]]
            tot += p
        x[idx] = tot
    return x


def small_tucker(seed, dims=(4, 3, 5), ranks=(2, 3, 2)):
    r = rng(seed)
    g = r.standard_normal(ranks)
    us = [r.standard_normal((n, k)) for n, k in zip(dims, ranks)]
    return g, us


def test_tucker_to_dense_elementwise():
    g, us = small_tucker(8)
    assert np.allclose(T.tucker_to_dense(g, us), tucker_elementwise(g, us), rtol=1e-13, atol=1e-13)


def test_prop1_unfolding_identity():
    """X_(k) = U_k G_(k) (U_d (x) ... (x) U_1, skipping k)^T."""
    g, us = small_tucker(9)
    x = tucker_elementwise(g, us)
    for k in range(3):
        kr = T.kron_list([us[j] for j in reversed(range(3)) if j != k])
        assert np.allclose(T.unfold(x, k), us[k] @ T.unfold(g, k) @ kr.T, rtol=1e-13, atol=1e-13)


def test_prop1_mttkrp_identity():
    """X_(k) (A_d (.) ... (.) A_1) = U_k G_(k) (U_d^T A_d (.) ... (.) U_1^T A_1)."""
    g, us = small_tucker(10)
    x = tucker_elementwise(g, us)
    r = rng(11)
    a = [r.standard_normal((u.shape[0], 6)) for u in us]
    for k in range(3):
        lhs = T.unfold(x, k) @ T.khatri_rao_list([a[j] for j in reversed(range(3)) if j != k])
        rhs = us[k] @ T.unfold(g, k) @ T.khatri_rao_list([us[j].T @ a[j] for j in reversed(range(3)) if j != k])
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_prop1_multi_ttm_identity():
    """X x_{j != k} B_j = G x_k U_k x_{j != k} (B_j U_j)."""
    g, us = small_tucker(12)
    x = tucker_elementwise(g, us)
    r = rng(13)
    b = [r.standard_normal((3, u.shape[0])) for u in us]
    for k in range(3):
        lhs = x
        rhs = T.ttm(g, us[k], k)
        for j in range(3):
            if j != k:
                lhs = ttm_elementwise(lhs, b[j], j)
                rhs = T.ttm(rhs, b[j] @ us[j], j)
        assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def tiny_sum(seed, dims=(5, 4, 6), ranks=((2, 3, 2), (1, 2, 3), (3, 1, 2)), coeffs=(1.0, -0.5, 2.0)):
    r = rng(seed)
    cores = [r.standard_normal(rk) for rk in ranks]
    facs = [[r.standard_normal((n, k)) for n, k in zip(dims, rk)] for rk in ranks]
    return {"dims": dims, "ranks": np.array(ranks), "cores": cores, "factors": facs,
            "coeffs": np.array(coeffs)}


def sketch_brute_krp(x, om, n):
    """Y_n[a, t] = sum over all other indices of X * prod_{j != n} Omega_j[i_j, t]."""
    shape = x.shape
    m = om[0].shape[1]
    y = np.zeros((shape[n], m))
    for idx in itertools.product(*[range(s) for s in shape]):
        for t in range(m):
            w = x[idx]
            for j in range(len(shape)):
                if j != n:
                    w *= om[j][idx[j], t]
            y[idx[n], t] += w
    return y


def test_structured_krp_sketch_equals_brute_force():
    ts = tiny_sum(14)
    r = rng(15)
    om = [r.standard_normal((n, 3)) for n in ts["dims"]]
    x = T.sum_to_dense(ts)
    ys = S.structured_sketch_krp(ts, om)
    for n in range(3):
        assert np.allclose(ys[n], sketch_brute_krp(x, om, n), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_structured_equals_dense_sketch(kind):
    ts = tiny_sum(16)
    r = rng(17)
    widths = [4, 4, 4] if kind == "krp" else [2, 3, 2]
    om = [r.standard_normal((n, w)) for n, w in zip(ts["dims"], widths)]
    ys = S.structured_sketch(ts, om, kind)
    yd = S.dense_sketch(ts, om, kind)
    for a, b in zip(ys, yd):
        assert a.shape == b.shape
        assert np.allclose(a, b, rtol=1e-12, atol=1e-12)


def test_kron_sketch_column_order_brute_force():
    """Kronecker sketch columns follow Omega_d (x) ... (x) Omega_1: the column
    of Y_n for (t_j)_{j != n} is first-remaining-mode fastest."""
    ts = tiny_sum(18)
    r = rng(19)
    om = [r.standard_normal((n, w)) for n, w in zip(ts["dims"], [2, 3, 2])]
    x = T.sum_to_dense(ts)
    ys = S.structured_sketch_kron(ts, om)
    n = 1
    for a in range(x.shape[1]):
        for t0 in range(2):
            for t2 in range(2):
                want = sum(x[i0, a, i2] * om[0][i0, t0] * om[2][i2, t2]
                           for i0 in range(x.shape[0]) for i2 in range(x.shape[2]))
                assert abs(ys[n][a, t0 + 2 * t2] - want) < 1e-12


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_sketch_linearity(kind):
    ts = tiny_sum(20)
    r = rng(21)
    widths = [4, 4, 4] if kind == "krp" else [2, 2, 3]
    om = [r.standard_normal((n, w)) for n, w in zip(ts["dims"], widths)]
    whole = S.structured_sketch(ts, om, kind)
    parts = []
    for i in range(3):
        one = dict(ts, cores=[ts["cores"][i]], factors=[ts["factors"][i]], coeffs=np.array([1.0]),
                   ranks=ts["ranks"][i:i + 1])
        parts.append(S.structured_sketch(one, om, kind))
    for n in range(3):
        acc = sum(ts["coeffs"][i] * parts[i][n] for i in range(3))
        assert np.allclose(whole[n], acc, rtol=1e-12, atol=1e-12)
    scaled = dict(ts, coeffs=2.5 * ts["coeffs"])
    for a, b in zip(S.structured_sketch(scaled, om, kind), whole):
        assert np.allclose(a, 2.5 * b, rtol=1e-13, atol=1e-13)


def test_d2_reduces_to_range_finder():
    """d = 2: Y_1 = X Omega_2 and Y_2 = X^T Omega_1 (randomized range finder)."""
    ts = tiny_sum(22, dims=(7, 6), ranks=((2, 3), (3, 2)), coeffs=(1.0, 1.0))
    r = rng(23)
    om = [r.standard_normal((7, 4)), r.standard_normal((6, 4))]
    x = T.sum_to_dense(ts)
    for kind in ("krp", "kron"):
        ys = S.structured_sketch(ts, om, kind)
        assert np.allclose(ys[0], x @ om[1], rtol=1e-12, atol=1e-12)
        assert np.allclose(ys[1], x.T @ om[0], rtol=1e-12, atol=1e-12)


def test_kron_identity_sketch_gives_unfolding():
    ts = tiny_sum(24)
    om = [np.eye(n) for n in ts["dims"]]
    x = T.sum_to_dense(ts)
    ys = S.structured_sketch_kron(ts, om)
    for n in range(3):
        assert np.allclose(ys[n], T.unfold(x, n), rtol=1e-13, atol=1e-13)


def test_tucker_rel_diff_matches_dense():
    """The basis-union difference used by the GPU parity tests equals the
    dense difference of the two reconstructions, for non-orthonormal
    factors of different widths too."""
    from helpers import tucker_rel_diff
    rng = np.random.default_rng(0)
    h = rng.standard_normal((5, 6, 7))
    q = [np.linalg.qr(rng.standard_normal((n, w)))[0] for n, w in ((9, 5), (10, 6), (11, 7))]
    h2 = h + 1e-9 * rng.standard_normal(h.shape)
    q2 = [x + 1e-10 * rng.standard_normal(x.shape) for x in q]
    a = RC.reconstruct(h, q)
    b = RC.reconstruct(h2, q2)
    want = np.linalg.norm(a - b) / np.linalg.norm(b)
    assert abs(tucker_rel_diff(h, q, h2, q2) - want) < 1e-6 * want
    h3 = rng.standard_normal((5, 4, 7))
    q3 = [q[0], rng.standard_normal((10, 4)), q[2]]
    b3 = RC.reconstruct(h3, q3)
    want3 = np.linalg.norm(a - b3) / np.linalg.norm(b3)
    assert abs(tucker_rel_diff(h, q, h3, q3) - want3) < 1e-10 * want3
