"""Pins for the oracle's hand adjoint: every gradient against FP64 central
finite differences of the forward (the paper has no gradients, so the
derivative of its own definition is the only reference)."""
import numpy as np
import pytest

import synth
from oracle import adjoint as AD
from oracle.recompress import thin_qr


def fd(f, x, idx, h=1e-6):
    old = x[idx]
    x[idx] = old + h
    fp = f()
    x[idx] = old - h
    fm = f()
    x[idx] = old
    return (fp - fm) / (2 * h)


def test_qr_adjoint_against_fd():
    rng = np.random.default_rng(0)
    y = rng.standard_normal((15, 6))
    C = rng.standard_normal((15, 6))
    q, r = thin_qr(y)
    yb = AD.qr_adjoint(q, r, C)
    f = lambda: float(np.sum(C * thin_qr(y)[0]))
    for idx in [(0, 0), (3, 2), (14, 5), (7, 1), (10, 4)]:
        assert abs(fd(f, y, idx) - yb[idx]) < 1e-7 * max(1.0, abs(yb[idx]))


def test_copyltu():
    M = np.arange(9.0).reshape(3, 3)
    S = AD.copyltu(M)
    assert np.array_equal(S, S.T)
    assert np.array_equal(np.tril(S), np.tril(M))


def small_problem(d=3, seed=0):
    if d == 3:
        ts = synth.random_sum(seed, (12, 10, 9), [[3, 2, 4], [2, 3, 2], [4, 4, 3]],
                              coeffs=[1.0, -0.6, 0.8])
        tg = synth.random_sum(seed + 50, (12, 10, 9), [[4, 4, 4]])
        m = 6
    else:
        ts = synth.random_sum(seed, (8, 7, 6, 7), [[3, 3, 3, 3], [2, 3, 2, 3]])
        tg = synth.random_sum(seed + 50, (8, 7, 6, 7), [[3, 3, 3, 3]])
        m = 5
    return ts, tg, m


def test_loss_gradients_wrt_H_and_Q_against_fd():
    ts, tg, m = small_problem()
    fw = AD.forward(ts, m, 3)
    H = fw["H"].copy()
    Q = [q.copy() for q in fw["Q"]]
    _, Hb, Qb = AD.tucker_loss(H, Q, tg)
    f = lambda: AD.tucker_loss(H, Q, tg)[0]
    for idx in [(0, 0, 0), (2, 3, 1), (5, 5, 5)]:
        assert abs(fd(f, H, idx) - Hb[idx]) < 1e-6 * max(1.0, abs(Hb[idx]))
    for k in range(3):
        for idx in [(0, 0), (4, 2), (8, 5)]:
            assert abs(fd(f, Q[k], idx) - Qb[k][idx]) < 1e-6 * max(1.0, abs(Qb[k][idx]))


@pytest.mark.parametrize("d", [3, 4])
def test_full_gradient_against_fd(d):
    ts, tg, m = small_problem(d)
    loss, Gb, Ub, fw = AD.loss_and_grad(ts, m, 11, tg)
    om = fw["omegas"]
    f = lambda: AD.loss_only(ts, m, 11, tg, om)
    rng = np.random.default_rng(1)
    checked = 0
    for i in range(len(ts["cores"])):
        g = ts["cores"][i]
        for _ in range(3):
            idx = tuple(int(rng.integers(0, n)) for n in g.shape)
            want = fd(f, g, idx)
            assert abs(want - Gb[i][idx]) < 1e-6 * max(1.0, abs(want)), (i, idx)
            checked += 1
        for k in range(d):
            u = ts["factors"][i][k]
            for _ in range(2):
                idx = (int(rng.integers(0, u.shape[0])), int(rng.integers(0, u.shape[1])))
                want = fd(f, u, idx)
                assert abs(want - Ub[i][k][idx]) < 1e-6 * max(1.0, abs(want)), (i, k, idx)
                checked += 1
    assert checked > 20


def test_loss_is_recompression_error():
    """The Tucker-form loss equals the dense squared error."""
    from oracle import tensor as T
    from oracle.recompress import reconstruct
    ts, tg, m = small_problem()
    fw = AD.forward(ts, m, 3)
    loss, _, _ = AD.tucker_loss(fw["H"], fw["Q"], tg)
    dense = np.sum((reconstruct(fw["H"], fw["Q"]) - T.sum_to_dense(tg)) ** 2)
    assert abs(loss - dense) < 1e-10 * max(1.0, dense)
