"""Differentiation form: the hand-written adjoint on the GPU against the
oracle's adjoint and against FP64 central finite differences."""
import numpy as np
import pytest

import synth
from helpers import np_of, rel, to_torch
from oracle import adjoint as AD

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as m
    return m


def torch_loss(H, Q, tg_core, tg_fac):
    """||[[H; Q]] - T||^2 in Tucker form, as the oracle computes it."""
    import torch

    def ttm(x, a, k):
        y = torch.tensordot(a, x, dims=([1], [k]))       # new mode first
        return torch.movedim(y, 0, k)
    d = H.dim()
    A = [q.T @ q for q in Q]
    B = [Q[k].T @ tg_fac[k] for k in range(d)]
    HA, TB, TT = H, tg_core, tg_core
    for k in range(d):
        HA = ttm(HA, A[k], k)
        TB = ttm(TB, B[k], k)
        TT = ttm(TT, tg_fac[k].T @ tg_fac[k], k)
    return (H * HA).sum() - 2 * (H * TB).sum() + (tg_core * TT).sum()


def gpu_grads(tsk, ts, tg, m, seed, dtype, prec):
    import torch
    cores, factors = to_torch(ts, DEV, dtype)
    for t in cores + [u for us in factors for u in us]:
        t.requires_grad_(True)
    H, Q = tsk.recompress(cores, factors, "krp", [m], seed, coeffs=ts["coeffs"], sketch_prec=prec)
    tc = torch.from_numpy(tg["cores"][0]).to(DEV, torch.float64)
    tf = [torch.from_numpy(u).to(DEV, torch.float64) for u in tg["factors"][0]]
    loss = torch_loss(H.double(), [q.double() for q in Q], tc, tf)
    loss.backward()
    torch.cuda.synchronize()
    return (loss.item(), [np_of(g.grad) for g in cores],
            [[np_of(u.grad) for u in us] for us in factors])


def small_problem():
    ts = synth.random_sum(0, (40, 36, 30), [[5, 4, 6], [4, 6, 5], [6, 5, 4]], coeffs=[1.0, -0.6, 0.8])
    tg = synth.random_sum(50, (40, 36, 30), [[6, 6, 6]])
    return ts, tg, 10


def test_fp64_gradient_matches_oracle_small(tsk):
    import torch
    ts, tg, m = small_problem()
    loss, gb, ub = gpu_grads(tsk, ts, tg, m, 3, torch.float64, "fp64")
    want_loss, wg, wu, _ = AD.loss_and_grad(ts, m, 3, tg)
    assert abs(loss - want_loss) < 1e-10 * max(1.0, abs(want_loss))
    for a, b in zip(gb, wg):
        assert rel(a, b) < 1e-9
    for us, ws in zip(ub, wu):
        for a, b in zip(us, ws):
            assert rel(a, b) < 1e-9


def test_backward_reports_singular_r(tsk):
    """A sum whose sketches have lower rank than the sketch width takes the
    Householder path, whose R is singular: the backward must report
    TSK_ERR_RANK_DEFICIENT rather than return meaningless gradients, and
    report it once (a following full-rank call is clean)."""
    import torch
    ts = synth.random_sum(4, (16, 18, 14), [[2, 2, 2]])
    tg = synth.random_sum(5, (16, 18, 14), [[2, 2, 2]])
    with pytest.raises(tsk.TskError) as err:
        gpu_grads(tsk, ts, tg, 6, 3, torch.float64, "fp64")
    assert err.value.name == "TSK_ERR_RANK_DEFICIENT"
    ts, tg, m = small_problem()
    gpu_grads(tsk, ts, tg, m, 3, torch.float64, "fp64")


def test_fp64_gradient_against_finite_differences(tsk):
    """64 random entries of cores and factors: GPU adjoint vs central FD of
    the GPU FP64 forward (h = 1e-6)."""
    import torch
    ts, tg, m = small_problem()
    loss, gb, ub = gpu_grads(tsk, ts, tg, m, 3, torch.float64, "fp64")
    cores, factors = to_torch(ts, DEV, torch.float64)
    tc = torch.from_numpy(tg["cores"][0]).to(DEV, torch.float64)
    tf = [torch.from_numpy(u).to(DEV, torch.float64) for u in tg["factors"][0]]

    def f():
        q, h = tsk.tucker_sum_recompress(cores, factors, "krp", [m], 3, coeffs=ts["coeffs"])
        return torch_loss(h, q, tc, tf).item()
    rng = np.random.default_rng(7)
    h = 1e-6
    for n_check in range(64):
        i = int(rng.integers(0, len(cores)))
        if n_check % 2 == 0:
            t = cores[i]
            idx = tuple(int(rng.integers(0, n)) for n in t.shape)
            want = gb[i][idx]
        else:
            k = int(rng.integers(0, 3))
            t = factors[i][k]
            idx = (int(rng.integers(0, t.shape[0])), int(rng.integers(0, t.shape[1])))
            want = ub[i][k][idx]
        old = t[idx].item()
        with torch.no_grad():
            t[idx] = old + h
        fp = f()
        with torch.no_grad():
            t[idx] = old - h
        fm = f()
        with torch.no_grad():
            t[idx] = old
        fd = (fp - fm) / (2 * h)
        assert abs(fd - want) < 1e-5 * max(1.0, abs(want)), (n_check, fd, want)


@pytest.mark.slow
@pytest.mark.parametrize("dtype_name,prec,tol", [("float64", "fp64", 1e-8), ("float32", "fp32", 1e-5)])
def test_gradient_workload(tsk, dtype_name, prec, tol):
    """d=3, 256^3, 6 terms with 24^3 cores, KRP m = 40, rank-32 target:
    gradients of every core and factor against the FP64 oracle adjoint."""
    import torch
    ts = synth.config_gradient()
    tg = synth.gradient_target()
    m = ts["ell"][0]
    loss, gb, ub = gpu_grads(tsk, ts, tg, m, ts["omega_seed"], getattr(torch, dtype_name), prec)
    want_loss, wg, wu, _ = AD.loss_and_grad(ts, m, ts["omega_seed"], tg)
    assert abs(loss - want_loss) < max(tol, 1e-10) * abs(want_loss) * 10
    worst = 0.0
    for a, b in zip(gb, wg):
        worst = max(worst, rel(a, b))
    for us, ws in zip(ub, wu):
        for a, b in zip(us, ws):
            worst = max(worst, rel(a, b))
    print(f"gradient workload {prec}: worst relative gradient error {worst:.3e}")
    assert worst < tol
