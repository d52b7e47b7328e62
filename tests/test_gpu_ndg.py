"""NDG transport steps (Section 5.3) on the GPU against the oracle.

From the rank-6 initial condition, both sides take forward-Euler steps in
which every node's update sum (1 + 4(k+1) Tucker terms) is recompressed by
the sketched sum: Stage 1 sizes from eps and p, Stages 2-3, Stage 4 with
eps.  The GPU runs each stage batched over all nodes; the oracle runs the
plain FP64 stages node by node, each from its own state.  Sketch sizes and
ranks are integers decided in FP64 on both sides and must agree; the states
agree to the eigenvector conditioning of the Stage-4 cuts (the GPU factors
mode Grams, the oracle takes SVDs), accumulated over the steps."""
import numpy as np
import pytest

from helpers import condition_bound, np_of, tucker_rel_diff
from oracle import recompress as RC
from oracle import tensor as T
from synth import ndg

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as m
    from paper_2603_13532_amd import ndg as gpu_ndg
    return m, gpu_ndg


def oracle_sum(states, tl, st):
    cores, factors, coeffs = [], [], []
    for c, src, kind in tl:
        g, us = states[src]
        us = list(us)
        if kind is not None:
            us[0] = st["scale"][kind][:, None] * us[0]
        cores.append(g)
        factors.append(us)
        coeffs.append(c)
    return {"dims": tuple(u.shape[0] for u in factors[0]),
            "ranks": np.array([g.shape for g in cores]), "cores": cores, "factors": factors,
            "coeffs": np.array(coeffs)}


def oracle_step(states, terms, st, eps, p, kind, seed):
    out, sizes, bounds = [], [], []
    for tl in terms:
        ts = oracle_sum(states, tl, st)
        ell = RC.effective_subranks(ts, eps, p)
        sz = [RC.krp_width(ell)] if kind == "krp" else RC.kron_sizes(ell)
        ref = RC.recompress(ts, kind, sz, seed)
        g, vs = RC.st_hosvd(ref["H"], eps)
        out.append((g, [q @ v for q, v in zip(ref["Q"], vs)]))
        sizes.append(list(sz))
        bounds.append(condition_bound(ref["H"], g.shape))
    return out, sizes, bounds


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_ndg_steps_match_oracle(tsk, kind):
    import torch
    m, gpu_ndg = tsk
    st = ndg.setup(nx=4, k=1, nxi=24, xi_max=6.0)
    eps, p, seed, steps = 1e-6, 5, 11, 3
    terms = ndg.euler_terms(st)
    init = ndg.initial_state(st)
    ref = [(s["core"], s["factors"]) for s in init]
    gpu = gpu_ndg.to_device(init, DEV)
    scales = {k: torch.from_numpy(v).to(DEV) for k, v in st["scale"].items()}
    acc = np.zeros(len(terms))
    for n in range(steps):
        print(f"step {n} ({kind})", flush=True)
        ref, rsz, bounds = oracle_step(ref, terms, st, eps, p, kind, seed)
        gpu, granks, gsz = gpu_ndg.euler_step(gpu, terms, scales, eps, p, kind=kind, seed=seed)
        torch.cuda.synchronize()
        acc += np.asarray(bounds)
        worst = 0.0
        for a, ((g, us), (rg, rus)) in enumerate(zip(gpu, ref)):
            assert gsz[a] == rsz[a], (n, a, gsz[a], rsz[a])
            assert tuple(granks[a]) == rg.shape, (n, a, granks[a], rg.shape)
            diff = tucker_rel_diff(np_of(g), [np_of(u) for u in us], rg, rus)
            worst = max(worst, diff / max(1e-12, 4 * acc[a]))
            assert diff <= max(1e-12, 4 * acc[a]), (n, a, diff, acc[a])
        print(f"  ranks {granks[0]} .. sizes {gsz[0]}, worst diff/bound {worst:.2e}")


def test_ndg_sketched_vs_deterministic(tsk):
    """One step of the sketched sum and of the deterministic baseline
    (TuckerAxby + TuckerRounding) from the same states, each against the
    dense sum.  TuckerRounding's error is at most tau ||X|| (ST-HOSVD with
    theta = tau^2 ||X||^2 / d); the sketched sum adds the projection error of
    sketches sized by Stage 1 (eps-rank plus oversampling), allowed one more
    eps."""
    import torch
    m, gpu_ndg = tsk
    st = ndg.setup(nx=4, k=1, nxi=24, xi_max=6.0)
    eps = 1e-6
    terms = ndg.euler_terms(st)
    init = ndg.initial_state(st)
    gpu = gpu_ndg.to_device(init, DEV)
    scales = {k: torch.from_numpy(v).to(DEV) for k, v in st["scale"].items()}
    a, _, _ = gpu_ndg.euler_step(gpu, terms, scales, eps, 5, kind="krp", seed=3)
    b, _ = gpu_ndg.euler_step_deterministic(gpu, terms, scales, eps)
    torch.cuda.synchronize()
    host = [(s["core"], s["factors"]) for s in init]
    for (ga, ua), (gb, ub), tl in zip(a, b, terms):
        exact = T.sum_to_dense(oracle_sum(host, tl, st))
        da = T.tucker_to_dense(np_of(ga), [np_of(u) for u in ua])
        db = T.tucker_to_dense(np_of(gb), [np_of(u) for u in ub])
        nx = np.linalg.norm(exact)
        assert np.linalg.norm(db - exact) <= 1.01 * eps * nx
        assert np.linalg.norm(da - exact) <= 2.0 * eps * nx
