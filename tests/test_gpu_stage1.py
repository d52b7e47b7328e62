"""Stage 1 on the GPU (tucker_sum_subranks, phase 1 of Algorithm 3) against
the oracle's effective_subranks, exactly; and the whole eps-driven sum of
Algorithms 4/5 (Stage 1 sizes, Stages 2-3, Stage 4) against the oracle run
with the same sizes."""
import numpy as np
import pytest

import synth
from helpers import np_of, to_torch, tucker_rel_diff
from oracle import recompress as RC

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def tsk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as m
    return m


CASES = {
    # sum of ranks per mode <= 96: Jacobi in LDS
    "tiny": lambda: synth.config_tiny(),
    "ragged": lambda: synth.random_sum(31, (130, 70, 90), [[30, 5, 33], [1, 46, 12], [40, 20, 40]],
                                       decay=0.15, coeffs=[1.5, -0.75, 2.0]),
    "four_modes": lambda: synth.random_sum(32, (40, 30, 20, 25), [[6, 5, 4, 7], [3, 8, 2, 5]],
                                           decay=0.2),
    "low_rank": lambda: synth.e1_low_rank_sum(seed=5, d=4, n=24, terms=20, r_true=10),
    # above 96: tridiagonal reduction and bisection
    "structured": lambda: synth.config_structured(),
    "gradient": lambda: synth.config_gradient(),
}


@pytest.mark.parametrize("eps", [1e-6, 1e-3, 1e-1])
@pytest.mark.parametrize("name", list(CASES))
def test_subranks_match_oracle(tsk, name, eps):
    import torch
    ts = CASES[name]()
    d = len(ts["dims"])
    p = [2] * d
    want = RC.effective_subranks(ts, eps, p)
    cores, factors = to_torch(ts, DEV)
    got = tsk.effective_subranks(cores, factors, eps, p, coeffs=ts["coeffs"])
    print(f"{name} eps {eps}: ell {got} (oracle {want})")
    assert got == want
    if name in ("tiny", "structured"):
        c32, f32 = to_torch(ts, DEV, torch.float32)
        want32 = RC.effective_subranks(
            {**ts, "cores": [g.astype(np.float32).astype(np.float64) for g in ts["cores"]],
             "factors": [[u.astype(np.float32).astype(np.float64) for u in us]
                         for us in ts["factors"]]}, eps, p)
        assert tsk.effective_subranks(c32, f32, eps, p, coeffs=ts["coeffs"]) == want32


def test_batch_sums_subranks(tsk):
    """Forty sums of the batch workload (sum of ranks up to 400 per mode)."""
    for one in synth.config_batch(count=40):
        cores, factors = to_torch(one, DEV)
        assert tsk.effective_subranks(cores, factors, 1e-4, 1) == \
            RC.effective_subranks(one, 1e-4, 1)


@pytest.mark.parametrize("kind", ["krp", "kron"])
def test_sketch_sum_end_to_end(tsk, kind):
    """Algorithm 5 (KRP) / 4 (Kronecker) with eps = 1e-3, p = 2 on the GPU:
    sizes from Stage 1, the recompression, the truncation; against the
    oracle with the same sizes and seed."""
    import torch
    ts = synth.random_sum(33, (120, 100, 80), [[12, 10, 8], [9, 11, 7], [6, 6, 6]], decay=0.15)
    eps, p, seed = 1e-3, [2, 2, 2], 44
    cores, factors = to_torch(ts, DEV)
    g, us, ranks, sizes = tsk.sketch_sum(cores, factors, kind, eps, p, seed, coeffs=ts["coeffs"])
    torch.cuda.synchronize()
    ell = RC.effective_subranks(ts, eps, p)
    want_sizes = [RC.krp_width(ell)] if kind == "krp" else RC.kron_sizes(ell)
    assert list(sizes) == list(want_sizes)
    ref = RC.recompress(ts, kind, sizes, seed)
    g_ref, v_ref = RC.st_hosvd(ref["H"], eps)
    assert tuple(ranks) == g_ref.shape
    diff = tucker_rel_diff(np_of(g), [np_of(u) for u in us], g_ref,
                           [q @ v for q, v in zip(ref["Q"], v_ref)])
    assert diff < 1e-11
    x_err = RC.rel_err_tucker(np_of(g), [np_of(u) for u in us], ts)
    print(f"{kind}: sizes {sizes}, ranks {ranks}, error vs the sum {x_err:.2e}")
    assert x_err < 10 * eps


def test_batched_subranks_match_oracle(tsk):
    """tucker_sum_subranks_batched over sums of different shapes and orders of
    magnitude in one launch sequence (widths below and above 96, so the LDS
    Jacobi and the tridiagonal path share a call), FP64 and FP32 inputs."""
    import torch
    sums = [CASES[k]() for k in ("tiny", "ragged", "low_rank", "structured")] + \
        synth.config_batch(count=24)[::3]
    for one in sums:
        one.setdefault("coeffs", np.ones(len(one["cores"])))
    for dtype in (torch.float64, torch.float32):
        batch = []
        for one in sums:
            cores, factors = to_torch(one, DEV, dtype)
            batch.append({"cores": cores, "factors": factors, "coeffs": one["coeffs"]})
        got = tsk.effective_subranks_batched(batch, 1e-3, 2)
        for one, g in zip(sums, got):
            ref = one if dtype == torch.float64 else {
                **one, "cores": [c.astype(np.float32).astype(np.float64) for c in one["cores"]],
                "factors": [[u.astype(np.float32).astype(np.float64) for u in us]
                            for us in one["factors"]]}
            assert g == RC.effective_subranks(ref, 1e-3, 2), (one["dims"], g)
