"""The entry point that allocates nothing (tucker_sum_recompress_noalloc),
called through the C ABI, against tucker_sum_recompress with a caller
workspace: two calls in a row on the shared static scratch, the second on a
smaller sum, each bit-identical to the workspace call (same plan, same
kernels) and within the FP64 tolerances of the oracle."""
import numpy as np
import pytest

import synth
from helpers import np_of, rel, to_torch
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


def outputs(tsk, shapes_q, shape_h, dtype):
    return ([tsk.empty_fortran(s, dtype, DEV) for s in shapes_q],
            tsk.empty_fortran(shape_h, dtype, DEV))


def one_call(tsk, ts, kind, sizes, seed, prec, dtype):
    import torch
    cores, factors = to_torch(ts, DEV, dtype)
    q_ref, h_ref, r_ref = tsk.tucker_sum_recompress(cores, factors, kind, sizes, seed,
                                                    coeffs=ts["coeffs"], sketch_prec=prec,
                                                    project_prec=prec, return_r=True)
    q_out, h_out = outputs(tsk, [tuple(q.shape) for q in q_ref], tuple(h_ref.shape), dtype)
    r_out = [tsk.empty_fortran(tuple(r.shape), torch.float64, DEV) for r in r_ref]
    for t in q_out + [h_out] + r_out:
        t.fill_(float("nan"))
    tsk.tucker_sum_recompress_noalloc(cores, factors, kind, sizes, seed, q_out, h_out,
                                      coeffs=ts["coeffs"], sketch_prec=prec, project_prec=prec,
                                      R_out=r_out)
    torch.cuda.synchronize()
    assert torch.equal(h_out, h_ref)
    for a, b in zip(q_out + r_out, q_ref + r_ref):
        assert torch.equal(a, b)
    return q_out, h_out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_workspace_call_twice(tsk, prec):
    import torch
    dtype = torch.float64 if prec == "fp64" else torch.float32
    big = synth.random_sum(41, (130, 70, 90), [[30, 5, 33], [12, 40, 12], [20, 20, 20]],
                           coeffs=[1.0, -0.5, 2.0])
    small = synth.random_sum(42, (40, 36, 30), [[5, 4, 6], [4, 6, 5]], coeffs=[0.7, 1.3])
    for ts, sizes, seed in ((big, [48], 7), (small, [8], 8)):
        print(f"no-alloc call {prec}: dims {ts['dims']}, m {sizes[0]}", flush=True)
        q, h = one_call(tsk, ts, "krp", sizes, seed, prec, dtype)
        if prec == "fp64":
            ref = RC.recompress(ts, "krp", sizes, seed)
            assert rel(np_of(h), ref["H"]) < 1e-11
            for a, b in zip(q, ref["Q"]):
                assert rel(np_of(a), b) < 1e-10


def test_noalloc_kron_tiny(tsk):
    import torch
    ts = synth.config_tiny()
    sizes = RC.kron_sizes(ts["ell"])
    q, h = one_call(tsk, ts, "kron", sizes, ts["omega_seed"], "fp64", torch.float64)
    ref = RC.recompress(ts, "kron", sizes, ts["omega_seed"])
    assert rel(np_of(h), ref["H"]) < 1e-11


def test_noalloc_rejects_a_problem_beyond_its_scratch(tsk):
    """d = 4, 256^4, 8 terms with 32^4 cores needs hundreds of MB of
    intermediates: refused before anything is enqueued."""
    import torch
    ts = synth.random_sum(3, (256,) * 4, np.full((8, 4), 32))
    cores, factors = to_torch(ts, DEV, torch.float64)
    q_out, h_out = outputs(tsk, [(256, 56)] * 4, (56,) * 4, torch.float64)
    with pytest.raises(tsk.TskError) as ei:
        tsk.tucker_sum_recompress_noalloc(cores, factors, "krp", [56], 3, q_out, h_out)
    assert ei.value.name == "TSK_ERR_WORKSPACE_TOO_SMALL"
