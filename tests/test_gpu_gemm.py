"""Kernel-level check of the grouped MFMA GEMM (every operand layout, ragged
tiles, K-splits, each arithmetic form) against float64 matmul on the CPU."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# relative Frobenius tolerances per arithmetic form (Gaussian data, K <= 300)
TOL = {"fp64": 1e-14, "fp32": 3e-6, "bf16x1": 1e-2, "bf16x3": 3e-5, "bf16x6": 3e-6}


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_13532_amd as tsk
    from paper_2603_13532_amd import _lib
    lib = _lib.load()
    fn = lib.tsk_debug_gemm
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                   ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                   ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
    return tsk, _lib, fn


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x1", "bf16x3", "bf16x6"])
@pytest.mark.parametrize("ta,tb", [(0, 0), (0, 1), (1, 0), (1, 1)])
@pytest.mark.parametrize("M,N,K,splits", [(16, 16, 4, 1), (70, 130, 37, 1), (129, 65, 300, 3),
                                          (1, 5, 1, 1)])
def test_gemm_layouts(env, prec, ta, tb, M, N, K, splits):
    import torch
    tsk, _lib, fn = env
    rng = np.random.default_rng(M * 1000 + N * 10 + K + ta * 2 + tb)
    a = rng.standard_normal((M, K))
    b = rng.standard_normal((K, N))
    want = a @ b
    dt = torch.float64 if prec == "fp64" else torch.float32
    # A stored as M x K (ta=0) or K x M (ta=1), column-major
    a_st = a if ta == 0 else a.T
    b_st = b if tb == 0 else b.T
    A = torch.from_numpy(np.asfortranarray(a_st)).to(DEV, dt)
    A = tsk.fortran(A)
    B = tsk.fortran(torch.from_numpy(np.asfortranarray(b_st)).to(DEV, dt))
    # strides: A[m][k] at m*a_sx + k*a_sk
    a_sx, a_sk = (1, M) if ta == 0 else (K, 1)
    b_sx, b_sk = (K, 1) if tb == 0 else (1, N)
    C = tsk.empty_fortran((M, N), torch.float64, DEV)
    ws = torch.empty(1 << 22, dtype=torch.uint8, device=DEV)
    h = tsk.Handle.get(DEV)
    st = fn(h.ptr, _lib.PRECISIONS[prec], M, N, K, A.data_ptr(), a_sx, a_sk, B.data_ptr(), b_sx, b_sk,
            C.data_ptr(), M, 1, splits, ws.data_ptr(), ws.numel(), None)
    assert st == 0
    torch.cuda.synchronize()
    got = C.cpu().numpy()
    if prec != "fp64":
        # reference on the operands as the form sees them (FP32 inputs)
        want = a.astype(np.float32).astype(np.float64) @ b.astype(np.float32).astype(np.float64)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    assert err < TOL[prec], err


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,N,K,splits", [(100, 70, 700, 10), (64, 130, 1100, 17), (65, 64, 96, 9)])
def test_gemm_many_splits(env, prec, M, N, K, splits):
    """Split-K reductions spanning more than one batch of eight partials per
    round trip (and splits that get no K-tile: 96 / 16 = 6 tiles for 9
    splits), against float64 matmul on the CPU."""
    import torch
    tsk, _lib, fn = env
    rng = np.random.default_rng(M + 7 * N + 13 * K + splits)
    a = rng.standard_normal((M, K))
    b = rng.standard_normal((K, N))
    dt = torch.float64 if prec == "fp64" else torch.float32
    A = tsk.fortran(torch.from_numpy(np.asfortranarray(a)).to(DEV, dt))
    B = tsk.fortran(torch.from_numpy(np.asfortranarray(b)).to(DEV, dt))
    C = tsk.empty_fortran((M, N), torch.float64, DEV)
    ws = torch.empty(1 << 24, dtype=torch.uint8, device=DEV)
    h = tsk.Handle.get(DEV)
    st = fn(h.ptr, _lib.PRECISIONS[prec], M, N, K, A.data_ptr(), 1, M, B.data_ptr(), K, 1,
            C.data_ptr(), M, 1, splits, ws.data_ptr(), ws.numel(), None)
    assert st == 0
    torch.cuda.synchronize()
    if prec == "fp64":
        want = a @ b
    else:
        want = a.astype(np.float32).astype(np.float64) @ b.astype(np.float32).astype(np.float64)
    err = np.linalg.norm(C.cpu().numpy() - want) / np.linalg.norm(want)
    assert err < TOL[prec], err
