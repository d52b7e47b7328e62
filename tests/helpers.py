"""Shared test utilities: moving seeded synthetic sums to torch tensors in
column-major layout, and relative errors."""
import numpy as np


def to_torch(tsum, device, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    from paper_2603_13532_amd import fortran

    def conv(a):
        t = torch.from_numpy(np.asfortranarray(a)).to(device=device, dtype=dtype)
        return fortran(t)
    cores = [conv(g) for g in tsum["cores"]]
    factors = [[conv(u) for u in us] for us in tsum["factors"]]
    return cores, factors


def np_of(t):
    return np.asfortranarray(t.detach().to("cpu").double().numpy())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    d = np.linalg.norm((a - b).ravel())
    return d / nb if nb > 0 else d
