"""Sketches Y_n = X_(n) S_n of a Tucker sum (Section 3.1).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two independent evaluations:
  dense_*       form the dense sum and the explicit sketching matrix S_n
                (Khatri-Rao eq. for S_k^KRP; Kronecker eq. for S_k^Kron) and
                multiply; tiny inputs only.
  structured_*  Stage 2 of Algorithm 5 (KRP) / Algorithm 4 (Kron), term by
                term and mode by mode, never forming X (eqs. for the KRP and
                Kronecker sketched unfoldings of a sum).
Mode indices are 0-based; "widths" is m for every mode (KRP) or q_k (Kron).
"""
import numpy as np

from .tensor import unfold, ttm, khatri_rao_list, kron_list, sum_to_dense


def sketch_matrix(omegas, n: int, kind: str) -> np.ndarray:
    """S_n = Omega_d (.) ... (.) Omega_1 skipping n, in reverse mode order
    (KRP, Section 3.1.1) or the same with Kronecker products (Section 3.1.2)."""
    mats = [omegas[j] for j in reversed(range(len(omegas))) if j != n]
    return khatri_rao_list(mats) if kind == "krp" else kron_list(mats)


def dense_sketch(tsum: dict, omegas, kind: str) -> list:
    """Y_n = X_(n) S_n with X formed densely."""
    x = sum_to_dense(tsum)
    return [unfold(x, n) @ sketch_matrix(omegas, n, kind) for n in range(len(tsum["dims"]))]


def structured_sketch_krp(tsum: dict, omegas) -> list:
    """Algorithm 5, Stage 2: for each term and mode, M_j = U_j^T Omega_j,
    V_(n) = G_(n) (M_d (.) ... (.) M_1 skipping n), Z = U_n V_(n);
    Y_n accumulates c_i Z over the terms."""
    d = len(tsum["dims"])
    ys = [np.zeros((tsum["dims"][n], omegas[0].shape[1])) for n in range(d)]
    for c, g, us in zip(tsum["coeffs"], tsum["cores"], tsum["factors"]):
        for n in range(d):
            ms = [us[j].T @ omegas[j] for j in range(d)]
            krp = khatri_rao_list([ms[j] for j in reversed(range(d)) if j != n])
            v = unfold(g, n) @ krp
            ys[n] += c * (us[n] @ v)
    return ys


def structured_sketch_kron(tsum: dict, omegas) -> list:
    """Algorithm 4, Stage 2: V = G x_j (Omega_j^T U_j) over j != n,
    Z = U_n V_(n); Y_n accumulates c_i Z over the terms."""
    d = len(tsum["dims"])
    widths = [int(np.prod([omegas[j].shape[1] for j in range(d) if j != n])) for n in range(d)]
    ys = [np.zeros((tsum["dims"][n], widths[n])) for n in range(d)]
    for c, g, us in zip(tsum["coeffs"], tsum["cores"], tsum["factors"]):
        for n in range(d):
            v = g
            for j in range(d):
                if j != n:
                    v = ttm(v, omegas[j].T @ us[j], j)
            ys[n] += c * (us[n] @ unfold(v, n))
    return ys


def structured_sketch(tsum: dict, omegas, kind: str) -> list:
    return structured_sketch_krp(tsum, omegas) if kind == "krp" else structured_sketch_kron(tsum, omegas)

