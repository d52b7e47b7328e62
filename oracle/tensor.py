"""Dense tensor algebra in FP64 (Section 2.1 and Section 2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Conventions (Section 2.1): arrays are Fortran ordered; the mode-k unfolding
X_(k) is n_k x prod_{j != k} n_j with the column index running over the
remaining modes first-mode-fastest (eq. for the unfolding index).  Products
over modes are written in reverse mode order, U_d (x) ... (x) U_1, as in
Proposition 1.
"""
import numpy as np


def unfold(x: np.ndarray, k: int) -> np.ndarray:
    """Mode-k unfolding (0-based k): rows i_k, column index
    sum_{m != k} i_m prod_{l < m, l != k} n_l (0-based form of the unfolding
    index equation)."""
    n = x.shape
    return np.reshape(np.moveaxis(x, k, 0), (n[k], -1), order="F")


def fold(mat: np.ndarray, k: int, shape) -> np.ndarray:
    """Inverse of `unfold` for a tensor of the given shape."""
    shape = tuple(shape)
    rest = (shape[k],) + tuple(s for j, s in enumerate(shape) if j != k)
    return np.asfortranarray(np.moveaxis(np.reshape(mat, rest, order="F"), 0, k))


def ttm(x: np.ndarray, a: np.ndarray, k: int) -> np.ndarray:
    """Mode-k tensor-times-matrix Y = X x_k A, defined by Y_(k) = A X_(k)."""
    shape = list(x.shape)
    shape[k] = a.shape[0]
    return fold(a @ unfold(x, k), k, shape)


def kron(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Kronecker product (Definition 1): (A (x) B)[i p + k, j q + l] = a_ij b_kl
    (0-based), built elementwise from the definition."""
    m, n = a.shape
    p, q = b.shape
    out = np.empty((m * p, n * q))
    for i in range(m):
        for j in range(n):
            out[i * p:(i + 1) * p, j * q:(j + 1) * q] = a[i, j] * b
    return out


def khatri_rao(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Khatri-Rao product (Definition 1): column t is a_t (x) b_t."""
    assert a.shape[1] == b.shape[1]
    cols = [np.kron(a[:, t], b[:, t]) for t in range(a.shape[1])]
    return np.stack(cols, axis=1)


def kron_list(mats) -> np.ndarray:
    """mats[0] (x) mats[1] (x) ... in the order given."""
    out = mats[0]
    for m in mats[1:]:
        out = kron(out, m)
    return out


def khatri_rao_list(mats) -> np.ndarray:
    out = mats[0]
    for m in mats[1:]:
        out = khatri_rao(out, m)
    return out


def tucker_to_dense(core: np.ndarray, factors) -> np.ndarray:
    """[[G; U_1, ..., U_d]] = G x_1 U_1 x_2 ... x_d U_d (Section 2.2)."""
    x = core
    for k, u in enumerate(factors):
        x = ttm(x, u, k)
    return x


def sum_to_dense(tsum: dict) -> np.ndarray:
    """Dense X = sum_i c_i [[G_i; U_1^(i), ..., U_d^(i)]]."""
    x = np.zeros(tsum["dims"], order="F")
    for c, g, us in zip(tsum["coeffs"], tsum["cores"], tsum["factors"]):
        x = x + c * tucker_to_dense(g, us)
    return x


def frob(x) -> float:
    return float(np.sqrt(np.sum(np.asarray(x, dtype=np.float64) ** 2)))


def rel_err(a, b) -> float:
    """||a - b||_F / ||b||_F (absolute when b == 0)."""
    nb = frob(b)
    d = frob(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return d / nb if nb > 0 else d
