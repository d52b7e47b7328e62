"""Recompression of a Tucker sum by sketching: Stages 2 and 3 of Algorithms
4 and 5 (range finder, thin QR, core projection), the sketch-size rules of
Section 3.2, and, beyond the hot path, Stage 1 (Algorithm 3) and Stage 4
(ST-HOSVD as in Algorithm 2, phase 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken where the paper is silent (each also listed in the design
notes): the thin QR is returned with diag(R) >= 0; its width is
min(n_k, sketch width); the output of the hot path is [[H; Q_1..Q_d]] with
no Stage-4 truncation; coefficients c_i scale the cores.
"""
import numpy as np

from .omega import omegas as make_omegas
from .sketch import structured_sketch, dense_sketch
from .tensor import ttm, unfold, sum_to_dense, tucker_to_dense


# ---------------------------------------------------------------- sizes
def kron_sizes(ell) -> list:
    """Kronecker sketch sizes, eq. for the heuristic sketch dimension:
    q_i = ceil(C / ell_i) with C = (prod_j ell_j)^(1/(d-1)).  Evaluated in
    integers as q_i = min{q >= 1 : (q ell_i)^(d-1) >= prod_j ell_j}, which is
    the same number without floating-point roots."""
    ell = [int(x) for x in ell]
    d = len(ell)
    prod = 1
    for x in ell:
        prod *= x
    out = []
    for li in ell:
        q = 1
        while (q * li) ** (d - 1) < prod:
            q += 1
        out.append(q)
    return out


def krp_width(ell) -> int:
    """KRP sketch width m = max_i ell_i (Section 3.2)."""
    return int(max(int(x) for x in ell))


def omega_widths(d: int, kind: str, sizes) -> list:
    """Columns of Omega_k: m for every mode (KRP) or q_k (Kron)."""
    if kind == "krp":
        return [int(sizes[0])] * d
    return [int(x) for x in sizes]


def sketch_widths(d: int, kind: str, sizes) -> list:
    """Columns of Y_n: m (KRP) or S_n = prod_{k != n} q_k (Kron)."""
    if kind == "krp":
        return [int(sizes[0])] * d
    return [int(np.prod([int(sizes[k]) for k in range(d) if k != n])) for n in range(d)]


def basis_widths(dims, kind: str, sizes) -> list:
    """Columns of Q_n: economy QR keeps min(n_n, sketch width)."""
    w = sketch_widths(len(dims), kind, sizes)
    return [min(int(dims[n]), w[n]) for n in range(len(dims))]


# ---------------------------------------------------------------- stage 2
def thin_qr(y: np.ndarray):
    """Economy QR of Y (Householder, LAPACK via numpy), signs fixed so that
    diag(R) >= 0."""
    q, r = np.linalg.qr(y, mode="reduced")
    sgn = np.sign(np.diag(r))
    sgn[sgn == 0] = 1.0
    return np.asfortranarray(q * sgn), r * sgn[:, None]


# ---------------------------------------------------------------- stage 3
def project_structured(tsum: dict, qs) -> np.ndarray:
    """H = sum_i c_i G^(i) x_1 (Q_1^T U_1^(i)) ... x_d (Q_d^T U_d^(i))
    (Section 3.3, projection of each summand by linearity)."""
    shape = tuple(q.shape[1] for q in qs)
    h = np.zeros(shape, order="F")
    for c, g, us in zip(tsum["coeffs"], tsum["cores"], tsum["factors"]):
        t = g
        for k, u in enumerate(us):
            t = ttm(t, qs[k].T @ u, k)
        h = h + c * t
    return h


def project_dense(x: np.ndarray, qs) -> np.ndarray:
    """H = X x_1 Q_1^T ... x_d Q_d^T (Stage 3 as written in Algorithms 4/5)."""
    h = x
    for k, q in enumerate(qs):
        h = ttm(h, q.T, k)
    return h


def reconstruct(h: np.ndarray, qs) -> np.ndarray:
    """Dense [[H; Q_1, ..., Q_d]]."""
    return tucker_to_dense(h, qs)


# ---------------------------------------------------------------- pipeline
def recompress(tsum: dict, kind: str, sizes, seed: int, structured: bool = True,
               omegas=None) -> dict:
    """Stages 2-3 of Algorithm 5 (kind='krp', sizes=(m,)) or Algorithm 4
    (kind='kron', sizes=(q_1..q_d)).  With structured=False, X is formed
    densely and sketched/projected by definition (tiny inputs only)."""
    d = len(tsum["dims"])
    if omegas is None:
        omegas = make_omegas(seed, tsum["dims"], omega_widths(d, kind, sizes))
    if structured:
        ys = structured_sketch(tsum, omegas, kind)
    else:
        ys = dense_sketch(tsum, omegas, kind)
    qr = [thin_qr(y) for y in ys]
    qs = [q for q, _ in qr]
    rs = [r for _, r in qr]
    if structured:
        h = project_structured(tsum, qs)
    else:
        h = project_dense(sum_to_dense(tsum), qs)
    return {"omegas": omegas, "Y": ys, "Q": qs, "R": rs, "H": h}


# ---------------------------------------------------------------- Tucker-form norms
def tucker_inner(core_a, facs_a, core_b, facs_b) -> float:
    """<[[A; U]], [[B; V]]> = <A, B x_k (U_k^T V_k)>."""
    t = core_b
    for k in range(len(facs_a)):
        t = ttm(t, facs_a[k].T @ facs_b[k], k)
    return float(np.sum(core_a * t))


def sum_norm_sq(tsum: dict) -> float:
    """||sum_i c_i [[G_i; U^(i)]]||_F^2 without forming the sum."""
    tot = 0.0
    n = len(tsum["cores"])
    for i in range(n):
        for j in range(n):
            tot += tsum["coeffs"][i] * tsum["coeffs"][j] * tucker_inner(
                tsum["cores"][i], tsum["factors"][i], tsum["cores"][j], tsum["factors"][j])
    return tot


def rel_err_tucker(h, qs, tsum: dict) -> float:
    """||[[H; Q]] - X|| / ||X|| from inner products (Q orthonormal), resolving
    relative errors down to about 1e-8."""
    xx = sum_norm_sq(tsum)
    hh = float(np.sum(np.asarray(h, dtype=np.float64) ** 2))
    hx = 0.0
    for c, g, us in zip(tsum["coeffs"], tsum["cores"], tsum["factors"]):
        hx += c * tucker_inner(h, qs, g, us)
    return float(np.sqrt(max(hh - 2.0 * hx + xx, 0.0) / xx))


# ---------------------------------------------------------------- beyond the hot path
def st_hosvd(h: np.ndarray, eps: float):
    """Stage 4: ST-HOSVD of H with relative tolerance eps (Algorithm 2,
    phase 2): theta = eps^2 ||H||^2 / d; per mode keep the smallest r whose
    discarded squared singular values sum to at most theta."""
    d = h.ndim
    theta = eps ** 2 * float(np.sum(h ** 2)) / d
    g = h
    vs = []
    for n in range(d):
        l, s, _ = np.linalg.svd(unfold(g, n), full_matrices=False)
        tail = np.concatenate([np.cumsum((s ** 2)[::-1])[::-1][1:], [0.0]])
        r = int(np.argmax(tail <= theta)) + 1
        p = l[:, :r]
        vs.append(p)
        g = ttm(g, p.T, n)
    return g, vs


def effective_subranks(tsum: dict, eps: float, p) -> list:
    """Stage 1, phase 1 of Algorithm 3: V_n = [||G^(i)|| U_n^(i)]_i,
    eigenvalues of V_n^T V_n clipped at 0 and sorted, smallest r with
    discarded sum <= eps^2/d * total, plus oversampling p_n.  The summands
    are c_i X^(i) (coefficients scale the cores), so the weight of term i is
    |c_i| ||G^(i)||_F."""
    d = len(tsum["dims"])
    p = np.broadcast_to(np.asarray(p), (d,))
    coeffs = tsum.get("coeffs")
    if coeffs is None:
        coeffs = np.ones(len(tsum["cores"]))
    ell = []
    for n in range(d):
        v = np.concatenate([abs(float(c)) * np.sqrt(np.sum(g ** 2)) * us[n]
                            for c, g, us in zip(coeffs, tsum["cores"], tsum["factors"])], axis=1)
        lam = np.sort(np.maximum(0.0, np.linalg.eigvalsh(v.T @ v)))[::-1]
        tau = eps ** 2 / d * float(np.sum(lam))
        tail = np.concatenate([np.cumsum(lam[::-1])[::-1][1:], [0.0]])
        r = int(np.argmax(tail <= tau)) + 1
        ell.append(r + int(p[n]))
    return ell
