"""Reverse mode of the Khatri-Rao recompression (Stages 2-3 of Algorithm 5)
and the Tucker-form loss ||[[H; Q]] - T||_F^2 used by the gradient workload.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no gradients; the rules below are derived from the forward
definitions in the order the forward computes them:

  P_k^(i) = U_k^(i)^T Omega_k                               (factor sketch)
  V_n^(i) = G^(i)_(n) KR_n^(i),  KR_n^(i) = P_d (.) ... (.) P_1, skipping n
  Y_n     = sum_i c_i U_n^(i) V_n^(i)                        (term expansion)
  Y_n     = Q_n R_n, diag R_n > 0                            (thin QR)
  W_k^(i) = Q_k^T U_k^(i)
  H       = sum_i c_i G^(i) x_1 W_1^(i) ... x_d W_d^(i)      (core projection)

Adjoints, with X_bar the gradient of the loss with respect to X:
  G_bar^(i)   += c_i H_bar x_k W_k^(i)T (all k)
  W_bar_k^(i)  = c_i (H_bar x_{j != k} W_j^(i)T)_(k) G^(i)_(k)^T
  Q_bar_k     += sum_i U_k^(i) W_bar_k^(i)T,   U_bar_k^(i) += Q_k W_bar_k^(i)
  Y_bar_n      = (Q_bar_n + Q_n copyltu(M)) R_n^-T,  M = -Q_bar_n^T Q_n
                 (R_bar = 0; copyltu keeps the lower triangle and mirrors it)
  U_bar_n^(i) += c_i Y_bar_n V_n^(i)T,   V_bar_n^(i) = c_i U_n^(i)T Y_bar_n
  G_bar^(i)_(n) += V_bar_n^(i) KR_n^(i)T
  P_bar_k^(i)  = sum_{n != k} (G^(i)_(k) KR of P_j (j != k, n) and V_bar_n at mode n)
  U_bar_k^(i) += Omega_k P_bar_k^(i)T
Every rule is checked against central finite differences in FP64.
"""
import numpy as np

from .omega import omegas as make_omegas
from .recompress import thin_qr
from .tensor import fold, khatri_rao_list, ttm, unfold


# ------------------------------------------------------------------ forward
def forward(tsum: dict, m: int, seed: int, omegas=None) -> dict:
    """KRP recompression (Algorithm 5, Stages 2-3) keeping the intermediates."""
    d = len(tsum["dims"])
    if omegas is None:
        omegas = make_omegas(seed, tsum["dims"], [m] * d)
    c = tsum["coeffs"]
    P = [[us[k].T @ omegas[k] for k in range(d)] for us in tsum["factors"]]
    V = []
    for i, g in enumerate(tsum["cores"]):
        row = []
        for n in range(d):
            kr = khatri_rao_list([P[i][j] for j in reversed(range(d)) if j != n])
            row.append(unfold(g, n) @ kr)
        V.append(row)
    Y = [sum(c[i] * tsum["factors"][i][n] @ V[i][n] for i in range(len(c))) for n in range(d)]
    QR = [thin_qr(y) for y in Y]
    Q = [q for q, _ in QR]
    R = [r for _, r in QR]
    W = [[Q[k].T @ us[k] for k in range(d)] for us in tsum["factors"]]
    H = 0
    for i, g in enumerate(tsum["cores"]):
        t = g
        for k in range(d):
            t = ttm(t, W[i][k], k)
        H = H + c[i] * t
    return {"omegas": omegas, "P": P, "V": V, "Y": Y, "Q": Q, "R": R, "W": W, "H": H}


# ------------------------------------------------------------------ loss
def tucker_loss(H, Q, target: dict):
    """L = ||[[H; Q]]||^2 - 2 <[[H; Q]], T> + ||T||^2 for a Tucker target T,
    with its gradients with respect to H and every Q_k (no orthonormality
    assumed, so the Q gradient is exact)."""
    d = H.ndim
    tg = target["cores"][0]
    tu = target["factors"][0]
    A = [q.T @ q for q in Q]
    B = [Q[k].T @ tu[k] for k in range(d)]
    HA = H
    for k in range(d):
        HA = ttm(HA, A[k], k)
    TB = tg
    for k in range(d):
        TB = ttm(TB, B[k], k)
    TT = tg
    for k in range(d):
        TT = ttm(TT, tu[k].T @ tu[k], k)
    loss = float(np.sum(H * HA) - 2.0 * np.sum(H * TB) + np.sum(tg * TT))
    H_bar = 2.0 * HA - 2.0 * TB
    Q_bar = []
    for k in range(d):
        C = H
        for j in range(d):
            if j != k:
                C = ttm(C, A[j], j)
        A_bar = unfold(H, k) @ unfold(C, k).T          # d<H, H x A>/dA_k
        Tk = tg
        for j in range(d):
            if j != k:
                Tk = ttm(Tk, B[j], j)
        B_bar = unfold(H, k) @ unfold(Tk, k).T          # d<H, T x B>/dB_k
        Q_bar.append(Q[k] @ (A_bar + A_bar.T) - 2.0 * tu[k] @ B_bar.T)
    return loss, H_bar, Q_bar


# ------------------------------------------------------------------ adjoints
def copyltu(M):
    """Symmetric matrix built from the lower triangle of M."""
    low = np.tril(M)
    return low + np.tril(M, -1).T


def qr_adjoint(Q, R, Q_bar):
    """Y_bar for Y = Q R (full column rank, diag R > 0) given Q_bar and R_bar = 0."""
    M = -Q_bar.T @ Q
    Z = Q_bar + Q @ copyltu(M)
    return np.linalg.solve(R, Z.T).T                   # Z R^-T


def backward(tsum: dict, fw: dict, H_bar, Q_bar):
    """Gradients of the loss with respect to every core and factor."""
    d = len(tsum["dims"])
    s = len(tsum["cores"])
    c = tsum["coeffs"]
    Q, R, W, P, V = fw["Q"], fw["R"], fw["W"], fw["P"], fw["V"]
    G_bar = [np.zeros_like(g) for g in tsum["cores"]]
    U_bar = [[np.zeros_like(u) for u in us] for us in tsum["factors"]]
    Qb = [np.array(q, dtype=np.float64) for q in Q_bar]
    # core projection
    for i, g in enumerate(tsum["cores"]):
        t = H_bar
        for k in range(d):
            t = ttm(t, W[i][k].T, k)
        G_bar[i] += c[i] * t
        for k in range(d):
            Z = H_bar
            for j in range(d):
                if j != k:
                    Z = ttm(Z, W[i][j].T, j)
            Wb = c[i] * unfold(Z, k) @ unfold(g, k).T
            Qb[k] += tsum["factors"][i][k] @ Wb.T
            U_bar[i][k] += Q[k] @ Wb
    # thin QR
    Y_bar = [qr_adjoint(Q[n], R[n], Qb[n]) for n in range(d)]
    # term expansion and core sketch
    P_bar = [[np.zeros_like(P[i][k]) for k in range(d)] for i in range(s)]
    for i, g in enumerate(tsum["cores"]):
        for n in range(d):
            U_bar[i][n] += c[i] * Y_bar[n] @ V[i][n].T
            Vb = c[i] * tsum["factors"][i][n].T @ Y_bar[n]
            kr = khatri_rao_list([P[i][j] for j in reversed(range(d)) if j != n])
            G_bar[i] += fold(Vb @ kr.T, n, g.shape)
            for k in range(d):
                if k == n:
                    continue
                F = [Vb if j == n else P[i][j] for j in range(d)]
                kr_k = khatri_rao_list([F[j] for j in reversed(range(d)) if j != k])
                P_bar[i][k] += unfold(g, k) @ kr_k
    # factor sketch
    for i in range(s):
        for k in range(d):
            U_bar[i][k] += fw["omegas"][k] @ P_bar[i][k].T
    return G_bar, U_bar


def loss_and_grad(tsum: dict, m: int, seed: int, target: dict):
    """Loss of the gradient workload and its gradients (cores, factors)."""
    fw = forward(tsum, m, seed)
    loss, H_bar, Q_bar = tucker_loss(fw["H"], fw["Q"], target)
    G_bar, U_bar = backward(tsum, fw, H_bar, Q_bar)
    return loss, G_bar, U_bar, fw


def loss_only(tsum: dict, m: int, seed: int, target: dict, omegas=None) -> float:
    fw = forward(tsum, m, seed, omegas)
    return tucker_loss(fw["H"], fw["Q"], target)[0]
