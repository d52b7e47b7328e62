"""NDG forward-Euler workload of Section 5.3: the transport equation
f_t + xi_x f_x = 0 on x in [0, 2 pi) (periodic), discretised in x by a
nodal discontinuous Galerkin method with upwind fluxes, each nodal value a
third-order Tucker tensor over the velocity grid (xi_x, xi_y, xi_z).

This module only describes the workload: the DG operator's coefficients,
the velocity grid, the rank-6 initial condition of Section 5.3 as Tucker
tensors, and, for one forward-Euler step, which Tucker tensors each node's
update sums (with their coefficients and the velocity factor that scales
their first mode).  It holds none of the recompression arithmetic: a caller
materialises each term (the state's core and factors, the first factor's
rows multiplied by the named velocity factor) and recompresses the sums.

Discretisation (Section 5.3, eq. for the weak form with the Lagrange basis
on the k+1 Gauss-Legendre nodes of each element): with the element width h,
nodes z_q and weights w_q on [-1, 1], L_q the Lagrange polynomials, and
xi+ = max(xi_x, 0), xi- = min(xi_x, 0),
  (h/2) w_p dC^i_p/dt = - L_p(1) [xi+ sum_q L_q(1) C^i_q + xi- sum_q L_q(-1) C^{i+1}_q]
                        + L_p(-1) [xi+ sum_q L_q(1) C^{i-1}_q + xi- sum_q L_q(-1) C^i_q]
                        + xi_x sum_q w_q L_p'(z_q) C^i_q,
and forward Euler C^{n+1} = C^n + dt dC/dt.  Writing xi_x = xi+ + xi- folds
the volume term into the two flux directions, so the update of node (i, p)
sums 1 + 4 (k+1) Tucker tensors: the state itself, xi+ C^i_q and xi- C^i_q
for every q, xi+ C^{i-1}_q and xi- C^{i+1}_q.  (The paper's count, 2 (k+1)
terms per stencil member and three members, also counts the upwind
direction that vanishes at each neighbour.)
"""
from __future__ import annotations

import numpy as np

# Section 5.3, rank-6 initial condition: (A_alpha, omega_alpha, beta_alpha)
A = (1 / 2, 1 / 4, 3 / 20, 1 / 5, 9 / 10, 1 / 100)
OMEGA = (1.0, 1 / 100, 2.0, 1 / 5, 7 / 10, 10.0)
BETA = ((-1 / 20, 0, 0), (1 / 20, 0, 0), (0, -3 / 40, 0), (0, 3 / 40, 0), (0, 0, -1 / 40),
        (0, 0, 1 / 40))


def lagrange(z: np.ndarray):
    """Values at -1 and +1 and the derivative matrix D[p, q] = L_p'(z_q) of
    the Lagrange polynomials on the nodes z."""
    n = len(z)

    def value(p, t):
        v = 1.0
        for j in range(n):
            if j != p:
                v *= (t - z[j]) / (z[p] - z[j])
        return v

    def deriv(p, t):
        tot = 0.0
        for m in range(n):
            if m == p:
                continue
            term = 1.0 / (z[p] - z[m])
            for j in range(n):
                if j != p and j != m:
                    term *= (t - z[j]) / (z[p] - z[j])
            tot += term
        return tot
    lm = np.array([value(p, -1.0) for p in range(n)])
    lp = np.array([value(p, 1.0) for p in range(n)])
    D = np.array([[deriv(p, z[q]) for q in range(n)] for p in range(n)])
    return lm, lp, D


def setup(nx: int = 32, k: int = 1, nxi: int = 100, xi_max: float = 12.0,
          dt_factor: float | None = None) -> dict:
    """Mesh, basis, velocity grid and time step.  The time step follows the
    speed-up runs of Section 5.3: dt = theta h with theta = 0.1 / ((2k + 1)
    xi_max) unless dt_factor overrides theta."""
    z, w = np.polynomial.legendre.leggauss(k + 1)
    h = 2 * np.pi / nx
    x = ((np.arange(nx) + 0.5) * h)[:, None] + 0.5 * h * z[None, :]
    lm, lp, D = lagrange(z)
    hv = 2 * xi_max / nxi
    xi = -xi_max + (np.arange(nxi) + 0.5) * hv
    theta = 0.1 / ((2 * k + 1) * xi_max) if dt_factor is None else dt_factor
    return {"nx": nx, "k": k, "nxi": nxi, "xi_max": xi_max, "z": z, "w": w, "h": h, "x": x,
            "lm": lm, "lp": lp, "D": D, "xi": xi, "dt": theta * h,
            "scale": {"plus": np.maximum(xi, 0.0), "minus": np.minimum(xi, 0.0)}}


def initial_state(st: dict) -> list:
    """The rank-6 initial condition at every node, node index i * (k+1) + p:
    a Tucker tensor with the diagonal 6 x 6 x 6 core of the coefficients
    (1 + A_a sin(omega_a x)) / (2 pi)^(3/2) and first/second/third factors
    exp(-(xi - beta_a,d)^2 / 2) (one column per a)."""
    xi = st["xi"]
    fac = [np.asfortranarray(np.stack([np.exp(-0.5 * (xi - b[d]) ** 2) for b in BETA], axis=1))
           for d in range(3)]
    out = []
    for i in range(st["nx"]):
        for p in range(st["k"] + 1):
            xv = st["x"][i, p]
            core = np.zeros((6, 6, 6), order="F")
            for a in range(6):
                core[a, a, a] = (1 + A[a] * np.sin(OMEGA[a] * xv)) / (2 * np.pi) ** 1.5
            out.append({"core": core, "factors": [f.copy(order="F") for f in fac]})
    return out


def euler_terms(st: dict) -> list:
    """For every node, the terms of its forward-Euler update: a list of
    (coefficient, source node, velocity factor of the first mode or None),
    the factor being "plus" (xi+) or "minus" (xi-)."""
    nx, k1 = st["nx"], st["k"] + 1
    lm, lp, D, w, h, dt = st["lm"], st["lp"], st["D"], st["w"], st["h"], st["dt"]
    out = []
    for i in range(nx):
        right, left = (i + 1) % nx, (i - 1) % nx
        for p in range(k1):
            s = dt * 2.0 / (h * w[p])
            terms = [(1.0, i * k1 + p, None)]
            for q in range(k1):
                vol = w[q] * D[p, q]
                terms.append((s * (vol - lp[p] * lp[q]), i * k1 + q, "plus"))
                terms.append((s * (vol + lm[p] * lm[q]), i * k1 + q, "minus"))
                terms.append((s * lm[p] * lp[q], left * k1 + q, "plus"))
                terms.append((-s * lp[p] * lm[q], right * k1 + q, "minus"))
            out.append(terms)
    return out


def step_matrix(st: dict, terms: list, xi0: float) -> np.ndarray:
    """The forward-Euler update of the nodal values at one velocity xi_x =
    xi0 as a dense matrix: C^{n+1} = M C^n over the N_x (k+1) nodes (the
    per-node sums evaluated on one velocity grid point)."""
    scale = {None: 1.0, "plus": max(xi0, 0.0), "minus": min(xi0, 0.0)}
    n = len(terms)
    M = np.zeros((n, n))
    for a, tl in enumerate(terms):
        for c, src, kind in tl:
            M[a, src] += c * scale[kind]
    return M
