"""The NDG transport workload (Section 5.3) against what the discretisation
fixes: the upwind DG scheme keeps constants, conserves mass on the periodic
mesh, converges at order k + 1 (the paper's NDG1-3 check), the initial
Tucker states hold the stated rank-6 condition, and the Tucker terms of a
node's update (velocity factors on the first mode) evaluate, point by point
in xi_x, to the scalar scheme's update."""
import numpy as np
import pytest

from synth import ndg
from oracle import tensor as T


def test_lagrange_basis():
    for k in range(4):
        z, _ = np.polynomial.legendre.leggauss(k + 1)
        lm, lp, D = ndg.lagrange(z)
        # interpolation of z^j at the ends and of its derivative at the nodes
        # is exact up to degree k (D[p, q] = L_p'(z_q))
        for j in range(k + 1):
            assert abs(lm @ z ** j - (-1.0) ** j) < 1e-13 and abs(lp @ z ** j - 1.0) < 1e-13
            deriv = j * z ** (j - 1) if j else np.zeros_like(z)
            assert np.allclose((z ** j) @ D, deriv, atol=1e-12)


@pytest.mark.parametrize("k", [0, 1, 2])
def test_constants_and_mass(k):
    st = ndg.setup(nx=6, k=k, nxi=4, xi_max=2.0)
    terms = ndg.euler_terms(st)
    assert all(len(t) == 1 + 4 * (k + 1) for t in terms)
    wts = np.tile(st["w"], st["nx"]) * st["h"] / 2
    rng = np.random.default_rng(0)
    for xi0 in (-1.5, -0.3, 0.0, 0.7, 2.0):
        M = ndg.step_matrix(st, terms, xi0)
        one = np.ones(M.shape[0])
        assert np.allclose(M @ one, one, atol=1e-13)  # f = const is a steady state
        c = rng.standard_normal(M.shape[0])
        assert abs(wts @ (M @ c) - wts @ c) < 1e-12 * np.abs(c).sum()  # mass


@pytest.mark.parametrize("k", [0, 1, 2])
def test_convergence_order(k):
    """L1 error of the smooth solution 1 + sin(x)/2 after T = 1 at xi_x = 1,
    dt = 0.1 / (2k + 3) h^(k+1): observed order k + 1."""
    errs = []
    for nx in (8, 16, 32):
        st = ndg.setup(nx=nx, k=k, nxi=4, xi_max=1.0)
        dt = 0.1 / (2 * k + 3) * st["h"] ** (k + 1)
        nst = int(np.ceil(1.0 / dt))
        st["dt"] = 1.0 / nst
        M = ndg.step_matrix(st, ndg.euler_terms(st), 1.0)
        x = st["x"].reshape(-1)
        c = 1 + 0.5 * np.sin(x)
        for _ in range(nst):
            c = M @ c
        wts = np.tile(st["w"], nx) * st["h"] / 2
        errs.append(np.sum(wts * np.abs(c - (1 + 0.5 * np.sin(x - 1.0)))))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > k + 1 - 0.15, (errs, orders)


def dense(state):
    return T.tucker_to_dense(state["core"], state["factors"])


def test_initial_condition():
    st = ndg.setup(nx=4, k=1, nxi=10, xi_max=3.0)
    states = ndg.initial_state(st)
    xi = st["xi"]
    X, Y, Z = np.meshgrid(xi, xi, xi, indexing="ij")
    for a in (0, 5):
        x = st["x"].reshape(-1)[a]
        want = sum((1 + A * np.sin(w * x)) / (2 * np.pi) ** 1.5 *
                   np.exp(-((X - b[0]) ** 2 + (Y - b[1]) ** 2 + (Z - b[2]) ** 2) / 2)
                   for A, w, b in zip(ndg.A, ndg.OMEGA, ndg.BETA))
        assert np.allclose(dense(states[a]), want, rtol=1e-13, atol=1e-16)


def test_terms_match_scalar_scheme():
    """Each node's sum of Tucker terms, evaluated densely, equals at every
    xi_x grid point the scalar scheme's update of that slice."""
    st = ndg.setup(nx=3, k=1, nxi=8, xi_max=3.0)
    states = ndg.initial_state(st)
    rng = np.random.default_rng(1)
    for s in states:  # perturb so that nodes differ in all modes
        s["core"] = s["core"] + 1e-3 * rng.standard_normal(s["core"].shape)
    terms = ndg.euler_terms(st)
    dn = [dense(s) for s in states]
    for a, tl in enumerate(terms):
        tot = 0
        for c, src, kind in tl:
            us = list(states[src]["factors"])
            if kind is not None:
                us[0] = st["scale"][kind][:, None] * us[0]
            tot = tot + c * T.tucker_to_dense(states[src]["core"], us)
        for j, xi0 in enumerate(st["xi"]):
            M = ndg.step_matrix(st, terms, xi0)
            want = sum(M[a, b] * dn[b][j] for b in range(len(states)))
            assert np.allclose(tot[j], want, rtol=1e-12, atol=1e-15)
