"""Pins of the oracle's reverse-mode derivative of the solve (multigrid.solve_adjoint):
central finite differences in b and in the vertex coefficient, and the homogeneity of
u = A^{-1} b in k (degree -1), which fixes sum_v k_v dJ/dk_v = -J without differencing."""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg


def _setup(bc, seed=0):
    xyz, tri = dec.square_grid(2)
    h = omg.Hierarchy(xyz, tri, 2, bc=bc)
    rng = np.random.default_rng(seed)
    nv = h.fine.nv
    kv = np.exp(0.3 * rng.standard_normal(nv))
    h.set_vertex_coeff(kv)
    b = h.rhs(rng.standard_normal(nv))
    g = rng.standard_normal(nv)
    if bc == "dirichlet":
        g[h.fine.bnd] = 0.0
    return h, kv, b, g


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_grad_k_finite_differences(bc):
    h, kv, b, g = _setup(bc)
    u = omg.direct_solve(h, b)
    _, gk = omg.solve_adjoint(h, u, g)
    eps = 1e-6
    fd = np.zeros_like(kv)
    for v in range(len(kv)):
        for s in (1, -1):
            kp = kv.copy()
            kp[v] += s * eps
            h.set_vertex_coeff(kp)
            fd[v] += s * float(g @ omg.direct_solve(h, b)) / (2 * eps)
    h.set_vertex_coeff(kv)
    assert np.abs(fd - gk).max() <= 1e-6 * np.abs(gk).max()


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_grad_b_finite_differences(bc):
    h, kv, b, g = _setup(bc, 1)
    u = omg.direct_solve(h, b)
    lam, _ = omg.solve_adjoint(h, u, g)
    rng = np.random.default_rng(5)
    d = h.rhs(rng.standard_normal(len(b)))
    eps = 1e-4
    fd = (g @ omg.direct_solve(h, b + eps * d) - g @ omg.direct_solve(h, b - eps * d)) / (2 * eps)
    assert abs(fd - lam @ d) <= 1e-9 * abs(fd)


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_grad_k_homogeneity(bc):
    h, kv, b, g = _setup(bc, 2)
    u = omg.direct_solve(h, b)
    _, gk = omg.solve_adjoint(h, u, g)
    J = float(g @ u)
    assert abs(kv @ gk + J) <= 1e-12 * abs(J) * 10


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_grad_w_finite_differences_and_homogeneity(bc):
    """dJ/dw for the finest operator's edge weights (the Hodge weights star1 k): central
    differences on a sample of edges, including edges whose weight is 0 (the right-grid
    diagonals), and sum_e w_e dJ/dw_e = -J (u is homogeneous of degree -1 in w)."""
    h, kv, b, g = _setup(bc)
    u = omg.direct_solve(h, b)
    gw = omg.solve_adjoint_weights(h, u, g)
    lv = h.fine
    w0 = lv.w.copy()
    J = float(g @ u)
    assert abs(float(w0 @ gw) + J) <= 1e-10 * abs(J)
    rng = np.random.default_rng(5)
    zero = np.nonzero(w0 == 0.0)[0]
    edges = np.concatenate([rng.choice(len(w0), 10, replace=False), zero[:2]])
    eps = 1e-6
    fd = np.zeros(len(edges))
    for i, e in enumerate(edges):
        for s in (1, -1):
            lv.w = w0.copy()
            lv.w[e] += s * eps
            h._assemble()
            fd[i] += s * float(g @ omg.direct_solve(h, b)) / (2 * eps)
    lv.w = w0
    h._assemble()
    assert np.abs(fd - gw[edges]).max() <= 1e-6 * np.abs(gw).max()
