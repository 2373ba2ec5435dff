"""Pins of the oracle's multicolour Gauss-Seidel smoother (multigrid.greedy_colors,
gauss_seidel, smoother="gs").

* Colouring: no two coupled vertices share a colour, each colour is the smallest one not used
  by a lower-numbered neighbour (checked by brute force), and on the right-triangle grid (the
  5-point operator once the zero diagonal couplings are dropped) the interior colours form the
  red-black checkerboard of the grid coordinates (i, j).
* One sweep equals lexicographic Gauss-Seidel in the order sorted by (colour, id): the forward
  sweep is x + (D + L)^{-1} (b - A x) and the backward sweep x + (D + U)^{-1} (b - A x), with
  L, U the strict triangles of the permuted operator (triangular solves, not the sweep code).
* The cycle with forward pre-smoothing and backward post-smoothing is symmetric:
  <M u, v> = <u, M v>, which CG preconditioning needs.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import dec
from oracle import multigrid as omg
import workloads as W


def _square(nsub=3, base=4):
    xyz, tri = dec.square_grid(base)
    return omg.Hierarchy(xyz, tri, nsub)


def _sphere(nsub=3):
    xyz, tri = dec.icosahedron()
    return omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")


@pytest.mark.parametrize("make", [_square, _sphere])
def test_coloring_valid_and_greedy(make):
    h = make()
    A = sp.csr_matrix(h.fine.A, copy=True)
    A.setdiag(0.0)
    A.eliminate_zeros()
    c = h.colors(h.top)
    for i in range(A.shape[0]):
        nb = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert not np.any(c[nb] == c[i])
        lower = {int(c[j]) for j in nb if j < i}
        assert c[i] == min(set(range(len(lower) + 1)) - lower)


def test_red_black_on_right_grid():
    h = _square()
    n = int(round(np.sqrt(h.fine.nv))) - 1
    c = h.colors(h.top)
    assert c.max() == 1
    ij = np.rint(h.fine.xyz[:, :2] * n).astype(int)
    parity = (ij[:, 0] + ij[:, 1]) % 2
    inner = ~h.fine.bnd
    # a connected bipartite graph has exactly two 2-colourings: the checkerboard or its swap
    assert np.all(c[inner] == parity[inner]) or np.all(c[inner] == 1 - parity[inner])


@pytest.mark.parametrize("make", [_square, _sphere])
@pytest.mark.parametrize("backward", [False, True])
def test_sweep_is_permuted_lexicographic(make, backward):
    h = make()
    A = sp.csr_matrix(h.fine.A)
    c = h.colors(h.top)
    n = A.shape[0]
    b = W.normal(n, 11)
    x0 = W.normal(n, 12)
    order = np.lexsort((np.arange(n), c))          # by colour, then id
    Ap = A[order][:, order]
    if backward:
        T = sp.triu(Ap, format="csr")
    else:
        T = sp.tril(Ap, format="csr")
    dx = spla.spsolve_triangular(T, (b - A @ x0)[order], lower=not backward)
    ref = x0.copy()
    ref[order] += dx
    x = omg.gauss_seidel(A, b, x0, c, 1, backward=backward)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("make", [_square, _sphere])
@pytest.mark.parametrize("kind", ["V", "W"])
def test_gs_cycle_symmetric(make, kind):
    h = make()
    n = h.fine.nv
    u, v = W.normal(n, 13), W.normal(n, 14)
    if h.bc == "dirichlet":
        u[h.fine.bnd] = 0.0
        v[h.fine.bnd] = 0.0
    else:
        u -= u.mean()
        v -= v.mean()
    Mu = omg.mgcycle(h, u, kind=kind, smoother="gs")
    Mv = omg.mgcycle(h, v, kind=kind, smoother="gs")
    assert abs(Mu @ v - u @ Mv) <= 1e-12 * abs(Mu @ v)


def test_gs_converges_faster_than_jacobi_per_cycle():
    h = _square(4)
    b = h.rhs(W.manufactured_c1(h.fine.xyz))
    _, kj, _ = omg.mg_solve(h, b)
    _, kg, _ = omg.mg_solve(h, b, smoother="gs")
    assert kg < kj
