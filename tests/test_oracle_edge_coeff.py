"""Pins of the oracle's edge-field Darcy coefficient (multigrid.Hierarchy.set_edge_coeff;
Sec. 3.2, Eq. dec_darcy with K given per edge): the finest level takes w = star1 k_e, and a
coarser edge the mean of the fine edges it was split into.

* For a coefficient that is linear in space, the edge field k_e = (k_lo + k_hi)/2 on the finest
  level coarsens to exactly the vertex rule on every level (a linear field's value at an edge
  point is the average of its endpoints'), on binary and on cubic subdivisions: the weights
  agree with set_vertex_coeff to rounding.
* A constant edge coefficient c scales every level's operator by c, so the solution is u/c.
* MG-PCG on a random positive edge field reaches the sparse direct solution.
"""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg
import workloads as W


def hier(schemes, bc="dirichlet"):
    xyz, tri = dec.square_grid(4)
    return omg.Hierarchy(xyz, tri, len(schemes), bc=bc, schemes=schemes)


@pytest.mark.parametrize("schemes", ["bbb", "cb", "bc"])
def test_linear_coefficient_matches_vertex_rule(schemes):
    a = hier(schemes)
    b = hier(schemes)
    xyz = a.fine.xyz
    kv = 1.0 + 0.3 * xyz[:, 0] + 0.2 * xyz[:, 1]
    a.set_vertex_coeff(kv)
    e = b.fine.edges
    b.set_edge_coeff(0.5 * (kv[e[:, 0]] + kv[e[:, 1]]))
    for la, lb in zip(a.levels, b.levels):
        assert np.abs(la.w - lb.w).max() <= 1e-14 * np.abs(la.w).max()
    assert np.array_equal(a.fine.w, b.fine.w)


def test_constant_coefficient_scales_the_solution():
    a = hier("bbb")
    b = hier("bbb")
    c = 2.5
    b.set_edge_coeff(np.full(b.fine.ne, c))
    for la, lb in zip(a.levels, b.levels):
        assert np.array_equal(lb.w, c * la.w)
    f = a.rhs(W.normal(a.fine.nv, 21))
    ua = omg.direct_solve(a, f)
    ub = omg.direct_solve(b, f)
    assert np.abs(ub - ua / c).max() <= 1e-13 * np.abs(ua).max()


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_mg_pcg_with_edge_coefficient(bc):
    h = hier("bbb", bc)
    ke = np.exp(0.5 * W.normal(h.fine.ne, 22))
    h.set_edge_coeff(ke)
    assert np.array_equal(h.fine.w, h.fine.star1 * ke)
    b = h.rhs(W.normal(h.fine.nv, 23))
    x, k, _ = omg.mg_pcg(h, b, rtol=1e-13)
    ref = omg.direct_solve(h, b)
    assert k < 40
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_maps_hierarchy_refuses_edge_coefficient():
    h = hier("b")
    meshes = [(lv.xyz, lv.tri) for lv in h.levels]
    h2 = omg.Hierarchy.from_maps(meshes, [h.fine.Mt.T])
    with pytest.raises(ValueError):
        h2.set_edge_coeff(np.ones(h2.fine.ne))
