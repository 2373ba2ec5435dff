"""Pins of the oracle's cubic (1-to-9) subdivision (dec.subdivide_cubic) and of mixed
binary/cubic hierarchies.

* Counts: V' = V + 2E + T, E' = 3E + 9T, T' = 9T; the paper's 105,625 vertices after 4 cubic
  subdivisions of the 4x4-cell square (tests/golden/paper_counts_cubic.txt).
* Geometry: flat children have the parent's orientation and 1/9 of its area; fine coordinates
  are M(f)^T applied to the coarse ones (barycentric consistency).
* Transfers: rows of M(f)^T sum to 1; linear functions are reproduced; the Galerkin product
  P^T L_f P equals the rediscretised L_c on flat meshes (nested piecewise-linear spaces).
* Functoriality (Prop. 2): for binary then cubic subdivision, M(g o f)^T = M(g)^T M(f)^T equals
  the barycentric coordinates of every fine vertex in the base mesh found by point location.
* Right-triangle grids stay right-triangle grids: star1 in {0, 1/2, 1} and L is the 5-point
  stencil, up to the rounding of coordinates in thirds.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dec
from oracle import multigrid as omg
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tri_area(xyz, tri):
    p, q, r = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    return 0.5 * ((q[:, 0] - p[:, 0]) * (r[:, 1] - p[:, 1]) - (q[:, 1] - p[:, 1]) * (r[:, 0] - p[:, 0]))


def test_counts_and_paper_vertices():
    xyz, tri = dec.square_grid(4)
    lv = omg.Level(xyz, tri)
    fxyz, ftri, _ = dec.subdivide_cubic(xyz, tri, lv.edges, lv.tri_edges)
    f = omg.Level(fxyz, ftri)
    assert f.nv == lv.nv + 2 * lv.ne + lv.nt
    assert f.ne == 3 * lv.ne + 9 * lv.nt
    assert f.nt == 9 * lv.nt
    rows = [list(map(int, l.split())) for l in open(os.path.join(GOLDEN, "paper_counts_cubic.txt"))
            if l.strip() and not l.startswith("#")]
    for base, nsub, V in rows:
        xyz, tri = dec.square_grid(base)
        nv, ne, nt = len(xyz), 3 * base * base + 2 * base, 2 * base * base
        for _ in range(nsub):
            nv, ne, nt = nv + 2 * ne + nt, 3 * ne + 9 * nt, 9 * nt
        assert nv == V
    h = omg.Hierarchy(*dec.square_grid(4), 2, schemes="cc")
    assert h.fine.nv == (4 * 9 + 1) ** 2


def test_geometry_and_barycentric_consistency():
    xyz, tri = dec.square_grid(3)
    xyz = xyz + 0.05 * np.column_stack([np.sin(7 * xyz[:, 1]), np.cos(5 * xyz[:, 0]), 0 * xyz[:, 0]])
    lv = omg.Level(xyz, tri)
    fxyz, ftri, Mt = dec.subdivide_cubic(xyz, tri, lv.edges, lv.tri_edges)
    a_c = _tri_area(xyz, tri)
    a_f = _tri_area(fxyz, ftri).reshape(-1, 9)
    assert np.all(a_f > 0)
    assert np.allclose(a_f, a_c[:, None] / 9.0, rtol=1e-12, atol=0)
    assert np.allclose(Mt @ xyz, fxyz, rtol=0, atol=1e-15)
    assert np.allclose(np.asarray(Mt.sum(axis=1)).ravel(), 1.0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("schemes", ["c", "cc", "bc", "cb"])
def test_galerkin_and_linear_reproduction(schemes):
    xyz, tri = dec.square_grid(3)
    h = omg.Hierarchy(xyz, tri, len(schemes), bc="natural", schemes=schemes)
    for l in range(1, h.top + 1):
        P = sp.csr_matrix(h.levels[l].Mt)
        G = (P.T @ h.levels[l].L @ P).toarray()
        Lc = h.levels[l - 1].L.toarray()
        assert np.abs(G - Lc).max() <= 1e-12 * np.abs(Lc).max()
        lin = 0.3 + 1.7 * h.levels[l - 1].xyz[:, 0] - 0.9 * h.levels[l - 1].xyz[:, 1]
        lin_f = 0.3 + 1.7 * h.levels[l].xyz[:, 0] - 0.9 * h.levels[l].xyz[:, 1]
        assert np.abs(P @ lin - lin_f).max() <= 1e-14


def _point_location(base_xyz, base_tri, pts):
    """Barycentric coordinates of each point in the base triangle containing it (brute force)."""
    out = np.zeros((len(pts), len(base_xyz)))
    for i, p in enumerate(pts):
        for t in base_tri:
            a, b, c = base_xyz[t[0], :2], base_xyz[t[1], :2], base_xyz[t[2], :2]
            T = np.column_stack([b - a, c - a])
            lam = np.linalg.solve(T, p[:2] - a)
            l0 = 1.0 - lam.sum()
            if min(l0, lam[0], lam[1]) >= -1e-12:
                out[i, t[0]], out[i, t[1]], out[i, t[2]] = l0, lam[0], lam[1]
                break
    return out


def test_functoriality_binary_then_cubic():
    xyz, tri = dec.square_grid(2)
    h = omg.Hierarchy(xyz, tri, 2, schemes="bc")
    comp = (h.levels[2].Mt @ h.levels[1].Mt).toarray()
    ref = _point_location(xyz, tri, h.fine.xyz)
    assert np.abs(comp - ref).max() <= 1e-13


def test_right_grid_stays_five_point():
    h = omg.Hierarchy(*dec.square_grid(2), 2, schemes="cc")
    s1 = h.fine.star1
    near = np.min(np.abs(s1[:, None] - np.array([0.0, 0.5, 1.0])[None, :]), axis=1)
    assert near.max() <= 1e-13
    n = 2 * 9
    L = h.fine.L.toarray()
    ij = np.rint(h.fine.xyz[:, :2] * n).astype(int)
    for v in range(h.fine.nv):
        i, j = ij[v]
        if 0 < i < n and 0 < j < n:
            assert abs(L[v, v] - 4.0) <= 1e-13
            nb = [u for u in range(h.fine.nv) if abs(ij[u][0] - i) + abs(ij[u][1] - j) == 1]
            for u in nb:
                assert abs(L[v, u] + 1.0) <= 1e-13
            assert abs(L[v].sum()) <= 1e-13
