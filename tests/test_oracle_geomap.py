"""Pins of the oracle's hierarchies over given meshes and geometric maps (Sec. 2.2.1, Def. 4,
Prop. 2), and of the non-nested input workload (independently jittered grids whose maps come
from point location).

* Given the meshes and maps of a subdivision hierarchy, ``Hierarchy.from_maps`` rebuilds the
  same operators and the same cycle bit for bit.
* The jittered maps are valid global barycentric coordinates: 1 to 3 nonnegative entries per
  column spanning one coarse simplex, summing to 1, and reproducing the fine coordinates.
* On the non-nested hierarchy MG-PCG reaches the sparse direct solution, and stand-alone
  cycles contract at an h-independent rate.
* Composition (Prop. 2): the identity is neutral, composed maps keep partition of unity and
  linear reproduction.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dec
from oracle import multigrid as omg
import workloads as W


@pytest.fixture(scope="module")
def maps_input():
    return W.maps_workload()


def test_from_maps_reproduces_subdivision():
    xyz, tri = dec.square_grid(3)
    h = omg.Hierarchy(xyz, tri, 3, schemes="bcb")
    meshes = [(lv.xyz, lv.tri) for lv in h.levels]
    maps = [h.levels[l].Mt.T for l in range(1, h.top + 1)]
    g = omg.Hierarchy.from_maps(meshes, maps)
    for a, b in zip(g.levels, h.levels):
        assert (a.A != b.A).nnz == 0
    b = W.normal(h.fine.nv, 3)
    x0 = W.normal(h.fine.nv, 4)
    assert np.array_equal(omg.mgcycle(g, b, x0.copy()), omg.mgcycle(h, b, x0.copy()))


def test_jittered_maps_are_barycentric(maps_input):
    meshes, maps = maps_input
    for k, M in enumerate(maps):
        xc, tc = meshes[k]
        xf, _ = meshes[k + 1]
        M = sp.csc_matrix(M)
        assert M.shape == (len(xc), len(xf))
        assert M.data.min() > 0.0
        counts = np.diff(M.indptr)
        assert counts.min() >= 1 and counts.max() <= 3
        assert np.abs(np.asarray(M.sum(axis=0)).ravel() - 1.0).max() <= 1e-15
        assert np.abs(M.T @ xc - xf).max() <= 1e-15
        tris = {tuple(sorted(t)) for t in tc.tolist()}
        for j in range(len(xf)):
            r = sorted(M.indices[M.indptr[j]:M.indptr[j + 1]].tolist())
            assert any(set(r) <= set(t) for t in tris) if len(r) > 1 else True
        # the maps are not nested: interior fine vertices are not coarse vertices
        assert np.count_nonzero(counts == 3) > len(xf) // 2


@pytest.mark.parametrize("bc", ["dirichlet", "natural"])
def test_nonnested_solve_reaches_direct_solution(maps_input, bc):
    meshes, maps = maps_input
    h = omg.Hierarchy.from_maps(meshes, maps, bc=bc)
    b = h.rhs(W.normal(h.fine.nv, 5))
    if bc == "natural":
        b -= b.mean()
    x, k, _ = omg.mg_pcg(h, b)
    xd = omg.direct_solve(h, b)
    assert k <= 20
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert omg.rel_residual(h, b, x) <= 1e-10


def test_nonnested_contraction_is_h_independent(maps_input):
    meshes, maps = maps_input
    rates = []
    for top in (3, 4):
        h = omg.Hierarchy.from_maps(meshes[:top + 1], maps[:top])
        b = h.rhs(W.normal(h.fine.nv, 6))
        _, k, hist = omg.mg_solve(h, b)
        rates.append((hist[-1] / hist[-4]) ** (1 / 3))
    assert max(rates) < 0.45 and abs(rates[0] - rates[1]) < 0.1


def test_composition(maps_input):
    meshes, maps = maps_input
    M01 = sp.csc_matrix(maps[0])
    M12 = sp.csc_matrix(maps[1])
    # identity is neutral (Prop. 2: M(id) = I)
    I0 = sp.identity(M01.shape[0], format="csc")
    assert (omg.compose(I0, M01) != M01).nnz == 0
    C = omg.compose(M01, M12)
    assert C.shape == (len(meshes[0][0]), len(meshes[2][0]))
    assert C.data.min() > 0.0
    assert np.abs(np.asarray(C.sum(axis=0)).ravel() - 1.0).max() <= 1e-15
    assert np.abs(C.T @ meshes[0][0] - meshes[2][0]).max() <= 1e-15
    # nested maps compose to point location in the coarsest mesh (binary then cubic)
    xyz, tri = dec.square_grid(2)
    h = omg.Hierarchy(xyz, tri, 2, schemes="bc")
    C = omg.compose(h.levels[1].Mt.T, h.levels[2].Mt.T).toarray()
    loc = W.grid_point_location(xyz, tri.astype(np.int32), 2, h.fine.xyz).toarray()
    assert np.abs(C - loc).max() <= 1e-15
