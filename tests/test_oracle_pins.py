"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: numbers printed in the
paper (``tests/golden``), closed forms, invariants, textbook special cases, brute force on
tiny inputs.  No GPU.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dec
from oracle import multigrid as mg
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _square_hier(n, nsub, bc="dirichlet"):
    xyz, tri = dec.square_grid(n)
    return mg.Hierarchy(xyz, tri, nsub, bc=bc)


def _sphere_hier(nsub):
    xyz, tri = dec.icosahedron()
    return mg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")


def _read_golden(name):
    sections, cur = {}, None
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("["):
            cur = line.strip("[]")
            sections[cur] = []
            continue
        sections[cur].append([float(v) for v in line.split()])
    return {k: np.array(v) for k, v in sections.items()}


# ------------------------------------------------------------ topology
@pytest.mark.parametrize("maker", ["square", "sphere", "sheared"])
def test_dd_is_zero_exactly(maker):
    """d1 d0 = 0 in integers (the mimetic property stated in Sec. 1)."""
    if maker == "sphere":
        h = _sphere_hier(3)
    elif maker == "square":
        h = _square_hier(4, 3)
    else:
        xyz, tri = dec.square_grid(5)
        xyz[:, 0] += 0.5 * xyz[:, 1]
        h = mg.Hierarchy(xyz, tri, 2)
    for lv in h.levels:
        prod = (lv.d1 @ lv.d0).tocoo()
        assert prod.dtype.kind == "i"
        assert np.all(prod.data == 0)
        assert set(np.unique(lv.d0.data)) <= {-1, 1}
        assert np.all(np.asarray(abs(lv.d0).sum(axis=1)).ravel() == 2)


def test_edge_numbering_bruteforce():
    """Edge ids, orientation and triangle signs against an explicit loop over triangles."""
    xyz, tri = dec.square_grid(3)
    edges, tri_edges, tri_sign = dec.edges_of(tri, len(xyz))
    seen = {}
    for t, (a, b, c) in enumerate(tri.tolist()):
        for k, (u, v) in enumerate(((a, b), (b, c), (c, a))):
            key = (min(u, v), max(u, v))
            if key not in seen:
                seen[key] = len(seen)
            assert tri_edges[t, k] == seen[key]
            assert tri_sign[t, k] == (1 if u < v else -1)
    assert [tuple(e) for e in edges.tolist()] == sorted(seen, key=seen.get)


@pytest.mark.parametrize("n,nsub", [(4, 3), (3, 2), (8, 2)])
def test_square_counts_closed_form(n, nsub):
    h = _square_hier(n, nsub)
    for l, lv in enumerate(h.levels):
        m = n * 2 ** l
        assert (lv.nv, lv.ne, lv.nt) == ((m + 1) ** 2, 3 * m * m + 2 * m, 2 * m * m)
        assert lv.nv - lv.ne + lv.nt == 1
        cnt = np.bincount(lv.tri_edges.ravel(), minlength=lv.ne)
        assert set(np.unique(cnt)) == {1, 2}
        assert np.count_nonzero(cnt == 1) == 4 * m
        assert np.count_nonzero(lv.bnd) == 4 * m


def test_icosphere_counts_closed_form():
    h = _sphere_hier(4)
    for l, lv in enumerate(h.levels):
        assert (lv.nv, lv.ne, lv.nt) == (10 * 4 ** l + 2, 30 * 4 ** l, 20 * 4 ** l)
        assert lv.nv - lv.ne + lv.nt == 2
        cnt = np.bincount(lv.tri_edges.ravel(), minlength=lv.ne)
        assert np.all(cnt == 2)
        assert not lv.bnd.any()
        assert np.allclose(np.linalg.norm(lv.xyz, axis=1), 1.0, atol=1e-15)


def _topology_only(n, nsub):
    xyz, tri = dec.square_grid(n)
    edges, tri_edges, _ = dec.edges_of(tri, len(xyz))
    for _ in range(nsub):
        xyz, tri, _ = dec.subdivide(xyz, tri, edges, tri_edges)
        edges, tri_edges, _ = dec.edges_of(tri, len(xyz))
    return len(xyz), len(edges), len(tri)


def _paper_counts():
    rows = []
    for line in open(os.path.join(GOLDEN, "paper_counts.txt")):
        if line.strip() and not line.startswith("#"):
            f = line.split()
            rows.append((int(f[0]), int(f[1]), int(f[2]), int(f[3]), int(f[4]),
                         None if f[5] == "-" else int(f[5])))
    return rows


@pytest.mark.parametrize("row", _paper_counts(), ids=lambda r: f"{r[0]}x{r[0]}-sub{r[1]}")
def test_paper_mesh_counts(row):
    """Vertex/edge/triangle counts and nnz(L) printed in Sec. 3 (golden/paper_counts.txt)."""
    n, nsub, V, E, T, nnz = row
    if V > 100000:
        pytest.importorskip("scipy")
    assert _topology_only(n, nsub) == (V, E, T)
    if nnz is not None:
        h = _square_hier(n, nsub, bc="natural")
        L = h.fine.L
        # structural nonzeros: the diagonal plus both off-diagonal slots of every edge
        assert L.shape[0] + 2 * h.fine.ne == nnz
        Ls = sp.csr_matrix((np.ones(L.nnz), L.indices, L.indptr), shape=L.shape)
        assert Ls.nnz <= nnz


# ------------------------------------------------------------ Hodge stars
def _edge_kinds(lv):
    d = lv.xyz[lv.edges[:, 1]] - lv.xyz[lv.edges[:, 0]]
    axis = (np.abs(d[:, 0]) < 1e-15) | (np.abs(d[:, 1]) < 1e-15)
    cnt = np.bincount(lv.tri_edges.ravel(), minlength=lv.ne)
    return axis, cnt == 1


def test_star1_right_grid_exact():
    """Right-triangle grids: star1 is 1 on interior axis edges, 1/2 on boundary axis edges
    and 0 on the diagonals, bit-exactly (cot 45 = 1, cot 90 = 0)."""
    h = _square_hier(4, 3)
    for lv in h.levels:
        axis, bnd_e = _edge_kinds(lv)
        assert np.all(lv.star1[axis & ~bnd_e] == 1.0)
        assert np.all(lv.star1[axis & bnd_e] == 0.5)
        assert np.all(lv.star1[~axis] == 0.0)


def test_star1_equilateral():
    """Equilateral triangles: interior edges carry 2 * (1/2) cot 60 = 1/sqrt(3) and boundary
    edges half of it.  Shearing x -> x - y/2, y -> y sqrt(3)/2 makes both triangles of every
    cell equilateral."""
    xyz, tri = dec.square_grid(6)
    xyz[:, 0] = xyz[:, 0] - 0.5 * xyz[:, 1]
    xyz[:, 1] = xyz[:, 1] * math.sqrt(3) / 2
    lv = mg.Level(xyz, tri)
    cnt = np.bincount(lv.tri_edges.ravel(), minlength=lv.ne)
    lens = np.linalg.norm(lv.xyz[lv.edges[:, 1]] - lv.xyz[lv.edges[:, 0]], axis=1)
    assert np.allclose(lens, 1 / 6, rtol=1e-12)
    assert np.allclose(lv.star1[cnt == 2], 1 / math.sqrt(3), rtol=1e-12)
    assert np.allclose(lv.star1[cnt == 1], 0.5 / math.sqrt(3), rtol=1e-12)


def _circumcenter(a, b, c):
    u, v = b - a, c - a
    w = np.cross(u, v)
    return a + (np.dot(u, u) * np.cross(v, w) + np.dot(v, v) * np.cross(w, u)) / (2 * np.dot(w, w))


def test_stars_against_explicit_circumcentric_dual():
    """Brute force on a small perturbed (acute) mesh: dual edge lengths and dual cell areas
    built from explicit circumcenters and edge midpoints."""
    rng = np.random.default_rng(11)
    xyz, tri = dec.square_grid(4)
    xyz[:, 0] = xyz[:, 0] - 0.5 * xyz[:, 1]                # equilateral cells ...
    xyz[:, 1] = xyz[:, 1] * math.sqrt(3) / 2
    xyz[:, :2] += 0.01 * rng.standard_normal((len(xyz), 2))  # ... perturbed, still acute
    xyz[:, 2] = 0.03 * rng.standard_normal(len(xyz))      # non-flat: a surface in R^3
    lv = mg.Level(xyz, tri)
    P = lv.xyz
    for i, j, k in lv.tri.tolist():
        for a, b, c in ((i, j, k), (j, k, i), (k, i, j)):
            assert np.dot(P[b] - P[a], P[c] - P[a]) > 0   # every angle acute
    star1 = np.zeros(lv.ne)
    star0 = np.zeros(lv.nv)
    for t, (i, j, k) in enumerate(lv.tri.tolist()):
        P = lv.xyz
        c = _circumcenter(P[i], P[j], P[k])
        for a in (i, j, k):
            assert abs(np.linalg.norm(c - P[a]) - np.linalg.norm(c - P[i])) < 1e-12
        for s, (a, b) in enumerate(((i, j), (j, k), (k, i))):
            m = 0.5 * (P[a] + P[b])
            e = lv.tri_edges[t, s]
            star1[e] += np.linalg.norm(c - m) / np.linalg.norm(P[b] - P[a])
        for a, b, d in ((i, j, k), (j, k, i), (k, i, j)):
            mab, mad = 0.5 * (P[a] + P[b]), 0.5 * (P[a] + P[d])
            star0[a] += 0.5 * np.linalg.norm(np.cross(mab - P[a], c - P[a]))
            star0[a] += 0.5 * np.linalg.norm(np.cross(c - P[a], mad - P[a]))
    assert np.allclose(lv.star1, star1, rtol=1e-12, atol=1e-14)
    assert np.allclose(lv.star0, star0, rtol=1e-12, atol=1e-14)


def test_star_sums():
    """sum star0 = area; sum star1 |e|^2 = 2 area (each triangle contributes its area
    twice); on the icosphere sum star0 increases towards 4 pi."""
    h = _square_hier(4, 3)
    for lv in h.levels:
        lens2 = np.sum((lv.xyz[lv.edges[:, 1]] - lv.xyz[lv.edges[:, 0]]) ** 2, axis=1)
        assert abs(lv.star0.sum() - 1.0) < 1e-13
        assert abs((lv.star1 * lens2).sum() - 2.0) < 1e-13
        interior = ~lv.bnd
        hh = 1.0 / (4 * 2 ** h.levels.index(lv))
        assert np.allclose(lv.star0[interior], hh * hh, rtol=1e-13)
    hs = _sphere_hier(5)
    sums = [lv.star0.sum() for lv in hs.levels]
    assert all(a < b for a, b in zip(sums, sums[1:]))
    deficit = [4 * math.pi - v for v in sums]
    assert all(3.8 < a / b < 4.2 for a, b in zip(deficit[2:], deficit[3:]))   # O(h^2)
    assert min(lv.star1.min() for lv in hs.levels) > 0.3


# ------------------------------------------------------------ Laplacian
def _five_point(lv, n):
    ij = np.rint(lv.xyz[:, :2] * n).astype(int)
    idx = {(int(i), int(j)): v for v, (i, j) in enumerate(ij)}
    rows, cols, vals = [], [], []
    for v, (i, j) in enumerate(ij.tolist()):
        nb = [(i + 1, j), (i - 1, j), (i, j + 1), (i, j - 1)]
        nb = [idx[q] for q in nb if q in idx]
        # the natural (Neumann) 5-point stencil on the square: half-weights on boundary sides
        for q in nb:
            both_bnd = (ij[q][0] in (0, n) and i in (0, n) and ij[q][0] == i) or \
                       (ij[q][1] in (0, n) and j in (0, n) and ij[q][1] == j)
            wgt = 0.5 if both_bnd else 1.0
            rows += [v, v]
            cols += [q, v]
            vals += [-wgt, wgt]
    return sp.csr_matrix((vals, (rows, cols)), shape=(lv.nv, lv.nv))


def test_laplacian_is_five_point_stencil():
    """On right-triangle grids L equals the 5-point stencil (boundary sides weighted 1/2)."""
    h = _square_hier(4, 3, bc="natural")
    for l, lv in enumerate(h.levels):
        S = _five_point(lv, 4 * 2 ** l)
        assert abs(lv.L - S).max() == 0.0


def test_laplacian_properties():
    rng = np.random.default_rng(5)
    for h in (_square_hier(4, 2, bc="natural"), _sphere_hier(3)):
        L = h.fine.L
        assert abs(L - L.T).max() == 0.0
        assert np.abs(L @ np.ones(L.shape[0])).max() < 1e-12
        ev = np.linalg.eigvalsh(L.toarray())
        assert ev.min() > -1e-12
        assert np.count_nonzero(ev < 1e-10) == 1          # connected: kernel = constants
    # linear precision: (L p)_i = 0 for linear p at interior vertices of a flat mesh
    xyz, tri = dec.square_grid(6)
    interior = (xyz[:, 0] > 0) & (xyz[:, 0] < 1) & (xyz[:, 1] > 0) & (xyz[:, 1] < 1)
    xyz[interior, :2] += 0.03 * rng.standard_normal((interior.sum(), 2))
    lv = mg.Level(xyz, tri)
    L = dec.laplacian(lv.d0, lv.star1)
    p = 0.3 + 1.7 * xyz[:, 0] - 0.9 * xyz[:, 1]
    assert np.abs((L @ p)[~lv.bnd]).max() < 1e-13


# ------------------------------------------------------------ transfers
def test_single_triangle_example_golden():
    """Interpolation and the row-normalised restriction of the worked example
    (golden/single_triangle_transfer.txt)."""
    g = _read_golden("single_triangle_transfer.txt")
    xyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    tri = np.array([[0, 1, 2]])
    edges, tri_edges, _ = dec.edges_of(tri, 3)
    _, _, Mt = dec.subdivide(xyz, tri, edges, tri_edges)
    # our ids of the paper's order a, ab, b, bc, c, ca
    mid = {tuple(sorted(e)): 3 + k for k, e in enumerate(edges.tolist())}
    order = [0, mid[(0, 1)], 1, mid[(1, 2)], 2, mid[(0, 2)]]
    assert np.array_equal(Mt.toarray()[order], g["interpolation"])
    R = dec.paper_restriction(Mt).toarray()            # V_c x V_f, fine -> coarse
    assert np.array_equal(R.T[order], g["restriction"])
    assert np.allclose(R.sum(axis=1), 1.0)


def test_transfer_invariants():
    h = _square_hier(4, 3)
    for lv in h.levels[1:]:
        Mt = lv.Mt
        assert np.array_equal(Mt @ np.ones(Mt.shape[1]), np.ones(Mt.shape[0]))
        Rp = dec.paper_restriction(Mt)
        assert np.allclose(Rp @ np.ones(Mt.shape[0]), 1.0, rtol=0, atol=1e-15)
        # interpolation reproduces linear functions on flat meshes
        nc = Mt.shape[1]
        lin = lambda X: 0.2 - 1.3 * X[:, 0] + 0.7 * X[:, 1]
        assert np.abs(Mt @ lin(lv.xyz[:nc]) - lin(lv.xyz)).max() < 1e-15
        # row sums of M(f) are 4 at interior coarse vertices of valence 6 (Sec. 2.2.1)
        coarse = h.levels[h.levels.index(lv) - 1]
        D = np.asarray(Mt.sum(axis=0)).ravel()
        assert np.all(D[~coarse.bnd] == 4.0)


def _barycentric_in(xyz_c, tri_c, p):
    """Global barycentric coordinates of point p in a flat coarse mesh, by brute force."""
    for a, b, c in tri_c.tolist():
        T = np.array([[xyz_c[a, 0], xyz_c[b, 0], xyz_c[c, 0]],
                      [xyz_c[a, 1], xyz_c[b, 1], xyz_c[c, 1]],
                      [1.0, 1.0, 1.0]])
        lam = np.linalg.solve(T, [p[0], p[1], 1.0])
        if np.all(lam > -1e-12):
            out = np.zeros(len(xyz_c))
            out[[a, b, c]] = np.where(np.abs(lam) < 1e-12, 0.0, lam)
            return out
    raise AssertionError("point outside mesh")


def test_functoriality_against_point_location():
    """M(g o f) = M(g) M(f) (Prop. 2): the composed matrix of two subdivisions equals the
    geometric barycentric coordinates of the finest vertices in the base mesh."""
    rng = np.random.default_rng(3)
    xyz, tri = dec.square_grid(2)
    xyz[4, :2] += 0.1 * rng.standard_normal(2)            # move the centre vertex
    h = mg.Hierarchy(xyz, tri, 2)
    M_comp = (h.levels[2].Mt @ h.levels[1].Mt).toarray()   # V_2 x V_0
    base = h.levels[0]
    for v in range(h.levels[2].nv):
        geo = _barycentric_in(base.xyz, base.tri, h.levels[2].xyz[v])
        assert np.allclose(M_comp[v], geo, atol=1e-12)
    # identity: the kept vertices map to themselves
    assert np.array_equal(M_comp[:base.nv], np.eye(base.nv))


def test_galerkin_equals_rediscretisation():
    """P^T L_f P = L_c exactly on nested flat right-triangle hierarchies."""
    h = _square_hier(4, 3, bc="natural")
    for l in range(1, h.top + 1):
        Mt = h.levels[l].Mt
        G = (Mt.T @ h.levels[l].L @ Mt).toarray()
        assert np.abs(G - h.levels[l - 1].L.toarray()).max() == 0.0


# ------------------------------------------------------------ solutions
def test_c1_discrete_closed_form():
    """sin(pi x) sin(pi y) is an eigenvector of the 5-point stencil: the discrete solution of
    L u = star0 f with f = 2 pi^2 sin sin is c(h) sin sin, c(h) = (pi h / 2)^2 / sin^2(pi h / 2)."""
    h = _square_hier(4, 4)
    b = h.rhs(W.manufactured_c1(h.fine.xyz))
    hh = 1 / 64
    c = (math.pi * hh / 2) ** 2 / math.sin(math.pi * hh / 2) ** 2
    exact = c * W.manufactured_c1_solution(h.fine.xyz)
    u = mg.direct_solve(h, b)
    assert np.abs(u - exact).max() < 1e-13
    x, k, hist = mg.mg_solve(h, b)
    assert hist[-1] <= 1e-10 and k <= 20
    assert np.abs(x - exact).max() < 1e-10
    # and c(h) - 1 = O(h^2): the max error against the continuous solution
    cont = W.manufactured_c1_solution(h.fine.xyz)
    assert abs(np.abs(u - cont).max() - (c - 1) * 1.0) < 1e-12


def test_matches_dense_lapack_on_tiny_meshes():
    for h in [_square_hier(4, s) for s in range(0, 3)] + [_sphere_hier(s) for s in range(1, 4)]:
        rng = np.random.default_rng(h.fine.nv)
        b = h.rhs(rng.standard_normal(h.fine.nv))
        A = h.fine.A.toarray()
        if h.bc == "dirichlet":
            ref = np.linalg.solve(A, b)
        else:
            b = b - b.mean()
            ref = np.linalg.pinv(A) @ b
        if h.top == 0:
            x = mg.coarse_solve(h, b)
        else:
            x, _, _ = mg.mg_pcg(h, b, rtol=1e-14)
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_contraction_factor_h_independent():
    """V(2,2) weighted-Jacobi (omega 0.8) cycles contract at a mesh-independent rate well
    below the smoothing factor max(|1 - omega/2|, |1 - 2 omega|) = 0.6 of that smoother."""
    rhos = []
    for nsub in (3, 4, 5):
        h = _square_hier(4, nsub)
        b = h.rhs(W.manufactured_c1(h.fine.xyz) + W.normal(h.fine.nv, 1))
        _, k, hist = mg.mg_solve(h, b, rtol=1e-11)
        rhos.append(mg.contraction_factor(hist))
    assert max(rhos) < 0.32 and min(rhos) > 0.2
    assert max(rhos) - min(rhos) < 0.03


def test_restriction_pairings_agree():
    """Row-normalised restriction with star0^{-1} L (Def. 6) and R = P^T with the stiffness
    L contract alike; row-normalised R with the stiffness L does not (it stalls)."""
    h = _square_hier(4, 4)
    b = h.rhs(W.normal(h.fine.nv, 2))
    _, _, hist = mg.mg_solve(h, b, rtol=1e-11)
    s0 = h.fine.star0.copy()
    s0[h.fine.bnd] = 1.0
    x = np.zeros_like(b)
    hp = [1.0]
    for _ in range(16):
        x = mg.vcycle_paper(h, b / s0, x)
        hp.append(np.linalg.norm(h.fine.A @ x - b) / np.linalg.norm(b))
    assert abs(mg.contraction_factor(hist) - mg.contraction_factor(hp)) < 0.02


def test_krylov_variants():
    """MG-PCG and FCG(1) take the same iterations with an exact V-cycle; refinement needs
    as many cycles as stand-alone MG; all reach the tolerance."""
    h = _square_hier(4, 4)
    b = h.rhs(W.manufactured_c1(h.fine.xyz))
    _, kp, hp = mg.mg_pcg(h, b)
    _, kf, hf = mg.mg_fcg(h, b)
    _, ki, hi = mg.mg_ir(h, b)
    _, km, hm = mg.mg_solve(h, b)
    assert kp == kf and abs(kp - 11) <= 1
    assert ki == km
    for hh in (hp, hf, hi, hm):
        assert hh[-1] <= 1e-10
    # FCG with a perturbed (float32-rounded) cycle still converges in about as many steps
    M32 = lambda r: mg.vcycle(h, r.astype(np.float32).astype(np.float64)).astype(np.float32).astype(np.float64)
    _, k32, h32 = mg.mg_fcg(h, b, precond=M32)
    assert h32[-1] <= 1e-10 and abs(k32 - kf) <= 2


def test_sphere_second_order_convergence():
    """-lap_S u = f with f a sum of spherical harmonics: the discrete solution converges to
    the continuous one at O(h^2) (error ratio near 4 per level)."""
    coeffs = W.sh_coefficients()
    errs = []
    for nsub in (3, 4, 5):
        h = _sphere_hier(nsub)
        b = h.rhs(W.sphere_rhs(h.fine.xyz, coeffs))
        x, k, hist = mg.mg_pcg(h, b, rtol=1e-12)
        ue = W.sphere_exact(h.fine.xyz, coeffs)
        errs.append(np.abs(x - (ue - ue.mean())).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.3 < r1 < 4.7 and 3.5 < r2 < 4.5


def test_mg_pcg_singular_zero_mean():
    h = _sphere_hier(3)
    b = h.rhs(W.normal(h.fine.nv, 8))
    x, k, hist = mg.mg_pcg(h, b)
    assert abs(x.mean()) < 1e-14
    assert mg.rel_residual(h, b, x) < 1e-9
    ref = mg.direct_solve(h, b)
    assert np.linalg.norm(x - ref) < 1e-8 * np.linalg.norm(ref)
