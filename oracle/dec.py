"""Meshes, subdivision maps and DEC operators -- plain FP64 reference.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the library.  It shares no code with the HIP
path.  Every function cites the passage of the paper (arXiv 2508.12501) it follows.

Conventions (an interface the library keeps too, so that results compare element-wise):

* Square grid with n cells per side: vertex (i, j) -> j*(n+1) + i at (i/n, j/n, 0); cell
  (i, j), j outer, i inner, with a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) gives the two
  counter-clockwise triangles (a,b,c), (a,c,d).
* Icosahedron: the 12 cyclic permutations of (0, +-1, +-phi) in a fixed order, normalised;
  faces are the vertex triples at mutual distance 2 (before normalising), in lexicographic
  order, each oriented so that its normal points away from the origin.
* Edges are numbered by first appearance while scanning triangles t = 0.. and, inside t =
  (v0, v1, v2), the sides (v0,v1), (v1,v2), (v2,v0); an edge is oriented from its smaller
  to its larger vertex id.
* One binary (1-to-4) subdivision keeps coarse vertex ids, puts the midpoint of coarse edge
  e at id V_c + e and replaces triangle t = (a,b,c) by 4t+0..3 = (a,ab,ca), (ab,b,bc),
  (ca,bc,c), (ab,bc,ca).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ------------------------------------------------------------------ base meshes
def square_grid(n: int):
    """Unit square, n x n cells, each split along its SW-NE diagonal (the right-triangle
    grids of the Poisson and porous-convection experiments, Sec. 3)."""
    j, i = np.mgrid[0:n + 1, 0:n + 1]
    xyz = np.zeros(((n + 1) ** 2, 3))
    xyz[:, 0] = i.ravel() / n
    xyz[:, 1] = j.ravel() / n
    tris = []
    for cj in range(n):
        for ci in range(n):
            a = cj * (n + 1) + ci
            b = a + 1
            c = a + n + 2
            d = a + n + 1
            tris.append((a, b, c))
            tris.append((a, c, d))
    return xyz, np.array(tris, dtype=np.int64)


def icosahedron():
    """Unit icosahedron (base of the sphere workloads): the 12 cyclic permutations of
    (0, +-1, +-phi), normalised, in the order listed below."""
    f = (1.0 + math.sqrt(5.0)) / 2.0
    raw = np.array([(-1, f, 0), (1, f, 0), (-1, -f, 0), (1, -f, 0),
                    (0, -1, f), (0, 1, f), (0, -1, -f), (0, 1, -f),
                    (f, 0, -1), (f, 0, 1), (-f, 0, -1), (-f, 0, 1)], dtype=np.float64)
    tris = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                dij = np.sum((raw[i] - raw[j]) ** 2)
                djk = np.sum((raw[j] - raw[k]) ** 2)
                dik = np.sum((raw[i] - raw[k]) ** 2)
                if abs(dij - 4) < 1e-9 and abs(djk - 4) < 1e-9 and abs(dik - 4) < 1e-9:
                    n = np.cross(raw[j] - raw[i], raw[k] - raw[i])
                    if np.dot(n, raw[i] + raw[j] + raw[k]) > 0:
                        tris.append((i, j, k))
                    else:
                        tris.append((i, k, j))
    r = np.sqrt(raw[:, 0] * raw[:, 0] + raw[:, 1] * raw[:, 1] + raw[:, 2] * raw[:, 2])
    return raw / r[:, None], np.array(tris, dtype=np.int64)


# ------------------------------------------------------------------ simplicial structure
def edges_of(tri: np.ndarray, nv: int):
    """Edge set E and face maps T -> E of the simplicial complex (Def. 1): returns
    ``edges`` (E,2) as (lo, hi), ``tri_edges`` (T,3) for the sides (v0v1, v1v2, v2v0) and
    ``tri_sign`` (T,3), +1 where the triangle's boundary cycle runs lo -> hi."""
    a = tri[:, [0, 1, 2]].ravel()
    b = tri[:, [1, 2, 0]].ravel()
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * nv + hi
    uniq, first, inv = np.unique(key, return_index=True, return_inverse=True)
    order = np.argsort(first, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(len(order))
    edges = np.stack([uniq[order] // nv, uniq[order] % nv], axis=1)
    tri_edges = rank[inv.ravel()].reshape(-1, 3)
    tri_sign = np.where(a < b, 1, -1).reshape(-1, 3)
    return edges, tri_edges, tri_sign


def d0_matrix(edges: np.ndarray, nv: int) -> sp.csr_matrix:
    """Exterior derivative on 0-forms, E x V: (d0 u)_e = u(hi) - u(lo) (Fig. dRC, Sec. 3.1)."""
    ne = len(edges)
    rows = np.repeat(np.arange(ne), 2)
    cols = edges.ravel()
    vals = np.tile([-1, 1], ne)
    return sp.csr_matrix((vals.astype(np.int64), (rows, cols)), shape=(ne, nv))


def d1_matrix(tri_edges: np.ndarray, tri_sign: np.ndarray, ne: int) -> sp.csr_matrix:
    """Exterior derivative on 1-forms, T x E: signed sum of a triangle's edges (Fig. dRC)."""
    nt = len(tri_edges)
    rows = np.repeat(np.arange(nt), 3)
    return sp.csr_matrix((tri_sign.ravel().astype(np.int64), (rows, tri_edges.ravel())),
                         shape=(nt, ne))


def boundary_vertices(tri_edges: np.ndarray, edges: np.ndarray, nv: int) -> np.ndarray:
    """Vertices on a boundary edge (an edge that is a face of exactly one triangle)."""
    count = np.bincount(tri_edges.ravel(), minlength=len(edges))
    bnd = np.zeros(nv, dtype=bool)
    bnd[edges[count == 1].ravel()] = True
    return bnd


# ------------------------------------------------------------------ geometric map
def subdivide(xyz, tri, edges, tri_edges, project: bool = False):
    """Binary subdivision (Sec. 2.2.1): each triangle splits into 4 through its edge
    midpoints.  Returns the fine mesh and M(f)^T, the V_f x V_c interpolation matrix whose
    row j holds the global barycentric coordinates of fine vertex j in the coarse mesh
    (Def. 3, Def. 4, Def. 5): 1 at a kept vertex, 1/2, 1/2 at an edge midpoint.  With
    ``project`` the midpoints are pushed radially onto the unit sphere (icosphere levels);
    the barycentric coordinates stay 1/2, 1/2."""
    nv, ne = len(xyz), len(edges)
    mid = 0.5 * (xyz[edges[:, 0]] + xyz[edges[:, 1]])
    if project:
        r = np.sqrt(mid[:, 0] * mid[:, 0] + mid[:, 1] * mid[:, 1] + mid[:, 2] * mid[:, 2])
        mid = mid / r[:, None]
    fxyz = np.vstack([xyz, mid])
    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    ab, bc, ca = nv + tri_edges[:, 0], nv + tri_edges[:, 1], nv + tri_edges[:, 2]
    ftri = np.stack([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                     np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], axis=1).reshape(-1, 3)
    rows = np.concatenate([np.arange(nv), nv + np.arange(ne), nv + np.arange(ne)])
    cols = np.concatenate([np.arange(nv), edges[:, 0], edges[:, 1]])
    vals = np.concatenate([np.ones(nv), np.full(ne, 0.5), np.full(ne, 0.5)])
    Mt = sp.csr_matrix((vals, (rows, cols)), shape=(nv + ne, nv))
    return fxyz, ftri, Mt


def subdivide_cubic(xyz, tri, edges, tri_edges, project: bool = False):
    """Cubic subdivision (Sec. 2.2.1, the 1-to-9 scheme of the paper's benchmarks): every edge
    gets two points at 1/3 and 2/3 of its length and every triangle its centroid; each triangle
    splits into 9 similar ones with the parent's orientation.  Numbering: coarse vertices keep
    their ids, edge e (oriented lo -> hi) adds V + 2e (the point next to lo) and V + 2e + 1
    (next to hi), triangle t adds V + 2E + t.  Returns the fine mesh and M(f)^T with the
    barycentric coordinates of each fine vertex: 1 at a kept vertex, (2/3, 1/3) on an edge,
    (1/3, 1/3, 1/3) at a centroid.  With ``project`` the new points are pushed radially onto the
    unit sphere (the barycentric coordinates stay those of the flat construction)."""
    nv, ne, nt = len(xyz), len(edges), len(tri)
    lo, hi = xyz[edges[:, 0]], xyz[edges[:, 1]]
    p1 = (2.0 * lo + hi) / 3.0
    p2 = (lo + 2.0 * hi) / 3.0
    cen = (xyz[tri[:, 0]] + xyz[tri[:, 1]] + xyz[tri[:, 2]]) / 3.0
    pts = np.empty((2 * ne, 3))
    pts[0::2] = p1
    pts[1::2] = p2
    new = np.vstack([pts, cen])
    if project:
        r = np.sqrt(new[:, 0] * new[:, 0] + new[:, 1] * new[:, 1] + new[:, 2] * new[:, 2])
        new = new / r[:, None]
    fxyz = np.vstack([xyz, new])

    def side(k, a_ids):
        """The two points of triangle side k ordered from the side's first vertex (a_ids)."""
        e = tri_edges[:, k]
        near_lo, near_hi = nv + 2 * e, nv + 2 * e + 1
        first_is_lo = edges[e, 0] == a_ids
        return np.where(first_is_lo, near_lo, near_hi), np.where(first_is_lo, near_hi, near_lo)

    a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
    ab1, ab2 = side(0, a)
    bc1, bc2 = side(1, b)
    ca1, ca2 = side(2, c)
    m = nv + 2 * ne + np.arange(nt)
    kids = [(a, ab1, ca2), (ab2, b, bc1), (ca1, bc2, c),
            (ab1, ab2, m), (bc1, bc2, m), (ca1, ca2, m),
            (ab1, m, ca2), (ab2, bc1, m), (bc2, ca1, m)]
    ftri = np.stack([np.stack(k, 1) for k in kids], axis=1).reshape(-1, 3)
    e_ids = np.arange(ne)
    rows = np.concatenate([np.arange(nv),
                           nv + 2 * e_ids, nv + 2 * e_ids, nv + 2 * e_ids + 1, nv + 2 * e_ids + 1,
                           m, m, m])
    cols = np.concatenate([np.arange(nv),
                           edges[:, 0], edges[:, 1], edges[:, 0], edges[:, 1],
                           a, b, c])
    vals = np.concatenate([np.ones(nv),
                           np.full(ne, 2.0 / 3.0), np.full(ne, 1.0 / 3.0),
                           np.full(ne, 1.0 / 3.0), np.full(ne, 2.0 / 3.0),
                           np.full(nt, 1.0 / 3.0), np.full(nt, 1.0 / 3.0), np.full(nt, 1.0 / 3.0)])
    Mt = sp.csr_matrix((vals, (rows, cols)), shape=(nv + 2 * ne + nt, nv))
    return fxyz, ftri, Mt


def paper_restriction(Mt: sp.spmatrix) -> sp.csr_matrix:
    """The restriction operator of Def. 6: the transpose of the row-normalisation of M(f).
    M(f) = Mt^T is V_c x V_f; as a column-vector operator it maps fine to coarse as
    rownorm(M(f)) r_f, so rows of the returned V_c x V_f matrix sum to 1."""
    M = sp.csr_matrix(Mt.T)
    rs = np.asarray(M.sum(axis=1)).ravel()
    return sp.csr_matrix(sp.diags(1.0 / rs) @ M)


# ------------------------------------------------------------------ Hodge stars
def _cot(pk, pi, pj):
    """cot of the angle at pk in the triangle (pk, pi, pj): (u.v)/|u x v|."""
    u = pi - pk
    v = pj - pk
    cr = np.cross(u, v)
    return np.sum(u * v, axis=1) / np.sqrt(np.sum(cr * cr, axis=1))


def hodge_stars(xyz, tri, tri_edges, ne: int):
    """Diagonal Hodge stars of the circumcentric dual (Sec. 3.1, Fig. pd-scs):
    star1[e] = |dual edge| / |primal edge| = (1/2) sum over triangles containing e of the
    cotangent of the angle opposite e (signed);
    star0[v] = area of the dual cell of v = sum over triangles (|e_vj|^2 cot th_k +
    |e_vk|^2 cot th_j) / 8 (signed)."""
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    c0 = _cot(p0, p1, p2)   # angle at v0, opposite side (v1,v2)
    c1 = _cot(p1, p2, p0)   # angle at v1, opposite side (v2,v0)
    c2 = _cot(p2, p0, p1)   # angle at v2, opposite side (v0,v1)
    star1 = (np.bincount(tri_edges[:, 1], 0.5 * c0, ne)
             + np.bincount(tri_edges[:, 2], 0.5 * c1, ne)
             + np.bincount(tri_edges[:, 0], 0.5 * c2, ne))
    l01 = np.sum((p1 - p0) ** 2, axis=1)
    l12 = np.sum((p2 - p1) ** 2, axis=1)
    l20 = np.sum((p0 - p2) ** 2, axis=1)
    nv = len(xyz)
    star0 = (np.bincount(tri[:, 0], (l01 * c2 + l20 * c1) / 8.0, nv)
             + np.bincount(tri[:, 1], (l12 * c0 + l01 * c2) / 8.0, nv)
             + np.bincount(tri[:, 2], (l20 * c1 + l12 * c0) / 8.0, nv))
    return star0, star1


# ------------------------------------------------------------------ Laplacian
def laplacian(d0: sp.spmatrix, w: np.ndarray) -> sp.csr_matrix:
    """Stiffness form of the 0-form Hodge Laplacian, L = d0^T diag(w) d0 with w = star1
    (times an edge coefficient for the Darcy operator).  The paper's Delta_0 =
    star0^{-1} d~1 star1 d0 (Eq. hodge0-laplacian) equals -star0^{-1} L, since d~1 is the
    negated transpose of d0."""
    d0f = sp.csr_matrix(d0, dtype=np.float64)
    return sp.csr_matrix(d0f.T @ sp.diags(w) @ d0f)


def dirichlet(L: sp.spmatrix, bnd: np.ndarray) -> sp.csr_matrix:
    """Zero-Dirichlet form L_D = M L M + (I - M), M = diag(interior): identity rows and
    columns at boundary vertices."""
    m = (~bnd).astype(np.float64)
    M = sp.diags(m)
    return sp.csr_matrix(M @ L @ M + sp.diags(1.0 - m))
