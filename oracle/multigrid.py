"""Geometric multigrid for the DEC 0-form Laplacian -- plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Follows Sec. 2.2.1 (interpolation
by M(f)^T, restriction), Sec. 3.1 (rediscretised Laplacian per level, V-cycles, relative
residual ||L u - b|| / ||b||, GMG as a CG preconditioner).  The smoother, cycle shape and
coarse solve are the ones of the workloads: V(nu1, nu2) weighted Jacobi and an exact dense
solve on the coarsest level.  Readings of the paper that are not spelled out there:

* Q1 sign: L = d0^T star1 d0 is positive semi-definite; -lap u = f becomes L u = star0 f.
* Q2 star1 = |dual edge| / |primal edge| (cotangent weights).
* Q4 restriction paired with the stiffness form L is R = M_c P^T (no row normalisation);
  ``pairing="paper"`` runs the row-normalised restriction of Def. 6 with star0^{-1} L.
* Q6 zero Dirichlet: identity rows/columns at boundary vertices, restricted residual zeroed
  at coarse boundary vertices.
* Q9 singular (closed surface, natural boundary): the plain vertex mean is removed from b,
  from every preconditioner output and from the final solution.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dec


class Level:
    """One mesh of the hierarchy with its rediscretised operators (Sec. 3.1: every DEC
    primitive is rebuilt on every level)."""

    def __init__(self, xyz, tri):
        self.xyz = xyz
        self.tri = tri
        self.nv = len(xyz)
        self.edges, self.tri_edges, self.tri_sign = dec.edges_of(tri, self.nv)
        self.ne = len(self.edges)
        self.nt = len(tri)
        self.d0 = dec.d0_matrix(self.edges, self.nv)
        self.star0, self.star1 = dec.hodge_stars(xyz, tri, self.tri_edges, self.ne)
        self.bnd = dec.boundary_vertices(self.tri_edges, self.edges, self.nv)
        self.Mt = None          # interpolation from the next coarser level (V x V_coarse)
        self.w = self.star1.copy()
        self.L = None
        self.A = None

    @property
    def d1(self):
        return dec.d1_matrix(self.tri_edges, self.tri_sign, self.ne)


class Hierarchy:
    """Meshes X_0 (coarsest) .. X_l (finest) related by binary subdivision maps (Fig. ex-subdiv),
    with L on each level and the transfer operators between neighbours."""

    def __init__(self, xyz, tri, nsub: int, project: bool = False, bc: str = "dirichlet",
                 schemes: str | None = None):
        """`schemes`: one letter per subdivision, "b" binary (1-to-4) or "c" cubic (1-to-9);
        default all binary."""
        assert bc in ("dirichlet", "natural")
        self.bc = bc
        self.schemes = schemes or "b" * nsub
        assert len(self.schemes) == nsub and set(self.schemes) <= {"b", "c"}
        self.levels = [Level(xyz, tri)]
        for k in range(nsub):
            c = self.levels[-1]
            sub = dec.subdivide_cubic if self.schemes[k] == "c" else dec.subdivide
            fxyz, ftri, Mt = sub(c.xyz, c.tri, c.edges, c.tri_edges, project)
            f = Level(fxyz, ftri)
            f.Mt = Mt
            self.levels.append(f)
        self._assemble()

    @classmethod
    def from_maps(cls, meshes, maps, bc: str = "dirichlet"):
        """A hierarchy over given meshes (coarsest first) related by given geometric maps
        (Sec. 2.2.1 with Def. 4): maps[l] is M(f) for f: mesh l+1 -> mesh l, a
        (coarse x fine) matrix whose column j holds the global barycentric coordinates of
        f(x_j).  Interpolation is M(f)^T and restriction M(f), as for subdivisions; the meshes
        need not be nested, and every level is rediscretised on its own mesh (Sec. 3.1)."""
        assert bc in ("dirichlet", "natural") and len(maps) == len(meshes) - 1
        self = cls.__new__(cls)
        self.bc = bc
        self.schemes = None
        self.levels = []
        for k, (xyz, tri) in enumerate(meshes):
            lv = Level(np.asarray(xyz, dtype=np.float64), np.asarray(tri))
            if k > 0:
                M = sp.csc_matrix(maps[k - 1])
                assert M.shape == (self.levels[-1].nv, lv.nv)
                lv.Mt = M.T.tocsr()
            self.levels.append(lv)
        self._assemble()
        return self

    # -- operators
    def _assemble(self):
        for lv in self.levels:
            lv.L = dec.laplacian(lv.d0, lv.w)
            lv.A = dec.dirichlet(lv.L, lv.bnd) if self.bc == "dirichlet" else lv.L

    def set_vertex_coeff(self, kv_fine: np.ndarray):
        """Edge coefficient for the Darcy operator: each level takes the vertex field at its
        own vertices (coarse vertex ids are kept by subdivision, so this is injection), sets
        k_e = (k_lo + k_hi) / 2 and w = star1 * k_e (reading Q13)."""
        for lv in self.levels:
            kv = kv_fine[:lv.nv]
            ke = 0.5 * (kv[lv.edges[:, 0]] + kv[lv.edges[:, 1]])
            lv.w = lv.star1 * ke
        self._assemble()

    def set_edge_coeff(self, ke_fine: np.ndarray):
        """The Darcy coefficient as an edge field (Sec. 3.2, Eq. dec_darcy: K multiplies the
        1-form d0 p edge by edge): the finest level uses w = star1 * k_e.  A coarser edge takes
        the mean of the fine edges it was split into: the two halves (lo, m), (m, hi) of a
        binary subdivision (m = nv_coarse + e), the three thirds (lo, p1), (p1, p2), (p2, hi) of
        a cubic one (p1 = nv_coarse + 2e, p2 = p1 + 1).  Hierarchies over given maps have no
        such correspondence and are refused."""
        if self.schemes is None:
            raise ValueError("edge coefficients need a subdivision hierarchy")
        ke = np.asarray(ke_fine, dtype=np.float64)
        assert ke.shape == (self.fine.ne,)
        for l in range(self.top, -1, -1):
            lv = self.levels[l]
            lv.w = lv.star1 * ke
            if l == 0:
                break
            fine, coarse = lv, self.levels[l - 1]
            index = {(int(a), int(b)): i for i, (a, b) in enumerate(fine.edges)}

            def eid(a, b):
                return index[(min(a, b), max(a, b))]

            nc = coarse.nv
            kc = np.empty(coarse.ne)
            for e, (a, b) in enumerate(coarse.edges):
                a, b = int(a), int(b)
                if self.schemes[l - 1] == "b":
                    m = nc + e
                    kc[e] = 0.5 * (ke[eid(a, m)] + ke[eid(m, b)])
                else:
                    p1, p2 = nc + 2 * e, nc + 2 * e + 1
                    kc[e] = (ke[eid(a, p1)] + ke[eid(p1, p2)] + ke[eid(p2, b)]) / 3.0
            ke = kc
        self._assemble()

    def colors(self, l: int) -> np.ndarray:
        """Greedy colour classes of level l's operator (cached; the sparsity does not change
        with the vertex coefficient)."""
        if not hasattr(self, "_colors"):
            self._colors = {}
        if l not in self._colors:
            self._colors[l] = greedy_colors(self.levels[l].A)
        return self._colors[l]

    @property
    def fine(self) -> Level:
        return self.levels[-1]

    @property
    def top(self) -> int:
        return len(self.levels) - 1

    def restrict(self, l: int, r: np.ndarray) -> np.ndarray:
        """R = M_c P^T from level l to l-1, zeroed at coarse Dirichlet vertices."""
        rc = self.levels[l].Mt.T @ r
        if self.bc == "dirichlet":
            rc[self.levels[l - 1].bnd] = 0.0
        return rc

    def prolong(self, l: int, ec: np.ndarray) -> np.ndarray:
        """Interpolation of Def. 5: values on level l-1 -> level l by M(f)^T."""
        return self.levels[l].Mt @ ec

    def rhs(self, f: np.ndarray) -> np.ndarray:
        """b = star0 f on the finest level (Dirichlet: zero on the boundary)."""
        b = self.fine.star0 * f
        if self.bc == "dirichlet":
            b[self.fine.bnd] = 0.0
        return b

    def unknowns(self) -> int:
        lv = self.fine
        return int(np.count_nonzero(~lv.bnd)) if self.bc == "dirichlet" else lv.nv


# ------------------------------------------------------------------ smoother and cycle
def jacobi(A, b, x, omega: float, nsweeps: int):
    """Weighted Jacobi: x <- x + omega D^{-1} (b - A x), D = diag(A)."""
    dinv = 1.0 / A.diagonal()
    for _ in range(nsweeps):
        x = x + omega * dinv * (b - A @ x)
    return x


def greedy_colors(A) -> np.ndarray:
    """Colour classes for a multicolour Gauss-Seidel sweep: vertices in increasing id, each
    taking the smallest colour not used by an already coloured neighbour, where neighbours are
    the couplings of A with a nonzero value (reading Q7b)."""
    G = sp.csr_matrix(A, copy=True)
    G.setdiag(0.0)
    G.eliminate_zeros()
    n = G.shape[0]
    color = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = {int(color[j]) for j in G.indices[G.indptr[i]:G.indptr[i + 1]] if color[j] >= 0}
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color


def gauss_seidel(A, b, x, colors, nsweeps: int, backward: bool = False):
    """Multicolour Gauss-Seidel: colour classes in increasing order (decreasing when
    `backward`); every vertex of a class takes x_i <- x_i + (b_i - (A x)_i) / A_ii with the
    latest values.  Vertices of one class are not coupled, so the order inside a class does not
    matter (the paper smooths with Gauss-Seidel, Sec. 3.1 and 3.2)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    x = x.copy()
    order = list(range(int(colors.max()) + 1))
    if backward:
        order.reverse()
    for _ in range(nsweeps):
        for c in order:
            for i in np.flatnonzero(colors == c):
                lo, hi = A.indptr[i], A.indptr[i + 1]
                x[i] = x[i] + (b[i] - A.data[lo:hi] @ x[A.indices[lo:hi]]) / d[i]
    return x


def cg_smooth(A, b, x, nsteps: int):
    """`nsteps` steps of unpreconditioned conjugate gradients on A x = b from x (CG smoothing,
    the smoother of the paper's V-cycle timings, Fig. time_per1vcycle).  Stops early on an
    exactly zero residual or a non-positive curvature."""
    x = x.copy()
    r = b - A @ x
    p = r.copy()
    rr = r @ r
    for _ in range(nsteps):
        q = A @ p
        pq = p @ q
        if not (rr > 0.0 and pq > 0.0):
            break
        alpha = rr / pq
        x = x + alpha * p
        r = r - alpha * q
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def smooth(h: Hierarchy, l: int, b, x, nsweeps: int, omega: float, smoother: str, post: bool):
    """The smoother of a cycle on level l: weighted Jacobi, or multicolour Gauss-Seidel with
    forward sweeps before the coarse-grid correction and backward sweeps after it (so the
    cycle stays symmetric)."""
    A = h.levels[l].A
    if smoother == "jacobi":
        return jacobi(A, b, x, omega, nsweeps)
    if smoother == "gs":
        return gauss_seidel(A, b, x, h.colors(l), nsweeps, backward=post)
    if smoother == "cg":
        return cg_smooth(A, b, x, nsweeps)
    raise ValueError(smoother)


def coarse_solve(h: Hierarchy, b: np.ndarray) -> np.ndarray:
    """Exact solve on the coarsest level: dense LU, or the minimum-norm least-squares
    solution (L^+ b) when L is singular."""
    A = h.levels[0].A.toarray()
    if h.bc == "dirichlet":
        return np.linalg.solve(A, b)
    return np.linalg.lstsq(A, b, rcond=None)[0]


def vcycle(h: Hierarchy, b, x=None, l=None, nu1=2, nu2=2, omega=0.8):
    """One V(nu1, nu2) cycle for A_l x = b: pre-smooth, restrict the residual, recurse with a
    zero initial guess, interpolate and correct, post-smooth (Sec. 2, Sec. 3.1)."""
    if l is None:
        l = h.top
    if l == 0:
        return coarse_solve(h, b)
    A = h.levels[l].A
    x = np.zeros_like(b) if x is None else x.copy()
    x = jacobi(A, b, x, omega, nu1)
    r = b - A @ x
    ec = vcycle(h, h.restrict(l, r), None, l - 1, nu1, nu2, omega)
    x = x + h.prolong(l, ec)
    x = jacobi(A, b, x, omega, nu2)
    return x


def mgcycle(h: Hierarchy, b, x=None, l=None, kind="V", nu1=2, nu2=2, omega=0.8,
            smoother="jacobi"):
    """One multigrid cycle of shape `kind` for A_l x = b (the V-, W- and F-cycles named in
    Sec. 2, textbook recursion): pre-smooth, restrict the residual, coarse-grid correction,
    interpolate and correct, post-smooth.  The coarse-grid correction is one cycle of the same
    shape from zero for V, two for W (the second starting from the first's result), and an
    F-cycle followed by a V-cycle for F.  On the coarsest level every shape is the exact solve.
    `smoother` is "jacobi" (weighted, omega), "gs" (multicolour Gauss-Seidel, see smooth) or
    "cg" (CG steps, which make the cycle a nonlinear map: use it inside FCG or IR)."""
    if l is None:
        l = h.top
    if l == 0:
        return coarse_solve(h, b)
    A = h.levels[l].A
    x = np.zeros_like(b) if x is None else x.copy()
    x = smooth(h, l, b, x, nu1, omega, smoother, post=False)
    r = b - A @ x
    rc = h.restrict(l, r)
    if kind == "V":
        ec = mgcycle(h, rc, None, l - 1, "V", nu1, nu2, omega, smoother)
    elif kind == "W":
        ec = mgcycle(h, rc, None, l - 1, "W", nu1, nu2, omega, smoother)
        ec = mgcycle(h, rc, ec, l - 1, "W", nu1, nu2, omega, smoother)
    elif kind == "F":
        ec = mgcycle(h, rc, None, l - 1, "F", nu1, nu2, omega, smoother)
        ec = mgcycle(h, rc, ec, l - 1, "V", nu1, nu2, omega, smoother)
    else:
        raise ValueError(kind)
    x = x + h.prolong(l, ec)
    x = smooth(h, l, b, x, nu2, omega, smoother, post=True)
    return x


def vcycle_paper(h: Hierarchy, f, x=None, l=None, nu1=2, nu2=2, omega=0.8):
    """The same cycle for the paper's scaling, star0^{-1} L x = f, with the row-normalised
    restriction of Def. 6 (Dirichlet identity rows kept unscaled)."""
    if l is None:
        l = h.top
    lv = h.levels[l]
    s0 = lv.star0.copy()
    if h.bc == "dirichlet":
        s0[lv.bnd] = 1.0
    A = sp.diags(1.0 / s0) @ lv.A
    if l == 0:
        A0 = A.toarray()
        if h.bc == "dirichlet":
            return np.linalg.solve(A0, f)
        return np.linalg.lstsq(A0, f, rcond=None)[0]
    x = np.zeros_like(f) if x is None else x.copy()
    x = jacobi(A, f, x, omega, nu1)
    r = f - A @ x
    rc = dec.paper_restriction(lv.Mt) @ r
    if h.bc == "dirichlet":
        rc[h.levels[l - 1].bnd] = 0.0
    ec = vcycle_paper(h, rc, None, l - 1, nu1, nu2, omega)
    x = x + h.prolong(l, ec)
    x = jacobi(A, f, x, omega, nu2)
    return x


# ------------------------------------------------------------------ solvers
def _project(h: Hierarchy, v):
    return v - v.mean() if h.bc == "natural" else v


def mg_solve(h: Hierarchy, b, rtol=1e-10, max_cycles=200, nu1=2, nu2=2, omega=0.8, cycle="V",
             smoother="jacobi"):
    """Stand-alone multigrid: repeat cycles from x = 0 until ||b - A x|| <= rtol ||b||.
    Returns (x, cycles, history of relative residuals)."""
    A = h.fine.A
    b = _project(h, b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    hist = [1.0]
    k = 0
    while hist[-1] > rtol and k < max_cycles and nb > 0:
        x = mgcycle(h, b, x, None, cycle, nu1, nu2, omega, smoother)
        k += 1
        hist.append(np.linalg.norm(b - A @ x) / nb)
    return _project(h, x), k, hist


def _precond(h, r, nu1, nu2, omega, cycle="V", smoother="jacobi"):
    return _project(h, mgcycle(h, r, None, None, cycle, nu1, nu2, omega, smoother))


def _true_residual_met(h: Hierarchy, A, b, x, nb, rtol):
    """The stopping test of Sec. 3.1 on the true relative residual ||b - A x|| / ||b||, for
    the (projected) iterate x.  Returns (met, x projected, b - A x)."""
    x = _project(h, x)
    r = b - A @ x
    return bool(np.linalg.norm(r) / nb <= rtol), x, r


def mg_pcg(h: Hierarchy, b, rtol=1e-10, max_iter=200, nu1=2, nu2=2, omega=0.8, cycle="V",
           smoother="jacobi"):
    """Conjugate gradients preconditioned by one V-cycle (Sec. 3.1, CG-GMG), x0 = 0.  The loop
    runs on the recursively updated residual; once that is below rtol, the true relative
    residual ||b - A x|| / ||b|| (the criterion of Sec. 3.1) decides, and if it is still above
    rtol the iteration restarts from x with r = b - A x and p = z.  Returns (x, iterations,
    history of the recursively updated relative residual)."""
    A = h.fine.A
    b = _project(h, b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0 if nb > 0 else 0.0]
    if nb == 0:
        return x, 0, hist
    z = _precond(h, r, nu1, nu2, omega, cycle, smoother)
    p = z.copy()
    rho = r @ z
    k = 0
    while k < max_iter:
        q = A @ p
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            met, x, r = _true_residual_met(h, A, b, x, nb, rtol)
            if met:
                break
            z = _precond(h, r, nu1, nu2, omega, cycle, smoother)
            p = z.copy()
            rho = r @ z
            continue
        z = _precond(h, r, nu1, nu2, omega, cycle, smoother)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return _project(h, x), k, hist


def mg_fcg(h: Hierarchy, b, rtol=1e-10, max_iter=200, nu1=2, nu2=2, omega=0.8, precond=None,
           cycle="V", smoother="jacobi"):
    """Flexible CG with one-vector truncation (FCG(1)): alpha = p^T r / p^T q,
    beta = -z^T q_prev / p_prev^T q_prev; stopped, and restarted when needed, on the true
    relative residual as mg_pcg is.  ``precond`` defaults to one V-cycle; passing
    another callable lets a test emulate a perturbed (e.g. lower precision) cycle."""
    A = h.fine.A
    b = _project(h, b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    r = b.copy()
    hist = [1.0 if nb > 0 else 0.0]
    if nb == 0:
        return x, 0, hist
    M = precond or (lambda v: mgcycle(h, v, None, None, cycle, nu1, nu2, omega, smoother))
    p_prev = q_prev = None
    k = 0
    while k < max_iter:
        z = _project(h, M(r))
        if p_prev is None:
            p = z
        else:
            p = z - ((z @ q_prev) / (p_prev @ q_prev)) * p_prev
        q = A @ p
        alpha = (p @ r) / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        k += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            # stop on the true relative residual (as mg_pcg); else restart from x
            met, x, r = _true_residual_met(h, A, b, x, nb, rtol)
            if met:
                break
            p_prev = q_prev = None
            continue
        p_prev, q_prev = p, q
    return _project(h, x), k, hist


def mg_ir(h: Hierarchy, b, rtol=1e-10, max_iter=200, nu1=2, nu2=2, omega=0.8, precond=None,
          cycle="V", smoother="jacobi"):
    """Iterative refinement: x <- x + M(b - A x) with the true residual recomputed each
    step."""
    A = h.fine.A
    b = _project(h, b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    M = precond or (lambda v: mgcycle(h, v, None, None, cycle, nu1, nu2, omega, smoother))
    r = b.copy()
    hist = [1.0 if nb > 0 else 0.0]
    k = 0
    while nb > 0 and hist[-1] > rtol and k < max_iter:
        x = x + _project(h, M(r))
        r = b - A @ x
        k += 1
        hist.append(np.linalg.norm(r) / nb)
    return _project(h, x), k, hist


def compose(Mg, Mf) -> sp.csc_matrix:
    """M(g o f) = M(g) M(f) for f: X -> Y and g: Y -> Z (Prop. 2): the matrix product."""
    return sp.csc_matrix(Mg @ Mf)


def rel_residual(h: Hierarchy, b, x) -> float:
    """||A x - b||_2 / ||b||_2 on the finest mesh (Sec. 3.1)."""
    b = _project(h, b)
    return float(np.linalg.norm(h.fine.A @ x - b) / np.linalg.norm(b))


def direct_solve(h: Hierarchy, b):
    """The plain definition u* = A^{-1} b (A^+ b, zero mean, when singular): sparse LU."""
    import scipy.sparse.linalg as spla
    b = _project(h, b)
    A = h.fine.A
    if h.bc == "dirichlet":
        return spla.spsolve(sp.csc_matrix(A), b)
    # natural boundary (Q9): b is compatible after the projection, so every solution differs
    # from A^+ b by a constant; ground vertex 0, solve the remaining nonsingular system, then
    # remove the mean
    A = sp.csc_matrix(A)
    x = np.zeros(A.shape[0])
    x[1:] = spla.spsolve(A[1:, 1:], b[1:])
    return x - x.mean()


def contraction_factor(hist, tail: int = 5) -> float:
    """Asymptotic residual reduction per cycle: geometric mean over the last ``tail``
    cycles of a residual history."""
    h = np.asarray(hist)
    h = h[h > 0]
    k = min(tail, len(h) - 1)
    return float((h[-1] / h[-1 - k]) ** (1.0 / k))


def solve_adjoint(h: Hierarchy, u, grad_u):
    """Reverse-mode derivative of the exact solve u = A^{-1} b (A^+ b when singular) for a
    loss J(u) with upstream gradient grad_u (an extension: the paper solves, it does not
    differentiate through the solver).

    lambda = A^{-T} grad_u = A^{-1} grad_u (A symmetric) is dJ/db.  With the finest-level
    edge weights w_e = star1_e k_e, k_e = (k_lo + k_hi) / 2 (reading Q13), dA/dk_e =
    star1_e (M d0_e)^T (M d0_e) where M masks Dirichlet vertices (identity otherwise), so
    dJ/dk_e = -lambda^T (dA/dk_e) u = -star1_e (d0 M lambda)_e (d0 M u)_e and
    dJ/dk_v = 1/2 sum over the edges at v of dJ/dk_e.  Coarser levels only shape the
    preconditioner and do not enter the exact solution.  Returns (dJ/db, dJ/dk_v)."""
    lv = h.fine
    lam = direct_solve(h, grad_u)
    m = np.ones(lv.nv)
    if h.bc == "dirichlet":
        m[lv.bnd] = 0.0
    d0 = sp.csr_matrix(lv.d0, dtype=np.float64)
    gk_e = -lv.star1 * (d0 @ (m * lam)) * (d0 @ (m * u))
    gk_v = 0.5 * (abs(d0).T @ gk_e)
    return lam, gk_v


def solve_adjoint_weights(h: Hierarchy, u, grad_u):
    """dJ/dw_e for the finest operator's edge weights w_e (L = d0^T diag(w) d0, the Hodge
    weights star1_e k_e), same setting as solve_adjoint: dA/dw_e = (M d0_e)^T (M d0_e), so
    dJ/dw_e = -(d0 M lambda)_e (d0 M u)_e with lambda = A^{-1} grad_u."""
    lv = h.fine
    lam = direct_solve(h, grad_u)
    m = np.ones(lv.nv)
    if h.bc == "dirichlet":
        m[lv.bnd] = 0.0
    d0 = sp.csr_matrix(lv.d0, dtype=np.float64)
    return -(d0 @ (m * lam)) * (d0 @ (m * u))
