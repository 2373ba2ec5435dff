"""GPU parity: the HIP path through the C-ABI against the FP64 oracle, element by element.

Tolerances (relative L2 unless stated):
* host build: integers and coordinates bit-exact, Hodge stars 1e-14;
* one kernel in FP64 (operator, sweep, restriction, interpolation): 1e-14;
* one V-cycle in FP64: 1e-13; FP32 kernels and cycles against the FP64 oracle: 1e-5;
* solves in FP64 run to the oracle's iteration count: 1e-12;
* the FP32-preconditioned FP64-refined solve must reach an FP64 relative residual of 1e-10
  (recomputed by the oracle's operator) and is reported against the oracle's solution.
"""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import dec  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


class Pair:
    """The same hierarchy built by the library and by the oracle."""

    def __init__(self, kind, nsub, base_cells=4, bc=None, order=mg.MG_ORDER_STRIPES):
        print(f"[parity] building {kind} base={base_cells} nsub={nsub} order={order}", flush=True)
        self.g = mg.Hierarchy(kind, nsub, base_cells=base_cells, bc=bc, order=order)
        if kind == "square":
            xyz, tri = dec.square_grid(base_cells)
            self.o = omg.Hierarchy(xyz, tri, nsub, bc="dirichlet" if bc in (None, 0) else "natural")
        else:
            xyz, tri = dec.icosahedron()
            self.o = omg.Hierarchy(xyz, tri, nsub, project=True,
                                   bc="natural" if bc in (None, 1) else "dirichlet")
        self.top = self.g.top


@pytest.fixture(scope="module")
def c1():
    return Pair("square", 4)


@pytest.fixture(scope="module")
def sphere():
    return Pair("sphere", 4)


@pytest.fixture(scope="module")
def ragged():
    # 3x3 base: level sizes are not multiples of 64 or 256 (ragged last slice and block)
    return Pair("square", 3, base_cells=3)


@pytest.fixture(scope="module")
def sphere_z():
    # the same icosphere laid out in Z-order instead of stripes
    return Pair("sphere", 4, order=mg.MG_ORDER_MORTON)


PAIRS = ["c1", "sphere", "ragged", "sphere_z"]


# ------------------------------------------------------------------ host build
@pytest.mark.parametrize("which", PAIRS)
def test_host_build_matches_oracle(which, request):
    P = request.getfixturevalue(which)
    for l, ol in enumerate(P.o.levels):
        ex = mg.mg_hierarchy_export(P.g.h, l)
        assert np.array_equal(ex["xyz"], ol.xyz), f"level {l} coordinates"
        assert np.array_equal(ex["tri"], ol.tri)
        assert np.array_equal(ex["edges"], ol.edges)
        assert np.array_equal(ex["tri_edges"], ol.tri_edges)
        assert np.array_equal(ex["tri_sign"], ol.tri_sign)
        assert np.array_equal(ex["boundary"].astype(bool), ol.bnd)
        assert np.abs(ex["star1"] - ol.star1).max() <= 1e-14 * np.abs(ol.star1).max()
        assert np.abs(ex["star0"] - ol.star0).max() <= 1e-14 * np.abs(ol.star0).max()
        if l > 0:
            Mt = ol.Mt.tocsr()
            par = ex["parents"]
            M = np.zeros((ol.nv, P.o.levels[l - 1].nv))
            M[np.arange(ol.nv), par[:, 0]] += 0.5
            M[np.arange(ol.nv), par[:, 1]] += 0.5
            assert np.array_equal(M, Mt.toarray())


# ------------------------------------------------------------------ kernels
def test_weight_storage(c1, sphere):
    """The row kernels read the narrowest exact copy of the weights: binary16 when every
    weight of a level is a binary16 number (grids: star1 in {0, 1/2, 1}), FP32 when every FP64
    weight is an FP32 number, FP64 otherwise (the sphere); a vertex coefficient that breaks
    the exactness switches back, and the operator still matches the oracle."""
    for l in range(c1.top + 1):
        i = mg.mg_hierarchy_info(c1.g.h, l)
        assert (i["weight_bytes32"], i["weight_bytes64"]) == (2, 2), (l, i)
    for l in range(sphere.top + 1):
        i = mg.mg_hierarchy_info(sphere.g.h, l)
        assert (i["weight_bytes32"], i["weight_bytes64"]) == (4, 8), (l, i)
    nv = c1.o.fine.nv
    k = np.exp(0.3 * W.normal(nv, 77))
    mg.mg_hierarchy_set_vertex_coeff(c1.g.h, gpu(k))
    try:
        i = mg.mg_hierarchy_info(c1.g.h, c1.top)
        assert (i["weight_bytes32"], i["weight_bytes64"]) == (4, 8)
        # the finest operator with edge coefficients (k_a + k_b) / 2, built independently;
        # Dirichlet form M L M + (I - M)
        import scipy.sparse as sp
        m = c1.o.fine
        x = W.normal(nv, 78)
        ke = 0.5 * (k[m.edges[:, 0]] + k[m.edges[:, 1]])
        L = (m.d0.T @ sp.diags(m.star1 * ke) @ m.d0).tocsr()
        xm = x.copy()
        xm[m.bnd] = 0.0
        ref = L @ xm
        ref[m.bnd] = x[m.bnd]
        y = torch.zeros(nv, dtype=torch.float64, device=DEV)
        mg.dec_laplacian_apply(c1.g.h, c1.top, gpu(x), y)
        assert rel(host(y), ref) <= 1e-13
    finally:
        mg.mg_hierarchy_set_vertex_coeff(c1.g.h, None)
    i = mg.mg_hierarchy_info(c1.g.h, c1.top)
    assert (i["weight_bytes32"], i["weight_bytes64"]) == (2, 2)


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_laplacian_apply(which, dt, request):
    P = request.getfixturevalue(which)
    tdt, tol = (torch.float64, 1e-14) if dt == "f64" else (torch.float32, 1e-5)
    for l, ol in enumerate(P.o.levels):
        x = W.normal(ol.nv, 100 + l)
        y = torch.zeros(ol.nv, dtype=tdt, device=DEV)
        mg.dec_laplacian_apply(P.g.h, l, gpu(x, tdt), y)
        ref = ol.A @ x
        assert rel(host(y), ref) <= tol, (l, rel(host(y), ref))


@pytest.mark.parametrize("which", PAIRS)
def test_star0_apply(which, request):
    P = request.getfixturevalue(which)
    f = W.normal(P.o.fine.nv, 7)
    b = torch.zeros_like(gpu(f))
    mg.dec_star0_apply(P.g.h, P.top, gpu(f), b)
    assert rel(host(b), P.o.rhs(f)) <= 1e-15


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_smoother(which, dt, request):
    P = request.getfixturevalue(which)
    tdt, tol = (torch.float64, 1e-14) if dt == "f64" else (torch.float32, 1e-5)
    for l, ol in enumerate(P.o.levels):
        b = W.normal(ol.nv, 200 + l)
        x0 = W.normal(ol.nv, 300 + l)
        x = gpu(x0, tdt)
        mg.mg_smooth(P.g.h, l, 3, 0.8, gpu(b, tdt), x)
        ref = omg.jacobi(ol.A, b, x0, 0.8, 3)
        assert rel(host(x), ref) <= tol, (l, rel(host(x), ref))


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_transfers(which, dt, request):
    P = request.getfixturevalue(which)
    tdt, tol = (torch.float64, 1e-15) if dt == "f64" else (torch.float32, 1e-6)
    for l in range(1, P.top + 1):
        ol, oc = P.o.levels[l], P.o.levels[l - 1]
        rf = W.normal(ol.nv, 400 + l)
        if P.o.bc == "dirichlet":
            rf[ol.bnd] = 0.0                  # boundary entries are not unknowns
        rc = torch.zeros(oc.nv, dtype=tdt, device=DEV)
        mg.mg_restrict(P.g.h, l, gpu(rf, tdt), rc)
        assert rel(host(rc), P.o.restrict(l, rf)) <= tol
        ec = W.normal(oc.nv, 500 + l)
        if P.o.bc == "dirichlet":
            ec[oc.bnd] = 0.0
        xf0 = W.normal(ol.nv, 600 + l)
        xf = gpu(xf0, tdt)
        mg.mg_prolong(P.g.h, l, gpu(ec, tdt), xf)
        assert rel(host(xf), xf0 + P.o.prolong(l, ec)) <= tol


# ------------------------------------------------------------------ cycles and solves
@pytest.mark.parametrize("which", PAIRS)
def test_vcycle(which, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default()
    for l in range(P.top + 1):
        ol = P.o.levels[l]
        b = W.normal(ol.nv, 700 + l)
        x0 = W.normal(ol.nv, 800 + l)
        ref = omg.vcycle(P.o, b, x0.copy(), l) if l > 0 else omg.coarse_solve(P.o, b)
        x = gpu(x0)
        mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
        assert rel(host(x), ref) <= 1e-13, (l, rel(host(x), ref))
        x32 = gpu(x0, torch.float32)
        mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
        assert rel(host(x32), ref) <= 1e-5, (l, rel(host(x32), ref))


def _rhs(P, which):
    xyz = P.o.fine.xyz
    if which.startswith("sphere"):
        f = W.sphere_rhs(xyz, W.sh_coefficients())
    elif which == "c1":
        f = W.manufactured_c1(xyz)
    else:
        f = W.normal(len(xyz), 9)
    return P.o.rhs(f)


@pytest.mark.parametrize("which", PAIRS)
def test_mg_solve(which, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, ho = omg.mg_solve(P.o, b)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_solve(P.g.h, mg.mg_opts_default(), gpu(b), x)
    print(f"[parity] mg_solve {which}: cycles gpu {res.iterations} oracle {ko}, "
          f"rel L2 vs oracle {rel(host(x), xo):.2e}, rel residual {res.rel_residual:.2e}")
    assert res.iterations == ko
    assert rel(host(x), xo) <= 1e-12
    assert res.rel_residual <= 1e-10
    assert omg.rel_residual(P.o, b, host(x)) <= 1e-10


def test_c1_closed_form(c1):
    b = _rhs(c1, "c1")
    x = torch.zeros(c1.o.fine.nv, dtype=torch.float64, device=DEV)
    mg.mg_pcg(c1.g.h, mg.mg_opts_default(rtol=1e-13), gpu(b), x)
    h = 1 / 64
    c = (math.pi * h / 2) ** 2 / math.sin(math.pi * h / 2) ** 2
    exact = c * W.manufactured_c1_solution(c1.o.fine.xyz)
    assert np.abs(host(x) - exact).max() < 1e-12


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("graph", [0, 1])
def test_pcg_fp64(which, graph, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, ho = omg.mg_pcg(P.o, b)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(use_graph=graph), gpu(b), x)
    print(f"[parity] pcg fp64 {which}: iters gpu {res.iterations} oracle {ko}, "
          f"rel L2 vs oracle {rel(host(x), xo):.2e}")
    assert res.iterations == ko
    assert rel(host(x), xo) <= 1e-12
    assert abs(res.rel_residual_loop - ho[-1]) <= 1e-3 * ho[-1]
    assert res.rel_residual <= 1e-10


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("outer", [mg.MG_OUTER_FCG, mg.MG_OUTER_IR, mg.MG_OUTER_CG])
@pytest.mark.parametrize("prec", [mg.MG_F64, mg.MG_F32])
def test_outer_methods(which, outer, prec, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    ref = omg.direct_solve(P.o, b)
    solver = {mg.MG_OUTER_FCG: omg.mg_fcg, mg.MG_OUTER_IR: omg.mg_ir, mg.MG_OUTER_CG: omg.mg_pcg}[outer]
    xo, ko, _ = solver(P.o, b)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=outer, precision=prec), gpu(b), x)
    xg = host(x)
    err = rel(xg, ref)
    print(f"[parity] {which} outer={outer} prec={prec}: iters gpu {res.iterations} oracle {ko} "
          f"residual {res.rel_residual:.2e} rel L2 vs direct {err:.2e} vs oracle {rel(xg, xo):.2e}")
    assert omg.rel_residual(P.o, b, xg) <= 1e-10 and res.rel_residual <= 1e-10
    if prec == mg.MG_F64:
        assert res.iterations == ko
        assert rel(xg, xo) <= 1e-12
    else:
        assert abs(res.iterations - ko) <= 2
        assert err <= 1e-7


def test_repeat_calls_are_bitwise_identical(c1):
    b = gpu(_rhs(c1, "c1"))
    outs = []
    for graph in (1, 1, 0):
        x = torch.zeros_like(b)
        mg.mg_pcg(c1.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32,
                                             use_graph=graph), b, x)
        outs.append(host(x))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_status_paths(c1):
    nv = c1.o.fine.nv
    b = gpu(_rhs(c1, "c1"))
    x = torch.zeros_like(b)
    res = mg.mg_pcg(c1.g.h, mg.mg_opts_default(max_iter=1), b, x, raise_on_error=False)
    assert res.status == mg.MG_ENOCONV and res.iterations == 1 and res.rel_residual > 1e-10
    with pytest.raises(mg.MGError) as e:
        mg.mg_pcg(c1.g.h, mg.mg_opts_default(max_iter=1), b, x)
    assert e.value.status == mg.MG_ENOCONV
    bn = b.clone()
    bn[nv // 2] = float("nan")
    res = mg.mg_pcg(c1.g.h, mg.mg_opts_default(), bn, x, raise_on_error=False)
    assert res.status == mg.MG_ENONFINITE
    z = torch.zeros_like(b)
    x.fill_(1.0)
    res = mg.mg_pcg(c1.g.h, mg.mg_opts_default(), z, x)
    assert res.iterations == 0 and torch.all(x == 0)
    with pytest.raises(mg.MGError):
        mg.mg_pcg(c1.g.h, mg.mg_opts_default(rtol=0.0), b, x)
    with pytest.raises(ValueError):
        mg.mg_pcg(c1.g.h, mg.mg_opts_default(), b[:-1].contiguous(), x[:-1].contiguous())


def test_smallest_meshes():
    """Degenerate sizes: a 1-cell Dirichlet square has no unknowns and is refused; a 2-cell one
    has a single unknown (the coarsest solve is the whole method); one subdivision of it gives
    a two-level hierarchy with 9 unknowns.  Each solve matches the oracle's direct solution."""
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy("square", 0, base_cells=1)
    assert e.value.status == mg.MG_EINVAL
    for nsub in (0, 1):
        g = mg.Hierarchy("square", nsub, base_cells=2)
        xyz, tri = dec.square_grid(2)
        o = omg.Hierarchy(xyz, tri, nsub)
        assert g.info[g.top]["n_unknowns"] == (1 if nsub == 0 else 9)
        b = o.rhs(W.manufactured_c1(o.fine.xyz))
        x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
        res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
        ref = omg.direct_solve(o, b)
        _, ko, _ = omg.mg_pcg(o, b)
        assert rel(host(x), ref) <= 1e-13 and res.iterations == ko
        x.zero_()
        mg.mg_pcg(g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32), gpu(b), x)
        assert omg.rel_residual(o, b, host(x)) <= 1e-10
        g.close()
