"""GPU parity on hierarchies with cubic (1-to-9) subdivisions, alone and mixed with binary ones
(Sec. 2.2.1; M(f) of Def. 5 with barycentric weights 2/3, 1/3 and 1/3, 1/3, 1/3), against the
oracle built with the same scheme string.

Tolerances as in test_gpu_parity.py, except the FP64 restriction: a cubic restriction row sums
up to 19 weighted terms (the kept vertex, two points on each incident edge, the centroid of
each incident triangle) in another order than the oracle's sparse product, so it is held to
1e-14 instead of 1e-15."""
import ctypes

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
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def mask(schemes):
    return sum(1 << k for k, s in enumerate(schemes) if s == "c")


class Pair:
    def __init__(self, kind, schemes, base_cells=4):
        nsub = len(schemes)
        print(f"[cubic] building {kind} base={base_cells} schemes={schemes}", flush=True)
        self.g = mg.Hierarchy(kind, nsub, base_cells=base_cells, cubic_mask=mask(schemes))
        if kind == "square":
            xyz, tri = dec.square_grid(base_cells)
            self.o = omg.Hierarchy(xyz, tri, nsub, schemes=schemes)
        else:
            xyz, tri = dec.icosahedron()
            self.o = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural", schemes=schemes)
        self.schemes = schemes
        self.top = self.g.top


@pytest.fixture(scope="module")
def ccb():
    # 4x4 base -> 12 -> 36 -> 72 cells per side: 73 x 73 vertices on the finest level
    return Pair("square", "ccb")


@pytest.fixture(scope="module")
def bcb():
    # 3x3 base -> 6 -> 18 -> 36: ragged slices and blocks on every level
    return Pair("square", "bcb", base_cells=3)


@pytest.fixture(scope="module")
def cbc():
    # icosphere 20 -> 180 -> 720 -> 6480 triangles, natural boundary
    return Pair("sphere", "cbc")


PAIRS = ["ccb", "bcb", "cbc"]


def _rhs(P, which):
    if which == "cbc":
        return P.o.rhs(W.sphere_rhs(P.o.fine.xyz, W.sh_coefficients()))
    return P.o.rhs(W.normal(P.o.fine.nv, 71))


@pytest.mark.parametrize("which", PAIRS)
def test_host_build_and_interpolation(which, request):
    P = request.getfixturevalue(which)
    for l, ol in enumerate(P.o.levels):
        info = mg.mg_hierarchy_info(P.g.h, l)
        assert info["scheme"] == (0 if l == 0 else {"b": 1, "c": 2}[P.schemes[l - 1]])
        ex = mg.mg_hierarchy_export(P.g.h, l)
        assert np.array_equal(ex["xyz"], ol.xyz), f"level {l} coordinates"
        assert np.array_equal(ex["tri"], ol.tri)
        assert np.array_equal(ex["edges"], ol.edges)
        assert np.array_equal(ex["boundary"].astype(bool), ol.bnd)
        assert np.abs(ex["star1"] - ol.star1).max() <= 1e-14 * np.abs(ol.star1).max()
        if l == 0:
            continue
        par, w = mg.mg_hierarchy_export_interp(P.g.h, l)
        M = np.zeros((ol.nv, P.o.levels[l - 1].nv))
        for q in range(3):
            np.add.at(M, (np.arange(ol.nv), par[:, q]), w[:, q])
        assert np.array_equal(M, ol.Mt.toarray()), f"level {l} interpolation"


def test_binary_parent_export_refused_on_cubic_level(ccb):
    nv = ccb.o.levels[1].nv
    par = np.empty((nv, 2), np.int32)
    st = mg.lib().mg_hierarchy_export(ccb.g.h, 1, None, None, None, None, None, None, None, None,
                                      par.ctypes.data_as(ctypes.c_void_p))
    assert st == mg.MG_EINVAL


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_operator_and_transfers(which, dt, request):
    P = request.getfixturevalue(which)
    tdt = torch.float64 if dt == "f64" else torch.float32
    t_op, t_r, t_p = (1e-14, 1e-14, 1e-15) if dt == "f64" else (1e-5, 1e-6, 1e-6)
    for l in range(P.top + 1):
        ol = P.o.levels[l]
        x = W.normal(ol.nv, 100 + l)
        y = torch.zeros(ol.nv, dtype=tdt, device=DEV)
        mg.dec_laplacian_apply(P.g.h, l, gpu(x, tdt), y)
        assert rel(host(y), ol.A @ x) <= t_op, (l, "operator")
        if l == 0:
            continue
        oc = P.o.levels[l - 1]
        rf = W.normal(ol.nv, 400 + l)
        if P.o.bc == "dirichlet":
            rf[ol.bnd] = 0.0
        rc = torch.zeros(oc.nv, dtype=tdt, device=DEV)
        mg.mg_restrict(P.g.h, l, gpu(rf, tdt), rc)
        assert rel(host(rc), P.o.restrict(l, rf)) <= t_r, (l, "restrict")
        ec = W.normal(oc.nv, 500 + l)
        if P.o.bc == "dirichlet":
            ec[oc.bnd] = 0.0
        xf0 = W.normal(ol.nv, 600 + l)
        xf = gpu(xf0, tdt)
        mg.mg_prolong(P.g.h, l, gpu(ec, tdt), xf)
        assert rel(host(xf), xf0 + P.o.prolong(l, ec)) <= t_p, (l, "prolong")


@pytest.mark.parametrize("shape", ["V", "W", "F"])
@pytest.mark.parametrize("which", PAIRS)
def test_one_cycle(which, shape, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default(cycle={"V": mg.MG_CYCLE_V, "W": mg.MG_CYCLE_W,
                                  "F": mg.MG_CYCLE_F}[shape])
    for l in range(1, P.top + 1):
        ol = P.o.levels[l]
        b = W.normal(ol.nv, 700 + l)
        x0 = W.normal(ol.nv, 800 + l)
        ref = omg.mgcycle(P.o, b, x0.copy(), l, shape)
        x = gpu(x0)
        mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
        assert rel(host(x), ref) <= 1e-13, (l, rel(host(x), ref))
        x32 = gpu(x0, torch.float32)
        mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
        assert rel(host(x32), ref) <= 1e-5, (l, rel(host(x32), ref))


@pytest.mark.parametrize("which", PAIRS)
def test_gs_cycle(which, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default(smoother=mg.MG_SMOOTH_GS)
    l = P.top
    b = W.normal(P.o.fine.nv, 901)
    if P.o.bc == "dirichlet":
        b[P.o.fine.bnd] = 0.0
    x0 = W.normal(P.o.fine.nv, 902)
    if P.o.bc == "dirichlet":
        x0[P.o.fine.bnd] = 0.0
    ref = omg.mgcycle(P.o, b, x0.copy(), l, "V", smoother="gs")
    x = gpu(x0)
    mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
    assert rel(host(x), ref) <= 1e-13


@pytest.mark.parametrize("which", PAIRS)
@pytest.mark.parametrize("graph", [0, 1])
def test_solves(which, graph, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, _ = omg.mg_pcg(P.o, b)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(use_graph=graph), gpu(b), x)
    e = rel(host(x), xo)
    print(f"[cubic] {which} FP64 MG-PCG: {res.iterations} iterations (oracle {ko}), rel L2 {e:.2e}")
    assert res.iterations == ko and e <= 1e-12
    xs, ks, _ = omg.mg_solve(P.o, b)
    x.zero_()
    res = mg.mg_solve(P.g.h, mg.mg_opts_default(use_graph=graph), gpu(b), x)
    assert res.iterations == ks and rel(host(x), xs) <= 1e-12
    x.zero_()
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32,
                                              use_graph=graph), gpu(b), x)
    r = omg.rel_residual(P.o, b, host(x))
    print(f"[cubic] {which} FP32-preconditioned FCG: {res.iterations} iterations, "
          f"FP64 rel residual {r:.2e}")
    assert r <= 1e-10


def test_batch_refuses_cubic(ccb):
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_create([ccb.g.h], mg.mg_opts_default(outer=mg.MG_OUTER_FCG))
    assert e.value.status == mg.MG_EINVAL


def test_cubic_mask_beyond_levels_rejected():
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy("square", 2, cubic_mask=0b100)
    assert e.value.status == mg.MG_EINVAL


def test_e1_fullsize_cycles():
    """The paper's largest V-cycle mesh: 4 cubic subdivisions of the 32-triangle square
    (325 x 325 = 105,625 vertices), b = L r with r ~ U[0,1) (zero on the boundary).  One V-cycle with three CG
    smoothing steps and one with Jacobi(2,2), each from x = 0, element by element against the
    oracle, and FP64 MG-PCG at the oracle's iteration count."""
    xyz, tri = dec.square_grid(4)
    print("[cubic] building the 105,625-vertex cubic hierarchy", flush=True)
    g = mg.Hierarchy("square", 4, base_cells=4, cubic_mask=0b1111)
    o = omg.Hierarchy(xyz, tri, 4, schemes="cccc")
    assert o.fine.nv == 105625 == g.nv()
    r = W.uniform01(o.fine.nv, W.SEED_E1)
    b = o.fine.A @ r
    b[o.fine.bnd] = 0.0     # zero Dirichlet data: the library's iterates then equal the oracle's
    for smoother, nu, code in (("cg", 3, mg.MG_SMOOTH_CG), ("jacobi", 2, mg.MG_SMOOTH_JACOBI)):
        opts = mg.mg_opts_default(smoother=code)
        opts.nu1 = opts.nu2 = nu
        ref = omg.mgcycle(o, b, np.zeros(o.fine.nv), o.top, "V", nu1=nu, nu2=nu,
                          smoother=smoother)
        x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
        mg.mg_vcycle(g.h, opts, g.top, gpu(b), x)
        e = rel(host(x), ref)
        print(f"[cubic] E1 V-cycle ({smoother}, {nu}): rel L2 vs oracle {e:.2e}")
        assert e <= 1e-12
    xo, ko, _ = omg.mg_pcg(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    g.close()
