"""GPU parity of hierarchies over given meshes and geometric maps (mg_hierarchy_build_maps) and
of map composition (mg_geomap_compose), against the oracle's Hierarchy.from_maps and compose.

Inputs: the non-nested workload (independently jittered 4..64-cell grids, maps by point
location, from the input generator) with zero Dirichlet and natural boundaries, and a nested
case whose meshes and maps are the library's own exports of a binary/cubic subdivision
hierarchy.  Tolerances as in test_gpu_parity.py (weighted restriction: 1e-14, as in
test_gpu_cubic.py); composition agrees with the sparse product to 1e-15 per entry."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

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


class Pair:
    def __init__(self, bc):
        print(f"[geomap] building the jittered-grid hierarchy, bc={bc}", flush=True)
        meshes, maps = W.maps_workload()
        self.meshes, self.maps = meshes, maps
        self.g = mg.Hierarchy.from_maps([m[0] for m in meshes], [m[1] for m in meshes], maps,
                                        bc=mg.MG_BC_DIRICHLET0 if bc == "dirichlet"
                                        else mg.MG_BC_NATURAL)
        self.o = omg.Hierarchy.from_maps(meshes, maps, bc=bc)
        self.top = self.g.top


@pytest.fixture(scope="module")
def jd():
    P = Pair("dirichlet")
    yield P
    P.g.close()


@pytest.fixture(scope="module")
def jn():
    P = Pair("natural")
    yield P
    P.g.close()


def _rhs(P):
    b = P.o.rhs(W.normal(P.o.fine.nv, 81))
    if P.o.bc == "natural":
        b -= b.mean()
    return b


@pytest.mark.parametrize("which", ["jd", "jn"])
def test_levels_and_interpolation(which, request):
    P = request.getfixturevalue(which)
    for l, ol in enumerate(P.o.levels):
        info = mg.mg_hierarchy_info(P.g.h, l)
        assert info["scheme"] == (0 if l == 0 else 3)
        ex = mg.mg_hierarchy_export(P.g.h, l)
        assert np.array_equal(ex["xyz"], ol.xyz)
        assert np.array_equal(ex["edges"], ol.edges)
        assert np.abs(ex["star1"] - ol.star1).max() <= 1e-14 * np.abs(ol.star1).max()
        if l:
            par, w = mg.mg_hierarchy_export_interp(P.g.h, l)
            M = np.zeros((ol.nv, P.o.levels[l - 1].nv))
            for q in range(3):
                np.add.at(M, (np.arange(ol.nv), par[:, q]), w[:, q])
            assert np.array_equal(M, ol.Mt.toarray())


@pytest.mark.parametrize("which", ["jd", "jn"])
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
        ec = W.normal(oc.nv, 500 + l)
        if P.o.bc == "dirichlet":
            rf[ol.bnd] = 0.0
            ec[oc.bnd] = 0.0
        rc = torch.zeros(oc.nv, dtype=tdt, device=DEV)
        mg.mg_restrict(P.g.h, l, gpu(rf, tdt), rc)
        assert rel(host(rc), P.o.restrict(l, rf)) <= t_r, (l, "restrict")
        xf0 = W.normal(ol.nv, 600 + l)
        if P.o.bc == "dirichlet":
            xf0[ol.bnd] = 0.0
        xf = gpu(xf0, tdt)
        mg.mg_prolong(P.g.h, l, gpu(ec, tdt), xf)
        assert rel(host(xf), xf0 + P.o.prolong(l, ec)) <= t_p, (l, "prolong")


@pytest.mark.parametrize("which", ["jd", "jn"])
def test_cycles(which, request):
    P = request.getfixturevalue(which)
    for shape, code in (("V", mg.MG_CYCLE_V), ("W", mg.MG_CYCLE_W)):
        o = mg.mg_opts_default(cycle=code)
        for l in range(1, P.top + 1):
            ol = P.o.levels[l]
            b = W.normal(ol.nv, 700 + l)
            x0 = W.normal(ol.nv, 800 + l)
            ref = omg.mgcycle(P.o, b, x0.copy(), l, shape)
            x = gpu(x0)
            mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
            assert rel(host(x), ref) <= 1e-13, (shape, l, rel(host(x), ref))
            x32 = gpu(x0, torch.float32)
            mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
            assert rel(host(x32), ref) <= 1e-5, (shape, l)


@pytest.mark.parametrize("which", ["jd", "jn"])
@pytest.mark.parametrize("graph", [0, 1])
def test_solves(which, graph, request):
    P = request.getfixturevalue(which)
    b = _rhs(P)
    xo, ko, _ = omg.mg_pcg(P.o, b)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(use_graph=graph), gpu(b), x)
    e = rel(host(x), xo)
    print(f"[geomap] {which} FP64 MG-PCG: {res.iterations} iterations (oracle {ko}), rel L2 {e:.2e}")
    assert res.iterations == ko and e <= 1e-12
    x.zero_()
    mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32,
                                        use_graph=graph), gpu(b), x)
    assert omg.rel_residual(P.o, b, host(x)) <= 1e-10


def test_vertex_coefficient_needs_kept_ids(jd):
    k = torch.ones(jd.o.fine.nv, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as e:
        mg.mg_hierarchy_set_vertex_coeff(jd.g.h, k)
    assert e.value.status == mg.MG_EINVAL


def test_batch_refuses_maps(jd):
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_create([jd.g.h], mg.mg_opts_default(outer=mg.MG_OUTER_FCG))
    assert e.value.status == mg.MG_EINVAL


def test_nested_maps_from_exports_match_subdivision():
    """Meshes and maps exported by a subdivision hierarchy, fed back as given maps: the
    solves follow the oracle's subdivision hierarchy, and the coefficient is accepted."""
    print("[geomap] nested maps from a bcb export", flush=True)
    src = mg.Hierarchy("square", 3, base_cells=3, cubic_mask=0b010)
    xyzs, tris, maps = [], [], []
    for l in range(src.n_levels):
        ex = mg.mg_hierarchy_export(src.h, l)
        xyzs.append(ex["xyz"])
        tris.append(ex["tri"])
        if l:
            par, w = mg.mg_hierarchy_export_interp(src.h, l)
            nv = len(ex["xyz"])
            keep = w.ravel() != 0.0
            M = sp.csc_matrix((w.ravel()[keep], (par.ravel()[keep], np.repeat(np.arange(nv), 3)[keep])),
                              shape=(len(xyzs[-2]), nv))
            maps.append(M)
    src.close()
    g = mg.Hierarchy.from_maps(xyzs, tris, maps)
    xyz, tri = dec.square_grid(3)
    o = omg.Hierarchy(xyz, tri, 3, schemes="bcb")
    b = o.rhs(W.normal(o.fine.nv, 91))
    xo, ko, _ = omg.mg_pcg(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    mg.mg_hierarchy_set_vertex_coeff(g.h, torch.ones(o.fine.nv, dtype=torch.float64, device=DEV))
    g.close()


def _bad_map_status(P, edit):
    M = sp.csc_matrix(P.maps[-1], copy=True)
    colptr, rowval, nzval = M.indptr.astype(np.int64), M.indices.copy(), M.data.copy()
    colptr, rowval, nzval = edit(colptr, rowval, nzval, M)
    maps = list(P.maps[:-1]) + [(colptr, rowval, nzval, M.shape)]
    with pytest.raises(mg.MGError) as e:
        mg.Hierarchy.from_maps([m[0] for m in P.meshes], [m[1] for m in P.meshes], maps)
    return e.value.status


def test_invalid_maps_rejected(jd):
    j = int(np.nonzero(np.diff(sp.csc_matrix(jd.maps[-1]).indptr) == 3)[0][0])

    def weights_off(cp, rv, nz, M):
        nz = nz.copy()
        nz[cp[j]] += 0.01
        return cp, rv, nz

    def not_a_simplex(cp, rv, nz, M):
        rv = rv.copy()
        far = (int(rv[cp[j]]) + M.shape[0] // 2) % M.shape[0]
        rv[cp[j] + 2] = far if far not in rv[cp[j]:cp[j] + 2] else (far + 1) % M.shape[0]
        return cp, rv, nz

    def row_out_of_range(cp, rv, nz, M):
        rv = rv.copy()
        rv[cp[j]] = M.shape[0]
        return cp, rv, nz

    def negative(cp, rv, nz, M):
        nz = nz.copy()
        nz[cp[j]] = -nz[cp[j]]
        return cp, rv, nz

    for edit in (weights_off, not_a_simplex, row_out_of_range, negative):
        assert _bad_map_status(jd, edit) == mg.MG_EINVAL, edit.__name__


def test_compose_matches_product(jd):
    maps = [sp.csc_matrix(M) for M in jd.maps]
    for a, b in ((0, 1), (1, 2), (2, 3)):
        # f: mesh b+1 -> mesh b, g: mesh b -> mesh a (a = b - 1)
        f, g = maps[b], maps[a]
        cp, rv, nz, shape = mg.mg_geomap_compose(g, f)
        C = sp.csc_matrix((nz, rv, cp), shape=shape)
        ref = omg.compose(g, f)
        assert C.shape == ref.shape and C.nnz == ref.nnz
        assert np.abs((C - ref).toarray()).max() <= 1e-15
        for j in range(shape[1]):
            assert np.all(np.diff(rv[cp[j]:cp[j + 1]]) > 0)
    # the whole chain: M(f_0 o ... o f_3)
    C = (maps[0].indptr, maps[0].indices, maps[0].data, maps[0].shape)
    for M in maps[1:]:
        C = mg.mg_geomap_compose(C, M)
    ref = maps[0] @ maps[1] @ maps[2] @ maps[3]
    got = sp.csc_matrix((C[2], C[1], C[0]), shape=C[3])
    assert np.abs((got - ref).toarray()).max() <= 1e-15
    assert np.abs(got.T @ jd.meshes[0][0] - jd.meshes[-1][0]).max() <= 1e-14


def test_compose_capacity_and_shape_errors(jd):
    f = sp.csc_matrix(jd.maps[1])
    g = sp.csc_matrix(jd.maps[0])
    gg, kg = mg._geomap(g)
    ff, kf = mg._geomap(f)
    nnz = ctypes.c_int64(0)
    assert mg.lib().mg_geomap_compose(ctypes.byref(gg), ctypes.byref(ff), None, None, None,
                                      ctypes.byref(nnz)) == 0
    small = ctypes.c_int64(nnz.value - 1)
    cp = np.empty(f.shape[1] + 1, np.int64)
    rv = np.empty(nnz.value, np.int32)
    nz = np.empty(nnz.value)
    assert mg.lib().mg_geomap_compose(ctypes.byref(gg), ctypes.byref(ff), cp.ctypes.data,
                                      rv.ctypes.data, nz.ctypes.data,
                                      ctypes.byref(small)) == mg.MG_EINVAL
    assert mg.lib().mg_geomap_compose(ctypes.byref(ff), ctypes.byref(ff), None, None, None,
                                      ctypes.byref(nnz)) == mg.MG_EINVAL
