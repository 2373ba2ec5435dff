"""The fused cycle legs on launch-bound binary levels (mg_opts.fuse_levels = 1): each workgroup
tile recomputes the rings of rows its leg needs around its own rows, and every value is formed
with the expressions and entry order of the one-launch-per-step kernels.  The results must
therefore equal those of fuse_levels = 0 bit for bit: one cycle of every shape, with several
sweep counts (those the tiles do not cover fall back per leg), in FP64 and FP32, and whole
solves with and without graph replay.  Agreement of the unfused path with the oracle is the
subject of the other parity tests (which now run fused by default).

Meshes: a 257 x 257 square (uniform slices, 4 entries per row), a ragged 97 x 97 square, the
icosphere (natural boundary, 6 entries per row), a fan disk whose centre has valence 8 (slices
of different widths: the tiles then carry each row's entry index), and two hierarchies with
cubic (weighted) transfers: cubic, cubic, binary subdivisions of the 4 x 4 square, and the
105,625-vertex mesh of four cubic subdivisions."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def fan_disk(m):
    xyz = [[0.0, 0.0, 0.0]] + [[math.cos(2 * math.pi * k / m), math.sin(2 * math.pi * k / m), 0.0]
                               for k in range(m)]
    tri = [[0, 1 + k, 1 + (k + 1) % m] for k in range(m)]
    return np.array(xyz), np.array(tri, dtype=np.int32)


def build(which):
    print(f"[tiles] building {which}", flush=True)
    if which == "sq":
        return mg.Hierarchy("square", 5, base_cells=8)
    if which == "rag":
        return mg.Hierarchy("square", 5, base_cells=3)
    if which == "sphere":
        return mg.Hierarchy("sphere", 5, bc=mg.MG_BC_NATURAL)
    if which == "cubic":
        return mg.Hierarchy("square", 3, base_cells=4, cubic_mask=0b011)
    if which == "e1":
        return mg.Hierarchy("square", 4, base_cells=4, cubic_mask=0b1111)
    xyz, tri = fan_disk(8)
    return mg.Hierarchy("arrays", 5, xyz=xyz, tri=tri)


MESHES = ["sq", "rag", "sphere", "fan8", "cubic", "e1"]


@pytest.fixture(scope="module")
def hier():
    cache = {}

    def get(which):
        if which not in cache:
            cache[which] = build(which)
        return cache[which]
    yield get
    for h in cache.values():
        h.close()


def tensor(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


@pytest.mark.parametrize("which", MESHES)
def test_tiles_present(which, hier):
    H = hier(which)
    for l in range(1, H.top + 1):
        info = mg.mg_hierarchy_info(H.h, l)
        n = info["n_unknowns"]
        # runs of the Morton order inside aligned blocks of at most 256 rows
        assert (n + 255) // 256 <= info["fused_tiles"] <= 2 * ((n + 255) // 256) + 64, (l, info)
        # own rows plus the overlap rings of compact patches
        assert n <= info["fused_tile_rows"] <= 4 * n, (l, info)
        print(f"[tiles] {which} level {l}: {n} rows, {info['fused_tiles']} tiles, "
              f"{info['fused_tile_rows'] / n:.2f} rows held per row")
    assert mg.mg_hierarchy_info(H.h, 0)["fused_tiles"] == 0


SWEEPS = [(2, 2), (1, 1), (0, 2), (2, 0), (1, 2), (3, 3)]


@pytest.mark.parametrize("which", MESHES)
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [mg.MG_CYCLE_V, mg.MG_CYCLE_W, mg.MG_CYCLE_F])
def test_cycle_bit_exact(which, dt, shape, hier):
    H = hier(which)
    n = H.nv()
    b = tensor(W.normal(n, 31), dt)
    x0 = tensor(W.normal(n, 32), dt)
    for nu1, nu2 in SWEEPS:
        out = []
        for fuse in (1, 0):
            o = mg.mg_opts_default(cycle=shape, fuse_levels=fuse)
            o.nu1, o.nu2 = nu1, nu2
            for start in (x0, torch.zeros_like(x0)):
                x = start.clone()
                mg.mg_vcycle(H.h, o, H.top, b, x)
                out.append(x)
        torch.cuda.synchronize()
        for a, c in ((out[0], out[2]), (out[1], out[3])):
            assert torch.isfinite(a).all()
            assert torch.equal(a, c), (which, dt, shape, nu1, nu2,
                                       float((a - c).abs().max()))


@pytest.mark.parametrize("which", MESHES)
@pytest.mark.parametrize("graph", [0, 1])
def test_solves_bit_exact(which, graph, hier):
    H = hier(which)
    n = H.nv()
    b = W.normal(n, 33)
    if which == "sphere":
        b = b - b.mean()
    bt = tensor(b, torch.float64)
    for outer, prec in ((mg.MG_OUTER_CG, mg.MG_F64), (mg.MG_OUTER_FCG, mg.MG_F32)):
        got = []
        for fuse in (1, 0):
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            res = mg.mg_pcg(H.h, mg.mg_opts_default(outer=outer, precision=prec,
                                                    use_graph=graph, fuse_levels=fuse), bt, x)
            got.append((res.iterations, res.rel_residual, x))
        assert got[0][0] == got[1][0] and got[0][1] == got[1][1]
        assert torch.equal(got[0][2], got[1][2])
        assert got[0][1] <= 1e-10
        # a second fused solve replays the captured iteration: same answer
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        res = mg.mg_pcg(H.h, mg.mg_opts_default(outer=outer, precision=prec, use_graph=graph),
                        bt, x)
        assert res.iterations == got[0][0] and torch.equal(x, got[0][2])


@pytest.mark.parametrize("which", MESHES)
@pytest.mark.parametrize("sweeps", [(2, 2), (1, 2)])
def test_mg_solve_bit_exact(which, sweeps, hier):
    """Stand-alone cycles: the finest level's fused up leg ends in the partner buffer, which
    the loop copies back (and so does an odd number of sweeps per cycle)."""
    H = hier(which)
    n = H.nv()
    b = W.normal(n, 34)
    if which == "sphere":
        b = b - b.mean()
    bt = tensor(b, torch.float64)
    got = []
    for fuse in (1, 0):
        o = mg.mg_opts_default(fuse_levels=fuse)
        o.nu1, o.nu2 = sweeps
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        res = mg.mg_solve(H.h, o, bt, x)
        got.append((res.iterations, res.rel_residual, x))
    assert got[0][0] == got[1][0] and got[0][1] == got[1][1] and got[0][1] <= 1e-10
    assert torch.equal(got[0][2], got[1][2])


def test_fuse_levels_validated(hier):
    H = hier("sq")
    n = H.nv()
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as e:
        mg.mg_vcycle(H.h, mg.mg_opts_default(fuse_levels=2), H.top, x.clone(), x)
    assert e.value.status == mg.MG_EINVAL
