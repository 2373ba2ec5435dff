"""The convergence check of the CG/FCG loop taken by one extra workgroup of the next
iteration's first kernel (the two Jacobi sweeps from zero on a row-pattern finest level), or
at the end of a batch of iterations, instead of by a launch of its own after the residual
update.  It is used with mg_opts.fuse_levels = 1 where the finest level opens its cycle with
those sweeps; fuse_levels = 0 runs the separate check.  The extra workgroup sums the partials
in the separate finaliser's order, so both must give the same bits: solution, iteration
count, status, loop and true residuals, residual history.  Cases: FCG and CG, FP32 and FP64
cycles, V- and W-cycles, graph replay and eager launches, host checks after every iteration,
an iteration limit that ends the loop, and the FP64 fallback after a forced breakdown, on a
1025 x 1025 grid (finest level 1,046,529 rows, untiled, 9 row patterns).  On finest levels cut
into workgroup tiles the check rides with the tiled down leg instead: FCG and CG, FP32 and
FP64 cycles, on a 129 x 129 grid (Dirichlet) and the level-6 icosphere (natural boundary,
mean-projected), each against fuse_levels = 0 (no tiles, separate check)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def grid():
    print("[fused-check] build 1025 x 1025", flush=True)
    g = mg.Hierarchy("square", 7, base_cells=8)
    top = g.info[g.top]
    assert top["fused_tiles"] == 0 and top["row_patterns"] > 0, top
    yield g
    g.close()


def rhs(g, seed):
    rng = np.random.default_rng(seed)
    return torch.as_tensor(rng.standard_normal(g.nv()), dtype=torch.float64, device=DEV)


def solve(g, b, **kw):
    x = torch.zeros_like(b)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(**kw), b, x, raise_on_error=False, history=64)
    torch.cuda.synchronize()
    return res, x.cpu().numpy()


def same(a, b):
    ra, xa = a
    rb, xb = b
    assert ra.status == rb.status
    assert ra.iterations == rb.iterations
    assert ra.rel_residual_loop == rb.rel_residual_loop
    assert ra.rel_residual == rb.rel_residual
    assert list(ra.hist) == list(rb.hist)
    assert ra.fp64_fallback == rb.fp64_fallback
    assert np.array_equal(xa, xb)


CASES = [
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32),
    dict(outer=mg.MG_OUTER_CG, precision=mg.MG_F32),
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F64),
    dict(outer=mg.MG_OUTER_CG, precision=mg.MG_F64),
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, cycle=mg.MG_CYCLE_W),
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, use_graph=0),
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, check_every=1),
    dict(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, nu1=3, nu2=1),
]


@pytest.mark.parametrize("kw", CASES, ids=[str(i) for i in range(len(CASES))])
def test_fused_check_matches_separate_check(grid, kw):
    b = rhs(grid, 21)
    print(f"  {kw}", flush=True)
    fused = solve(grid, b, fuse_levels=1, **kw)
    plain = solve(grid, b, fuse_levels=0, **kw)
    print(f"  iterations {fused[0].iterations}, loop residual {fused[0].rel_residual_loop:.3e}",
          flush=True)
    assert fused[0].status == mg.MG_OK and fused[0].rel_residual <= 1e-10
    same(fused, plain)
    # again on the same hierarchy (the first batch is sized from this solve's count)
    same(fused, solve(grid, b, fuse_levels=1, **kw))


@pytest.mark.parametrize("limit", [1, 3])
def test_iteration_limit(grid, limit):
    b = rhs(grid, 22)
    fused = solve(grid, b, fuse_levels=1, precision=mg.MG_F32, max_iter=limit)
    plain = solve(grid, b, fuse_levels=0, precision=mg.MG_F32, max_iter=limit)
    assert fused[0].status == mg.MG_ENOCONV and fused[0].iterations == limit
    same(fused, plain)


def test_fallback_after_breakdown(grid):
    b = rhs(grid, 23)
    ref = solve(grid, b, fuse_levels=1)
    mg.mg_hierarchy_set_debug(grid.h, mg.MG_DEBUG_ZERO_PRECOND32)
    try:
        fused = solve(grid, b, fuse_levels=1, precision=mg.MG_F32)
        plain = solve(grid, b, fuse_levels=0, precision=mg.MG_F32)
    finally:
        mg.mg_hierarchy_set_debug(grid.h, 0)
    print(f"  fallback {fused[0].fp64_fallback} iterations {fused[0].iterations} "
          f"(FP64 alone {ref[0].iterations})", flush=True)
    assert fused[0].status == mg.MG_OK and fused[0].fp64_fallback == 1
    assert fused[0].iterations == ref[0].iterations
    assert np.array_equal(fused[1], ref[1])
    same(fused, plain)


TILED = [("square", mg.MG_OUTER_FCG, mg.MG_F32), ("square", mg.MG_OUTER_CG, mg.MG_F64),
         ("square", mg.MG_OUTER_FCG, mg.MG_F64), ("sphere", mg.MG_OUTER_FCG, mg.MG_F32),
         ("sphere", mg.MG_OUTER_CG, mg.MG_F64)]


@pytest.mark.parametrize("kind,outer,precision", TILED)
def test_fused_check_in_tiled_down_leg(kind, outer, precision):
    print(f"[fused-check] tiled {kind} outer={outer} precision={precision}", flush=True)
    g = mg.Hierarchy("square", 5, base_cells=4) if kind == "square" else mg.Hierarchy("sphere", 6)
    try:
        assert g.info[g.top]["fused_tiles"] > 0, g.info[g.top]
        rng = np.random.default_rng(24)
        bh = rng.standard_normal(g.nv())
        if kind == "sphere":
            bh -= bh.mean()
        b = torch.as_tensor(bh, dtype=torch.float64, device=DEV)
        fused = solve(g, b, fuse_levels=1, outer=outer, precision=precision)
        plain = solve(g, b, fuse_levels=0, outer=outer, precision=precision)
        print(f"  iterations {fused[0].iterations}", flush=True)
        assert fused[0].status == mg.MG_OK and fused[0].rel_residual <= 1e-10
        same(fused, plain)
        same(fused, solve(g, b, fuse_levels=1, outer=outer, precision=precision, use_graph=0))
    finally:
        g.close()
