"""GPU tests of the FP64 fallback of the FP32-preconditioned solve (mg_opts.stall_checks),
forced from the host with the zero-preconditioner fault (MG_DEBUG_ZERO_PRECOND32):

* FCG and CG: a zero FP32 cycle gives p = 0, so p^T A p = 0 (FCG) or z^T r = 0 (CG), a
  breakdown in the first iteration before x moves; the solve goes on from x = 0 with the FP64
  cycle and must reproduce the plain FP64 solve bit for bit, with its iteration count, on a
  Dirichlet square and on the natural-boundary sphere;
* iterative refinement: x stays put and the loop residual stays flat; after the first check
  and stall_checks flat ones (check_every iterations each) the FP64 cycle takes over, and the
  result is the plain FP64 refinement's, bit for bit, after the wasted iterations;
* stall_checks = 0 turns the fallback off: FCG reports MG_EBREAKDOWN, refinement MG_ENOCONV;
* iterations captured as graphs before the fault was set are not reused, and clearing it
  restores the plain mixed solve, which does not fall back;
* the solution meets the oracle's to the solve's tolerance.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import dec  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def problem(kind):
    print(f"[fallback] {kind}", flush=True)
    if kind == "square":
        g = mg.Hierarchy("square", 5, base_cells=4)
        xyz, tri = dec.square_grid(4)
        o = omg.Hierarchy(xyz, tri, 5)
        b = o.rhs(W.manufactured_c1(o.fine.xyz))
    else:
        g = mg.Hierarchy("sphere", 4)
        xyz, tri = dec.icosahedron()
        o = omg.Hierarchy(xyz, tri, 4, project=True, bc="natural")
        b = o.rhs(W.sphere_rhs(o.fine.xyz, W.sh_coefficients(4, 7)))
    return g, o, torch.tensor(b, device=DEV)


def solve(g, b, **kw):
    x = torch.zeros_like(b)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(**kw), b, x, raise_on_error=False)
    return res, host(x)


@pytest.mark.parametrize("kind,outer", [("square", mg.MG_OUTER_FCG), ("square", mg.MG_OUTER_CG),
                                        ("sphere", mg.MG_OUTER_FCG)])
def test_krylov_breakdown_falls_back_to_fp64(kind, outer):
    g, o, b = problem(kind)
    ref, x64 = solve(g, b, outer=outer)
    assert ref.status == mg.MG_OK and ref.fp64_fallback == 0
    mixed, xm = solve(g, b, outer=outer, precision=mg.MG_F32)
    assert mixed.status == mg.MG_OK and mixed.fp64_fallback == 0
    mg.mg_hierarchy_set_debug(g.h, mg.MG_DEBUG_ZERO_PRECOND32)
    res, x = solve(g, b, outer=outer, precision=mg.MG_F32)
    print(f"  outer={outer}: fallback {res.fp64_fallback} status {res.status} "
          f"iterations {res.iterations} (FP64 alone {ref.iterations})", flush=True)
    assert res.status == mg.MG_OK and res.fp64_fallback == 1
    assert res.iterations == ref.iterations
    assert np.array_equal(x, x64)
    assert res.rel_residual <= 1e-10
    # without the fallback the breakdown is reported
    off, _ = solve(g, b, outer=outer, precision=mg.MG_F32, stall_checks=0)
    assert off.status == mg.MG_EBREAKDOWN and off.fp64_fallback == 0
    # the fault cleared: the plain mixed solve again
    mg.mg_hierarchy_set_debug(g.h, 0)
    again, xa = solve(g, b, outer=outer, precision=mg.MG_F32)
    assert again.fp64_fallback == 0 and again.iterations == mixed.iterations
    assert np.array_equal(xa, xm)
    ref_o = omg.direct_solve(o, b.cpu().numpy())
    assert np.linalg.norm(x - ref_o) <= 1e-8 * np.linalg.norm(ref_o)
    g.close()


def test_refinement_stagnation_falls_back_to_fp64():
    g, o, b = problem("square")
    ref, x64 = solve(g, b, outer=mg.MG_OUTER_IR)
    assert ref.status == mg.MG_OK
    mg.mg_hierarchy_set_debug(g.h, mg.MG_DEBUG_ZERO_PRECOND32)
    every, stall = 4, 3
    res, x = solve(g, b, outer=mg.MG_OUTER_IR, precision=mg.MG_F32, check_every=every,
                   stall_checks=stall)
    print(f"  IR: fallback {res.fp64_fallback} status {res.status} iterations {res.iterations} "
          f"(FP64 alone {ref.iterations})", flush=True)
    assert res.status == mg.MG_OK and res.fp64_fallback == 1
    # the first check sets the level, `stall` flat checks follow; then the FP64 loop from x = 0
    assert res.iterations == (1 + stall) * every + ref.iterations
    assert np.array_equal(x, x64)
    # no fallback: refinement on a zero correction never converges
    off, xo = solve(g, b, outer=mg.MG_OUTER_IR, precision=mg.MG_F32, stall_checks=0,
                    max_iter=20)
    assert off.status == mg.MG_ENOCONV and off.iterations == 20 and off.fp64_fallback == 0
    assert not np.any(xo)
    # a budget that ends inside the stagnating stretch: no room left for the FP64 loop
    short, _ = solve(g, b, outer=mg.MG_OUTER_IR, precision=mg.MG_F32, check_every=every,
                     stall_checks=stall, max_iter=(1 + stall) * every)
    assert short.status == mg.MG_ENOCONV and short.iterations == (1 + stall) * every
    g.close()


def test_stall_checks_validated():
    g, _, b = problem("square")
    x = torch.zeros_like(b)
    with pytest.raises(mg.MGError, match="stall_checks"):
        mg.mg_pcg(g.h, mg.mg_opts_default(stall_checks=-1), b, x)
    with pytest.raises(mg.MGError, match="debug flag"):
        mg.mg_hierarchy_set_debug(g.h, 2)
    g.close()
