"""Full-size parity: the 2049 x 2049 grid (8x8 base, 8 subdivisions, 4.2 M vertices) that
bench.py times, and the level-7 icosphere (163,842 vertices), against the FP64 oracle.

The oracle is fast enough at these sizes (about 20 s to build the 9-level grid hierarchy, under
1 s per V-cycle) to compare whole vectors element by element, with the same launch
configuration as the benchmark (graph replay, default options)."""
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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


@pytest.fixture(scope="module")
def c3():
    print("[fullsize] building the 2049x2049 hierarchy (library and oracle)", flush=True)
    g = mg.Hierarchy("square", W.C3["nsub"], base_cells=W.C3["base_cells"])
    xyz, tri = dec.square_grid(W.C3["base_cells"])
    o = omg.Hierarchy(xyz, tri, W.C3["nsub"])
    b = o.rhs(W.normal(o.fine.nv, W.SEED_C3))
    print("[fullsize] built", flush=True)
    yield g, o, b
    g.close()


def test_c3_rhs_and_kernels(c3):
    g, o, b = c3
    top = g.top
    f = W.normal(o.fine.nv, W.SEED_C3)
    bg = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    mg.dec_star0_apply(g.h, top, gpu(f), bg)
    assert rel(host(bg), b) <= 1e-15
    x0 = W.normal(o.fine.nv, 31)
    y = torch.zeros_like(bg)
    mg.dec_laplacian_apply(g.h, top, gpu(x0), y)
    assert rel(host(y), o.fine.A @ x0) <= 1e-14
    x = gpu(x0)
    mg.mg_smooth(g.h, top, 1, 0.8, bg, x)
    ref = omg.jacobi(o.fine.A, b, x0, 0.8, 1)
    assert rel(host(x), ref) <= 1e-14
    x32 = gpu(x0, torch.float32)
    mg.mg_smooth(g.h, top, 1, 0.8, gpu(b, torch.float32), x32)
    assert rel(host(x32), ref) <= 1e-6


def test_c3_vcycle(c3):
    g, o, b = c3
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    mg.mg_vcycle(g.h, mg.mg_opts_default(), g.top, gpu(b), x)
    ref = omg.vcycle(o, b)
    assert rel(host(x), ref) <= 1e-13
    x32 = torch.zeros(o.fine.nv, dtype=torch.float32, device=DEV)
    mg.mg_vcycle(g.h, mg.mg_opts_default(), g.top, gpu(b, torch.float32), x32)
    e32 = rel(host(x32), ref)
    print(f"[fullsize] FP32 V-cycle vs FP64 oracle cycle: rel L2 {e32:.2e}")
    assert e32 <= 1e-5


def test_c3_fp64_pcg_matches_oracle(c3):
    g, o, b = c3
    xo, ko, ho = omg.mg_pcg(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    err = rel(host(x), xo)
    print(f"[fullsize] C3 FP64 MG-PCG: iterations {res.iterations} (oracle {ko}), "
          f"rel residual {res.rel_residual:.3e}, rel L2 vs oracle {err:.2e}")
    assert res.iterations == ko
    assert err <= 1e-12


def test_c3_mixed_fcg(c3):
    g, o, b = c3
    xo, ko, _ = omg.mg_pcg(o, b, rtol=1e-13)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32), gpu(b), x)
    xg = host(x)
    resid = omg.rel_residual(o, b, xg)
    err = rel(xg, xo)
    print(f"[fullsize] C3 FCG + FP32 V-cycle: iterations {res.iterations}, "
          f"FP64 rel residual (oracle operator) {resid:.3e}, rel L2 vs oracle u* {err:.2e}")
    assert resid <= 1e-10
    assert abs(res.iterations - (ko - 2)) <= 4
    assert err <= 1e-8


def test_c3_morton_order_matches(c3):
    """The same solve with the Z-order layout, whose neighbour offsets at this size do not fit
    16 bits (absolute 32-bit column path), against the oracle."""
    g, o, b = c3
    gm = mg.Hierarchy("square", W.C3["nsub"], base_cells=W.C3["base_cells"], order=mg.MG_ORDER_MORTON)
    x0 = W.normal(o.fine.nv, 41)
    y = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    mg.dec_laplacian_apply(gm.h, gm.top, gpu(x0), y)
    assert rel(host(y), o.fine.A @ x0) <= 1e-14
    xo, ko, _ = omg.mg_pcg(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(gm.h, mg.mg_opts_default(), gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    x.zero_()
    mg.mg_pcg(gm.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32), gpu(b), x)
    assert omg.rel_residual(o, b, host(x)) <= 1e-10
    gm.close()


def test_c2_sphere_fullsize():
    xyz, tri = dec.icosahedron()
    o = omg.Hierarchy(xyz, tri, W.C2["sphere_level"], project=True, bc="natural")
    g = mg.Hierarchy("sphere", W.C2["sphere_level"])
    b = o.rhs(W.sphere_rhs(o.fine.xyz, W.sh_coefficients()))
    xo, ko, _ = omg.mg_pcg(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    err = rel(host(x), xo)
    print(f"[fullsize] C2 icosphere-7 FP64 MG-PCG: iterations {res.iterations} (oracle {ko}), "
          f"rel L2 vs oracle {err:.2e}")
    assert res.iterations == ko and err <= 1e-12
    assert abs(host(x).mean()) <= 1e-14 * np.abs(host(x)).max()
    x.zero_()
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32), gpu(b), x)
    assert omg.rel_residual(o, b, host(x)) <= 1e-10
    ue = W.sphere_exact(o.fine.xyz, W.sh_coefficients())
    print(f"[fullsize] C2 max error vs continuous solution {np.abs(host(x) - (ue - ue.mean())).max():.3e}")
    g.close()
