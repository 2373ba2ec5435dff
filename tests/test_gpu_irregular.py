"""GPU parity on an irregular mesh: a disk triangulated as a fan of 11 triangles around its
centre, subdivided 5 times (zero Dirichlet boundary).  The centre keeps valence 11, so one
operator slice is 11 wide while the others are at most 6 wide: the layout stays sliced (slice
bounds loaded, not a uniform width), rows take the generic entry loop past 8 entries, and the
fused coarse cycle (levels up to 2048 rows) runs its generic path while the finest level runs
the separate kernels.  Same tolerances as test_gpu_parity.py."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NSUB = 5


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def fan_disk(m=11):
    xyz = [[0.0, 0.0, 0.0]] + [[math.cos(2 * math.pi * k / m), math.sin(2 * math.pi * k / m), 0.0]
                               for k in range(m)]
    tri = [[0, 1 + k, 1 + (k + 1) % m] for k in range(m)]
    return np.array(xyz), np.array(tri, dtype=np.int32)


@pytest.fixture(scope="module")
def fan():
    xyz, tri = fan_disk()
    print("[irregular] building the fan-disk hierarchy", flush=True)
    g = mg.Hierarchy("arrays", NSUB, xyz=xyz, tri=tri)
    o = omg.Hierarchy(xyz, tri, NSUB)
    yield g, o
    g.close()


def test_fan_operator_and_smoother(fan):
    g, o = fan
    nv = o.fine.nv
    x0 = W.normal(nv, 61)
    for dt, tol in ((torch.float64, 1e-14), (torch.float32, 1e-6)):
        y = torch.zeros(nv, dtype=dt, device=DEV)
        mg.dec_laplacian_apply(g.h, g.top, gpu(x0, dt), y)
        assert rel(host(y), o.fine.A @ x0) <= tol
    b = o.rhs(W.normal(nv, 62))
    x = gpu(x0)
    mg.mg_smooth(g.h, g.top, 2, 0.8, gpu(b), x)
    assert rel(host(x), omg.jacobi(o.fine.A, b, x0, 0.8, 2)) <= 1e-14


def test_fan_vcycle_and_solves(fan):
    g, o = fan
    b = o.rhs(W.normal(o.fine.nv, 63))
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    mg.mg_vcycle(g.h, mg.mg_opts_default(), g.top, gpu(b), x)
    assert rel(host(x), omg.vcycle(o, b)) <= 1e-13
    xo, ko, _ = omg.mg_pcg(o, b)
    x.zero_()
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    e = rel(host(x), xo)
    print(f"[irregular] FP64 MG-PCG: {res.iterations} iterations (oracle {ko}), rel L2 {e:.2e}")
    assert res.iterations == ko and e <= 1e-12
    x.zero_()
    mg.mg_pcg(g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32), gpu(b), x)
    assert omg.rel_residual(o, b, host(x)) <= 1e-10
