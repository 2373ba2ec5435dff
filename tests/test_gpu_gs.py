"""GPU parity of the multicolour Gauss-Seidel smoother (mg_opts.smoother = MG_SMOOTH_GS)
against the oracle (multigrid.mgcycle with smoother="gs").  A different colouring or sweep
order would change every iterate, so cycle parity also checks the colouring.  Tolerances as
in test_gpu_parity.py."""
import math

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


class Pair:
    def __init__(self, kind, nsub, base_cells=4):
        print(f"[gs] building {kind} nsub={nsub}", flush=True)
        if kind == "square":
            self.g = mg.Hierarchy("square", nsub, base_cells=base_cells)
            xyz, tri = dec.square_grid(base_cells)
            self.o = omg.Hierarchy(xyz, tri, nsub)
        elif kind == "sphere":
            self.g = mg.Hierarchy("sphere", nsub)
            xyz, tri = dec.icosahedron()
            self.o = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")
        else:   # fan disk with a valence-11 centre
            m = 11
            xyz = np.array([[0.0, 0.0, 0.0]] + [[math.cos(2 * math.pi * k / m),
                                                 math.sin(2 * math.pi * k / m), 0.0]
                                                for k in range(m)])
            tri = np.array([[0, 1 + k, 1 + (k + 1) % m] for k in range(m)], dtype=np.int32)
            self.g = mg.Hierarchy("arrays", nsub, xyz=xyz, tri=tri)
            self.o = omg.Hierarchy(xyz, tri, nsub)
        self.top = self.g.top


@pytest.fixture(scope="module")
def sq():
    return Pair("square", 4)


@pytest.fixture(scope="module")
def sph():
    return Pair("sphere", 4)


@pytest.fixture(scope="module")
def fan():
    return Pair("fan", 4)


PAIRS = ["sq", "sph", "fan"]
GS = dict(smoother=mg.MG_SMOOTH_GS)


@pytest.mark.parametrize("which", PAIRS)
def test_gs_cycle(which, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default(**GS)
    for l in range(1, P.top + 1):
        ol = P.o.levels[l]
        b = W.normal(ol.nv, 1100 + l)
        x0 = W.normal(ol.nv, 1150 + l)
        ref = omg.mgcycle(P.o, b, x0.copy(), l, "V", smoother="gs")
        x = gpu(x0)
        mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
        assert rel(host(x), ref) <= 1e-13, (l, rel(host(x), ref))
        x32 = gpu(x0, torch.float32)
        mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
        assert rel(host(x32), ref) <= 1e-5, (l, rel(host(x32), ref))


def _rhs(P, which):
    if which == "sph":
        return P.o.rhs(W.sphere_rhs(P.o.fine.xyz, W.sh_coefficients()))
    return P.o.rhs(W.normal(P.o.fine.nv, 41))


@pytest.mark.parametrize("which", PAIRS)
def test_gs_solvers(which, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, _ = omg.mg_pcg(P.o, b, smoother="gs")
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(**GS), gpu(b), x)
    print(f"[gs] {which} PCG with Gauss-Seidel: {res.iterations} iterations (oracle {ko})")
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    xs, ks, _ = omg.mg_solve(P.o, b, smoother="gs")
    x.zero_()
    res = mg.mg_solve(P.g.h, mg.mg_opts_default(nu1=1, nu2=2, **GS), gpu(b), x)
    xs, ks, _ = omg.mg_solve(P.o, b, nu1=1, nu2=2, smoother="gs")
    assert res.iterations == ks and rel(host(x), xs) <= 1e-12
    xw, kw, _ = omg.mg_pcg(P.o, b, cycle="W", smoother="gs")
    x.zero_()
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(cycle=mg.MG_CYCLE_W, **GS), gpu(b), x)
    assert res.iterations == kw and rel(host(x), xw) <= 1e-12
    x.zero_()
    mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, **GS),
              gpu(b), x)
    assert omg.rel_residual(P.o, b, host(x)) <= 1e-10


def test_gs_rejected_by_batch(sq):
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_create([sq.g.h], mg.mg_opts_default(outer=mg.MG_OUTER_FCG, **GS))
    assert e.value.status == mg.MG_EINVAL
