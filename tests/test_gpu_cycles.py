"""GPU parity of the W- and F-cycle shapes (mg_opts.cycle) against the oracle's mgcycle, the
solvers that use them, and the batched solve with a W-cycle.  Tolerances as in
test_gpu_parity.py: one FP64 cycle 1e-13, FP32 cycle 1e-5, FP64 solves at the oracle's
iteration count 1e-12."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import dec  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SHAPES = {"W": mg.MG_CYCLE_W, "F": mg.MG_CYCLE_F}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


class Pair:
    def __init__(self, kind, nsub, base_cells=4):
        print(f"[cycles] building {kind} nsub={nsub}", flush=True)
        self.g = mg.Hierarchy(kind, nsub, base_cells=base_cells)
        if kind == "square":
            xyz, tri = dec.square_grid(base_cells)
            self.o = omg.Hierarchy(xyz, tri, nsub)
        else:
            xyz, tri = dec.icosahedron()
            self.o = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")
        self.top = self.g.top


@pytest.fixture(scope="module")
def sq():
    return Pair("square", 4)


@pytest.fixture(scope="module")
def sph():
    return Pair("sphere", 4)


@pytest.fixture(scope="module")
def rag():
    return Pair("square", 3, base_cells=3)


PAIRS = ["sq", "sph", "rag"]


@pytest.mark.parametrize("shape", ["W", "F"])
@pytest.mark.parametrize("which", PAIRS)
def test_one_cycle(which, shape, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default(cycle=SHAPES[shape])
    for l in range(1, P.top + 1):
        ol = P.o.levels[l]
        b = W.normal(ol.nv, 900 + l)
        x0 = W.normal(ol.nv, 950 + l)
        ref = omg.mgcycle(P.o, b, x0.copy(), l, shape)
        x = gpu(x0)
        mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
        assert rel(host(x), ref) <= 1e-13, (l, rel(host(x), ref))
        x32 = gpu(x0, torch.float32)
        mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
        assert rel(host(x32), ref) <= 1e-5, (l, rel(host(x32), ref))


def _rhs(P, which):
    if which == "sph":
        return P.o.rhs(W.sphere_rhs(P.o.fine.xyz, W.sh_coefficients()))
    return P.o.rhs(W.normal(P.o.fine.nv, 31))


@pytest.mark.parametrize("which", PAIRS)
def test_w_cycle_pcg_and_standalone(which, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, _ = omg.mg_pcg(P.o, b, cycle="W")
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(cycle=mg.MG_CYCLE_W), gpu(b), x)
    print(f"[cycles] {which} W-cycle PCG: {res.iterations} iterations (oracle {ko})")
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    xs, ks, _ = omg.mg_solve(P.o, b, cycle="W")
    x.zero_()
    res = mg.mg_solve(P.g.h, mg.mg_opts_default(cycle=mg.MG_CYCLE_W), gpu(b), x)
    assert res.iterations == ks and rel(host(x), xs) <= 1e-12


@pytest.mark.parametrize("which", PAIRS)
def test_f_cycle_fcg_and_mixed(which, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    xo, ko, _ = omg.mg_fcg(P.o, b, cycle="F")
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, cycle=mg.MG_CYCLE_F),
                    gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    for shape in (mg.MG_CYCLE_W, mg.MG_CYCLE_F):
        x.zero_()
        mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32,
                                            cycle=shape), gpu(b), x)
        assert omg.rel_residual(P.o, b, host(x)) <= 1e-10


def test_batch_w_cycle(sq, rag):
    hs, bs, refs = [], [], []
    for i, P in enumerate([sq, rag, sq, rag, sq]):
        b = P.o.rhs(W.normal(P.o.fine.nv, 4100 + i))
        hs.append(P.g.h)
        bs.append(gpu(b))
        refs.append((P, b))
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, cycle=mg.MG_CYCLE_W)
    bt = mg.mg_batch_create(hs, o)
    xs = [torch.zeros_like(b) for b in bs]
    res = mg.mg_batch_solve(bt, bs, xs)
    for i, (P, b) in enumerate(refs):
        xo, ko, _ = omg.mg_fcg(P.o, b, cycle="W")
        assert res[i].iterations == ko and rel(host(xs[i]), xo) <= 1e-12
    mg.mg_batch_free(bt)


def test_bad_cycle_rejected(sq):
    x = torch.zeros(sq.o.fine.nv, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as e:
        mg.mg_pcg(sq.g.h, mg.mg_opts_default(cycle=7), x.clone(), x)
    assert e.value.status == mg.MG_EINVAL
