"""GPU parity of CG smoothing (mg_opts.smoother = MG_SMOOTH_CG) against the oracle
(multigrid.mgcycle with smoother="cg").  Right-hand sides and initial guesses are zero on the
Dirichlet boundary (the smoother iterates on the unknowns; the oracle's identity rows then
carry zero residual) and have zero mean on the sphere.  Tolerances: one FP64 cycle 1e-12, FP32 cycle 1e-4 (the CG coefficients
are data dependent), FP64 FCG/IR solves and stand-alone cycles at the oracle's iteration count
1e-12 (the same algorithm: nonlinear cycles, but the rounding of the CG coefficients stays at
the level of the operator products it divides, ~1e-15 measured)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import dec  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CG = dict(smoother=mg.MG_SMOOTH_CG, nu1=3, nu2=3)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


class Pair:
    def __init__(self, kind, nsub):
        print(f"[cgs] building {kind} nsub={nsub}", flush=True)
        if kind == "square":
            self.g = mg.Hierarchy("square", nsub)
            xyz, tri = dec.square_grid(4)
            self.o = omg.Hierarchy(xyz, tri, nsub)
        else:
            self.g = mg.Hierarchy("sphere", nsub)
            xyz, tri = dec.icosahedron()
            self.o = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")
        self.top = self.g.top


@pytest.fixture(scope="module")
def sq():
    return Pair("square", 4)


@pytest.fixture(scope="module")
def sph():
    return Pair("sphere", 4)


def _zero_bnd(P, l, v):
    """Zero on the Dirichlet boundary; zero mean on a closed surface (a consistent singular
    system: CG on an inconsistent one drifts in the null space and amplifies rounding)."""
    v = v.copy()
    if P.o.bc == "dirichlet":
        v[P.o.levels[l].bnd] = 0.0
    else:
        v -= v.mean()
    return v


@pytest.mark.parametrize("which", ["sq", "sph"])
@pytest.mark.parametrize("shape", ["V", "W"])
def test_cg_smoothed_cycle(which, shape, request):
    P = request.getfixturevalue(which)
    o = mg.mg_opts_default(cycle=mg.MG_CYCLE_W if shape == "W" else mg.MG_CYCLE_V, **CG)
    for l in range(1, P.top + 1):
        ol = P.o.levels[l]
        b = _zero_bnd(P, l, W.normal(ol.nv, 1300 + l))
        x0 = _zero_bnd(P, l, W.normal(ol.nv, 1350 + l))
        ref = omg.mgcycle(P.o, b, x0.copy(), l, shape, nu1=3, nu2=3, smoother="cg")
        x = gpu(x0)
        mg.mg_vcycle(P.g.h, o, l, gpu(b), x)
        assert rel(host(x), ref) <= 1e-12, (l, rel(host(x), ref))
        x32 = gpu(x0, torch.float32)
        mg.mg_vcycle(P.g.h, o, l, gpu(b, torch.float32), x32)
        assert rel(host(x32), ref) <= 1e-4, (l, rel(host(x32), ref))


def _rhs(P, which):
    if which == "sph":
        return P.o.rhs(W.sphere_rhs(P.o.fine.xyz, W.sh_coefficients()))
    return P.o.rhs(W.normal(P.o.fine.nv, 71))


@pytest.mark.parametrize("which", ["sq", "sph"])
def test_cg_smoothed_solvers(which, request):
    P = request.getfixturevalue(which)
    b = _rhs(P, which)
    x = torch.zeros(P.o.fine.nv, dtype=torch.float64, device=DEV)
    for outer, ofun in ((mg.MG_OUTER_FCG, omg.mg_fcg), (mg.MG_OUTER_IR, omg.mg_ir)):
        xo, ko, _ = ofun(P.o, b, nu1=3, nu2=3, smoother="cg")
        x.zero_()
        res = mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=outer, **CG), gpu(b), x)
        print(f"[cgs] {which} outer {outer}: {res.iterations} iterations (oracle {ko}), "
              f"rel L2 {rel(host(x), xo):.2e}")
        assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    xs, ks, _ = omg.mg_solve(P.o, b, nu1=3, nu2=3, smoother="cg")
    x.zero_()
    res = mg.mg_solve(P.g.h, mg.mg_opts_default(**CG), gpu(b), x)
    print(f"[cgs] {which} cycles: {res.iterations} (oracle {ks}), rel L2 {rel(host(x), xs):.2e}")
    assert res.iterations == ks and rel(host(x), xs) <= 1e-12
    x.zero_()
    mg.mg_pcg(P.g.h, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, **CG),
              gpu(b), x)
    assert omg.rel_residual(P.o, b, host(x)) <= 1e-10


def test_cg_smoothing_needs_flexible_outer(sq):
    x = torch.zeros(sq.o.fine.nv, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as e:
        mg.mg_pcg(sq.g.h, mg.mg_opts_default(**CG), x.clone(), x)
    assert e.value.status == mg.MG_EINVAL
