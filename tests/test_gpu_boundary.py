"""GPU tests of the C-ABI pieces around the solve (Sec. 3.1 and Sec. 3.2), against the oracle:

* stopping on the true relative residual (Sec. 3.1): at rtol 4e-15 on the 65 x 65 square the
  recursively updated residual passes at iteration 14 while the true one does not, so CG and
  FCG restart and stop at iteration 15 with the oracle, whose solution they match to 1e-12;
  an unattainable rtol (1e-15) ends in MG_ENOCONV at max_iter;
* the residual history in mg_result against the oracle's history, entry by entry (1e-10
  relative, iterates that agree to 1e-12);
* MG_EINCOMPAT, when asked for (mg_opts.compat_check), for a natural-boundary right-hand side
  outside the range, and none for a compatible one, without the check, or for the adjoint's
  upstream gradient (which is projected);
* the Darcy coefficient as an edge field (Eq. dec_darcy): FP64 MG-PCG at the oracle's
  iteration count to 1e-12, Dirichlet and natural, binary and cubic levels; the refusals;
* k = exp(g) formed by the library and the chain rule dJ/dg = k dJ/dk.
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def pair(kind="square", nsub=4, bc=None, schemes=None):
    print(f"[boundary] {kind} nsub={nsub} bc={bc} schemes={schemes}", flush=True)
    cubic = 0
    if schemes:
        cubic = sum(1 << k for k, c in enumerate(schemes) if c == "c")
    if kind == "square":
        g = mg.Hierarchy("square", nsub, base_cells=4,
                         bc=mg.MG_BC_NATURAL if bc == "natural" else None, cubic_mask=cubic)
        xyz, tri = dec.square_grid(4)
        o = omg.Hierarchy(xyz, tri, nsub, bc=bc or "dirichlet", schemes=schemes)
    else:
        g = mg.Hierarchy("sphere", nsub)
        xyz, tri = dec.icosahedron()
        o = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")
    return g, o


@pytest.fixture(scope="module")
def c1():
    g, o = pair()
    yield g, o, o.rhs(W.normal(o.fine.nv, 5))
    g.close()


OUTERS = {"cg": (omg.mg_pcg, mg.MG_OUTER_CG), "fcg": (omg.mg_fcg, mg.MG_OUTER_FCG)}


@pytest.mark.parametrize("outer", sorted(OUTERS))
def test_restart_on_the_true_residual(c1, outer):
    g, o, b = c1
    solver, code = OUTERS[outer]
    rtol = 4e-15
    xo, ko, ho = solver(o, b, rtol=rtol, max_iter=60)
    first = next(i for i, v in enumerate(ho) if v <= rtol)
    assert (first, ko) == (14, 15)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=code, rtol=rtol, max_iter=60), gpu(b), x)
    print(f"[boundary] {outer} rtol 4e-15: iterations {res.iterations} (oracle {ko}), true "
          f"{res.rel_residual:.2e}, loop {res.rel_residual_loop:.2e}")
    assert res.iterations == ko
    assert res.rel_residual <= rtol
    assert rel(host(x), xo) <= 1e-12


@pytest.mark.parametrize("outer", sorted(OUTERS))
def test_unattainable_tolerance_is_enoconv(c1, outer):
    g, o, b = c1
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=OUTERS[outer][1], rtol=1e-15, max_iter=40),
                    gpu(b), x, raise_on_error=False)
    assert res.status == mg.MG_ENOCONV and res.iterations == 40
    assert res.rel_residual > 1e-15


@pytest.mark.parametrize("outer", sorted(OUTERS))
def test_residual_history(c1, outer):
    g, o, b = c1
    solver, code = OUTERS[outer]
    xo, ko, ho = solver(o, b)
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=code), gpu(b), x, history=64)
    assert res.history_len == res.iterations == ko
    h = res.hist
    assert h.shape == (ko,)
    e = np.abs(h - np.asarray(ho[1:])) / np.asarray(ho[1:])
    print(f"[boundary] {outer} history: max relative difference {e.max():.2e}")
    assert e.max() <= 1e-10
    # a shorter buffer takes the first entries only
    x.zero_()
    res = mg.mg_pcg(g.h, mg.mg_opts_default(outer=code), gpu(b), x, history=3)
    assert res.history_len == 3 and np.array_equal(res.hist, h[:3])
    # mg_solve records the residual after each cycle (the true one)
    x.zero_()
    res = mg.mg_solve(g.h, mg.mg_opts_default(), gpu(b), x, history=64)
    xs, ks, hs = omg.mg_solve(o, b)
    assert res.history_len == res.iterations == ks
    # true residuals: near convergence b - A x cancels, so the entries agree to rounding in
    # units of ||b|| (the iterates agree to 1e-13), not relative to themselves
    e = np.abs(res.hist - np.asarray(hs[1:]))
    print(f"[boundary] mg_solve history: max difference {e.max():.2e} (units of ||b||)")
    assert e.max() <= 1e-14


def test_incompatible_rhs():
    g, o = pair("sphere", 3)
    nv = o.fine.nv
    f = W.normal(nv, 31)
    x = torch.zeros(nv, dtype=torch.float64, device=DEV)
    bad = gpu(f + 0.5)          # mean far from zero: no solution
    strict = mg.mg_opts_default(compat_check=1)
    for fn in (mg.mg_pcg, mg.mg_solve):
        x.fill_(3.0)
        with pytest.raises(mg.MGError) as e:
            fn(g.h, strict, bad, x)
        assert e.value.status == mg.MG_EINCOMPAT
        assert np.all(host(x) == 0.0)
    good = gpu(f - f.mean())    # compatible up to rounding
    res = mg.mg_pcg(g.h, strict, good, x)
    assert res.status == mg.MG_OK
    # without the check the right-hand side is projected: L^+ b
    res = mg.mg_pcg(g.h, mg.mg_opts_default(rtol=1e-12), bad, x)
    assert res.status == mg.MG_OK
    assert rel(host(x), omg.direct_solve(o, f + 0.5)) <= 1e-9
    # the adjoint projects its upstream gradient instead of refusing it
    gb = torch.empty_like(x)
    res = mg.mg_pcg_adjoint(g.h, mg.mg_opts_default(), x, bad, gb)
    assert res.status == mg.MG_OK
    ref = omg.direct_solve(o, f + 0.5)
    assert rel(host(gb), ref) <= 1e-8
    g.close()


CASES = [("square", 4, None, None), ("square", 4, "natural", None), ("square", 3, None, "bcb")]


@pytest.mark.parametrize("case", CASES, ids=["dirichlet", "natural", "cubic"])
def test_edge_coefficient(case):
    kind, nsub, bc, schemes = case
    g, o = pair(kind, nsub, bc, schemes)
    ne = o.fine.ne
    ke = np.exp(0.6 * W.normal(ne, 41))
    o.set_edge_coeff(ke)
    mg.mg_hierarchy_set_edge_coeff(g.h, gpu(ke))
    b = o.rhs(W.normal(o.fine.nv, 42))
    for opts, solver in ((mg.mg_opts_default(), omg.mg_pcg),
                         (mg.mg_opts_default(outer=mg.MG_OUTER_FCG), omg.mg_fcg)):
        xo, ko, _ = solver(o, b)
        x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
        res = mg.mg_pcg(g.h, opts, gpu(b), x)
        e = rel(host(x), xo)
        print(f"[boundary] edge coefficient {case}: iterations {res.iterations} (oracle {ko}), "
              f"rel L2 {e:.2e}")
        assert res.iterations == ko and e <= 1e-12
    # vertex-coefficient gradients are refused while an edge coefficient is set
    x = torch.zeros(o.fine.nv, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as err:
        mg.mg_pcg_adjoint(g.h, mg.mg_opts_default(), x, gpu(b), torch.empty_like(x),
                          torch.zeros_like(x))
    assert err.value.status == mg.MG_EINVAL
    with pytest.raises(mg.MGError) as err:
        mg.mg_hierarchy_set_edge_coeff(g.h, gpu(-ke))
    assert err.value.status == mg.MG_EINVAL
    # back to k = 1
    mg.mg_hierarchy_set_edge_coeff(g.h, None)
    o2 = pair(kind, nsub, bc, schemes)
    xo, ko, _ = omg.mg_pcg(o2[1], b)
    o2[0].close()
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    g.close()


def test_edge_coefficient_refused_on_maps_hierarchy():
    xyz, tri = dec.square_grid(4)
    o = omg.Hierarchy(xyz, tri, 1)
    meshes = [(lv.xyz, lv.tri) for lv in o.levels]
    g = mg.Hierarchy.from_maps([m[0] for m in meshes], [m[1] for m in meshes], [o.fine.Mt.T])
    with pytest.raises(mg.MGError) as err:
        mg.mg_hierarchy_set_edge_coeff(g.h, gpu(np.ones(o.fine.ne)))
    assert err.value.status == mg.MG_EINVAL
    g.close()


def test_log_coefficient_and_chain_rule():
    g, o = pair("square", 3, "natural")
    nv = o.fine.nv
    gv = 0.7 * W.normal(nv, 51)
    mg.mg_hierarchy_set_log_coeff(g.h, gpu(gv))
    o.set_vertex_coeff(np.exp(gv))
    b = o.rhs(W.normal(nv, 52))
    xo, ko, _ = omg.mg_pcg(o, b)
    x = torch.zeros(nv, dtype=torch.float64, device=DEV)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(), gpu(b), x)
    assert res.iterations == ko and rel(host(x), xo) <= 1e-12
    gk = W.normal(nv, 53)
    acc = W.normal(nv, 54)
    gg = gpu(acc)
    mg.mg_hierarchy_coeff_grad_log(g.h, gpu(gk), gg)
    ref = acc + np.exp(gv) * gk
    assert np.abs(host(gg) - ref).max() <= 4e-16 * np.abs(ref).max() * 4
    # unit coefficient: dJ/dg = dJ/dk
    mg.mg_hierarchy_set_vertex_coeff(g.h, None)
    gg = torch.zeros(nv, dtype=torch.float64, device=DEV)
    mg.mg_hierarchy_coeff_grad_log(g.h, gpu(gk), gg)
    assert np.array_equal(host(gg), gk)
    g.close()
