"""The allocation-free integration entry point, porous_integrate_noalloc, against
porous_integrate on the paper's porous-convection setup (Sec. 3.2; the E4 rectangle with its
Gaussian initial temperature and walls at +-100): the same accepted and rejected steps and the
same states, bit for bit, on two calls in a row (the 65 x 65 mesh, then the smaller 33 x 33
one), since both run the same kernels in the same order (the pressure solves of the
allocation-free form run eagerly, which replays the captured iteration's launches).  Also its
refusals: a hierarchy without porous set-up, and one too large for the static work area."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
E = W.E4
Y_LEN = E["y_range"][1] - E["y_range"][0]


def e4_hierarchy(nsub):
    base = mg.Hierarchy("square", 0, base_cells=E["base_cells"], bc=mg.MG_BC_NATURAL)
    ex = mg.mg_hierarchy_export(base.h, 0)
    base.close()
    return mg.Hierarchy("arrays", nsub, xyz=W.e4_coords(ex["xyz"]), tri=ex["tri"],
                        bc=mg.MG_BC_NATURAL)


def params(use_graph):
    return mg.porous_params_make(E["Ra"], E["phi"], 1e-4,
                                 mg.mg_opts_default(rtol=1e-12, use_graph=use_graph),
                                 delta_T=E["delta_T"], y_len=Y_LEN)


def run(g, T0, noalloc, use_graph, t_end=0.02, t_save=(0.005, 0.01)):
    n = g.nv()
    o = mg.porous_rk_opts_make(params(use_graph), t_end, rtol=E["rtol"], atol=E["atol"])
    Ts = torch.full((len(t_save), n), np.nan, dtype=torch.float64, device=DEV)
    Te = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    st = mg.porous_integrate(g.h, o, T0, Te, t_save, Ts, noalloc=noalloc)
    torch.cuda.synchronize()
    return st, Te, Ts


def test_noalloc_matches_porous_integrate_twice():
    for nsub in (4, 3):   # the second call has the smaller input
        print(f"[noalloc] E4 rectangle nsub={nsub}", flush=True)
        g = e4_hierarchy(nsub)
        n = g.nv()
        xyz = mg.mg_hierarchy_export(g.h, g.top)["xyz"]
        T0 = torch.as_tensor(W.e4_initial_temperature(xyz), dtype=torch.float64, device=DEV)
        # set-up: the first porous call builds the hierarchy's porous data
        mg.porous_rhs(g.h, params(1), T0, torch.empty(n, dtype=torch.float64, device=DEV))
        got = run(g, T0, noalloc=True, use_graph=1)
        for use_graph in (0, 1):
            ref = run(g, T0, noalloc=False, use_graph=use_graph)
            a, b = got[0].as_dict(), ref[0].as_dict()
            print(f"[noalloc] nsub={nsub} graph={use_graph}: noalloc {a} reference {b}",
                  flush=True)
            assert a == b
            assert torch.equal(got[1], ref[1]) and torch.equal(got[2], ref[2])
        assert got[0].t == 0.02 and got[0].accepted > 3
        assert bool(torch.isfinite(got[1]).all())
        # and once more on the same hierarchy: the static area starts cleared again
        again = run(g, T0, noalloc=True, use_graph=0)
        assert torch.equal(again[1], got[1]) and torch.equal(again[2], got[2])
        g.close()


def test_noalloc_refusals():
    print("[noalloc] refusals", flush=True)
    g = e4_hierarchy(2)
    n = g.nv()
    T0 = torch.zeros(n, dtype=torch.float64, device=DEV)
    Te = torch.empty(n, dtype=torch.float64, device=DEV)
    o = mg.porous_rk_opts_make(params(0), 0.01, rtol=E["rtol"], atol=E["atol"])
    with pytest.raises(mg.MGError) as e:
        mg.porous_integrate(g.h, o, T0, Te, noalloc=True)
    assert e.value.status == mg.MG_EINVAL and "not set up" in str(e.value)
    g.close()
    # 513 x 513 = 263,169 unknowns: more than the static work area holds
    g = e4_hierarchy(7)
    n = g.nv()
    T0 = torch.zeros(n, dtype=torch.float64, device=DEV)
    Te = torch.empty(n, dtype=torch.float64, device=DEV)
    with pytest.raises(mg.MGError) as e:
        mg.porous_integrate(g.h, o, T0, Te, noalloc=True)
    assert e.value.status == mg.MG_EINVAL and "static area" in str(e.value)
    g.close()
