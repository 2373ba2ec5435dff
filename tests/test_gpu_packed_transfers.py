"""The packed transfer index forms against the int32 ones they stand in for.

On the configured grids the per-step interpolation reads its two parents as int16 offsets from
a per-slice base (one 32-bit word per row) and the per-step restriction reads int16 offsets from
the kept vertex.  The int32 kernels remain for levels whose offsets do not fit; building with
DECMG_NO_PACKED_TRANSFERS set selects them everywhere.  Both forms do the same arithmetic in
the same order, so transfers, cycles and whole solves must agree bit for bit; a fan disk whose
centre has twelve incident edges keeps int32 restriction lists on its first level (the width
exceeds 8) and is checked against the oracle."""
import math
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
from oracle import multigrid as omg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
ENV = "DECMG_NO_PACKED_TRANSFERS"


def build(packed, **kw):
    print(f"[packed] building square packed={packed} {kw}", flush=True)
    if packed:
        return mg.Hierarchy("square", 5, **kw)
    os.environ[ENV] = "1"
    try:
        return mg.Hierarchy("square", 5, **kw)
    finally:
        del os.environ[ENV]


@pytest.fixture(scope="module", params=[dict(base_cells=8), dict(base_cells=3),
                                        dict(base_cells=8, order=mg.MG_ORDER_MORTON)],
                ids=["sq", "ragged", "morton"])
def pair(request):
    a, b = build(True, **request.param), build(False, **request.param)
    # stripes order keeps every offset within 16 bits; Z-order may not (neighbours across the
    # curve's quadrant boundaries lie far apart), and then the int32 forms are used anyway
    a.expect_packed = "order" not in request.param
    yield a, b
    a.close()
    b.close()


def tensor(a, dt):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


def test_forms_reported(pair):
    a, b = pair
    for l in range(1, a.top + 1):
        ia, ib = mg.mg_hierarchy_info(a.h, l), mg.mg_hierarchy_info(b.h, l)
        if a.expect_packed:
            assert ia["interp_packed16"] == 1 and ia["restrict_offsets16"] == 1, ia
        assert ib["interp_packed16"] == 0 and ib["restrict_offsets16"] == 0, ib
    i0 = mg.mg_hierarchy_info(a.h, 0)
    assert i0["interp_packed16"] == 0 and i0["restrict_offsets16"] == 0


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_transfers_bit_exact(pair, dt):
    a, b = pair
    for l in range(1, a.top + 1):
        nf = mg.mg_hierarchy_info(a.h, l)["nv"]
        nc = mg.mg_hierarchy_info(a.h, l - 1)["nv"]
        rf = tensor(W.normal(nf, 700 + l), dt)
        out = [torch.zeros(nc, dtype=dt, device=DEV) for _ in range(2)]
        mg.mg_restrict(a.h, l, rf, out[0])
        mg.mg_restrict(b.h, l, rf, out[1])
        ec = tensor(W.normal(nc, 800 + l), dt)
        xf = [tensor(W.normal(nf, 900 + l), dt) for _ in range(2)]
        mg.mg_prolong(a.h, l, ec, xf[0])
        mg.mg_prolong(b.h, l, ec, xf[1])
        torch.cuda.synchronize()
        assert torch.equal(out[0], out[1]), (l, dt)
        assert torch.equal(xf[0], xf[1]), (l, dt)


@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_cycles_and_solves_bit_exact(pair, dt):
    a, b = pair
    n = a.nv()
    rhs = tensor(W.normal(n, 41), dt)
    got = []
    for H in (a, b):
        x = torch.zeros(n, dtype=dt, device=DEV)
        mg.mg_vcycle(H.h, mg.mg_opts_default(), H.top, rhs, x)
        got.append(x)
    torch.cuda.synchronize()
    assert torch.equal(got[0], got[1])
    bt = tensor(W.normal(n, 42), torch.float64)
    res = []
    for H in (a, b):
        x = torch.zeros(n, dtype=torch.float64, device=DEV)
        prec = mg.MG_F32 if dt == torch.float32 else mg.MG_F64
        r = mg.mg_pcg(H.h, mg.mg_opts_default(precision=prec), bt, x)
        res.append((r.iterations, r.rel_residual, x))
    assert res[0][0] == res[1][0] and res[0][1] == res[1][1] and res[0][1] <= 1e-10
    assert torch.equal(res[0][2], res[1][2])


def test_wide_restriction_lists_keep_int32():
    m = 12
    xyz = np.array([[0.0, 0.0, 0.0]] + [[math.cos(2 * math.pi * k / m),
                                         math.sin(2 * math.pi * k / m), 0.0] for k in range(m)])
    tri = np.array([[0, 1 + k, 1 + (k + 1) % m] for k in range(m)], dtype=np.int32)
    print("[packed] building fan12", flush=True)
    g = mg.Hierarchy("arrays", 3, xyz=xyz, tri=tri)
    o = omg.Hierarchy(xyz, tri, 3, bc="dirichlet")
    try:
        assert mg.mg_hierarchy_info(g.h, 1)["restrict_offsets16"] == 0
        for l in range(1, 4):
            ol, oc = o.levels[l], o.levels[l - 1]
            rf = W.normal(ol.nv, 1000 + l)
            rf[ol.bnd] = 0.0
            rc = torch.zeros(oc.nv, dtype=torch.float64, device=DEV)
            mg.mg_restrict(g.h, l, tensor(rf, torch.float64), rc)
            ref = o.restrict(l, rf)
            got = rc.cpu().numpy()
            assert np.linalg.norm(got - ref) <= 1e-15 * max(np.linalg.norm(ref), 1.0), l
            ec = W.normal(oc.nv, 1100 + l)
            ec[oc.bnd] = 0.0
            xf0 = W.normal(ol.nv, 1200 + l)
            xf = tensor(xf0, torch.float64)
            mg.mg_prolong(g.h, l, tensor(ec, torch.float64), xf)
            ref = xf0 + o.prolong(l, ec)
            assert np.linalg.norm(xf.cpu().numpy() - ref) <= 1e-15 * np.linalg.norm(ref), l
    finally:
        g.close()
