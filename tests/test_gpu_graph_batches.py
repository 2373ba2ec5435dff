"""Batches of CG/FCG iterations are launched as replayed graphs of several iterations each
(up to 16), the first iteration after a start from p = q = 0 in a graph of its own kind.
Whatever the graph sizes, a solve must equal the same solve with eager launches
(use_graph = 0) bit for bit: solution, iteration count, status, residuals and residual
history.  The batch sizes are set with check_every on fresh hierarchies (the first batch of a
hierarchy's first solve has check_every iterations): sizes 1, 2, 3, 5, 7, 8 and 13, on a
Dirichlet grid (FCG, CG) and on a sphere (natural boundary)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def make(kind):
    return mg.Hierarchy("square", 5, base_cells=4) if kind == "square" else mg.Hierarchy("sphere", 5)


def rhs(g, seed):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(g.nv())
    if g.bc == mg.MG_BC_NATURAL:
        b -= b.mean()
    return torch.as_tensor(b, dtype=torch.float64, device=DEV)


def solve(g, b, **kw):
    x = torch.zeros_like(b)
    res = mg.mg_pcg(g.h, mg.mg_opts_default(**kw), b, x, raise_on_error=False, history=64)
    torch.cuda.synchronize()
    return res, x.cpu().numpy()


@pytest.mark.parametrize("kind,outer,precision", [("square", mg.MG_OUTER_FCG, mg.MG_F32),
                                                  ("square", mg.MG_OUTER_CG, mg.MG_F64),
                                                  ("sphere", mg.MG_OUTER_FCG, mg.MG_F32)])
@pytest.mark.parametrize("every", [1, 2, 3, 5, 7, 8, 13])
def test_graph_batches_match_eager(kind, outer, precision, every):
    print(f"[graph-batches] {kind} outer={outer} precision={precision} check_every={every}",
          flush=True)
    ge, gg = make(kind), make(kind)
    try:
        b = rhs(ge, 31)
        kw = dict(outer=outer, precision=precision, check_every=every)
        eager = solve(ge, b, use_graph=0, **kw)
        graph = solve(gg, b, use_graph=1, **kw)
        ra, xa = eager
        rb, xb = graph
        assert ra.status == rb.status == mg.MG_OK
        assert ra.iterations == rb.iterations
        assert ra.rel_residual_loop == rb.rel_residual_loop
        assert ra.rel_residual == rb.rel_residual
        assert list(ra.hist) == list(rb.hist)
        assert np.array_equal(xa, xb)
        # a second solve on the graph hierarchy starts with a batch of the last count
        again = solve(gg, b, use_graph=1, **kw)
        assert again[0].iterations == ra.iterations and np.array_equal(again[1], xa)
    finally:
        ge.close()
        gg.close()
