"""The oracle's stopping rule (Sec. 3.1: the solve stops on the relative residual
||b - A x|| / ||b||).  CG and FCG(1) update the residual recursively; when the recursive value
has fallen below rtol but the true one has not (rounding makes the two drift apart near the
attainable accuracy), the loop restarts from x with r = b - A x.  Pins, on the 65 x 65 square
with a seeded N(0,1) right-hand side:
* at rtol 1e-10 the recursive and true residuals agree and no restart happens;
* at rtol 4e-15 the recursive residual passes first at iteration 14 while the true one is
  5.4e-15; one restart later (iteration 15) the true residual is 2.3e-15: the returned x meets
  rtol on the true residual;
* at rtol 1e-15, below the attainable accuracy (~2e-15), the loop runs to max_iter and the
  returned x does not meet it (the library reports MG_ENOCONV there).
The true residual is recomputed here from its definition with the oracle's assembled A."""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg
import workloads as W


@pytest.fixture(scope="module")
def c1():
    xyz, tri = dec.square_grid(4)
    o = omg.Hierarchy(xyz, tri, 4)
    return o, o.rhs(W.normal(o.fine.nv, 5))


def true_rel(o, b, x):
    return float(np.linalg.norm(b - o.fine.A @ x) / np.linalg.norm(b))


@pytest.mark.parametrize("solver", [omg.mg_pcg, omg.mg_fcg])
def test_no_restart_at_1e_10(c1, solver):
    o, b = c1
    x, k, hist = solver(o, b, rtol=1e-10)
    first = next(i for i, v in enumerate(hist) if v <= 1e-10)
    assert k == first == 10
    assert true_rel(o, b, x) <= 1e-10


@pytest.mark.parametrize("solver", [omg.mg_pcg, omg.mg_fcg])
def test_restart_on_the_true_residual(c1, solver):
    o, b = c1
    rtol = 4e-15
    x, k, hist = solver(o, b, rtol=rtol, max_iter=60)
    first = next(i for i, v in enumerate(hist) if v <= rtol)
    assert first == 14 and k == 15
    assert true_rel(o, b, x) <= rtol
    # without the restart the iterate of iteration 14 would have been returned: it does not
    # meet rtol on the true residual
    x14, k14, _ = solver(o, b, rtol=rtol, max_iter=14)
    assert k14 == 14 and true_rel(o, b, x14) > rtol


@pytest.mark.parametrize("solver", [omg.mg_pcg, omg.mg_fcg])
def test_unattainable_tolerance_runs_to_max_iter(c1, solver):
    o, b = c1
    x, k, hist = solver(o, b, rtol=1e-15, max_iter=40)
    assert k == 40
    assert true_rel(o, b, x) > 1e-15
    assert min(hist) <= 1e-15   # the recursive residual alone would have stopped
