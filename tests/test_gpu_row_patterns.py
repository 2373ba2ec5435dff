"""Row patterns (DevOperator.pat): on levels whose rows take at most 256 distinct sequences of
(column offset, weight) -- grids with a unit coefficient -- the two-row sweep, residual, apply
and direction-update kernels read one byte per row naming the row's pattern instead of its
offsets and weights.  The patterns hold the same values in the same order as the SELL entries,
so every result must equal that of a hierarchy built without them (DECMG_NO_ROW_PATTERNS)
bit for bit: cycles in FP64 and FP32, whole FP64 PCG and FP32-preconditioned FCG solves, and
after a coefficient change that makes the patterns too many (the kernels fall back to the SELL
arrays) and back.  Agreement of the SELL path with the oracle is the subject of the parity
tests, which run with patterns wherever the level allows them."""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2508_12501_amd as mg  # noqa: E402
import workloads as W  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"

# grids of 4 x 2^k and 8 x 2^k cells have dyadic coordinates, so their weights are exactly
# 1/2 and 1 and the rows take 9 patterns; on the 96 x 96 grid (3 x 3 base) the coordinates
# round, the weights differ in their last bits and there are too many patterns (none used)
MESHES = {"c1": (4, 4), "ragged": (3, 5), "c3": (8, 8)}
DYADIC = {"c1", "c3"}


def build(which, patterns):
    base, nsub = MESHES[which]
    print(f"[patterns] {which} patterns={patterns}", flush=True)
    if patterns:
        os.environ.pop("DECMG_NO_ROW_PATTERNS", None)
    else:
        os.environ["DECMG_NO_ROW_PATTERNS"] = "1"
    try:
        return mg.Hierarchy("square", nsub, base_cells=base)
    finally:
        os.environ.pop("DECMG_NO_ROW_PATTERNS", None)


@pytest.fixture(scope="module")
def pairs():
    cache = {}

    def get(which):
        if which not in cache:
            cache[which] = (build(which, True), build(which, False))
        return cache[which]
    yield get
    for a, b in cache.values():
        a.close()
        b.close()


def tensor(a, dt=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=DEV)


@pytest.mark.parametrize("which", sorted(MESHES))
def test_patterns_present(which, pairs):
    P, S = pairs(which)
    for l in range(P.top + 1):
        ip, is_ = mg.mg_hierarchy_info(P.h, l), mg.mg_hierarchy_info(S.h, l)
        assert is_["row_patterns"] == 0
        if which in DYADIC and ip["uniform_width"] >= 1 and ip["index_bytes"] == 2:
            assert 1 <= ip["row_patterns"] <= 256, (l, ip)
        assert ip["row_patterns"] <= 256
    print(f"[patterns] {which}: finest level {P.info[P.top]['n_unknowns']} rows, "
          f"{mg.mg_hierarchy_info(P.h, P.top)['row_patterns']} patterns")


@pytest.mark.parametrize("which", sorted(MESHES))
@pytest.mark.parametrize("dt", [torch.float64, torch.float32])
def test_cycles_bit_exact(which, dt, pairs):
    P, S = pairs(which)
    n = P.nv()
    b = tensor(W.normal(n, 61), dt)
    x0 = tensor(W.normal(n, 62), dt)
    for shape in (mg.MG_CYCLE_V, mg.MG_CYCLE_W):
        outs = []
        for H in (P, S):
            x = x0.clone()
            mg.mg_vcycle(H.h, mg.mg_opts_default(cycle=shape), H.top, b, x)
            outs.append(x)
        assert torch.equal(outs[0], outs[1]), (which, dt, shape)


@pytest.mark.parametrize("which", sorted(MESHES))
def test_solves_bit_exact(which, pairs):
    P, S = pairs(which)
    n = P.nv()
    b = tensor(W.normal(n, 63))
    for opts in (mg.mg_opts_default(), mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)):
        got = []
        for H in (P, S):
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            res = mg.mg_pcg(H.h, opts, b, x)
            got.append((res.iterations, res.rel_residual, x))
        assert got[0][0] == got[1][0] and got[0][1] == got[1][1]
        assert torch.equal(got[0][2], got[1][2])
        assert got[0][1] <= 1e-10


def test_coefficient_change_drops_and_restores_patterns(pairs):
    P, S = pairs("c1")
    n = P.nv()
    b = tensor(W.normal(n, 64))
    k = tensor(np.exp(0.5 * W.normal(n, 65)))
    opts = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)
    x = torch.zeros(n, dtype=torch.float64, device=DEV)
    mg.mg_pcg(P.h, opts, b, x)               # captures graphs with patterns
    for coeff in (k, None):
        for H in (P, S):
            mg.mg_hierarchy_set_vertex_coeff(H.h, coeff)
        npat = mg.mg_hierarchy_info(P.h, P.top)["row_patterns"]
        assert (npat == 0) if coeff is not None else (npat > 0)
        got = []
        for H in (P, S):
            x = torch.zeros(n, dtype=torch.float64, device=DEV)
            res = mg.mg_pcg(H.h, opts, b, x)
            got.append((res.iterations, x))
        assert got[0][0] == got[1][0] and torch.equal(got[0][1], got[1][1])
