"""GPU parity of the batched solve (mg_batch_*) through the C-ABI.

* Every instance against the FP64 oracle: with the FP64 cycle, the batch runs the oracle's
  FCG(1) (multigrid.mg_fcg) column by column, so iteration counts match and solutions agree to
  1e-12 (relative L2); with the FP32 cycle, each solution reaches an FP64 relative residual of
  1e-10 under the oracle's operator and agrees with the exact solve to 1e-8.
* Different groupings (column widths 1..64, padded or exact groups, 1 or 4 streams) give the
  same solutions to 1e-12 and the same iteration counts.
* W- and F-cycles (FP64) match the oracle's FCG with the same cycle: iteration counts and
  1e-12.
* The tuner returns a valid tuning, and a batch created from its cache file uses it.
"""
import os

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


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


class Mix:
    """Three hierarchies (a 17x17 Dirichlet square, a ragged 25x25 Dirichlet square, a
    642-vertex natural-BC icosphere) and `n` instances cycling over them."""

    SPECS = [("square", 2, 4), ("square", 3, 3), ("sphere", 3, None)]

    def __init__(self, n):
        print(f"[batch] building the {n}-instance mix", flush=True)
        self.g, self.o = [], []
        for kind, nsub, base in self.SPECS:
            if kind == "square":
                self.g.append(mg.Hierarchy("square", nsub, base_cells=base))
                xyz, tri = dec.square_grid(base)
                self.o.append(omg.Hierarchy(xyz, tri, nsub))
            else:
                self.g.append(mg.Hierarchy("sphere", nsub))
                xyz, tri = dec.icosahedron()
                self.o.append(omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural"))
        self.kind = [i % 3 if i % 5 else 0 for i in range(n)]   # more squares-17 than others
        self.b = []
        for i, k in enumerate(self.kind):
            o = self.o[k]
            self.b.append(o.rhs(W.normal(o.fine.nv, 4000 + i)))
        self.hs = [self.g[k].h for k in self.kind]

    def tensors(self):
        bs = [gpu(b) for b in self.b]
        xs = [torch.full_like(b, 7.0) for b in bs]   # overwritten entirely by the solve
        return bs, xs


@pytest.fixture(scope="module")
def mix():
    m = Mix(23)
    yield m
    for g in m.g:
        g.close()


def test_batch_fp64_cycle_matches_oracle_fcg(mix):
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F64)
    bt = mg.mg_batch_create(mix.hs, o)
    bs, xs = mix.tensors()
    res = mg.mg_batch_solve(bt, bs, xs)
    for i, k in enumerate(mix.kind):
        xo, ko, _ = omg.mg_fcg(mix.o[k], mix.b[i])
        e = rel(host(xs[i]), xo)
        assert res[i].iterations == ko, (i, res[i].iterations, ko)
        assert e <= 1e-12, (i, e)
        assert res[i].status == mg.MG_OK and res[i].rel_residual <= 1e-10
    print(f"[batch] FP64 cycle: {len(mix.kind)} instances match the oracle FCG")
    mg.mg_batch_free(bt)


@pytest.mark.parametrize("shape", ["W", "F"])
def test_batch_cycle_shapes_match_oracle_fcg(mix, shape):
    # W- and F-cycles: below the tiled levels the register-resident bottom runs once per column
    # (stride-M access), the second coarse cycle of each visit starting from the first's result
    kind = {"W": mg.MG_CYCLE_W, "F": mg.MG_CYCLE_F}[shape]
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F64, cycle=kind)
    bt = mg.mg_batch_create(mix.hs, o)
    bs, xs = mix.tensors()
    res = mg.mg_batch_solve(bt, bs, xs)
    for i, k in enumerate(mix.kind):
        xo, ko, _ = omg.mg_fcg(mix.o[k], mix.b[i], cycle=shape)
        e = rel(host(xs[i]), xo)
        assert res[i].iterations == ko, (i, res[i].iterations, ko)
        assert e <= 1e-12, (i, e)
    print(f"[batch] FP64 {shape}-cycle: {len(mix.kind)} instances match the oracle FCG")
    mg.mg_batch_free(bt)


def test_batch_mixed_precision(mix):
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)
    bt = mg.mg_batch_create(mix.hs, o)
    bs, xs = mix.tensors()
    res = mg.mg_batch_solve(bt, bs, xs)
    worst = 0.0
    for i, k in enumerate(mix.kind):
        xg = host(xs[i])
        r = omg.rel_residual(mix.o[k], mix.b[i], xg)
        assert r <= 1e-10, (i, r)
        worst = max(worst, rel(xg, omg.direct_solve(mix.o[k], mix.b[i])))
        # the single-instance solve with the same options takes the same number of iterations
        x1 = torch.zeros_like(bs[i])
        r1 = mg.mg_pcg(mix.g[k].h, o, bs[i], x1)
        assert abs(r1.iterations - res[i].iterations) <= 1
    print(f"[batch] FP32 cycle: worst rel L2 vs exact solve {worst:.2e}")
    assert worst <= 1e-8
    mg.mg_batch_free(bt)


@pytest.mark.parametrize("max_cols,pad,streams", [(1, 1, 1), (4, 0, 4), (64, 1, 2), (8, 0, 1)])
def test_batch_groupings_agree(mix, max_cols, pad, streams):
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)
    ref = mg.mg_batch_create(mix.hs, o, mg.mg_batch_tuning(32, 1, 4, 0))
    bs, xs0 = mix.tensors()
    r0 = mg.mg_batch_solve(ref, bs, xs0)
    bt = mg.mg_batch_create(mix.hs, o, mg.mg_batch_tuning(max_cols, pad, streams, 0))
    t, ng = mg.mg_batch_info(bt)
    assert (t.max_cols, t.pad_groups, t.streams) == (max_cols, pad, streams)
    _, xs = mix.tensors()
    r1 = mg.mg_batch_solve(bt, bs, xs)
    # twice: the second call starts from the learnt iteration counts
    r2 = mg.mg_batch_solve(bt, bs, xs)
    for i in range(len(bs)):
        assert rel(host(xs[i]), host(xs0[i])) <= 1e-9
        assert abs(r1[i].iterations - r0[i].iterations) <= 1
        assert r2[i].iterations == r1[i].iterations
    print(f"[batch] grouping {max_cols}/{pad}/{streams}: {ng} groups agree")
    mg.mg_batch_free(ref)
    mg.mg_batch_free(bt)


def test_batch_autotune_and_cache(mix, tmp_path):
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)
    bt = mg.mg_batch_create(mix.hs, o)
    bs, xs = mix.tensors()
    cache = str(tmp_path / "tune.txt")
    chosen, ms = mg.mg_batch_autotune(bt, bs, xs, reps=1, tune_cache=cache)
    print(f"[batch] tuner chose {chosen.as_dict()} at {ms:.3f} ms")
    assert chosen.max_cols in (8, 16, 32, 64) and chosen.streams in (1, 2, 4)
    assert os.path.exists(cache)
    t, _ = mg.mg_batch_info(bt)
    assert t.as_dict() == chosen.as_dict()
    res = mg.mg_batch_solve(bt, bs, xs)
    assert all(r.status == mg.MG_OK for r in res)
    b2 = mg.mg_batch_create(mix.hs, o, tune_cache=cache)
    t2, _ = mg.mg_batch_info(b2)
    assert t2.as_dict() == chosen.as_dict()
    mg.mg_batch_free(bt)
    mg.mg_batch_free(b2)


def test_batch_status_paths(mix):
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_create(mix.hs, mg.mg_opts_default(outer=mg.MG_OUTER_CG))
    assert e.value.status == mg.MG_EINVAL
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_create(mix.hs, mg.mg_opts_default(outer=mg.MG_OUTER_FCG),
                           mg.mg_batch_tuning(3, 1, 1, 0))
    assert e.value.status == mg.MG_EINVAL
    bt = mg.mg_batch_create(mix.hs, mg.mg_opts_default(outer=mg.MG_OUTER_FCG, max_iter=2))
    bs, xs = mix.tensors()
    res = mg.mg_batch_solve(bt, bs, xs, raise_on_error=False)
    assert all(r.status == mg.MG_ENOCONV and r.iterations == 2 for r in res)
    with pytest.raises(mg.MGError) as e:
        mg.mg_batch_solve(bt, bs, xs)
    assert e.value.status == mg.MG_ENOCONV
    mg.mg_batch_free(bt)


def test_c4_fullsize_batch():
    """The 256-instance mix (icospheres of levels 4..7 and squares of 33..513 vertices a side),
    FP32 cycle: every instance reaches 1e-10; one instance of each mesh type, the 163,842-vertex
    icosphere and the 513 x 513 square included, is checked against the oracle's operator and
    exact solve."""
    insts = W.c4_instances()
    hier, oh = {}, {}
    hs, bs, keys = [], [], []
    for i, d in enumerate(insts):
        key = (d["kind"], d["nsub"])
        if key not in hier:
            print(f"[batch] C4 hierarchy {key}", flush=True)
            if d["kind"] == "sphere":
                hier[key] = mg.Hierarchy("sphere", d["nsub"])
            else:
                hier[key] = mg.Hierarchy("square", d["nsub"], base_cells=d["base_cells"])
        g = hier[key]
        nv = g.nv()
        f = gpu(W.normal(nv, d["rhs_seed"]))
        b = torch.zeros_like(f)
        mg.dec_star0_apply(g.h, g.top, f, b)
        hs.append(g.h)
        bs.append(b)
        keys.append(key)
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32)
    bt = mg.mg_batch_create(hs, o)
    xs = [torch.zeros_like(b) for b in bs]
    res = mg.mg_batch_solve(bt, bs, xs)
    _, ng = mg.mg_batch_info(bt)
    dof = sum(hier[k].info[hier[k].top]["n_unknowns"] for k in keys)
    print(f"[batch] C4: {len(bs)} instances, {dof} unknowns, {ng} groups, "
          f"iterations {min(r.iterations for r in res)}..{max(r.iterations for r in res)}")
    assert all(r.status == mg.MG_OK and r.rel_residual <= 1e-10 for r in res)
    seen = set()
    for i, key in enumerate(keys):
        if key in seen:
            continue
        seen.add(key)
        kind, nsub = key
        if kind == "sphere":
            xyz, tri = dec.icosahedron()
            oo = omg.Hierarchy(xyz, tri, nsub, project=True, bc="natural")
        else:
            xyz, tri = dec.square_grid(4)
            oo = omg.Hierarchy(xyz, tri, nsub)
        bo = oo.rhs(W.normal(oo.fine.nv, insts[i]["rhs_seed"]))
        xg = host(xs[i])
        r = omg.rel_residual(oo, bo, xg)
        e = rel(xg, omg.direct_solve(oo, bo))
        print(f"[batch] C4 instance {i} {key}: oracle rel residual {r:.2e}, rel L2 vs exact {e:.2e}",
              flush=True)
        assert r <= 1e-10 and e <= 1e-8
    mg.mg_batch_free(bt)
    for g in hier.values():
        g.close()
