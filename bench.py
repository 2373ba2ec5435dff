"""Benchmark: DEC multigrid solve throughput on one MI355X.

Workload: unit square, 8x8-cell right-triangle base, 8 binary subdivisions (2049 x 2049 =
4,198,401 vertices, 4,190,209 interior unknowns, 9 levels), circumcentric Hodge stars,
f ~ N(0,1) per vertex (seed 3), b = star0 f, zero Dirichlet boundary.  One step = one
complete solve from x = 0 to a relative residual of 1e-10: flexible CG in FP64 with one
FP32 V(2,2) weighted-Jacobi (omega 0.8) cycle as preconditioner.  The plain FP64 MG-PCG
solve of the same system is timed beside it.

Prints one JSON line.  --gpus N > 1 exits: the solver runs on a single GPU (no sharded path).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--kernel-reps", type=int, default=50)
    p.add_argument("--probe-steps", type=int, default=3,
                   help="eager solves during which the finest-level FP32 sweeps are timed with "
                        "hipEvents (the roofline figure)")
    p.add_argument("--isolated", action="store_true",
                   help="also time back-to-back launches of single kernels (warm caches)")
    p.add_argument("--order", choices=["stripes", "morton"], default="stripes")
    p.add_argument("--no-porous", action="store_true",
                   help="skip the porous-convection rollout and gradient timing")
    p.add_argument("--no-variants", action="store_true",
                   help="skip the W/F-cycle, Gauss-Seidel and CG-smoothing timings")
    p.add_argument("--only", choices=["e4", "cubic", "batch"], default=None,
                   help="run only one secondary workload and print its record (for profiling)")
    p.add_argument("--no-e4", action="store_true",
                   help="skip the adaptive porous-convection run to t = 0.5")
    p.add_argument("--no-cubic", action="store_true",
                   help="skip the V-cycle timing on the 4-fold cubic subdivision")
    p.add_argument("--no-batch", action="store_true",
                   help="skip the 256-instance batched solve timing")
    p.add_argument("--profile-kernels", action="store_true",
                   help="only launch the finest-level kernels (and a plain copy of known size "
                        "that calibrates the HBM counters) a few times each, for rocprofv3 --pmc")
    p.add_argument("--no-c2", action="store_true",
                   help="skip the FP64 MG-PCG timing on the level-7 icosphere")
    p.add_argument("--no-large", action="store_true",
                   help="skip the sweep rates on the 4097 x 4097 grid (working set > MALL)")
    p.add_argument("--batch-tuning", default=None,
                   help="with --only batch: max_cols,pad_groups,streams instead of the tuner")
    p.add_argument("--cpu-baseline-worker", type=int, default=0, help=argparse.SUPPRESS)
    return p.parse_args()


def profile_kernels(reps=5):
    """Short program for counter runs: C3 finest-level sweeps/applies and a 256 MiB copy."""
    import torch

    import paper_2508_12501_amd as mg
    import workloads as W
    H = mg.Hierarchy("square", W.C3["nsub"], base_cells=W.C3["base_cells"])
    top = H.top
    src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0")   # 256 MiB
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    for kern, dt in ((mg.KERNEL_JACOBI, mg.MG_F32), (mg.KERNEL_JACOBI, mg.MG_F64),
                     (mg.KERNEL_APPLY, mg.MG_F64), (mg.KERNEL_RESTRICT, mg.MG_F32),
                     (mg.KERNEL_PROLONG, mg.MG_F32)):
        ms = mg.mg_time_kernel(H.h, kern, top, dt, reps)
        print(f"[profile] kernel {kern} dtype {dt}: {ms:.4f} ms/launch", file=sys.stderr, flush=True)
    info = H.info[top]
    H.close()
    # a finest level whose working set exceeds the 256 MB MALL, and one with general weights
    L = mg.Hierarchy("square", W.C3["nsub"] + 1, base_cells=W.C3["base_cells"])
    for tag in ("unit k", "general k"):
        for dt in (mg.MG_F32, mg.MG_F64):
            ms = mg.mg_time_kernel(L.h, mg.KERNEL_JACOBI, L.top, dt, reps)
            print(f"[profile] 4097^2 sweep ({tag}) dtype {dt}: {ms:.4f} ms/launch", file=sys.stderr,
                  flush=True)
        if tag == "unit k":
            g = torch.tensor(W.normal(L.nv(), 5), device="cuda:0")
            mg.mg_smooth(L.h, L.top, 20, 0.8, torch.zeros_like(g), g)
            mg.mg_hierarchy_set_log_coeff(L.h, g)
    L.close()
    S = mg.Hierarchy("sphere", W.C2["sphere_level"])
    ms = mg.mg_time_kernel(S.h, mg.KERNEL_JACOBI, S.top, mg.MG_F32, reps)
    print(f"[profile] icosphere-7 sweep FP32: {ms:.4f} ms/launch", file=sys.stderr, flush=True)
    S.close()
    print(json.dumps({"copy_bytes_read": src.numel() * 8, "copy_bytes_written": src.numel() * 8,
                      "n_unknowns": info["n_unknowns"], "nnz_operator": info["nnz_operator"]}))


def kernel_bytes(info, dtype_bytes, kind):
    """Algorithmic bytes of one launch on a level: each stored coupling read once (column
    index of the level's width + the weight in the format the kernels of that precision read),
    each vector entry read or written once, gathers at perfect reuse."""
    n, nnz, ib = info["n_unknowns"], info["nnz_operator"], info["index_bytes"]
    wb = info["weight_bytes32"] if dtype_bytes == 4 else info["weight_bytes64"]
    if kind not in ("jacobi", "spmv"):
        raise ValueError(kind)
    nvec = {"jacobi": 3, "spmv": 2}[kind]   # x, b read, x' written / x read, y written
    if info.get("row_patterns", 0) > 0:
        # one pattern byte per row, and the pattern table (16-bit offset + weight per entry)
        return n * (1 + nvec * dtype_bytes) + info["row_patterns"] * info["uniform_width"] * (
            2 + dtype_bytes)
    return nnz * (ib + wb) + n * nvec * dtype_bytes


def transfer_bytes(fine, coarse, dtype_bytes, kind):
    """Algorithmic bytes of one per-step transfer launch between level `fine` and its coarse
    level, each array read or written once: the restriction reads per coarse row the kept
    vertex's id and its midpoint list (16-bit offsets or 32-bit ids, padded to the uniform
    width), each fine residual entry once, and writes each coarse entry once; the interpolation
    reads per fine row its two parents (one packed 32-bit word, or two 32-bit ids; plus a 32-bit
    base per 64 rows when packed) and x, writes x, and reads each coarse entry once."""
    nf, nc = fine["n_unknowns"], coarse["n_unknowns"]
    if kind == "restrict":
        ib = 2 if fine["restrict_offsets16"] else 4
        return nc * (4 + fine["restrict_width"] * ib + dtype_bytes) + nf * dtype_bytes
    if kind != "prolong":
        raise ValueError(kind)
    packed = fine["interp_packed16"]
    return (nf * ((4 if packed else 8) + 2 * dtype_bytes) + nc * dtype_bytes
            + (4 * ((nf + 63) // 64) if packed else 0))


def transfer_rates(mg, H, level, reps):
    """FP32 per-step restriction and interpolation of `level`, timed back to back."""
    fine = mg.mg_hierarchy_info(H.h, level)
    coarse = mg.mg_hierarchy_info(H.h, level - 1)
    out = {}
    for name, kern in (("restrict_fp32", mg.KERNEL_RESTRICT), ("prolong_fp32", mg.KERNEL_PROLONG)):
        ms = mg.mg_time_kernel(H.h, kern, level, mg.MG_F32, reps)
        by = transfer_bytes(fine, coarse, 4, name.split("_")[0])
        out[name] = {"ms_per_launch": ms, "bytes_per_launch": by,
                     "GB/s": by / (ms * 1e-3) / 1e9, "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    return out


def sweep_kernel_name(info):
    """The FP32 finest-level sweep's instantiation: over row patterns, or one or two rows per
    thread with int16 or int32 columns and binary16 or FP32 weights."""
    if info.get("row_patterns", 0) > 0:
        return "k_rows2p<float, 2>"
    return "%s<float, 2, %s, %s>" % ("k_rows2" if info["rows_per_thread"] == 2 else "k_rows",
                                    "true" if info["index_bytes"] == 2 else "false",
                                    "Half16" if info["weight_bytes32"] == 2 else "float")


def sweep_grid(info):
    """Threads launched by the finest-level sweep: 256-thread blocks of 256 rows per thread row."""
    rows = 256 * info["rows_per_thread"]
    return (info["n_unknowns"] + rows - 1) // rows * 256


def recorded_traffic(kernel_key):
    """HBM bytes per launch of `kernel_key` from the committed rocprofv3 --pmc summary, or None
    when the kernels have changed since the counters were taken (source hash differs)."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "c3_finest_kernels_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2508_12501_amd", "csrc", "kernels.hip")
    try:
        text = open(path).read()
        rec = json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))
    except Exception:
        return None
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["kernels_hip_sha256"]:
        return None
    k = rec["kernels"].get(kernel_key)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "host_cpus": os.cpu_count(), "usable_cpus": usable}


def cpu_baseline_worker(nproc):
    """Runs in a child process that never touches the GPU: builds the oracle's C3 hierarchy
    once, then forks `nproc` processes that each run the oracle's FP64 MG-PCG on the same
    system at the same time (one thread each); prints their aggregate unknowns per second."""
    import multiprocessing as mp

    import numpy as np
    os.environ["OMP_NUM_THREADS"] = "1"
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    import workloads as W
    from oracle import dec
    from oracle import multigrid as omg
    xyz, tri = dec.square_grid(W.C3["base_cells"])
    o = omg.Hierarchy(xyz, tri, W.C3["nsub"])
    b = o.rhs(W.normal(o.fine.nv, W.SEED_C3))
    ctx = mp.get_context("fork")
    start = ctx.Barrier(nproc + 1)
    q = ctx.Queue()

    def solve(i):
        start.wait()
        t = time.perf_counter()
        _, k, _ = omg.mg_pcg(o, b, rtol=1e-10)
        q.put((time.perf_counter() - t, k))

    procs = [ctx.Process(target=solve, args=(i,)) for i in range(nproc)]
    for p_ in procs:
        p_.start()
    start.wait()
    t0 = time.perf_counter()
    res = [q.get() for _ in procs]
    wall = time.perf_counter() - t0
    for p_ in procs:
        p_.join()
    print(json.dumps({"wall": wall, "unknowns": o.unknowns(), "solves": nproc,
                      "iterations": res[0][1], "per_solve_s": [r[0] for r in res]}))


def cpu_baseline_parallel():
    """The oracle on the host's cores: one FP64 MG-PCG solve of C3 per core, all at once, in a
    child process (which never initialises the GPU); aggregate unknowns per second."""
    import subprocess
    host = host_cpu()
    nproc = max(1, min(16, host["usable_cpus"]))
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                        str(nproc)], capture_output=True, text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError("cpu baseline worker failed: " + r.stderr[-2000:])
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    return rec, host


def cpu_baseline(b_nat_np, rtol):
    """The FP64 oracle's MG-PCG on the same system, one thread, timed on the host."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    import numpy as np

    from oracle import dec
    from oracle import multigrid as omg
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        t0 = time.perf_counter()
        xyz, tri = dec.square_grid(8)
        o = omg.Hierarchy(xyz, tri, 8)
        t_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, k, hist = omg.mg_pcg(o, b_nat_np, rtol=rtol)
        t_solve = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    return dict(x=x, iters=k, t_solve=t_solve, t_build=t_build, hier=o,
                final=hist[-1], unknowns=o.unknowns())


def porous_bench(mg, W, torch, np, with_oracle):
    """The porous-convection rollout (257 x 257 vertices, 200 forward-Euler steps, pressure by
    MG-PCG FP64 to 1e-10) and its discrete-adjoint gradient with checkpoints every 20 steps."""
    from paper_2508_12501_amd import autograd as mga
    C = W.C5
    H = mg.Hierarchy("square", C["nsub"], base_cells=C["base_cells"], bc=mg.MG_BC_NATURAL)
    nv = H.nv()
    g = torch.tensor(W.c5_logk_noise(nv), device="cuda:0")
    mg.mg_smooth(H.h, H.top, C["g_smooth_sweeps"], C["g_smooth_omega"], torch.zeros_like(g), g)
    xyz = mg.mg_hierarchy_export(H.h, H.top)["xyz"]
    T0 = torch.tensor(W.c5_initial_temperature(xyz), device="cuda:0")
    w = torch.tensor(W.c5_loss_weights(nv), device="cuda:0")
    # dt = 1/2 min(h^2 phi Ra / 4, 2 phi / (Ra k_max^2)), h the shortest edge (1/256 here)
    h = 1.0 / (C["base_cells"] * 2 ** C["nsub"])
    kmax = float(torch.exp(g).max())
    dt = 0.5 * min(h * h * C["phi"] * C["Ra"] / 4, 2 * C["phi"] / (C["Ra"] * kmax ** 2))
    steps, ckpt = C["steps"], C["ckpt"]
    prm = mg.porous_params_make(C["Ra"], C["phi"], dt, mg.mg_opts_default(rtol=1e-10))
    mg.mg_hierarchy_set_vertex_coeff(H.h, torch.exp(g))
    Ta, Tb = T0.clone(), torch.empty_like(T0)
    for _ in range(3):
        mg.porous_step(H.h, prm, Ta, Tb)
    torch.cuda.synchronize()
    t = time.perf_counter()
    Ta.copy_(T0)
    iters = 0
    for _ in range(steps):
        r = mg.porous_step(H.h, prm, Ta, Tb)
        iters += r.iterations
        Ta, Tb = Tb, Ta
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t
    gq = g.clone().requires_grad_(True)
    T0q = T0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    TN = mga.porous_rollout(H, T0q, gq, steps, C["Ra"], C["phi"], dt, ckpt=ckpt,
                            solve=mg.mg_opts_default(rtol=1e-10))
    J = (TN * w).sum()
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t
    out = {"workload": "porous convection, unit square 4x4 base x 6 subdivisions (257x257), "
                       "Ra 1000, phi 0.1, 200 forward-Euler steps, checkpoints every 20",
           "vertices": nv, "dt": dt, "steps_per_s": steps / t_fwd,
           "ms_per_step": 1e3 * t_fwd / steps, "pressure_iterations_mean": iters / steps,
           "gradient_s": t_grad, "loss": float(J.detach())}
    if with_oracle:
        from oracle import dec
        from oracle import multigrid as omg
        from oracle import porous as op
        xyz_o, tri = dec.square_grid(C["base_cells"])
        o = omg.Hierarchy(xyz_o, tri, C["nsub"], bc="natural")
        g_ref = op.smooth_logk(o, W.c5_logk_noise(nv), C["g_smooth_sweeps"], C["g_smooth_omega"])
        m = op.PorousModel(o, g_ref, Ra=C["Ra"], phi=C["phi"], dt=dt)
        t = time.perf_counter()
        Jo, gg, gT = m.loss_and_grad(W.c5_initial_temperature(o.fine.xyz), W.c5_loss_weights(nv),
                                     steps, ckpt)
        t_o = time.perf_counter() - t
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        out["cpu_baseline"] = {"value": 1.0 / t_o, "unit": "gradients/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one full 200-step loss + adjoint gradient ({t_o:.1f} s)"}
        out["parity"] = {"loss_rel": abs(float(J.detach()) - Jo) / abs(Jo),
                         "grad_g_rel_l2": rel(gq.grad.cpu().numpy(), gg),
                         "grad_T0_rel_l2": rel(T0q.grad.cpu().numpy(), gT)}
    H.close()
    return out


def cubic_bench(mg, W, torch, np, steps):
    """V-cycles on the 105,625-vertex mesh (4 cubic subdivisions of the 32-triangle square) with
    b = L r, r ~ U[0,1): time per cycle for CG smoothing (3 steps each side) and Jacobi(2,2),
    and the FP32-preconditioned FCG solve to 1e-10 on the same hierarchy."""
    dev = torch.device("cuda:0")
    H = mg.Hierarchy("square", W.E1_CUBIC["nsub"], base_cells=W.E1_CUBIC["base_cells"],
                     cubic_mask=W.E1_CUBIC["cubic_mask"])
    top, nv = H.top, H.nv()
    r = torch.tensor(W.uniform01(nv, W.SEED_E1), device=dev)
    b = torch.zeros_like(r)
    mg.dec_laplacian_apply(H.h, top, r, b)
    x = torch.zeros_like(b)
    y = torch.zeros_like(b)
    out = {"workload": "4x4-cell square (32 triangles) after 4 cubic (1-to-9) subdivisions: "
                       "325x325 = 105,625 vertices, zero Dirichlet, b = L r with r ~ U[0,1) "
                       "seed %d" % W.SEED_E1, "vertices": nv, "levels": H.n_levels}
    ncyc = max(10, 4 * steps)
    for name, smo, nu in (("cg_smoothing_3", mg.MG_SMOOTH_CG, 3),
                          ("jacobi_2_2", mg.MG_SMOOTH_JACOBI, 2)):
        o = mg.mg_opts_default(smoother=smo)
        o.nu1 = o.nu2 = nu
        x.zero_()
        for _ in range(3):
            mg.mg_vcycle(H.h, o, top, b, x)
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(ncyc):
            mg.mg_vcycle(H.h, o, top, b, x)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / ncyc
        mg.dec_laplacian_apply(H.h, top, x, y)
        res = float(torch.linalg.norm(b - y) / torch.linalg.norm(b))
        out[name] = {"s_per_cycle": dt, "vertex_cycles_per_s": nv / dt, "cycles": ncyc,
                     "rel_residual_after": res}
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, rtol=1e-10)
    for _ in range(2):
        mg.mg_pcg(H.h, o, b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = mg.mg_pcg(H.h, o, b, x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out["mixed_fcg"] = {"iterations": res.iterations, "rel_residual": res.rel_residual,
                        "ms_per_solve": 1e3 * dt, "value": H.info[top]["n_unknowns"] / dt,
                        "unit": "DOF/s"}
    H.close()
    return out


def e4_bench(mg, W, torch, np):
    """The paper's porous-convection run: 16,641 vertices, adaptive Dormand-Prince 5(4) to
    t = 0.5 at relative tolerance 1e-9 (absolute 1e-6), one FP64 MG-PCG pressure solve
    (rtol 1e-12) per right-hand side, ten save times."""
    E = W.E4
    dev = torch.device("cuda:0")
    base = mg.Hierarchy("square", 0, base_cells=E["base_cells"], bc=mg.MG_BC_NATURAL)
    ex = mg.mg_hierarchy_export(base.h, 0)
    base.close()
    H = mg.Hierarchy("arrays", E["nsub"], xyz=W.e4_coords(ex["xyz"]), tri=ex["tri"],
                     bc=mg.MG_BC_NATURAL)
    xyz = mg.mg_hierarchy_export(H.h, H.top)["xyz"]
    nv = len(xyz)
    y_len = E["y_range"][1] - E["y_range"][0]
    prm = mg.porous_params_make(E["Ra"], E["phi"], 1e-4, mg.mg_opts_default(rtol=1e-12),
                                delta_T=E["delta_T"], y_len=y_len)
    T0 = torch.tensor(W.e4_initial_temperature(xyz), device=dev)
    ts = W.e4_save_times()
    Ts = torch.empty(len(ts), nv, dtype=torch.float64, device=dev)
    Te = torch.empty_like(T0)
    warm = mg.porous_rk_opts_make(prm, 0.002, rtol=E["rtol"], atol=E["atol"])
    mg.porous_integrate(H.h, warm, T0, Te)
    o = mg.porous_rk_opts_make(prm, E["t_end"], rtol=E["rtol"], atol=E["atol"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = mg.porous_integrate(H.h, o, T0, Te, ts, Ts)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    H.close()
    return {"workload": "porous convection, 128x128-cell 40x20 rectangle (16,641 vertices), "
                        "Gaussian T0 x400, walls +-100, Ra 1000, phi 0.1, kappa 40; "
                        "Dormand-Prince 5(4) to t = 0.5, rtol 1e-9, atol 1e-6; pressure by "
                        "FP64 MG-PCG (rtol 1e-12)",
            "vertices": nv, "seconds": dt, **st.as_dict(),
            "ms_per_rhs": 1e3 * dt / st.rhs_evals,
            "pressure_iterations_per_solve": st.pressure_iterations / st.rhs_evals,
            "paper": {"rhs_evals": 7677, "accepted": 1275, "gmg_seconds": 167,
                      "note": "Tsit5 on a laptop CPU; context only"}}


def c2_bench(mg, W, torch, np, steps, with_oracle):
    """FP64 MG-PCG on the level-7 icosphere (163,842 vertices, natural boundary): f = sum of
    real spherical harmonics of degree 1..8 with N(0,1) coefficients (seed 2), b = star0 f with
    its mean removed; median solve time to 1e-10, rel L2 against the oracle's MG-PCG.  Also the
    finest-level FP32 and FP64 sweep rates on this level, whose weights are general (no
    binary16 copy) and whose rows have 6 couplings."""
    dev = torch.device("cuda:0")
    H = mg.Hierarchy("sphere", W.C2["sphere_level"])
    top = H.top
    info = H.info[top]
    xyz = mg.mg_hierarchy_export(H.h, top)["xyz"]
    f = torch.tensor(W.sphere_rhs(xyz, W.sh_coefficients()), device=dev)
    b = torch.zeros_like(f)
    mg.dec_star0_apply(H.h, top, f, b)
    b -= b.mean()
    x = torch.zeros_like(b)
    o = mg.mg_opts_default(rtol=1e-10)
    for _ in range(2):
        mg.mg_pcg(H.h, o, b, x)
    times = []
    torch.cuda.synchronize()
    for _ in range(steps):
        t = time.perf_counter()
        res = mg.mg_pcg(H.h, o, b, x)
        times.append(time.perf_counter() - t)
    ms = 1e3 * float(np.median(times))
    out = {"workload": "icosphere level 7 (163,842 vertices, 8 levels), natural boundary, f = "
                       "sum of real spherical harmonics l = 1..8 with N(0,1) coefficients seed 2, "
                       "b = star0 f mean removed; FP64 MG-PCG V(2,2) Jacobi(0.8) to 1e-10",
           "unknowns": info["n_unknowns"], "iterations": res.iterations,
           "rel_residual": res.rel_residual, "ms_median": ms,
           "value": info["n_unknowns"] / (ms * 1e-3), "unit": "DOF/s"}
    sweeps = {}
    for name, dt, nb in (("fp32", mg.MG_F32, 4), ("fp64", mg.MG_F64, 8)):
        msk = mg.mg_time_kernel(H.h, mg.KERNEL_JACOBI, top, dt, 50)
        by = kernel_bytes(info, nb, "jacobi")
        sweeps[name] = {"ms_per_launch": msk, "bytes_per_launch": by,
                        "GB/s": by / (msk * 1e-3) / 1e9,
                        "frac": by / (msk * 1e-3) / 1e9 / HBM_PEAK_GBS,
                        "weight_bytes": info["weight_bytes32" if nb == 4 else "weight_bytes64"],
                        "couplings_per_row": info["nnz_operator"] / info["n_unknowns"]}
    out["finest_sweeps_general_weights"] = sweeps
    if with_oracle:
        from oracle import dec
        from oracle import multigrid as omg
        xo_, tri = dec.icosahedron()
        oh = omg.Hierarchy(xo_, tri, W.C2["sphere_level"], project=True, bc="natural")
        bo = oh.rhs(W.sphere_rhs(oh.fine.xyz, W.sh_coefficients()))
        bo = bo - bo.mean()
        t = time.perf_counter()
        xo, ko, _ = omg.mg_pcg(oh, bo, rtol=1e-10)
        t_o = time.perf_counter() - t
        xg = x.cpu().numpy()
        out["parity"] = {"rel_l2_vs_oracle": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                         "oracle_iterations": ko}
        out["cpu_baseline"] = {"value": info["n_unknowns"] / t_o, "unit": "DOF/s", "cores": 1,
                               "kind": "oracle", "sample": f"one FP64 MG-PCG solve ({t_o:.2f} s)"}
    H.close()
    return out


def large_sweeps(mg, W, torch, reps=20):
    """Finest-level sweep rates on the 4097 x 4097 grid (8 x 8 base, 9 subdivisions, 16.8 M
    unknowns), whose working sets are above the 256 MB MALL, so that back-to-back launches are
    served from HBM: with the unit coefficient (row patterns: 13 B per row in FP32, 25 B in
    FP64), and with a general coefficient k = exp(g), g from 20 Jacobi sweeps of N(0,1) noise
    (seed 5), whose weights are distinct per edge (FP32 / FP64 weights and 16-bit offsets: 36 B
    and 56 B per row, 604 MB and 939 MB)."""
    L = mg.Hierarchy("square", W.C3["nsub"] + 1, base_cells=W.C3["base_cells"])
    out = {"workload": "unit square 8x8 base x 9 subdivisions (4097x4097), finest level",
           "unknowns": L.info[L.top]["n_unknowns"]}

    def rates(tag):
        info = mg.mg_hierarchy_info(L.h, L.top)
        for name, dt, nb in (("fp32", mg.MG_F32, 4), ("fp64", mg.MG_F64, 8)):
            ms = mg.mg_time_kernel(L.h, mg.KERNEL_JACOBI, L.top, dt, reps)
            by = kernel_bytes(info, nb, "jacobi")
            out[tag + name] = {"ms_per_launch": ms, "bytes_per_launch": by,
                               "GB/s": by / (ms * 1e-3) / 1e9,
                               "frac": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                               "row_patterns": info["row_patterns"],
                               "weight_bytes": info["weight_bytes32" if nb == 4 else "weight_bytes64"]}
    rates("")
    out.update(transfer_rates(mg, L, L.top, reps))
    g = torch.tensor(W.normal(L.nv(), 5), device="cuda:0")
    mg.mg_smooth(L.h, L.top, 20, 0.8, torch.zeros_like(g), g)
    mg.mg_hierarchy_set_log_coeff(L.h, g)
    rates("general_k_")
    L.close()
    return out


def batch_bench(mg, W, torch, np, steps, fixed=None):
    """The 256-instance mix (icospheres of levels 4..7, squares of 33..513 vertices a side,
    seeded types), FP32-preconditioned FCG to 1e-10 for every instance, solved as one batch
    after the tuner has picked the grouping; aggregate unknowns per second."""
    insts = W.c4_instances()
    hier, hs, bs = {}, [], []
    t0 = time.perf_counter()
    for d in insts:
        key = (d["kind"], d["nsub"])
        if key not in hier:
            hier[key] = (mg.Hierarchy("sphere", d["nsub"]) if d["kind"] == "sphere"
                         else mg.Hierarchy("square", d["nsub"], base_cells=d["base_cells"]))
        g = hier[key]
        f = torch.tensor(W.normal(g.nv(), d["rhs_seed"]), device="cuda:0")
        b = torch.zeros_like(f)
        mg.dec_star0_apply(g.h, g.top, f, b)
        hs.append(g.h)
        bs.append(b)
    dof = sum(hier[(d["kind"], d["nsub"])].info[-1]["n_unknowns"] for d in insts)
    t_build = time.perf_counter() - t0
    xs = [torch.zeros_like(b) for b in bs]
    o = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, rtol=1e-10)
    t0 = time.perf_counter()
    if fixed:
        # a given grouping (no tuner runs: for a kernel trace of the solves alone)
        bt = mg.mg_batch_create(hs, o, mg.mg_batch_tuning(*fixed, 0))
        chosen, _ = mg.mg_batch_info(bt)
    else:
        bt = mg.mg_batch_create(hs, o)
        chosen, tune_ms = mg.mg_batch_autotune(bt, bs, xs, reps=1)
    t_tune = time.perf_counter() - t0
    _, ngroups = mg.mg_batch_info(bt)
    mg.mg_batch_solve(bt, bs, xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = mg.mg_batch_solve(bt, bs, xs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    its = [r.iterations for r in res]
    out = {"workload": "256 instances: icospheres level 4..7 (natural) and squares 33..513 a side "
                       "(Dirichlet), seeded mix, f~N(0,1) seeds 4000+i; FCG + FP32 V(2,2) to 1e-10",
           "instances": len(insts), "unknowns": dof, "value": dof / dt, "unit": "DOF/s",
           "ms_per_batch": 1e3 * dt, "groups": ngroups, "tuning": chosen.as_dict(),
           "tuning_s": t_tune, "build_s": t_build, "iterations_min": min(its),
           "iterations_max": max(its),
           "max_rel_residual": max(r.rel_residual for r in res)}
    # per-instance error against the oracle's exact (sparse direct) solve: the first instance
    # of every mesh type (nine of them, the 163,842-vertex icosphere and 513 x 513 square
    # included)
    from oracle import dec
    from oracle import multigrid as omg
    errs, seen = [], set()
    t0 = time.perf_counter()
    for i, d in enumerate(insts):
        key = (d["kind"], d["nsub"])
        if key in seen:
            continue
        seen.add(key)
        if d["kind"] == "sphere":
            xyz, tri = dec.icosahedron()
            oo = omg.Hierarchy(xyz, tri, d["nsub"], project=True, bc="natural")
        else:
            xyz, tri = dec.square_grid(d["base_cells"])
            oo = omg.Hierarchy(xyz, tri, d["nsub"])
        bo = oo.rhs(W.normal(oo.fine.nv, d["rhs_seed"]))
        ue = omg.direct_solve(oo, bo)
        errs.append(float(np.linalg.norm(xs[i].cpu().numpy() - ue) / np.linalg.norm(ue)))
    out["rel_l2_vs_oracle_exact"] = {"max": max(errs), "median": float(np.median(errs)),
                                     "instances_checked": len(errs),
                                     "rule": "first instance of each of the nine mesh types",
                                     "oracle_s": time.perf_counter() - t0}
    mg.mg_batch_free(bt)
    for g in hier.values():
        g.close()
    return out


def main():
    a = parse()
    if a.cpu_baseline_worker:
        cpu_baseline_worker(a.cpu_baseline_worker)
        return
    if a.profile_kernels:
        profile_kernels()
        return
    if a.gpus != 1:
        print(json.dumps({"error": "the solver runs on a single GPU (no sharded path); --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2508_12501_amd as mg
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.only:
        if a.only == "e4":
            rec = e4_bench(mg, W, torch, np)
        elif a.only == "cubic":
            rec = cubic_bench(mg, W, torch, np, max(3, a.steps // 2))
        else:
            fixed = (tuple(int(v) for v in a.batch_tuning.split(",")) if a.batch_tuning
                     else None)
            rec = batch_bench(mg, W, torch, np, max(3, a.steps // 2), fixed)
        print(json.dumps({"only": a.only, **rec}))
        return
    t0 = time.perf_counter()
    order = mg.MG_ORDER_MORTON if a.order == "morton" else mg.MG_ORDER_STRIPES
    H = mg.Hierarchy("square", W.C3["nsub"], base_cells=W.C3["base_cells"], order=order)
    t_hier = time.perf_counter() - t0
    top = H.top
    info = H.info[top]
    nv, unknowns = info["nv"], info["n_unknowns"]
    print(f"[bench] hierarchy built in {t_hier:.1f}s: levels={H.n_levels} nv={nv} "
          f"unknowns={unknowns} nnz={info['nnz_operator']}", file=sys.stderr, flush=True)

    f = torch.tensor(W.normal(nv, W.SEED_C3), device=dev)
    b = torch.zeros_like(f)
    mg.dec_star0_apply(H.h, top, f, b)
    x = torch.zeros_like(b)
    rtol = 1e-10
    mixed = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, rtol=rtol)
    fp64 = mg.mg_opts_default(outer=mg.MG_OUTER_CG, precision=mg.MG_F64, rtol=rtol)

    def timed(opts, steps, warmup):
        # each step is one complete solve from x = 0 (mg_pcg zeroes its iterate and overwrites
        # every entry of x); the K steps are bracketed by one synchronize on each side
        for _ in range(warmup):
            mg.mg_pcg(H.h, opts, b, x)
        times, res = [], None
        torch.cuda.synchronize()
        t_all = time.perf_counter()
        for _ in range(steps):
            t = time.perf_counter()
            res = mg.mg_pcg(H.h, opts, b, x)
            times.append(time.perf_counter() - t)
        torch.cuda.synchronize()
        total = time.perf_counter() - t_all
        return times, total, res

    times_m, total_m, res_m = timed(mixed, a.steps, a.warmup)
    x_mixed = x.clone()
    print(f"[bench] mixed FCG: {res_m.iterations} it, residual {res_m.rel_residual:.3e}, "
          f"median {1e3 * np.median(times_m):.3f} ms", file=sys.stderr, flush=True)
    n64 = max(3, a.steps // 2)
    times_d, total_d, res_d = timed(fp64, n64, 1)
    x_fp64 = x.clone()
    print(f"[bench] fp64 PCG: {res_d.iterations} it, residual {res_d.rel_residual:.3e}, "
          f"median {1e3 * np.median(times_d):.3f} ms", file=sys.stderr, flush=True)

    # the other cycle shapes with the same mixed-precision FCG (C3, timed like the headline)
    variants = {}
    for vname, cyc, smo in () if a.no_variants else (("mixed_W_cycle", mg.MG_CYCLE_W, mg.MG_SMOOTH_JACOBI),
                            ("mixed_F_cycle", mg.MG_CYCLE_F, mg.MG_SMOOTH_JACOBI),
                            ("mixed_V_gauss_seidel", mg.MG_CYCLE_V, mg.MG_SMOOTH_GS),
                            ("mixed_W_gauss_seidel", mg.MG_CYCLE_W, mg.MG_SMOOTH_GS),
                            ("mixed_V_cg_smoothing_3", mg.MG_CYCLE_V, mg.MG_SMOOTH_CG)):
        ov = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, rtol=rtol, cycle=cyc,
                                smoother=smo)
        if smo == mg.MG_SMOOTH_CG:
            ov.nu1 = ov.nu2 = 3
        tv, totv, rv = timed(ov, max(3, a.steps // 2), 1)
        variants[vname] = {"iterations": rv.iterations, "rel_residual": rv.rel_residual,
                           "ms_median": 1e3 * float(np.median(tv)),
                           "value": unknowns / (totv / len(tv))}
        print(f"[bench] {vname}: {rv.iterations} it, median {1e3 * np.median(tv):.3f} ms",
              file=sys.stderr, flush=True)

    cubic = None
    if not a.no_cubic:
        cubic = cubic_bench(mg, W, torch, np, max(3, a.steps // 2))
        print(f"[bench] cubic 105,625-vertex V-cycle (CG 3): "
              f"{1e6 * cubic['cg_smoothing_3']['s_per_cycle']:.1f} us/cycle; mixed FCG "
              f"{cubic['mixed_fcg']['iterations']} it {cubic['mixed_fcg']['ms_per_solve']:.3f} ms",
              file=sys.stderr, flush=True)

    e4 = None
    if not a.no_e4:
        e4 = e4_bench(mg, W, torch, np)
        print(f"[bench] E4 porous run to t=0.5: {e4['seconds']:.2f} s, {e4['accepted']} accepted, "
              f"{e4['rejected']} rejected, {e4['rhs_evals']} right-hand sides, "
              f"{e4['ms_per_rhs']:.3f} ms each", file=sys.stderr, flush=True)

    c2 = None
    if not a.no_c2:
        c2 = c2_bench(mg, W, torch, np, max(5, a.steps), not a.no_cpu_baseline)
        print(f"[bench] C2 icosphere-7 FP64 MG-PCG: {c2['iterations']} it, median "
              f"{c2['ms_median']:.3f} ms, {c2['value'] / 1e6:.0f} M DOF/s", file=sys.stderr,
              flush=True)
    large = None
    if not a.no_large:
        large = large_sweeps(mg, W, torch)
        print(f"[bench] 4097^2 finest sweeps: FP32 {large['fp32']['GB/s']:.0f} GB/s, FP64 "
              f"{large['fp64']['GB/s']:.0f} GB/s; general k: FP32 "
              f"{large['general_k_fp32']['GB/s']:.0f} GB/s, FP64 "
              f"{large['general_k_fp64']['GB/s']:.0f} GB/s; transfers: restriction "
              f"{large['restrict_fp32']['GB/s']:.0f} GB/s, interpolation "
              f"{large['prolong_fp32']['GB/s']:.0f} GB/s", file=sys.stderr, flush=True)

    ms_step = 1e3 * total_m / a.steps
    value = unknowns / (total_m / a.steps)
    value_fp64 = unknowns / (total_d / n64)

    # dominant kernel: the FP32 Jacobi sweep on the finest level, timed with hipEvents on the
    # solve's stream around each of its launches inside eager (non-graph) mixed solves
    eager = mg.mg_opts_default(outer=mg.MG_OUTER_FCG, precision=mg.MG_F32, rtol=rtol, use_graph=0)
    mg.mg_probe_begin(H.h, top, mg.MG_F32)
    t_eager = []
    for _ in range(a.probe_steps):
        t = time.perf_counter()
        mg.mg_pcg(H.h, eager, b, x)
        t_eager.append(time.perf_counter() - t)
    ms_j32, n_probe = mg.mg_probe_end(H.h)
    by_j32 = kernel_bytes(info, 4, "jacobi")
    gbs = lambda by, ms: by / (ms * 1e-3) / 1e9
    achieved = gbs(by_j32, ms_j32)
    print(f"[bench] probe: {n_probe} finest-level FP32 sweeps in {a.probe_steps} eager solves, "
          f"{1e3 * ms_j32:.2f} us each, {achieved:.0f} GB/s", file=sys.stderr, flush=True)
    # the finest transfers back to back (the 2049^2 working sets fit in the MALL)
    others = {"transfers_back_to_back": transfer_rates(mg, H, top, a.kernel_reps)}
    tr = others["transfers_back_to_back"]
    print(f"[bench] finest transfers back to back: restriction {tr['restrict_fp32']['GB/s']:.0f}"
          f" GB/s, interpolation {tr['prolong_fp32']['GB/s']:.0f} GB/s", file=sys.stderr,
          flush=True)
    if a.isolated:
        by_j64 = kernel_bytes(info, 8, "jacobi")
        by_a64 = kernel_bytes(info, 8, "spmv")
        ms_w32 = mg.mg_time_kernel(H.h, mg.KERNEL_JACOBI, top, mg.MG_F32, a.kernel_reps)
        ms_j64 = mg.mg_time_kernel(H.h, mg.KERNEL_JACOBI, top, mg.MG_F64, a.kernel_reps)
        ms_a64 = mg.mg_time_kernel(H.h, mg.KERNEL_APPLY, top, mg.MG_F64, a.kernel_reps)
        others.update({"isolated_warm_jacobi_f32": {"GB/s": gbs(by_j32, ms_w32), "ms": ms_w32},
                  "isolated_warm_jacobi_f64": {"GB/s": gbs(by_j64, ms_j64), "ms": ms_j64, "bytes": by_j64},
                  "isolated_warm_apply_f64": {"GB/s": gbs(by_a64, ms_a64), "ms": ms_a64, "bytes": by_a64}})

    out = {
        "metric": "MG solve DOF/s to 1e-10 rel residual: FP32-precond+FP64-refine vs FP64",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": "unit-square right-triangle grid 8x8 base x 8 subdivisions "
                        "(2049x2049, 9 levels), f~N(0,1) seed 3, zero Dirichlet; "
                        "FCG(FP64) + FP32 V(2,2) Jacobi(0.8) preconditioner to 1e-10",
            "unknowns": unknowns,
            "levels": H.n_levels,
            "order": a.order,
        },
        "mixed": {"iterations": res_m.iterations, "rel_residual": res_m.rel_residual,
                  "ms_median": 1e3 * float(np.median(times_m))},
        "fp64": {"iterations": res_d.iterations, "rel_residual": res_d.rel_residual,
                 "ms_median": 1e3 * float(np.median(times_d)), "value": value_fp64},
        "speedup_mixed_vs_fp64": value / value_fp64,
        "variants": variants,
        "cubic_vcycle": cubic,
        "porous_e4_adaptive": e4,
        "roofline": {
            "bound": "hbm",
            "kernel": sweep_kernel_name(info) + " (FP32 weighted-Jacobi sweep, finest level)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": recorded_traffic("%s@%d" % (sweep_kernel_name(info), sweep_grid(info))),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE, copy-calibrated)",
            "bytes_per_launch": by_j32,
            "ms_per_launch": ms_j32,
            "launches_timed": n_probe,
            "timed_in": f"{a.probe_steps} eager mixed solves (hipEvents on the solve stream)",
            "eager_solve_ms_median": 1e3 * float(np.median(t_eager)),
            # the same launch priced with the generic layout (int32 columns, FP32 weights, the
            # 48 B per row of a deg-4 FP32 sweep): this layout moves less than that, so the
            # ratio is not a bandwidth fraction
            "bytes_per_launch_generic_layout": 48 * unknowns,
            "generic_layout_ratio": 48 * unknowns / (ms_j32 * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "others": others,
        },
        "c2_sphere_fp64": c2,
        "large_grid_sweeps": large,
    }
    if not a.no_cpu_baseline:
        print("[bench] oracle baseline (FP64 MG-PCG, 1 thread) ...", file=sys.stderr, flush=True)
        bn = b.cpu().numpy()
        cb = cpu_baseline(bn, rtol)
        xo = cb["x"]
        print("[bench] oracle baseline on the host's cores ...", file=sys.stderr, flush=True)
        par, host = cpu_baseline_parallel()
        out["cpu_baseline"] = {
            "value": par["solves"] * par["unknowns"] / par["wall"], "unit": "DOF/s",
            "cores": par["solves"], "kind": "oracle",
            "sample": f"{par['solves']} simultaneous FP64 MG-PCG solves of the same system, one "
                      f"per core, one thread each ({par['iterations']} iterations, "
                      f"{par['wall']:.1f} s wall; hierarchy build excluded)",
            **host,
            "single_thread_value": cb["unknowns"] / cb["t_solve"],
            "single_thread_sample": f"one solve, {cb['t_solve']:.1f} s",
        }
        den = float(np.linalg.norm(xo))
        out["parity"] = {
            "mixed_rel_l2_vs_oracle": float(np.linalg.norm(x_mixed.cpu().numpy() - xo)) / den,
            "fp64_rel_l2_vs_oracle": float(np.linalg.norm(x_fp64.cpu().numpy() - xo)) / den,
            "oracle_iterations": cb["iters"],
        }
    if not a.no_porous:
        print("[bench] porous-convection rollout and gradient ...", file=sys.stderr, flush=True)
        out["porous"] = porous_bench(mg, W, torch, np, not a.no_cpu_baseline)
        print(f"[bench] porous: {out['porous']['ms_per_step']:.3f} ms/step, gradient "
              f"{out['porous']['gradient_s']:.3f} s", file=sys.stderr, flush=True)
    if not a.no_batch:
        print("[bench] batched 256-instance solve (tuning first) ...", file=sys.stderr, flush=True)
        out["batch"] = batch_bench(mg, W, torch, np, max(3, a.steps // 2))
        print(f"[bench] batch: {out['batch']['ms_per_batch']:.3f} ms per batch, "
              f"{out['batch']['value'] / 1e6:.0f} M DOF/s", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
