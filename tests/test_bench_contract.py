"""Host-side checks of bench.py's contract (no GPU needed): a run on more than one GPU is
refused with a message, the roofline's algorithmic bytes follow their per-row model on the
2049 x 2049 headline level, and the recorded HBM traffic is read back only while the kernel
source matches the one the counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    rec = json.loads(p.stdout.strip().splitlines()[-1])
    assert "single GPU" in rec["error"] and rec["n_gpus"] == 2


def test_headline_sweep_bytes():
    # 2049 x 2049 grid, zero Dirichlet: 2047^2 unknowns, 4 stored couplings per interior row
    # less the boundary-adjacent ones (the level's reported nnz), int16 column offsets; the
    # weights (star1 in {1/2, 1}) are read as binary16 by both precisions
    info = {"n_unknowns": 4190209, "nnz_operator": 16760836, "index_bytes": 2,
            "weight_bytes32": 2, "weight_bytes64": 2, "rows_per_thread": 2}
    assert bench.kernel_bytes(info, 4, "jacobi") == 16760836 * 4 + 4190209 * 12 == 117325852
    assert bench.kernel_bytes(info, 8, "spmv") == 16760836 * 4 + 4190209 * 16
    assert bench.sweep_kernel_name(info) == "k_rows2<float, 2, true, Half16>"
    assert bench.sweep_grid(info) == 2095360 and bench.sweep_grid(dict(info, rows_per_thread=1)) == 4190464
    assert bench.sweep_kernel_name(dict(info, index_bytes=4, rows_per_thread=1)) == \
        "k_rows<float, 2, false, Half16>"
    # general weights: FP32 for FP32 kernels, FP64 for FP64 kernels
    info.update(weight_bytes32=4, weight_bytes64=8)
    assert bench.kernel_bytes(info, 4, "jacobi") == 16760836 * 6 + 4190209 * 12 == 150847524
    assert bench.kernel_bytes(info, 8, "spmv") == 16760836 * 10 + 4190209 * 16
    assert bench.sweep_kernel_name(dict(info, rows_per_thread=1)) == "k_rows<float, 2, true, float>"
    with pytest.raises(ValueError):
        bench.kernel_bytes(info, 4, "other")
    # row patterns: one byte per row names the row's pattern (offsets and weights come from a
    # table of at most 256 patterns of uw entries)
    info.update(row_patterns=9, uniform_width=4)
    assert bench.kernel_bytes(info, 4, "jacobi") == 4190209 * 13 + 9 * 4 * 6
    assert bench.kernel_bytes(info, 8, "spmv") == 4190209 * 17 + 9 * 4 * 10
    assert bench.sweep_kernel_name(info) == "k_rows2p<float, 2>"


def test_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    # the headline sweep as bench.py names it on the C3 finest level (row patterns, two rows
    # per thread: 2,095,360 threads)
    info = {"row_patterns": 9, "n_unknowns": 4190209, "rows_per_thread": 2}
    key = "%s@%d" % (bench.sweep_kernel_name(info), bench.sweep_grid(info))
    assert key == "k_rows2p<float, 2>@2095360"
    prof = os.path.join(ROOT, "profiles", "c3_finest_kernels_hbm_traffic.md")
    # a copy of the repository layout whose kernel source differs from the recorded hash
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "c3_finest_kernels_hbm_traffic.md").write_text(open(prof).read())
    src_dir = tmp_path / "paper_2508_12501_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (src_dir / "kernels.hip").write_text("// not the measured source\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic(key) is None
    # the same layout with the measured source: the record comes back
    src = os.path.join(ROOT, "paper_2508_12501_amd", "csrc", "kernels.hip")
    (src_dir / "kernels.hip").write_bytes(open(src, "rb").read())
    import hashlib
    import re
    rec = json.loads(re.search(r"```json\n(.*?)\n```", open(prof).read(), re.S).group(1))
    if hashlib.sha256(open(src, "rb").read()).hexdigest() == rec["kernels_hip_sha256"]:
        got = bench.recorded_traffic(key)
        assert got is not None and got > 0
