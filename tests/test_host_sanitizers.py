"""The host mesh and geometric-map code (csrc/mesh.cpp, csrc/geomap.cpp) built with
AddressSanitizer, UndefinedBehaviorSanitizer and libstdc++ bounds assertions, and run over its
construction paths (square grids, icosahedra, binary and cubic subdivisions, sphere projection)
and its validation cases (degenerate, duplicate and isolated-vertex meshes, non-finite
coordinates, edges of three triangles; maps with bad shapes, column pointers, rows, entry
counts, weights or supports; the composition's capacity protocol).  The driver is
tests/sanitize/host_mesh_driver.cpp; any sanitizer report aborts it.  CPU only (host g++)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_12501_amd", "csrc")


def test_mesh_and_map_code_under_asan_ubsan(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host g++")
    exe = tmp_path / "host_mesh_driver"
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-D_GLIBCXX_ASSERTIONS",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
           os.path.join(ROOT, "tests", "sanitize", "host_mesh_driver.cpp"),
           os.path.join(CSRC, "mesh.cpp"), os.path.join(CSRC, "geomap.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host-mesh-driver ok" in r.stdout
    assert int(r.stdout.split()[-1]) > 500
