"""C-ABI checks that need no GPU: the library loads, exports every function the header
declares, and the host-only mesh entry points validate their inputs."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import paper_2508_12501_amd as mg


def test_library_exports_every_declared_symbol():
    L = mg.lib()
    names = mg.header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(mg._PROTOS), set(names) ^ set(mg._PROTOS)
    assert L.mg_abi_version() == 4


def test_opts_default():
    o = mg.mg_opts_default()
    assert (o.nu1, o.nu2, o.omega, o.rtol, o.outer, o.precision) == (2, 2, 0.8, 1e-10, 0, 0)
    assert (o.compat_check, o.stall_checks) == (0, 3)


def test_struct_layouts_match_the_header(tmp_path):
    # the binding's ctypes mirrors against the header as the host compiler lays it out
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    src = tmp_path / "layout.cpp"
    src.write_text(
        '#include <cstddef>\n#include <cstdio>\n#include "decmg.h"\n'
        "int main() { std::printf(\"%zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(mg_opts),\n"
        "  offsetof(mg_opts, stall_checks), sizeof(mg_result), offsetof(mg_result, history_len),\n"
        "  offsetof(mg_result, fp64_fallback), sizeof(mg_level_info),\n"
        "  offsetof(mg_level_info, restrict_width)); }\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cxx, "-std=c++17", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    assert got == [ctypes.sizeof(mg.mg_opts), mg.mg_opts.stall_checks.offset,
                   ctypes.sizeof(mg.mg_result), mg.mg_result.history_len.offset,
                   mg.mg_result.fp64_fallback.offset, ctypes.sizeof(mg.mg_level_info),
                   mg.mg_level_info.restrict_width.offset]


def test_debug_flags_validated():
    L = mg.lib()
    assert L.mg_hierarchy_set_debug(None, 0) == mg.MG_EINVAL


def test_mesh_constructors_and_validation():
    m = mg.dec_mesh_square_grid(4)
    mg.dec_mesh_free(m)
    m = mg.dec_mesh_icosahedron()
    mg.dec_mesh_free(m)
    xyz = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    m = mg.dec_mesh_from_arrays(xyz, [[0, 1, 2], [1, 3, 2]])
    mg.dec_mesh_free(m)
    bad = [
        ([[0, 1, 2], [0, 1, 4]], "out of range"),
        ([[0, 1, 1], [1, 3, 2]], "degenerate"),
        ([[0, 1, 2], [1, 3, 2], [2, 1, 0]], "duplicate"),
        ([[0, 1, 2]], "in no triangle"),
    ]
    for tri, msg in bad:
        with pytest.raises(mg.MGError) as e:
            mg.dec_mesh_from_arrays(xyz, tri)
        assert e.value.status == mg.MG_EINVAL and msg in str(e.value)
    # an edge shared by three triangles
    xyz5 = np.vstack([xyz, [[0.5, -1, 0]]])
    with pytest.raises(mg.MGError, match="more than two"):
        mg.dec_mesh_from_arrays(xyz5, [[0, 1, 2], [1, 3, 2], [1, 2, 4]])
    nan = xyz.copy()
    nan[3, 0] = np.nan
    with pytest.raises(mg.MGError, match="non-finite"):
        mg.dec_mesh_from_arrays(nan, [[0, 1, 2], [1, 3, 2]])
    with pytest.raises(mg.MGError):
        mg.dec_mesh_square_grid(0)


def test_null_arguments_rejected():
    L = mg.lib()
    assert L.dec_mesh_square_grid(4, None) == mg.MG_EINVAL
    assert L.mg_hierarchy_info(None, 0, None) == mg.MG_EINVAL
    assert L.mg_pcg(None, None, None, None, None, None) == mg.MG_EINVAL
    assert b"null" in L.mg_last_error()
