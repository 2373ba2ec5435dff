"""decmg: geometric multigrid for the DEC 0-form Laplacian on MI355X (gfx950).

A thin ctypes binding of ``libdecmg.so`` (declared in ``include/decmg.h``).  Functions carry
the C names and only marshal arguments: every step of the path runs in the library's HIP
kernels.  Vectors are contiguous torch tensors on the GPU (float64, or float32 where the C
call takes a dtype), one entry per vertex of the named level in the natural numbering.  Work
is enqueued on torch's current stream.

If the library has not been built, importing works but the first call raises
``LibraryMissing``; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdecmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "decmg.h")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_ENOCONV, MG_EBREAKDOWN, MG_ENONFINITE, MG_EINCOMPAT = range(8)
STATUS_NAMES = ["MG_OK", "MG_EINVAL", "MG_ENOMEM", "MG_EDEVICE", "MG_ENOCONV", "MG_EBREAKDOWN",
                "MG_ENONFINITE", "MG_EINCOMPAT"]
MG_F64, MG_F32 = 0, 1
MG_BC_DIRICHLET0, MG_BC_NATURAL = 0, 1
MG_OUTER_CG, MG_OUTER_FCG, MG_OUTER_IR = 0, 1, 2
MG_ORDER_STRIPES, MG_ORDER_MORTON = 0, 1
MG_CYCLE_V, MG_CYCLE_W, MG_CYCLE_F = 0, 1, 2
MG_SMOOTH_JACOBI, MG_SMOOTH_GS, MG_SMOOTH_CG = 0, 1, 2
MG_DEBUG_ZERO_PRECOND32 = 1
KERNEL_JACOBI, KERNEL_APPLY, KERNEL_RESIDUAL, KERNEL_RESTRICT, KERNEL_PROLONG = range(5)


class LibraryMissing(ImportError):
    pass


class MGError(RuntimeError):
    def __init__(self, status: int, message: str, result=None):
        self.status = status
        self.result = result
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{name}: {message}")


class mg_hier_opts(ctypes.Structure):
    _fields_ = [("n_subdiv", ctypes.c_int32), ("project_sphere", ctypes.c_int32),
                ("bc", ctypes.c_int32), ("order", ctypes.c_int32),
                ("cubic_mask", ctypes.c_int32)]


class mg_level_info(ctypes.Structure):
    _fields_ = [("n_levels", ctypes.c_int32), ("level", ctypes.c_int32),
                ("nv", ctypes.c_int64), ("ne", ctypes.c_int64), ("nt", ctypes.c_int64),
                ("n_unknowns", ctypes.c_int64), ("nnz_operator", ctypes.c_int64),
                ("index_bytes", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("fused_tiles", ctypes.c_int32), ("fused_tile_rows", ctypes.c_int32),
                ("weight_bytes32", ctypes.c_int32), ("weight_bytes64", ctypes.c_int32),
                ("uniform_width", ctypes.c_int32), ("rows_per_thread", ctypes.c_int32),
                ("interp_packed16", ctypes.c_int32), ("restrict_offsets16", ctypes.c_int32),
                ("row_patterns", ctypes.c_int32), ("restrict_width", ctypes.c_int32)]


class mg_opts(ctypes.Structure):
    _fields_ = [("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("omega", ctypes.c_double),
                ("precision", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("cycle", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("fuse_levels", ctypes.c_int32), ("compat_check", ctypes.c_int32),
                ("stall_checks", ctypes.c_int32)]


class mg_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("rel_residual_loop", ctypes.c_double),
                ("history", ctypes.c_void_p), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("fp64_fallback", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_
                if f not in ("history", "history_cap", "history_len")}


def _result(history: int):
    """An mg_result, with a host buffer for `history` iterations when history > 0 (kept on the
    result as .hist, a numpy array trimmed to history_len by _trim)."""
    res = mg_result()
    if history > 0:
        buf = np.zeros(int(history), dtype=np.float64)
        res.history = buf.ctypes.data
        res.history_cap = int(history)
        res._hist_buf = buf
    return res


def _trim(res):
    buf = getattr(res, "_hist_buf", None)
    res.hist = None if buf is None else buf[:res.history_len].copy()
    return res


class mg_geomap(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowval", ctypes.c_void_p),
                ("nzval", ctypes.c_void_p)]


class mg_batch_tuning(ctypes.Structure):
    _fields_ = [("max_cols", ctypes.c_int32), ("pad_groups", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class porous_params(ctypes.Structure):
    _fields_ = [("Ra", ctypes.c_double), ("phi", ctypes.c_double), ("dt", ctypes.c_double),
                ("solve", mg_opts), ("delta_T", ctypes.c_double), ("y_len", ctypes.c_double)]


class porous_rk_opts(ctypes.Structure):
    _fields_ = [("model", porous_params), ("t_end", ctypes.c_double), ("rtol", ctypes.c_double),
                ("atol", ctypes.c_double), ("h0", ctypes.c_double), ("max_steps", ctypes.c_int32),
                ("fixed_step", ctypes.c_int32)]


class porous_rk_stats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("rejected", ctypes.c_int32),
                ("rhs_evals", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("pressure_iterations", ctypes.c_int64), ("t", ctypes.c_double),
                ("h_min", ctypes.c_double), ("h_max", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_PROTOS = {
    "mg_last_error": (ctypes.c_char_p, []),
    "mg_abi_version": (_i32, []),
    "dec_mesh_from_arrays": (_i32, [_i64, _vp, _i64, _vp, ctypes.POINTER(_vp)]),
    "dec_mesh_square_grid": (_i32, [_i32, ctypes.POINTER(_vp)]),
    "dec_mesh_icosahedron": (_i32, [ctypes.POINTER(_vp)]),
    "dec_mesh_free": (None, [_vp]),
    "mg_hierarchy_build": (_i32, [_vp, ctypes.POINTER(mg_hier_opts), _vp, ctypes.POINTER(_vp)]),
    "mg_hierarchy_build_maps": (_i32, [_i32, ctypes.POINTER(_vp), ctypes.POINTER(mg_geomap),
                                       ctypes.POINTER(mg_hier_opts), _vp, ctypes.POINTER(_vp)]),
    "mg_geomap_compose": (_i32, [ctypes.POINTER(mg_geomap), ctypes.POINTER(mg_geomap), _vp, _vp,
                                 _vp, ctypes.POINTER(_i64)]),
    "mg_hierarchy_free": (None, [_vp]),
    "mg_hierarchy_info": (_i32, [_vp, _i32, ctypes.POINTER(mg_level_info)]),
    "mg_hierarchy_export": (_i32, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mg_hierarchy_export_interp": (_i32, [_vp, _i32, _vp, _vp]),
    "mg_hierarchy_set_vertex_coeff": (_i32, [_vp, _vp, _vp]),
    "mg_hierarchy_set_log_coeff": (_i32, [_vp, _vp, _vp]),
    "mg_hierarchy_coeff_grad_log": (_i32, [_vp, _vp, _vp, _vp]),
    "mg_hierarchy_set_edge_coeff": (_i32, [_vp, _vp, _vp]),
    "mg_hierarchy_set_debug": (_i32, [_vp, _i32]),
    "dec_star0_apply": (_i32, [_vp, _i32, _vp, _vp, _vp]),
    "dec_laplacian_apply": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "mg_smooth": (_i32, [_vp, _i32, _i32, _i32, _d, _vp, _vp, _vp]),
    "mg_restrict": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "mg_prolong": (_i32, [_vp, _i32, _i32, _vp, _vp, _vp]),
    "mg_opts_default": (None, [ctypes.POINTER(mg_opts)]),
    "mg_vcycle": (_i32, [_vp, ctypes.POINTER(mg_opts), _i32, _i32, _vp, _vp, _vp]),
    "mg_solve": (_i32, [_vp, ctypes.POINTER(mg_opts), _vp, _vp, ctypes.POINTER(mg_result), _vp]),
    "mg_pcg": (_i32, [_vp, ctypes.POINTER(mg_opts), _vp, _vp, ctypes.POINTER(mg_result), _vp]),
    "mg_pcg_adjoint": (_i32, [_vp, ctypes.POINTER(mg_opts), _vp, _vp, _vp, _vp, _vp,
                              ctypes.POINTER(mg_result), _vp]),
    "porous_step": (_i32, [_vp, ctypes.POINTER(porous_params), _vp, _vp, _vp,
                           ctypes.POINTER(mg_result), _vp]),
    "porous_step_adjoint": (_i32, [_vp, ctypes.POINTER(porous_params), _vp, _vp, _vp, _vp, _vp,
                                   _vp, _vp]),
    "porous_rhs": (_i32, [_vp, ctypes.POINTER(porous_params), _vp, _vp, _vp,
                          ctypes.POINTER(mg_result), _vp]),
    "porous_integrate": (_i32, [_vp, ctypes.POINTER(porous_rk_opts), _vp, _i32, _vp, _vp, _vp,
                                ctypes.POINTER(porous_rk_stats), _vp]),
    "porous_integrate_noalloc": (_i32, [_vp, ctypes.POINTER(porous_rk_opts), _vp, _i32, _vp, _vp,
                                        _vp, ctypes.POINTER(porous_rk_stats), _vp]),
    "mg_batch_create": (_i32, [ctypes.POINTER(_vp), _i32, ctypes.POINTER(mg_opts),
                               ctypes.POINTER(mg_batch_tuning), ctypes.c_char_p,
                               ctypes.POINTER(_vp)]),
    "mg_batch_solve": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp),
                              ctypes.POINTER(mg_result), _vp]),
    "mg_batch_autotune": (_i32, [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _i32,
                                 ctypes.c_char_p, ctypes.POINTER(mg_batch_tuning),
                                 ctypes.POINTER(_d)]),
    "mg_batch_info": (_i32, [_vp, ctypes.POINTER(mg_batch_tuning), ctypes.POINTER(_i32)]),
    "mg_batch_free": (None, [_vp]),
    "mg_time_kernel": (_i32, [_vp, _i32, _i32, _i32, _i32, _vp, ctypes.POINTER(_d)]),
    "mg_probe_begin": (_i32, [_vp, _i32, _i32]),
    "mg_probe_end": (_i32, [_vp, ctypes.POINTER(_d), ctypes.POINTER(_i32)]),
}

_LIB = None


def lib():
    """Load libdecmg.so (once).  Raises LibraryMissing if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is missing: run `python -m paper_2508_12501_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def header_functions() -> list:
    """Names of the functions declared in include/decmg.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return re.findall(r"^\s*(?:const\s+)?[\w]+\*?\s+\**(\w+)\s*\(", src, flags=re.M)


def _check(st: int, result=None):
    if st != MG_OK:
        raise MGError(st, lib().mg_last_error().decode(), result)


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, dtype=None, numel=None, name="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _dtype_code(t):
    import torch
    if t.dtype == torch.float64:
        return MG_F64
    if t.dtype == torch.float32:
        return MG_F32
    raise ValueError("vectors must be float64 or float32")


# ----------------------------------------------------------------- meshes
def dec_mesh_square_grid(ncells: int):
    out = _vp()
    _check(lib().dec_mesh_square_grid(int(ncells), ctypes.byref(out)))
    return out


def dec_mesh_icosahedron():
    out = _vp()
    _check(lib().dec_mesh_icosahedron(ctypes.byref(out)))
    return out


def dec_mesh_from_arrays(xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    if xyz.ndim != 2 or xyz.shape[1] != 3 or tri.ndim != 2 or tri.shape[1] != 3:
        raise ValueError("xyz must be (nv, 3) and tri (nt, 3)")
    out = _vp()
    _check(lib().dec_mesh_from_arrays(xyz.shape[0], xyz.ctypes.data, tri.shape[0],
                                      tri.ctypes.data, ctypes.byref(out)))
    return out


def dec_mesh_free(m):
    lib().dec_mesh_free(m)


# ----------------------------------------------------------------- hierarchy
def mg_hierarchy_build(mesh, n_subdiv: int, project_sphere: bool = False,
                       bc: int = MG_BC_DIRICHLET0, stream=None, order: int = MG_ORDER_STRIPES,
                       cubic_mask: int = 0):
    """cubic_mask: bit k set makes the (k+1)-th subdivision 1-to-9 instead of 1-to-4."""
    o = mg_hier_opts(int(n_subdiv), int(bool(project_sphere)), int(bc), int(order),
                     int(cubic_mask))
    out = _vp()
    _check(lib().mg_hierarchy_build(mesh, ctypes.byref(o), _stream(stream), ctypes.byref(out)))
    return out


def _geomap(M):
    """A geometric map as (mg_geomap, arrays kept alive): M is a scipy sparse matrix
    (n_rows x n_cols, column j = barycentric coordinates of the image of vertex j) or a tuple
    (colptr, rowval, nzval, (n_rows, n_cols))."""
    if isinstance(M, tuple):
        colptr, rowval, nzval, shape = M
    else:
        c = M.tocsc()
        colptr, rowval, nzval, shape = c.indptr, c.indices, c.data, c.shape
    keep = (np.ascontiguousarray(colptr, dtype=np.int64),
            np.ascontiguousarray(rowval, dtype=np.int32),
            np.ascontiguousarray(nzval, dtype=np.float64))
    g = mg_geomap(int(shape[0]), int(shape[1]), keep[0].ctypes.data, keep[1].ctypes.data,
                  keep[2].ctypes.data)
    return g, keep


def mg_hierarchy_build_maps(meshes, maps, bc: int = MG_BC_DIRICHLET0, stream=None,
                            order: int = MG_ORDER_STRIPES):
    """meshes: mesh handles, coarsest first; maps[l]: M(f) of f: mesh l+1 -> mesh l."""
    if len(maps) != len(meshes) - 1:
        raise ValueError("need one map per pair of neighbouring meshes")
    gs = [_geomap(M) for M in maps]
    arr = (mg_geomap * max(len(gs), 1))(*[g for g, _ in gs])
    mp = (_vp * len(meshes))(*meshes)
    o = mg_hier_opts(0, 0, int(bc), int(order), 0)
    out = _vp()
    _check(lib().mg_hierarchy_build_maps(len(meshes), mp, arr, ctypes.byref(o), _stream(stream),
                                         ctypes.byref(out)))
    return out


def mg_geomap_compose(g, f):
    """M(g) M(f) as (colptr, rowval, nzval, shape) from two maps given like _geomap's input."""
    gg, kg = _geomap(g)
    ff, kf = _geomap(f)
    nnz = _i64(0)
    _check(lib().mg_geomap_compose(ctypes.byref(gg), ctypes.byref(ff), None, None, None,
                                   ctypes.byref(nnz)))
    colptr = np.empty(ff.n_cols + 1, np.int64)
    rowval = np.empty(max(nnz.value, 1), np.int32)
    nzval = np.empty(max(nnz.value, 1))
    _check(lib().mg_geomap_compose(ctypes.byref(gg), ctypes.byref(ff), colptr.ctypes.data,
                                   rowval.ctypes.data, nzval.ctypes.data, ctypes.byref(nnz)))
    return colptr, rowval[:nnz.value], nzval[:nnz.value], (gg.n_rows, ff.n_cols)


def mg_hierarchy_free(h):
    lib().mg_hierarchy_free(h)


def mg_hierarchy_info(h, level: int) -> dict:
    info = mg_level_info()
    _check(lib().mg_hierarchy_info(h, int(level), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in info._fields_}


def mg_hierarchy_export(h, level: int) -> dict:
    i = mg_hierarchy_info(h, level)
    nv, ne, nt = i["nv"], i["ne"], i["nt"]
    out = dict(xyz=np.empty((nv, 3)), tri=np.empty((nt, 3), np.int32),
               edges=np.empty((ne, 2), np.int32), tri_edges=np.empty((nt, 3), np.int32),
               tri_sign=np.empty((nt, 3), np.int8), star0=np.empty(nv), star1=np.empty(ne),
               boundary=np.empty(nv, np.uint8))
    parents = np.empty((nv, 2), np.int32) if level > 0 and i["scheme"] == 1 else None
    _check(lib().mg_hierarchy_export(
        h, int(level), *(out[k].ctypes.data for k in
                         ("xyz", "tri", "edges", "tri_edges", "tri_sign", "star0", "star1", "boundary")),
        parents.ctypes.data if parents is not None else None))
    out["parents"] = parents
    return out


def mg_hierarchy_export_interp(h, level: int):
    """(parents, weights), each (nv, 3): row j of M(f)^T for level >= 1 of either scheme."""
    nv = mg_hierarchy_info(h, level)["nv"]
    par = np.empty((nv, 3), np.int32)
    w = np.empty((nv, 3))
    _check(lib().mg_hierarchy_export_interp(h, int(level), par.ctypes.data, w.ctypes.data))
    return par, w


def mg_hierarchy_set_vertex_coeff(h, k_vertex, stream=None):
    import torch
    ptr = None if k_vertex is None else _ptr(k_vertex, torch.float64, _nv(h, _top(h)), "k_vertex")
    _check(lib().mg_hierarchy_set_vertex_coeff(h, ptr, _stream(stream)))


def mg_hierarchy_set_log_coeff(h, g_vertex, stream=None):
    """k = exp(g) at the finest level's vertices (the library forms the exponential)."""
    import torch
    _check(lib().mg_hierarchy_set_log_coeff(h, _ptr(g_vertex, torch.float64, _nv(h, _top(h)), "g"),
                                            _stream(stream)))


def mg_hierarchy_coeff_grad_log(h, grad_k, grad_g, stream=None):
    """grad_g += k * grad_k (chain rule through k = exp(g); accumulates into grad_g)."""
    import torch
    n = _nv(h, _top(h))
    _check(lib().mg_hierarchy_coeff_grad_log(h, _ptr(grad_k, torch.float64, n, "grad_k"),
                                             _ptr(grad_g, torch.float64, n, "grad_g"),
                                             _stream(stream)))


def mg_hierarchy_set_edge_coeff(h, k_edge, stream=None):
    """Darcy coefficient per finest-level edge (natural edge order); None restores k = 1."""
    import torch
    top = _top(h)
    ptr = None if k_edge is None else _ptr(k_edge, torch.float64,
                                           mg_hierarchy_info(h, top)["ne"], "k_edge")
    _check(lib().mg_hierarchy_set_edge_coeff(h, ptr, _stream(stream)))


def mg_hierarchy_set_debug(h, flags: int):
    """Fault injection for failure-handling tests (MG_DEBUG_ bits; 0 clears)."""
    _check(lib().mg_hierarchy_set_debug(h, int(flags)))


# ----------------------------------------------------------------- operators
def _nv(h, level):
    return mg_hierarchy_info(h, level)["nv"]


def _top(h):
    return mg_hierarchy_info(h, 0)["n_levels"] - 1


def dec_star0_apply(h, level: int, f, b, stream=None):
    import torch
    n = _nv(h, level)
    _check(lib().dec_star0_apply(h, int(level), _ptr(f, torch.float64, n, "f"),
                                 _ptr(b, torch.float64, n, "b"), _stream(stream)))


def dec_laplacian_apply(h, level: int, x, y, stream=None):
    n = _nv(h, level)
    _check(lib().dec_laplacian_apply(h, int(level), _dtype_code(x), _ptr(x, y.dtype, n, "x"),
                                     _ptr(y, x.dtype, n, "y"), _stream(stream)))


def mg_smooth(h, level: int, nsweeps: int, omega: float, b, x, stream=None):
    n = _nv(h, level)
    _check(lib().mg_smooth(h, int(level), _dtype_code(x), int(nsweeps), float(omega),
                           _ptr(b, x.dtype, n, "b"), _ptr(x, None, n, "x"), _stream(stream)))


def mg_restrict(h, level: int, r_fine, r_coarse, stream=None):
    nf, nc = _nv(h, level), _nv(h, max(level - 1, 0))
    _check(lib().mg_restrict(h, int(level), _dtype_code(r_fine), _ptr(r_fine, None, nf, "r_fine"),
                             _ptr(r_coarse, r_fine.dtype, nc, "r_coarse"), _stream(stream)))


def mg_prolong(h, level: int, e_coarse, x_fine, stream=None):
    nf, nc = _nv(h, level), _nv(h, max(level - 1, 0))
    _check(lib().mg_prolong(h, int(level), _dtype_code(x_fine),
                            _ptr(e_coarse, x_fine.dtype, nc, "e_coarse"),
                            _ptr(x_fine, None, nf, "x_fine"), _stream(stream)))


# ----------------------------------------------------------------- solvers
def mg_opts_default(**kw) -> mg_opts:
    o = mg_opts()
    lib().mg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def mg_vcycle(h, opts: mg_opts, level: int, b, x, stream=None):
    n = _nv(h, level)
    _check(lib().mg_vcycle(h, ctypes.byref(opts), int(level), _dtype_code(x),
                           _ptr(b, x.dtype, n, "b"), _ptr(x, None, n, "x"), _stream(stream)))


def mg_solve(h, opts: mg_opts, b, x, stream=None, raise_on_error=True, history=0) -> mg_result:
    """history > 0: the result's .hist holds the relative residual after each cycle."""
    import torch
    res = _result(history)
    n = _nv(h, _top(h))
    st = lib().mg_solve(h, ctypes.byref(opts), _ptr(b, torch.float64, n, "b"),
                        _ptr(x, torch.float64, n, "x"), ctypes.byref(res), _stream(stream))
    _trim(res)
    if raise_on_error:
        _check(st, res)
    return res


def mg_pcg(h, opts: mg_opts, b, x, stream=None, raise_on_error=True, history=0) -> mg_result:
    """history > 0: the result's .hist holds the loop's relative residual per iteration."""
    import torch
    res = _result(history)
    n = _nv(h, _top(h))
    st = lib().mg_pcg(h, ctypes.byref(opts), _ptr(b, torch.float64, n, "b"),
                      _ptr(x, torch.float64, n, "x"), ctypes.byref(res), _stream(stream))
    _trim(res)
    if raise_on_error:
        _check(st, res)
    return res


def _opt_ptr(t, dtype, n, name):
    return ctypes.c_void_p(None) if t is None else _ptr(t, dtype, n, name)


def mg_pcg_adjoint(h, opts: mg_opts, u, grad_u, grad_b, grad_k=None, stream=None,
                   raise_on_error=True, grad_w=None) -> mg_result:
    """grad_b = A^-1 grad_u; grad_k (if given) += dJ/dk at the vertices and grad_w (if given,
    one entry per finest-level edge) += dJ/dw for the edge weights w = star1 k (accumulate)."""
    import torch
    res = mg_result()
    top = _top(h)
    n = _nv(h, top)
    ne = mg_hierarchy_info(h, top)["ne"]
    st = lib().mg_pcg_adjoint(h, ctypes.byref(opts), _opt_ptr(u, torch.float64, n, "u"),
                              _ptr(grad_u, torch.float64, n, "grad_u"),
                              _ptr(grad_b, torch.float64, n, "grad_b"),
                              _opt_ptr(grad_k, torch.float64, n, "grad_k"),
                              _opt_ptr(grad_w, torch.float64, ne, "grad_w"), ctypes.byref(res),
                              _stream(stream))
    if raise_on_error:
        _check(st, res)
    return res


def porous_params_make(Ra: float, phi: float, dt: float, solve: mg_opts | None = None,
                       delta_T: float = 1.0, y_len: float = 1.0) -> porous_params:
    """kappa = delta_T * y_len / (phi * Ra); delta_T = y_len = 1 is the scaled form."""
    p = porous_params()
    p.Ra, p.phi, p.dt = float(Ra), float(phi), float(dt)
    p.solve = solve if solve is not None else mg_opts_default()
    p.delta_T, p.y_len = float(delta_T), float(y_len)
    return p


def porous_rhs(h, prm: porous_params, T, dTdt, p=None, stream=None) -> mg_result:
    import torch
    res = mg_result()
    n = _nv(h, _top(h))
    _check(lib().porous_rhs(h, ctypes.byref(prm), _ptr(T, torch.float64, n, "T"),
                            _ptr(dTdt, torch.float64, n, "dTdt"), _opt_ptr(p, torch.float64, n, "p"),
                            ctypes.byref(res), _stream(stream)), res)
    return res


def porous_rk_opts_make(model: porous_params, t_end: float, rtol: float = 1e-9,
                        atol: float = 1e-6, h0: float = 0.0, max_steps: int = 100000,
                        fixed_step: bool = False) -> porous_rk_opts:
    o = porous_rk_opts()
    o.model = model
    o.t_end, o.rtol, o.atol, o.h0 = float(t_end), float(rtol), float(atol), float(h0)
    o.max_steps, o.fixed_step = int(max_steps), int(bool(fixed_step))
    return o


def porous_integrate(h, opts: porous_rk_opts, T0, T_end, t_save=(), T_save=None, stream=None,
                     raise_on_error=True, noalloc=False) -> porous_rk_stats:
    """T_save: (len(t_save), nv) float64 device tensor (rows = save times), or None.
    noalloc=True calls porous_integrate_noalloc (no device allocation; static work area)."""
    import torch
    n = _nv(h, _top(h))
    ts = np.ascontiguousarray(np.asarray(t_save, dtype=np.float64))
    if len(ts) and (T_save is None or tuple(T_save.shape) != (len(ts), n)):
        raise ValueError("T_save must be (len(t_save), nv)")
    st = porous_rk_stats()
    fn = lib().porous_integrate_noalloc if noalloc else lib().porous_integrate
    code = fn(h, ctypes.byref(opts), _ptr(T0, torch.float64, n, "T0"),
                                  len(ts), ts.ctypes.data if len(ts) else None,
                                  _ptr(T_save, torch.float64, n * len(ts), "T_save") if len(ts) else None,
                                  _ptr(T_end, torch.float64, n, "T_end"), ctypes.byref(st),
                                  _stream(stream))
    if raise_on_error:
        _check(code)
    return st


def porous_step(h, prm: porous_params, T, T_out, p=None, stream=None, raise_on_error=True) -> mg_result:
    import torch
    res = mg_result()
    n = _nv(h, _top(h))
    st = lib().porous_step(h, ctypes.byref(prm), _ptr(T, torch.float64, n, "T"),
                           _ptr(T_out, torch.float64, n, "T_out"), _opt_ptr(p, torch.float64, n, "p"),
                           ctypes.byref(res), _stream(stream))
    if raise_on_error:
        _check(st, res)
    return res


def porous_step_adjoint(h, prm: porous_params, T, p, lam, lam_out, grad_k=None, stream=None,
                        psi=None):
    """psi (optional tensor): receives the adjoint pressure."""
    import torch
    n = _nv(h, _top(h))
    _check(lib().porous_step_adjoint(h, ctypes.byref(prm), _ptr(T, torch.float64, n, "T"),
                                     _opt_ptr(p, torch.float64, n, "p"),
                                     _ptr(lam, torch.float64, n, "lambda"),
                                     _ptr(lam_out, torch.float64, n, "lambda_out"),
                                     _opt_ptr(grad_k, torch.float64, n, "grad_k"),
                                     _opt_ptr(psi, torch.float64, n, "psi"), _stream(stream)))


class BatchRef:
    """A batch handle with the vertex count of each instance (for argument checks)."""

    def __init__(self, ptr, nvs):
        self._as_parameter_ = ctypes.c_void_p(ptr)
        self.nvs = list(nvs)
        self.n = len(self.nvs)


def mg_batch_create(hs, opts: mg_opts, tune: mg_batch_tuning | None = None,
                    tune_cache: str | None = None) -> BatchRef:
    """hs: one hierarchy handle per instance (repeat a handle to share its hierarchy)."""
    n = len(hs)
    arr = (_vp * n)(*[h.value if isinstance(h, ctypes.c_void_p) else h for h in hs])
    out = _vp()
    _check(lib().mg_batch_create(arr, n, ctypes.byref(opts),
                                 ctypes.byref(tune) if tune is not None else None,
                                 tune_cache.encode() if tune_cache else None, ctypes.byref(out)))
    return BatchRef(out.value, [_nv(h, _top(h)) for h in hs])


def _ptr_arrays(bt: BatchRef, bs, xs):
    import torch
    if len(bs) != bt.n or len(xs) != bt.n:
        raise ValueError(f"need {bt.n} right-hand sides and solutions")
    pb = (_vp * bt.n)(*[_ptr(b, torch.float64, nv, "b").value for b, nv in zip(bs, bt.nvs)])
    px = (_vp * bt.n)(*[_ptr(x, torch.float64, nv, "x").value for x, nv in zip(xs, bt.nvs)])
    return pb, px


def mg_batch_solve(bt: BatchRef, bs, xs, stream=None, raise_on_error=True):
    """Solves every instance; returns the list of mg_result."""
    pb, px = _ptr_arrays(bt, bs, xs)
    res = (mg_result * bt.n)()
    st = lib().mg_batch_solve(bt, pb, px, res, _stream(stream))
    out = list(res)
    if raise_on_error:
        _check(st, out)
    return out


def mg_batch_autotune(bt: BatchRef, bs, xs, reps: int = 2, tune_cache: str | None = None):
    """Returns (chosen mg_batch_tuning, best time in ms)."""
    pb, px = _ptr_arrays(bt, bs, xs)
    chosen = mg_batch_tuning()
    ms = ctypes.c_double()
    _check(lib().mg_batch_autotune(bt, pb, px, int(reps),
                                   tune_cache.encode() if tune_cache else None,
                                   ctypes.byref(chosen), ctypes.byref(ms)))
    return chosen, ms.value


def mg_batch_info(bt: BatchRef):
    """Returns (mg_batch_tuning, number of groups)."""
    t = mg_batch_tuning()
    ng = ctypes.c_int32()
    _check(lib().mg_batch_info(bt, ctypes.byref(t), ctypes.byref(ng)))
    return t, ng.value


def mg_batch_free(bt: BatchRef):
    if bt is not None and bt._as_parameter_.value:
        lib().mg_batch_free(bt)
        bt._as_parameter_ = ctypes.c_void_p(None)


def mg_time_kernel(h, kernel: int, level: int, dtype: int, reps: int, stream=None) -> float:
    ms = ctypes.c_double()
    _check(lib().mg_time_kernel(h, int(kernel), int(level), int(dtype), int(reps), _stream(stream),
                                ctypes.byref(ms)))
    return ms.value


def mg_probe_begin(h, level: int, dtype: int):
    _check(lib().mg_probe_begin(h, int(level), int(dtype)))


def mg_probe_end(h):
    """Returns (mean ms per probed sweep launch, number of launches)."""
    ms = ctypes.c_double()
    n = ctypes.c_int32()
    _check(lib().mg_probe_end(h, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ----------------------------------------------------------------- convenience
class Hierarchy:
    """Owns a mesh and a hierarchy handle; frees both when closed or collected."""

    def __init__(self, kind: str, n_subdiv: int, base_cells: int = 4, bc=None, xyz=None, tri=None,
                 order: int = MG_ORDER_STRIPES, cubic_mask: int = 0):
        if kind == "square":
            self.mesh = dec_mesh_square_grid(base_cells)
            bc = MG_BC_DIRICHLET0 if bc is None else bc
            project = False
        elif kind == "sphere":
            self.mesh = dec_mesh_icosahedron()
            bc = MG_BC_NATURAL if bc is None else bc
            project = True
        elif kind == "arrays":
            self.mesh = dec_mesh_from_arrays(xyz, tri)
            bc = MG_BC_DIRICHLET0 if bc is None else bc
            project = False
        else:
            raise ValueError(kind)
        self.bc = bc
        self.h = mg_hierarchy_build(self.mesh, n_subdiv, project, bc, order=order,
                                    cubic_mask=cubic_mask)
        self.n_levels = mg_hierarchy_info(self.h, 0)["n_levels"]
        self.top = self.n_levels - 1
        self.info = [mg_hierarchy_info(self.h, l) for l in range(self.n_levels)]

    @classmethod
    def from_maps(cls, xyz_list, tri_list, maps, bc=MG_BC_DIRICHLET0,
                  order: int = MG_ORDER_STRIPES):
        """Hierarchy over given meshes (coarsest first) related by geometric maps M(f)."""
        self = cls.__new__(cls)
        self.meshes = [dec_mesh_from_arrays(x, t) for x, t in zip(xyz_list, tri_list)]
        self.mesh = None
        self.bc = bc
        self.h = mg_hierarchy_build_maps(self.meshes, maps, bc, order=order)
        self.n_levels = mg_hierarchy_info(self.h, 0)["n_levels"]
        self.top = self.n_levels - 1
        self.info = [mg_hierarchy_info(self.h, l) for l in range(self.n_levels)]
        return self

    def nv(self, level=None):
        return self.info[self.top if level is None else level]["nv"]

    def close(self):
        if getattr(self, "h", None):
            mg_hierarchy_free(self.h)
            self.h = None
        if getattr(self, "mesh", None):
            dec_mesh_free(self.mesh)
            self.mesh = None
        for m in getattr(self, "meshes", None) or []:
            dec_mesh_free(m)
        self.meshes = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
