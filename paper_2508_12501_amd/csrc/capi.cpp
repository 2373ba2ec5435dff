// extern "C" entry points of libdecmg.so (declared in include/decmg.h).  Validation happens
// here, before any launch; exceptions from the host code become status codes.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "batch.hpp"
#include "decmg.h"
#include "geomap.hpp"
#include "hier.hpp"
#include "solver.hpp"
#include "util.hpp"

struct dec_mesh {
  decmg::Mesh m;
};
struct mg_hierarchy {
  std::unique_ptr<decmg::Hierarchy> h;
};
struct mg_batch {
  std::unique_ptr<decmg::Batch> b;
};

namespace {
thread_local std::string g_err;

mg_status fail(mg_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define API_BEGIN try {
#define API_END                                                              \
  }                                                                          \
  catch (const decmg::DeviceError& e) {                                      \
    const std::string w = e.what();                                          \
    return fail(w.find("out of memory") != std::string::npos ? MG_ENOMEM     \
                                                             : MG_EDEVICE,   \
                w);                                                          \
  }                                                                          \
  catch (const std::bad_alloc&) {                                            \
    return fail(MG_ENOMEM, "out of host memory");                            \
  }                                                                          \
  catch (const std::exception& e) {                                          \
    return fail(MG_EINVAL, e.what());                                        \
  }

hipStream_t S(void* p) { return reinterpret_cast<hipStream_t>(p); }

mg_status check_level(const mg_hierarchy* h, int32_t level, bool need_coarser = false) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  const int nl = int(h->h->lv.size());
  if (level < 0 || level >= nl) return fail(MG_EINVAL, "level out of range");
  if (need_coarser && level < 1) return fail(MG_EINVAL, "level 0 has no coarser level");
  return MG_OK;
}

mg_status check_dtype(int32_t dtype) {
  if (dtype != MG_F64 && dtype != MG_F32) return fail(MG_EINVAL, "dtype must be MG_F64 or MG_F32");
  return MG_OK;
}

mg_status check_opts(const mg_opts* o) {
  if (!o) return fail(MG_EINVAL, "null options");
  if (o->nu1 < 0 || o->nu2 < 0 || o->nu1 > 64 || o->nu2 > 64)
    return fail(MG_EINVAL, "nu1/nu2 must be in 0..64");
  if (!(o->omega > 0.0 && o->omega < 2.0)) return fail(MG_EINVAL, "omega must be in (0, 2)");
  if (o->precision != MG_F64 && o->precision != MG_F32)
    return fail(MG_EINVAL, "precision must be MG_F64 or MG_F32");
  if (o->outer != MG_OUTER_CG && o->outer != MG_OUTER_FCG && o->outer != MG_OUTER_IR)
    return fail(MG_EINVAL, "unknown outer method");
  if (!(o->rtol > 0.0) || !std::isfinite(o->rtol)) return fail(MG_EINVAL, "rtol must be > 0");
  if (o->max_iter < 1) return fail(MG_EINVAL, "max_iter must be >= 1");
  if (o->cycle != MG_CYCLE_V && o->cycle != MG_CYCLE_W && o->cycle != MG_CYCLE_F)
    return fail(MG_EINVAL, "cycle must be MG_CYCLE_V, MG_CYCLE_W or MG_CYCLE_F");
  if (o->smoother != MG_SMOOTH_JACOBI && o->smoother != MG_SMOOTH_GS &&
      o->smoother != MG_SMOOTH_CG)
    return fail(MG_EINVAL, "smoother must be MG_SMOOTH_JACOBI, MG_SMOOTH_GS or MG_SMOOTH_CG");
  if (o->fuse_levels != 0 && o->fuse_levels != 1) return fail(MG_EINVAL, "fuse_levels must be 0 or 1");
  if (o->compat_check != 0 && o->compat_check != 1)
    return fail(MG_EINVAL, "compat_check must be 0 or 1");
  if (o->stall_checks < 0 || o->stall_checks > 1000)
    return fail(MG_EINVAL, "stall_checks must be in 0..1000");
  return MG_OK;
}

// Options of a Krylov solve (mg_pcg and what runs it): CG needs a linear, symmetric cycle.
mg_status check_krylov_opts(const mg_opts* o) {
  if (mg_status st = check_opts(o); st != MG_OK) return st;
  if (o->smoother == MG_SMOOTH_CG && o->outer == MG_OUTER_CG)
    return fail(MG_EINVAL, "CG smoothing makes the cycle nonlinear: use MG_OUTER_FCG or MG_OUTER_IR");
  return MG_OK;
}


template <typename T>
void op_vcycle(decmg::Hierarchy& H, const mg_opts& o, int level, const void* b, void* x,
               hipStream_t s) {
  using namespace decmg;
  Level& L = *H.lv[level];
  LevelVecs<T>& V = vecs<T>(L);
  const T* bn = static_cast<const T*>(b);
  T* xn = static_cast<T*>(x);
  const int32_t nb = int32_t(L.bnd_h.size());
  k::gather<T>(L.perm, L.n, bn, V.b, s);
  if (level == 0) {
    k::coarse<T>(H, V.b, V.x, nullptr, s);
    k::scatter<T>(L.perm, L.n, V.x, xn, s);
    k::bnd_copy<T>(L.bnd_ids, nb, bn, xn, s);
    return;
  }
  k::gather<T>(L.perm, L.n, xn, V.x, s);
  T* cur = vcycle<T>(H, level, V.b, V.x, o, nullptr, s);
  k::scatter<T>(L.perm, L.n, cur, xn, s);
  // the identity rows of non-unknowns under the same smoother: Jacobi moves x towards b by
  // omega per sweep; Gauss-Seidel and CG smoothing set x = b
  if (o.smoother != MG_SMOOTH_JACOBI) {
    if (o.nu1 + o.nu2 > 0) k::bnd_copy<T>(L.bnd_ids, nb, bn, xn, s);
  } else {
    for (int i = 0; i < o.nu1 + o.nu2; ++i) k::bnd_jacobi<T>(L.bnd_ids, nb, bn, xn, o.omega, s);
  }
}

template <typename T>
void op_smooth(decmg::Hierarchy& H, int level, int nsweeps, double omega, const void* b, void* x,
               hipStream_t s) {
  using namespace decmg;
  Level& L = *H.lv[level];
  LevelVecs<T>& V = vecs<T>(L);
  const T* bn = static_cast<const T*>(b);
  T* xn = static_cast<T*>(x);
  k::gather<T>(L.perm, L.n, bn, V.b, s);
  k::gather<T>(L.perm, L.n, xn, V.x, s);
  T *cur = V.x, *oth = V.t;
  for (int i = 0; i < nsweeps; ++i) {
    k::jacobi<T>(L, cur, V.b, oth, omega, nullptr, s);
    std::swap(cur, oth);
  }
  k::scatter<T>(L.perm, L.n, cur, xn, s);
  for (int i = 0; i < nsweeps; ++i)
    k::bnd_jacobi<T>(L.bnd_ids, int32_t(L.bnd_h.size()), bn, xn, omega, s);
}

template <typename T>
void op_apply(decmg::Hierarchy& H, int level, const void* x, void* y, hipStream_t s) {
  using namespace decmg;
  Level& L = *H.lv[level];
  LevelVecs<T>& V = vecs<T>(L);
  k::gather<T>(L.perm, L.n, static_cast<const T*>(x), V.x, s);
  k::spmv<T>(L, V.x, V.r, nullptr, s);
  k::scatter<T>(L.perm, L.n, V.r, static_cast<T*>(y), s);
  k::bnd_copy<T>(L.bnd_ids, int32_t(L.bnd_h.size()), static_cast<const T*>(x), static_cast<T*>(y), s);
}

template <typename T>
void op_restrict(decmg::Hierarchy& H, int level, const void* rf, void* rc, hipStream_t s) {
  using namespace decmg;
  Level& F = *H.lv[level];
  Level& C = *H.lv[level - 1];
  k::gather<T>(F.perm, F.n, static_cast<const T*>(rf), vecs<T>(F).r, s);
  k::restrict_<T>(F, C, vecs<T>(F).r, vecs<T>(C).b, nullptr, s);
  k::scatter<T>(C.perm, C.n, vecs<T>(C).b, static_cast<T*>(rc), s);
  k::bnd_zero<T>(C.bnd_ids, int32_t(C.bnd_h.size()), static_cast<T*>(rc), s);
}

template <typename T>
void op_prolong(decmg::Hierarchy& H, int level, const void* ec, void* xf, hipStream_t s) {
  using namespace decmg;
  Level& F = *H.lv[level];
  Level& C = *H.lv[level - 1];
  k::gather<T>(C.perm, C.n, static_cast<const T*>(ec), vecs<T>(C).x, s);
  k::gather<T>(F.perm, F.n, static_cast<const T*>(xf), vecs<T>(F).x, s);
  k::prolong<T>(F, C, vecs<T>(C).x, vecs<T>(F).x, nullptr, s);
  k::scatter<T>(F.perm, F.n, vecs<T>(F).x, static_cast<T*>(xf), s);
}

}  // namespace

extern "C" {

const char* mg_last_error(void) { return g_err.c_str(); }
int32_t mg_abi_version(void) { return 4; }

mg_status dec_mesh_from_arrays(int64_t nv, const double* xyz, int64_t nt, const int32_t* tri,
                               dec_mesh** out) {
  API_BEGIN
  if (!out || !xyz || !tri) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if (nv < 3 || nt < 1) return fail(MG_EINVAL, "mesh needs nv >= 3 and nt >= 1");
  if (nv > (int64_t(1) << 30) || nt > (int64_t(1) << 30)) return fail(MG_EINVAL, "mesh too large");
  auto m = std::make_unique<dec_mesh>();
  m->m.nv = nv;
  m->m.nt = nt;
  m->m.xyz.assign(xyz, xyz + 3 * nv);
  m->m.tri.assign(tri, tri + 3 * nt);
  for (int64_t i = 0; i < 3 * nt; ++i)
    if (tri[i] < 0 || tri[i] >= nv) return fail(MG_EINVAL, "triangle index out of range");
  std::string err = m->m.validate_vertices();
  if (err.empty()) err = m->m.build_topology();
  if (!err.empty()) return fail(MG_EINVAL, err);
  *out = m.release();
  API_END
  return MG_OK;
}

mg_status dec_mesh_square_grid(int32_t ncells, dec_mesh** out) {
  API_BEGIN
  if (!out) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if (ncells < 1 || ncells > 32768) return fail(MG_EINVAL, "ncells must be in 1..32768");
  auto m = std::make_unique<dec_mesh>();
  m->m = decmg::square_grid(ncells);
  std::string err = m->m.build_topology();
  if (!err.empty()) return fail(MG_EINVAL, err);
  *out = m.release();
  API_END
  return MG_OK;
}

mg_status dec_mesh_icosahedron(dec_mesh** out) {
  API_BEGIN
  if (!out) return fail(MG_EINVAL, "null argument");
  auto m = std::make_unique<dec_mesh>();
  m->m = decmg::icosahedron();
  std::string err = m->m.build_topology();
  if (!err.empty()) return fail(MG_EINVAL, err);
  *out = m.release();
  API_END
  return MG_OK;
}

void dec_mesh_free(dec_mesh* m) { delete m; }

mg_status mg_hierarchy_build(const dec_mesh* base, const mg_hier_opts* opts, void* stream,
                             mg_hierarchy** out) {
  API_BEGIN
  (void)stream;
  if (!base || !opts || !out) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if (opts->n_subdiv < 0 || opts->n_subdiv > 12) return fail(MG_EINVAL, "n_subdiv must be in 0..12");
  if (opts->bc != MG_BC_DIRICHLET0 && opts->bc != MG_BC_NATURAL)
    return fail(MG_EINVAL, "bc must be MG_BC_DIRICHLET0 or MG_BC_NATURAL");
  if (opts->order != MG_ORDER_STRIPES && opts->order != MG_ORDER_MORTON)
    return fail(MG_EINVAL, "order must be MG_ORDER_STRIPES or MG_ORDER_MORTON");
  if (opts->cubic_mask < 0 || (opts->n_subdiv < 31 && (opts->cubic_mask >> opts->n_subdiv) != 0))
    return fail(MG_EINVAL, "cubic_mask has bits beyond n_subdiv");
  double growth = 1.0;
  for (int32_t i = 0; i < opts->n_subdiv; ++i) growth *= ((opts->cubic_mask >> i) & 1) ? 9.0 : 4.0;
  if (double(base->m.nt) * growth > double(int64_t(1) << 30))
    return fail(MG_EINVAL, "finest level would exceed 2^30 triangles");
  auto h = std::make_unique<mg_hierarchy>();
  h->h.reset(decmg::build_hierarchy(base->m, *opts));
  *out = h.release();
  API_END
  return MG_OK;
}

mg_status mg_hierarchy_build_maps(int32_t n_levels, const dec_mesh* const* meshes,
                                  const mg_geomap* maps, const mg_hier_opts* opts, void* stream,
                                  mg_hierarchy** out) {
  API_BEGIN
  (void)stream;
  if (!meshes || !opts || !out || (n_levels > 1 && !maps)) return fail(MG_EINVAL, "null argument");
  *out = nullptr;
  if (n_levels < 1 || n_levels > 32) return fail(MG_EINVAL, "n_levels must be in 1..32");
  if (opts->n_subdiv != 0 || opts->project_sphere != 0 || opts->cubic_mask != 0)
    return fail(MG_EINVAL, "n_subdiv, project_sphere and cubic_mask must be 0 for given maps");
  if (opts->bc != MG_BC_DIRICHLET0 && opts->bc != MG_BC_NATURAL)
    return fail(MG_EINVAL, "bc must be MG_BC_DIRICHLET0 or MG_BC_NATURAL");
  if (opts->order != MG_ORDER_STRIPES && opts->order != MG_ORDER_MORTON)
    return fail(MG_EINVAL, "order must be MG_ORDER_STRIPES or MG_ORDER_MORTON");
  std::vector<decmg::Mesh> ms;
  bool nested = true;
  for (int32_t l = 0; l < n_levels; ++l) {
    if (!meshes[l]) return fail(MG_EINVAL, "null mesh");
    ms.push_back(meshes[l]->m);
    ms.back().scheme = 0;
    ms.back().parent.clear();
    ms.back().parent3.clear();
    ms.back().pweight.clear();
    if (l == 0) continue;
    const std::string err = decmg::check_geomap(ms[l - 1], ms[l].nv, maps[l - 1]);
    if (!err.empty()) return fail(MG_EINVAL, "map " + std::to_string(l - 1) + ": " + err);
    decmg::set_interp_from_geomap(ms[l], maps[l - 1]);
    nested = nested && decmg::geomap_keeps_ids(maps[l - 1]);
  }
  if (double(ms.back().nt) > double(int64_t(1) << 30))
    return fail(MG_EINVAL, "finest level exceeds 2^30 triangles");
  auto h = std::make_unique<mg_hierarchy>();
  h->h.reset(decmg::build_hierarchy_maps(std::move(ms), nested, *opts));
  *out = h.release();
  API_END
  return MG_OK;
}

mg_status mg_geomap_compose(const mg_geomap* g, const mg_geomap* f, int64_t* colptr,
                            int32_t* rowval, double* nzval, int64_t* nnz) {
  API_BEGIN
  if (!g || !f || !nnz) return fail(MG_EINVAL, "null argument");
  const std::string err = decmg::compose_geomaps(*g, *f, colptr, rowval, nzval, nnz);
  if (!err.empty()) return fail(MG_EINVAL, err);
  API_END
  return MG_OK;
}

void mg_hierarchy_free(mg_hierarchy* h) { delete h; }

mg_status mg_hierarchy_info(const mg_hierarchy* h, int32_t level, mg_level_info* out) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (!out) return fail(MG_EINVAL, "null argument");
  const decmg::Level& L = *h->h->lv[level];
  out->n_levels = int32_t(h->h->lv.size());
  out->level = level;
  out->nv = L.mesh.nv;
  out->ne = L.mesh.ne;
  out->nt = L.mesh.nt;
  out->n_unknowns = L.n;
  out->nnz_operator = L.nnz;
  out->index_bytes = L.op.col16 ? 2 : 4;
  out->scheme = L.mesh.scheme;
  out->row_patterns = L.op.npat;
  out->restrict_width = (level >= 1 && !L.tr.weighted) ? L.tr.r_uw : -1;
  out->fused_tiles = L.tiles.ntiles;
  out->fused_tile_rows = int32_t(L.tiles.rows_total);
  out->weight_bytes32 = L.op.w_exact16 ? 2 : 4;
  out->weight_bytes64 = L.op.w_exact16 ? 2 : (L.op.w_exact32 ? 4 : 8);
  out->uniform_width = L.op.uw;
  out->rows_per_thread = (L.op.uw >= 1 && L.op.uw <= 8) ? 2 : 1;
  out->interp_packed16 = L.tr.p_ab16 ? 1 : 0;
  out->restrict_offsets16 = L.tr.r_col16 ? 1 : 0;
  return MG_OK;
}

mg_status mg_hierarchy_export(const mg_hierarchy* h, int32_t level, double* xyz, int32_t* tri,
                              int32_t* edges, int32_t* tri_edges, int8_t* tri_sign,
                              double* star0, double* star1, uint8_t* boundary,
                              int32_t* parents) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  const decmg::Mesh& m = h->h->lv[level]->mesh;
  auto cp = [](auto* dst, const auto& v) {
    if (dst && !v.empty()) std::memcpy(dst, v.data(), v.size() * sizeof(v[0]));
  };
  cp(xyz, m.xyz);
  cp(tri, m.tri);
  cp(edges, m.edge);
  cp(tri_edges, m.tri_edge);
  cp(tri_sign, m.tri_sign);
  cp(star0, m.star0);
  cp(star1, m.star1);
  cp(boundary, m.bnd);
  if (parents) {
    if (level == 0) return fail(MG_EINVAL, "level 0 has no parents");
    if (m.scheme != 1) return fail(MG_EINVAL, "not a binary level: use mg_hierarchy_export_interp");
    cp(parents, m.parent);
  }
  return MG_OK;
}

mg_status mg_hierarchy_export_interp(const mg_hierarchy* h, int32_t level, int32_t* parents,
                                     double* weights) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (level == 0) return fail(MG_EINVAL, "level 0 has no parents");
  const decmg::Mesh& m = h->h->lv[level]->mesh;
  if (parents) std::memcpy(parents, m.parent3.data(), m.parent3.size() * sizeof(int32_t));
  if (weights) std::memcpy(weights, m.pweight.data(), m.pweight.size() * sizeof(double));
  return MG_OK;
}

extern "C++" {  // helpers with C++ types, internal to this file
namespace {
// The finest level's vertex coefficient (host copy of a device array of nv values), checked.
mg_status set_vertex_field(decmg::Hierarchy& H, std::vector<double> kv) {
  for (double v : kv)
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(MG_EINVAL, "vertex coefficients must be finite and positive");
  H.kvert_h = std::move(kv);
  H.kedge_h.clear();
  const size_t nv = H.kvert_h.size();
  if (!H.kvert_d)
    decmg::check_hip(hipMalloc(&H.kvert_d, nv * sizeof(double)), "hipMalloc");
  decmg::check_hip(hipMemcpy(H.kvert_d, H.kvert_h.data(), nv * sizeof(double),
                             hipMemcpyHostToDevice),
                   "hipMemcpy");
  ++H.kversion;
  decmg::upload_weights(H);
  return MG_OK;
}

std::vector<double> to_host(const double* d, size_t n, void* stream) {
  std::vector<double> h(n);
  decmg::check_hip(hipStreamSynchronize(S(stream)), "hipStreamSynchronize");
  decmg::check_hip(hipMemcpy(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy");
  return h;
}
}  // namespace
}  // extern "C++"

mg_status mg_hierarchy_set_vertex_coeff(mg_hierarchy* h, const double* k_vertex, void* stream) {
  API_BEGIN
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  decmg::Hierarchy& H = *h->h;
  if (k_vertex && !H.nested_ids)
    return fail(MG_EINVAL, "the vertex coefficient is injected by vertex id: the maps of this "
                           "hierarchy do not keep the coarse vertex ids");
  if (!k_vertex) {
    H.kvert_h.clear();
    H.kedge_h.clear();
    ++H.kversion;
    decmg::upload_weights(H);
    return MG_OK;
  }
  return set_vertex_field(H, to_host(k_vertex, size_t(H.lv.back()->nv), stream));
  API_END
  return MG_OK;
}

mg_status mg_hierarchy_set_log_coeff(mg_hierarchy* h, const double* g_vertex, void* stream) {
  API_BEGIN
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  decmg::Hierarchy& H = *h->h;
  if (!g_vertex) return fail(MG_EINVAL, "null g");
  if (!H.nested_ids)
    return fail(MG_EINVAL, "the vertex coefficient is injected by vertex id: the maps of this "
                           "hierarchy do not keep the coarse vertex ids");
  std::vector<double> k = to_host(g_vertex, size_t(H.lv.back()->nv), stream);
  for (double& v : k) {
    if (!std::isfinite(v)) return fail(MG_EINVAL, "g must be finite");
    v = std::exp(v);
  }
  return set_vertex_field(H, std::move(k));
  API_END
  return MG_OK;
}

mg_status mg_hierarchy_coeff_grad_log(mg_hierarchy* h, const double* grad_k, double* grad_g,
                                      void* stream) {
  API_BEGIN
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (!grad_k || !grad_g) return fail(MG_EINVAL, "null vector");
  decmg::Hierarchy& H = *h->h;
  if (!H.kedge_h.empty())
    return fail(MG_EINVAL, "the hierarchy holds an edge coefficient, not a vertex one");
  decmg::k::mul_acc(H.lv.back()->nv, H.kvert_h.empty() ? nullptr : H.kvert_d, grad_k, grad_g,
                    S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status mg_hierarchy_set_debug(mg_hierarchy* h, int32_t flags) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (flags & ~int32_t(MG_DEBUG_ZERO_PRECOND32)) return fail(MG_EINVAL, "unknown debug flag");
  API_BEGIN
  decmg::Hierarchy& H = *h->h;
  if (H.debug_flags != flags) {
    // captured iterations hold the old behaviour
    for (auto& kv : H.graphs) (void)hipGraphExecDestroy(kv.second);
    H.graphs.clear();
    H.debug_flags = flags;
  }
  API_END
  return MG_OK;
}

mg_status mg_hierarchy_set_edge_coeff(mg_hierarchy* h, const double* k_edge, void* stream) {
  API_BEGIN
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  decmg::Hierarchy& H = *h->h;
  if (!k_edge) {
    H.kvert_h.clear();
    H.kedge_h.clear();
    ++H.kversion;
    decmg::upload_weights(H);
    return MG_OK;
  }
  for (const auto& L : H.lv)
    if (L->mesh.scheme != 1 && L->mesh.scheme != 2 && L.get() != H.lv.front().get())
      return fail(MG_EINVAL, "edge coefficients need a hierarchy of subdivisions: the levels of "
                             "mg_hierarchy_build_maps have no edge correspondence");
  std::vector<double> ke = to_host(k_edge, size_t(H.lv.back()->mesh.ne), stream);
  for (double v : ke)
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(MG_EINVAL, "edge coefficients must be finite and positive");
  H.kedge_h = decmg::coarsen_edge_coeff(H, std::move(ke));
  H.kvert_h.clear();
  ++H.kversion;
  decmg::upload_weights(H);
  API_END
  return MG_OK;
}

mg_status dec_star0_apply(mg_hierarchy* h, int32_t level, const double* f, double* b, void* stream) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (!f || !b) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  decmg::k::star0_apply(*h->h->lv[level], h->h->bc, f, b, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status dec_laplacian_apply(mg_hierarchy* h, int32_t level, int32_t dtype, const void* x, void* y,
                              void* stream) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (!x || !y) return fail(MG_EINVAL, "null vector");
  if (x == y) return fail(MG_EINVAL, "x and y must not alias");
  API_BEGIN
  if (dtype == MG_F64)
    op_apply<double>(*h->h, level, x, y, S(stream));
  else
    op_apply<float>(*h->h, level, x, y, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status mg_smooth(mg_hierarchy* h, int32_t level, int32_t dtype, int32_t nsweeps, double omega,
                    const void* b, void* x, void* stream) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (!b || !x) return fail(MG_EINVAL, "null vector");
  if (nsweeps < 0) return fail(MG_EINVAL, "nsweeps must be >= 0");
  if (!(omega > 0.0 && omega < 2.0)) return fail(MG_EINVAL, "omega must be in (0, 2)");
  API_BEGIN
  if (dtype == MG_F64)
    op_smooth<double>(*h->h, level, nsweeps, omega, b, x, S(stream));
  else
    op_smooth<float>(*h->h, level, nsweeps, omega, b, x, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status mg_restrict(mg_hierarchy* h, int32_t level, int32_t dtype, const void* r_fine,
                      void* r_coarse, void* stream) {
  if (mg_status st = check_level(h, level, true); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (!r_fine || !r_coarse) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  if (dtype == MG_F64)
    op_restrict<double>(*h->h, level, r_fine, r_coarse, S(stream));
  else
    op_restrict<float>(*h->h, level, r_fine, r_coarse, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status mg_prolong(mg_hierarchy* h, int32_t level, int32_t dtype, const void* e_coarse,
                     void* x_fine, void* stream) {
  if (mg_status st = check_level(h, level, true); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (!e_coarse || !x_fine) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  if (dtype == MG_F64)
    op_prolong<double>(*h->h, level, e_coarse, x_fine, S(stream));
  else
    op_prolong<float>(*h->h, level, e_coarse, x_fine, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

void mg_opts_default(mg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->nu1 = 2;
  o->nu2 = 2;
  o->omega = 0.8;
  o->precision = MG_F64;
  o->outer = MG_OUTER_CG;
  o->rtol = 1e-10;
  o->max_iter = 200;
  o->check_every = 4;
  o->use_graph = 1;
  o->fuse_levels = 1;
  o->stall_checks = 3;
}

mg_status mg_vcycle(mg_hierarchy* h, const mg_opts* o, int32_t level, int32_t dtype, const void* b,
                    void* x, void* stream) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (mg_status st = check_opts(o); st != MG_OK) return st;
  if (!b || !x) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  if (dtype == MG_F64)
    op_vcycle<double>(*h->h, *o, level, b, x, S(stream));
  else
    op_vcycle<float>(*h->h, *o, level, b, x, S(stream));
  decmg::check_hip(hipGetLastError(), "kernel launch");
  API_END
  return MG_OK;
}

mg_status mg_solve(mg_hierarchy* h, const mg_opts* o, const double* b, double* x, mg_result* res,
                   void* stream) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (mg_status st = check_opts(o); st != MG_OK) return st;
  if (!b || !x) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  const int st = decmg::run_mg(*h->h, *o, b, x, res, S(stream));
  if (st != MG_OK) return fail(mg_status(st), "mg_solve stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status mg_pcg(mg_hierarchy* h, const mg_opts* o, const double* b, double* x, mg_result* res,
                 void* stream) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (mg_status st = check_krylov_opts(o); st != MG_OK) return st;
  if (!b || !x) return fail(MG_EINVAL, "null vector");
  API_BEGIN
  const int st = decmg::run_pcg(*h->h, *o, b, x, res, S(stream), false, o->compat_check != 0);
  if (st != MG_OK) return fail(mg_status(st), "mg_pcg stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status mg_pcg_adjoint(mg_hierarchy* h, const mg_opts* o, const double* u_fine,
                         const double* grad_u, double* grad_b, double* grad_k, double* grad_w,
                         mg_result* res, void* stream) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (mg_status st = check_krylov_opts(o); st != MG_OK) return st;
  if (!grad_u || !grad_b) return fail(MG_EINVAL, "null vector");
  if ((grad_k || grad_w) && !u_fine)
    return fail(MG_EINVAL, "grad_k and grad_w need the forward solution u_fine");
  if (grad_k && !h->h->kedge_h.empty())
    return fail(MG_EINVAL, "grad_k is the vertex-coefficient gradient; with an edge coefficient "
                           "use grad_w");
  API_BEGIN
  const int st = decmg::run_pcg_adjoint(*h->h, *o, u_fine, grad_u, grad_b, grad_k, grad_w, res,
                                        S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "mg_pcg_adjoint stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

extern "C++" {  // helpers with C++ types, internal to this file
namespace {
mg_status check_porous(const mg_hierarchy* h, const porous_params* p, bool need_dt = true) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  if (!p) return fail(MG_EINVAL, "null parameters");
  if (h->h->bc != MG_BC_NATURAL)
    return fail(MG_EINVAL, "the porous step needs a hierarchy with natural boundaries");
  if (!(p->Ra > 0) || !(p->phi > 0) || !std::isfinite(p->Ra) || !std::isfinite(p->phi) ||
      !(p->delta_T > 0) || !(p->y_len > 0) || !std::isfinite(p->delta_T) ||
      !std::isfinite(p->y_len))
    return fail(MG_EINVAL, "Ra, phi, delta_T and y_len must be finite and positive");
  if (need_dt && (!(p->dt > 0) || !std::isfinite(p->dt)))
    return fail(MG_EINVAL, "dt must be finite and positive");
  return check_krylov_opts(&p->solve);
}
decmg::PorousParams porous_of(const porous_params* p) { return decmg::porous_params_of(*p); }
}  // namespace
}  // extern "C++"

mg_status porous_step(mg_hierarchy* h, const porous_params* prm, const double* T, double* T_out,
                      double* p, mg_result* res, void* stream) {
  if (mg_status st = check_porous(h, prm); st != MG_OK) return st;
  if (!T || !T_out) return fail(MG_EINVAL, "null vector");
  if (T == T_out) return fail(MG_EINVAL, "T_out must not alias T");
  API_BEGIN
  const int st = decmg::run_porous_step(*h->h, porous_of(prm), T, T_out, p, res, S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "porous_step pressure solve stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status porous_rhs(mg_hierarchy* h, const porous_params* prm, const double* T, double* dTdt,
                     double* p, mg_result* res, void* stream) {
  if (mg_status st = check_porous(h, prm, false); st != MG_OK) return st;
  if (!T || !dTdt) return fail(MG_EINVAL, "null vector");
  if (T == dTdt) return fail(MG_EINVAL, "dTdt must not alias T");
  API_BEGIN
  const int st = decmg::run_porous_rhs(*h->h, porous_of(prm), T, dTdt, p, res, S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "porous_rhs pressure solve stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

extern "C++" {  // helpers with C++ types, internal to this file
namespace {
mg_status check_integrate(mg_hierarchy* h, const porous_rk_opts* o, const double* T0,
                          int32_t n_save, const double* t_save, double* T_save, double* T_end) {
  if (!o) return fail(MG_EINVAL, "null options");
  if (mg_status st = check_porous(h, &o->model, false); st != MG_OK) return st;
  if (!T0 || !T_end) return fail(MG_EINVAL, "null vector");
  if (!(o->t_end > 0) || !std::isfinite(o->t_end)) return fail(MG_EINVAL, "t_end must be > 0");
  if (o->max_steps < 1) return fail(MG_EINVAL, "max_steps must be >= 1");
  if (o->fixed_step != 0 && o->fixed_step != 1) return fail(MG_EINVAL, "fixed_step must be 0 or 1");
  if (!(o->h0 >= 0) || !std::isfinite(o->h0)) return fail(MG_EINVAL, "h0 must be >= 0");
  if (o->fixed_step && !(o->h0 > 0)) return fail(MG_EINVAL, "fixed steps need h0 > 0");
  if (!o->fixed_step && (!(o->rtol > 0) || !(o->atol > 0) || !std::isfinite(o->rtol) ||
                         !std::isfinite(o->atol)))
    return fail(MG_EINVAL, "rtol and atol must be finite and positive");
  if (n_save < 0 || (n_save > 0 && (!t_save || !T_save)))
    return fail(MG_EINVAL, "save times need t_save and T_save");
  for (int32_t i = 0; i < n_save; ++i)
    if (!(t_save[i] > (i ? t_save[i - 1] : 0.0)) || !(t_save[i] <= o->t_end))
      return fail(MG_EINVAL, "save times must increase strictly within (0, t_end]");
  return MG_OK;
}
}  // namespace
}  // extern "C++"

mg_status porous_integrate(mg_hierarchy* h, const porous_rk_opts* o, const double* T0,
                           int32_t n_save, const double* t_save, double* T_save, double* T_end,
                           porous_rk_stats* stats, void* stream) {
  if (mg_status st = check_integrate(h, o, T0, n_save, t_save, T_save, T_end); st != MG_OK)
    return st;
  API_BEGIN
  const int st = decmg::run_porous_integrate(*h->h, *o, T0, n_save, t_save, T_save, T_end, stats,
                                             S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "porous_integrate stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status porous_integrate_noalloc(mg_hierarchy* h, const porous_rk_opts* o, const double* T0,
                                   int32_t n_save, const double* t_save, double* T_save,
                                   double* T_end, porous_rk_stats* stats, void* stream) {
  if (mg_status st = check_integrate(h, o, T0, n_save, t_save, T_save, T_end); st != MG_OK)
    return st;
  API_BEGIN
  const int st = decmg::run_porous_integrate_noalloc(*h->h, *o, T0, n_save, t_save, T_save,
                                                     T_end, stats, S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "porous_integrate_noalloc stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status porous_step_adjoint(mg_hierarchy* h, const porous_params* prm, const double* T,
                              const double* p, const double* lambda, double* lambda_out,
                              double* grad_k, double* psi, void* stream) {
  if (mg_status st = check_porous(h, prm); st != MG_OK) return st;
  if (!T || !lambda || !lambda_out) return fail(MG_EINVAL, "null vector");
  if (lambda == lambda_out) return fail(MG_EINVAL, "lambda_out must not alias lambda");
  if (grad_k && !h->h->kedge_h.empty())
    return fail(MG_EINVAL, "grad_k is the vertex-coefficient gradient; the hierarchy holds an "
                           "edge coefficient");
  API_BEGIN
  const int st = decmg::run_porous_adjoint(*h->h, porous_of(prm), T, p, lambda, lambda_out,
                                           grad_k, psi, S(stream));
  if (st != MG_OK)
    return fail(mg_status(st), "porous_step_adjoint solve stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

extern "C++" {  // helpers with C++ types, internal to this file
namespace {
mg_status check_tuning(const mg_batch_tuning* t) {
  const int mc = t->max_cols;
  if (mc < 1 || mc > decmg::kBatchMaxCols || (mc & (mc - 1)) != 0)
    return fail(MG_EINVAL, "max_cols must be a power of two in 1..64");
  if (t->pad_groups != 0 && t->pad_groups != 1) return fail(MG_EINVAL, "pad_groups must be 0 or 1");
  if (t->streams < 1 || t->streams > 4) return fail(MG_EINVAL, "streams must be in 1..4");
  return MG_OK;
}
mg_status check_ptrs(const mg_batch* bt, const double* const* b, double* const* x) {
  if (!bt || !bt->b) return fail(MG_EINVAL, "null batch");
  if (!b || !x) return fail(MG_EINVAL, "null pointer array");
  for (size_t i = 0; i < bt->b->inst_h.size(); ++i)
    if (!b[i] || !x[i]) return fail(MG_EINVAL, "null vector for instance " + std::to_string(i));
  return MG_OK;
}
}  // namespace
}  // extern "C++"

mg_status mg_batch_create(mg_hierarchy* const* h, int32_t n, const mg_opts* o,
                          const mg_batch_tuning* tune, const char* tune_cache, mg_batch** out) {
  if (!out) return fail(MG_EINVAL, "null output handle");
  *out = nullptr;
  if (!h || n < 1) return fail(MG_EINVAL, "need at least one instance");
  if (mg_status st = check_opts(o); st != MG_OK) return st;
  if (o->outer != MG_OUTER_FCG) return fail(MG_EINVAL, "batched solves run FCG(1): outer must be MG_OUTER_FCG");
  if (o->smoother != MG_SMOOTH_JACOBI) return fail(MG_EINVAL, "batched solves smooth with Jacobi");
  for (int32_t i = 0; i < n; ++i)
    if (h[i] && h[i]->h)
      for (const auto& L : h[i]->h->lv)
        if (L->tr.weighted) return fail(MG_EINVAL, "batched solves take binary hierarchies only");
  if (tune)
    if (mg_status st = check_tuning(tune); st != MG_OK) return st;
  for (int32_t i = 0; i < n; ++i)
    if (!h[i] || !h[i]->h) return fail(MG_EINVAL, "null hierarchy for instance " + std::to_string(i));
  API_BEGIN
  auto B = std::make_unique<decmg::Batch>();
  B->opts = *o;
  for (int32_t i = 0; i < n; ++i) B->inst_h.push_back(h[i]->h.get());
  B->signature = decmg::batch_signature(*B);
  if (tune) {
    B->tune = decmg::BatchTuning{tune->max_cols, tune->pad_groups, tune->streams};
  } else {
    decmg::BatchTuning t;
    if (decmg::batch_cache_lookup(tune_cache, B->signature, t)) {
      const mg_batch_tuning ct{t.max_cols, t.pad_groups, t.streams, 0};
      if (check_tuning(&ct) == MG_OK) B->tune = t;
    }
  }
  decmg::batch_setup(*B);
  auto* r = new mg_batch;
  r->b = std::move(B);
  *out = r;
  API_END
  return MG_OK;
}

mg_status mg_batch_solve(mg_batch* bt, const double* const* b, double* const* x, mg_result* res,
                         void* stream) {
  if (mg_status st = check_ptrs(bt, b, x); st != MG_OK) return st;
  API_BEGIN
  const int st = decmg::batch_solve(*bt->b, b, x, res, S(stream));
  if (st != MG_OK) return fail(mg_status(st), "an instance of the batch stopped with status " + std::to_string(st));
  API_END
  return MG_OK;
}

mg_status mg_batch_autotune(mg_batch* bt, const double* const* b, double* const* x, int32_t reps,
                            const char* tune_cache, mg_batch_tuning* chosen, double* best_ms) {
  if (mg_status st = check_ptrs(bt, b, x); st != MG_OK) return st;
  if (reps < 1 || reps > 100) return fail(MG_EINVAL, "reps must be in 1..100");
  API_BEGIN
  const double ms = decmg::batch_autotune(*bt->b, b, x, reps, tune_cache);
  if (chosen) *chosen = mg_batch_tuning{bt->b->tune.max_cols, bt->b->tune.pad_groups, bt->b->tune.streams, 0};
  if (best_ms) *best_ms = ms;
  API_END
  return MG_OK;
}

mg_status mg_batch_info(const mg_batch* bt, mg_batch_tuning* tune, int32_t* n_groups) {
  if (!bt || !bt->b) return fail(MG_EINVAL, "null batch");
  if (tune) *tune = mg_batch_tuning{bt->b->tune.max_cols, bt->b->tune.pad_groups, bt->b->tune.streams, 0};
  if (n_groups) *n_groups = int32_t(bt->b->groups.size());
  return MG_OK;
}

void mg_batch_free(mg_batch* bt) { delete bt; }

mg_status mg_time_kernel(mg_hierarchy* h, int32_t kernel, int32_t level, int32_t dtype, int32_t reps,
                         void* stream, double* ms_per_launch) {
  if (mg_status st = check_level(h, level, kernel >= 3); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  if (kernel < 0 || kernel > 4) return fail(MG_EINVAL, "kernel must be 0..4");
  if (reps < 1 || !ms_per_launch) return fail(MG_EINVAL, "reps >= 1 and a result pointer needed");
  API_BEGIN
  using namespace decmg;
  Hierarchy& H = *h->h;
  Level& L = *H.lv[level];
  hipStream_t s = S(stream);
  hipEvent_t e0, e1;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  auto launch = [&](auto tag) {
    using T = decltype(tag);
    LevelVecs<T>& V = vecs<T>(L);
    switch (kernel) {
      case 0: k::jacobi<T>(L, V.x, V.b, V.t, 0.8, nullptr, s); break;
      case 1: k::spmv<T>(L, V.x, V.r, nullptr, s); break;
      case 2: k::residual<T>(L, V.x, V.b, V.r, nullptr, s); break;
      case 3: k::restrict_<T>(L, *H.lv[level - 1], V.r, vecs<T>(*H.lv[level - 1]).b, nullptr, s); break;
      case 4: k::prolong<T>(L, *H.lv[level - 1], vecs<T>(*H.lv[level - 1]).x, V.t, nullptr, s); break;
    }
  };
  auto run = [&]() {
    for (int i = 0; i < reps; ++i) {
      if (dtype == MG_F64) launch(double(0)); else launch(float(0));
    }
  };
  run();  // warm-up pass
  check_hip(hipEventRecord(e0, s), "hipEventRecord");
  run();
  check_hip(hipEventRecord(e1, s), "hipEventRecord");
  check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
  float ms = 0.f;
  check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  check_hip(hipGetLastError(), "kernel launch");
  *ms_per_launch = double(ms) / reps;
  API_END
  return MG_OK;
}

mg_status mg_probe_begin(mg_hierarchy* h, int32_t level, int32_t dtype) {
  if (mg_status st = check_level(h, level); st != MG_OK) return st;
  if (mg_status st = check_dtype(dtype); st != MG_OK) return st;
  decmg::Hierarchy::Probe& P = h->h->probe;
  for (auto& e : P.ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  P.ev.clear();
  P.on = true;
  P.level = level;
  P.dtype = dtype;
  P.stream = nullptr;
  return MG_OK;
}

mg_status mg_probe_end(mg_hierarchy* h, double* ms_per_launch, int32_t* launches) {
  if (!h || !h->h) return fail(MG_EINVAL, "null hierarchy");
  API_BEGIN
  decmg::Hierarchy::Probe& P = h->h->probe;
  P.on = false;
  double total = 0.0;
  if (!P.ev.empty()) decmg::check_hip(hipStreamSynchronize(P.stream), "hipStreamSynchronize");
  for (auto& e : P.ev) {
    float ms = 0.f;
    decmg::check_hip(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
    total += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  const int32_t n = int32_t(P.ev.size());
  P.ev.clear();
  if (launches) *launches = n;
  if (ms_per_launch) *ms_per_launch = n ? total / n : 0.0;
  API_END
  return MG_OK;
}

}  // extern "C"
