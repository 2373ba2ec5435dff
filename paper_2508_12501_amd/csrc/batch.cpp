// Host orchestration of the batched solve: grouping, buffers, per-group iteration graphs,
// concurrent replay over a few streams, and the tuner that picks the grouping and stream count.
//
// Each column runs the FCG(1) recurrence of mg_pcg with a V(nu1, nu2) weighted-Jacobi cycle as
// preconditioner (FP32 on a power-of-two-scaled FP32 copy of the FP64 residual, or FP64), the
// dense FP64 coarsest solve, and, on natural-boundary hierarchies, the removal of the vertex
// mean from b, from every preconditioned vector and from x.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <stdexcept>

#include "batch.hpp"
#include "util.hpp"

namespace decmg {

namespace {

template <typename T>
T* dalloc(size_t n) {
  T* p = nullptr;
  check_hip(hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)), "hipMalloc");
  check_hip(hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)), "hipMemset");
  return p;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

int pow2_ceil(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}
int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p <<= 1;
  return p;
}

template <typename T> std::vector<BatchLevelVecs<T>>& bvecs(BatchGroup& G);
template <> std::vector<BatchLevelVecs<float>>& bvecs<float>(BatchGroup& G) { return G.v32; }
template <> std::vector<BatchLevelVecs<double>>& bvecs<double>(BatchGroup& G) { return G.v64; }

// One cycle of shape `kind` (V, W or F, as in the single-column solver) on level l, from zero
// or from x_init (a buffer of this level).
template <typename T>
T* cycle_b(const mg_opts& o, BatchGroup& G, int l, const T* b, T* x_init, int kind,
           hipStream_t s) {
  Hierarchy& H = *G.H;
  Level& L = *H.lv[l];
  BatchLevelVecs<T>& V = bvecs<T>(G)[l];
  const int M = G.M;
  const BatchFlag* fl = G.flag;
  if (l == 0) {
    bk::coarse<T>(M, H, b, V.x, fl, s);
    return V.x;
  }
  if (k::coarse_cycle_general_ok<T>(H, l, false)) {
    // levels l..0 in one launch, one workgroup per column (the register-resident bottom of the
    // single solve, reading the columns with stride M)
    T* xo = x_init ? x_init : V.x;
    k::coarse_cycle_columns<T>(H, l, b, xo, x_init != nullptr, o.omega, o.nu1, o.nu2, kind, M,
                               &fl->all_done, s);
    return xo;
  }
  T* cur;
  T* oth;
  int pre = o.nu1;
  if (x_init) {
    cur = x_init;
    oth = (x_init == V.t) ? V.x : V.t;
  } else {
    cur = V.x;
    oth = V.t;
    if (pre >= 1) {
      bk::jacobi_zero<T>(M, L, b, cur, o.omega, fl, s);
      --pre;
    } else {
      bk::zero(cur, size_t(L.n) * M * sizeof(T), s);
    }
  }
  for (; pre > 0; --pre) {
    bk::rows<T>(2, M, L, cur, b, oth, o.omega, fl, s);
    std::swap(cur, oth);
  }
  Level& C = *H.lv[l - 1];
  BatchLevelVecs<T>& VC = bvecs<T>(G)[l - 1];
  bk::rows<T>(1, M, L, cur, b, V.r, 0.0, fl, s);
  bk::restrict_<T>(M, L, C, V.r, VC.b, fl, s);
  T* ec;
  if (kind == MG_CYCLE_W) {
    ec = cycle_b<T>(o, G, l - 1, VC.b, nullptr, MG_CYCLE_W, s);
    ec = cycle_b<T>(o, G, l - 1, VC.b, ec, MG_CYCLE_W, s);
  } else if (kind == MG_CYCLE_F) {
    ec = cycle_b<T>(o, G, l - 1, VC.b, nullptr, MG_CYCLE_F, s);
    ec = cycle_b<T>(o, G, l - 1, VC.b, ec, MG_CYCLE_V, s);
  } else {
    ec = cycle_b<T>(o, G, l - 1, VC.b, nullptr, MG_CYCLE_V, s);
  }
  int post = o.nu2;
  if (post >= 1 && int64_t(L.n) * M <= kLaunchBoundRows) {
    bk::prolong_sweep<T>(M, L, ec, cur, b, oth, o.omega, fl, s);
    std::swap(cur, oth);
    --post;
  } else {
    bk::prolong<T>(M, L, C, ec, cur, fl, s);
  }
  for (; post > 0; --post) {
    bk::rows<T>(2, M, L, cur, b, oth, o.omega, fl, s);
    std::swap(cur, oth);
  }
  return cur;
}

// One FCG(1) iteration of every column of group G.
void enqueue_iter(const mg_opts& o, BatchGroup& G, hipStream_t s) {
  Hierarchy& H = *G.H;
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  const int M = G.M;
  const int top = int(H.lv.size()) - 1;
  const int natural = H.bc == MG_BC_NATURAL ? 1 : 0;
  BatchFlag* fl = G.flag;
  double* P0 = G.part;
  double* P1 = G.part + size_t(G.part_blocks) * M;
  const int nb = bk::red_blocks(n, M);
  float* r32 = nullptr;
  if (o.precision == MG_F32) {
    r32 = G.v32[top].b;
    float* z = cycle_b<float>(o, G, top, r32, nullptr, o.cycle, s);
    if (natural) {
      bk::colsum32(M, n, z, G.col, P0, nb, fl, s);
      bk::finalize(bk::FIN_MEAN, M, nb, P0, nullptr, G.col, fl, 0, s);
    }
    bk::zdot<float>(M, n, G.col, z, G.Q, P0, nb, natural, fl, s);
    bk::finalize(bk::FIN_BETA_FCG, M, nb, P0, nullptr, G.col, fl, 0, s);
    bk::pupd<float>(M, n, G.col, z, G.P, G.X, natural, fl, s);
  } else {
    double* z = cycle_b<double>(o, G, top, G.R, nullptr, o.cycle, s);
    if (natural) {
      bk::colsum(M, n, z, P0, nb, fl, s);
      bk::finalize(bk::FIN_MEAN, M, nb, P0, nullptr, G.col, fl, 0, s);
    }
    bk::zdot<double>(M, n, G.col, z, G.Q, P0, nb, natural, fl, s);
    bk::finalize(bk::FIN_BETA_FCG, M, nb, P0, nullptr, G.col, fl, 0, s);
    bk::pupd<double>(M, n, G.col, z, G.P, G.X, natural, fl, s);
  }
  bk::spmv_dot2(M, F, G.P, G.Q, G.R, P0, P1, nb, fl, s);
  bk::finalize(bk::FIN_ALPHA_FCG, M, nb, P0, P1, G.col, fl, 0, s);
  bk::update_r(M, n, G.col, G.Q, G.R, r32, P0, nb, fl, s);
  bk::finalize(bk::FIN_CHECK, M, nb, P0, nullptr, G.col, fl, 0, s);
}

// b (natural, caller's) -> B (blocked); norms, projection, x = p = q = 0, r = b.
void enqueue_setup(const mg_opts& o, BatchGroup& G, hipStream_t s) {
  Hierarchy& H = *G.H;
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  const int M = G.M;
  const int top = int(H.lv.size()) - 1;
  bk::init_cols(G.col, G.flag, M, G.ncols, o.rtol, o.max_iter, double(n), s);
  bk::gather_in(M, G.ncols, F.perm, n, G.bptr, G.B, s);
  const int nb = bk::red_blocks(n, M);
  if (H.bc == MG_BC_NATURAL) {
    bk::colsum(M, n, G.B, G.part, nb, nullptr, s);
    bk::finalize(bk::FIN_MEAN, M, nb, G.part, nullptr, G.col, G.flag, 1, s);
    bk::sub_mean(M, n, G.col, G.B, s);
    bk::dot(M, n, G.B, G.B, G.part, nb, nullptr, s);
    bk::finalize(bk::FIN_BNORM, M, nb, G.part, nullptr, G.col, G.flag, 0, s);
  } else {
    const int nbv = std::min(2048, (F.nv + 255) / 256);
    bk::nat_sumsq(M, G.ncols, F.nv, G.bptr, G.part, nbv, s);
    bk::finalize(bk::FIN_BNORM, M, nbv, G.part, nullptr, G.col, G.flag, 0, s);
  }
  bk::start(M, n, G.col, G.B, G.X, G.R, G.P, G.Q,
            o.precision == MG_F32 ? G.v32[top].b : nullptr, s);
}

void enqueue_finish(BatchGroup& G, hipStream_t s) {
  Hierarchy& H = *G.H;
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  const int M = G.M;
  const int nb = bk::red_blocks(n, M);
  bk::apply_pending(M, n, G.col, G.P, G.X, s);   // each column's last solution step
  if (H.bc == MG_BC_NATURAL) {
    bk::colsum(M, n, G.X, G.part, nb, nullptr, s);
    bk::finalize(bk::FIN_MEAN, M, nb, G.part, nullptr, G.col, G.flag, 1, s);
    bk::sub_mean(M, n, G.col, G.X, s);
  }
  bk::residual_norm(M, F, G.X, G.B, G.part, nb, s);
  bk::finalize(bk::FIN_RNORM, M, nb, G.part, nullptr, G.col, G.flag, 1, s);
  bk::scatter_out(M, G.ncols, F.perm, n, F.bnd_ids, int32_t(F.bnd_h.size()), G.X, G.bptr, G.xptr,
                  s);
}

hipGraphExec_t capture(const mg_opts& o, BatchGroup& G, hipStream_t cs, int m = 1) {
  hipGraph_t g = nullptr;
  check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  for (int i = 0; i < m; ++i) enqueue_iter(o, G, cs);
  check_hip(hipStreamEndCapture(cs, &g), "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  check_hip(e, "hipGraphInstantiate");
  return ex;
}

}  // namespace

void batch_release_groups(Batch& B) {
  for (BatchGroup& G : B.groups) {
    for (hipGraphExec_t& ge : G.graph)
      if (ge) {
        (void)hipGraphExecDestroy(ge);
        ge = nullptr;
      }
    for (auto& v : G.v32)
      for (void* p : {(void*)v.x, (void*)v.t, (void*)v.r, (void*)v.b}) dfree(p);
    for (auto& v : G.v64)
      for (void* p : {(void*)v.x, (void*)v.t, (void*)v.r, (void*)v.b}) dfree(p);
    for (void* p : {(void*)G.X, (void*)G.R, (void*)G.P, (void*)G.Q, (void*)G.B, (void*)G.Z,
                    (void*)G.part, (void*)G.col, (void*)G.flag, (void*)G.bptr, (void*)G.xptr})
      dfree(p);
  }
  B.groups.clear();
  for (hipStream_t s : B.streams) (void)hipStreamDestroy(s);
  B.streams.clear();
  for (hipEvent_t e : B.ev_done) (void)hipEventDestroy(e);
  B.ev_done.clear();
  if (B.col_host) (void)hipHostFree(B.col_host);
  if (B.ptr_host) (void)hipHostFree(B.ptr_host);
  B.col_host = nullptr;
  B.ptr_host = nullptr;
}

Batch::~Batch() {
  batch_release_groups(*this);
  if (capture_stream) (void)hipStreamDestroy(capture_stream);
  if (ev_start) (void)hipEventDestroy(ev_start);
}

void batch_setup(Batch& B) {
  batch_release_groups(B);
  if (!B.capture_stream)
    check_hip(hipStreamCreateWithFlags(&B.capture_stream, hipStreamNonBlocking), "hipStreamCreate");
  if (!B.ev_start) check_hip(hipEventCreateWithFlags(&B.ev_start, hipEventDisableTiming), "hipEventCreate");
  // instances per hierarchy, in order of first appearance
  std::vector<Hierarchy*> order;
  std::map<Hierarchy*, std::vector<int>> by_h;
  for (int i = 0; i < int(B.inst_h.size()); ++i) {
    Hierarchy* h = B.inst_h[i];
    if (!by_h.count(h)) order.push_back(h);
    by_h[h].push_back(i);
  }
  const BatchTuning& t = B.tune;
  for (Hierarchy* h : order) {
    const std::vector<int>& ids = by_h[h];
    size_t pos = 0;
    while (pos < ids.size()) {
      const int rem = int(ids.size() - pos);
      BatchGroup G;
      G.H = h;
      G.M = t.pad_groups ? std::min(t.max_cols, pow2_ceil(rem)) : std::min(t.max_cols, pow2_floor(rem));
      G.ncols = std::min(G.M, rem);
      G.inst.assign(ids.begin() + pos, ids.begin() + pos + G.ncols);
      pos += G.ncols;
      B.groups.push_back(std::move(G));
    }
  }
  const int nstreams = std::max(1, std::min<int>(t.streams, int(B.groups.size())));
  for (int k = 0; k < nstreams; ++k) {
    hipStream_t s = nullptr;
    check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
    B.streams.push_back(s);
    hipEvent_t e = nullptr;
    check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate");
    B.ev_done.push_back(e);
  }
  // largest groups first over the streams, so the streams carry similar work
  std::vector<size_t> idx(B.groups.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
    return int64_t(B.groups[a].H->lv.back()->n) * B.groups[a].M >
           int64_t(B.groups[b].H->lv.back()->n) * B.groups[b].M;
  });
  std::vector<int64_t> load(nstreams, 0);
  for (size_t i : idx) {
    BatchGroup& G = B.groups[i];
    const int k = int(std::min_element(load.begin(), load.end()) - load.begin());
    G.stream_slot = k;
    load[k] += int64_t(G.H->lv.back()->n) * G.M;
  }
  const bool f32 = B.opts.precision == MG_F32;
  for (BatchGroup& G : B.groups) {
    Hierarchy& H = *G.H;
    const int M = G.M;
    const int nl = int(H.lv.size());
    if (f32)
      G.v32.resize(nl);
    else
      G.v64.resize(nl);
    for (int l = 0; l < nl; ++l) {
      const size_t sz = size_t(H.lv[l]->n + 1) * M;
      if (f32) {
        auto& v = G.v32[l];
        v.x = dalloc<float>(sz);
        v.t = dalloc<float>(sz);
        v.r = dalloc<float>(sz);
        v.b = dalloc<float>(sz);
      } else {
        auto& v = G.v64[l];
        v.x = dalloc<double>(sz);
        v.t = dalloc<double>(sz);
        v.r = dalloc<double>(sz);
        v.b = dalloc<double>(sz);
      }
    }
    const Level& F = *H.lv.back();
    const size_t sz = size_t(F.n + 1) * M;
    G.X = dalloc<double>(sz);
    G.R = dalloc<double>(sz);
    G.P = dalloc<double>(sz);
    G.Q = dalloc<double>(sz);
    G.B = dalloc<double>(sz);
    G.part_blocks = std::max(bk::red_blocks(F.n, M), std::min(2048, (F.nv + 255) / 256));
    G.part = dalloc<double>(size_t(2) * G.part_blocks * M);
    G.col = dalloc<BatchCol>(M);
    G.flag = dalloc<BatchFlag>(1);
    G.bptr = const_cast<const double**>(dalloc<double*>(M));
    G.xptr = dalloc<double*>(M);
  }
  check_hip(hipHostMalloc(reinterpret_cast<void**>(&B.col_host),
                          std::max<size_t>(B.groups.size(), 1) * kBatchMaxCols * sizeof(BatchCol), 0),
            "hipHostMalloc");
  check_hip(hipHostMalloc(reinterpret_cast<void**>(&B.ptr_host),
                          std::max<size_t>(B.groups.size(), 1) * 2 * kBatchMaxCols * sizeof(void*), 0),
            "hipHostMalloc");
  if (B.opts.use_graph)
    for (BatchGroup& G : B.groups) {
      G.graph[0] = capture(B.opts, G, B.capture_stream);
      G.graph_epoch = G.H->weight_epoch;
    }
}

int batch_solve(Batch& B, const double* const* b, double* const* x, mg_result* res, hipStream_t s) {
  const mg_opts& o = B.opts;
  const size_t ng = B.groups.size();
  // a hierarchy whose coefficient changed the form of its weights since a group's graph was
  // captured: capture that group's iteration again
  for (BatchGroup& G : B.groups)
    if (G.graph[0] && G.graph_epoch != G.H->weight_epoch) {
      check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      for (hipGraphExec_t& ge : G.graph)
        if (ge) {
          (void)hipGraphExecDestroy(ge);
          ge = nullptr;
        }
      G.graph[0] = capture(o, G, B.capture_stream);
      G.graph_epoch = G.H->weight_epoch;
    }
  check_hip(hipEventRecord(B.ev_start, s), "hipEventRecord");
  for (hipStream_t st : B.streams) check_hip(hipStreamWaitEvent(st, B.ev_start, 0), "hipStreamWaitEvent");
  for (size_t g = 0; g < ng; ++g) {
    BatchGroup& G = B.groups[g];
    hipStream_t st = B.streams[G.stream_slot];
    void** tab = B.ptr_host + g * 2 * kBatchMaxCols;
    for (int c = 0; c < G.M; ++c) {
      const bool live = c < G.ncols;
      tab[c] = live ? const_cast<double*>(b[G.inst[c]]) : nullptr;
      tab[kBatchMaxCols + c] = live ? x[G.inst[c]] : nullptr;
    }
    check_hip(hipMemcpyAsync(G.bptr, tab, G.M * sizeof(void*), hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
    check_hip(hipMemcpyAsync(G.xptr, tab + kBatchMaxCols, G.M * sizeof(void*),
                             hipMemcpyHostToDevice, st),
              "hipMemcpyAsync");
    enqueue_setup(o, G, st);
  }
  // rounds of speculative iterations; a finished group's launches are no-ops
  std::vector<char> active(ng, 1);
  size_t left = ng;
  bool first = true;
  int total = 0;
  while (left > 0) {
    for (size_t g = 0; g < ng; ++g) {
      if (!active[g]) continue;
      BatchGroup& G = B.groups[g];
      hipStream_t st = B.streams[G.stream_slot];
      const int reps = first && G.last_iters > 0 ? G.last_iters : std::max(1, o.check_every);
      if (G.graph[0]) {
        // reps iterations as graphs of 8, 4, 2 and 1 iterations: one launch gap per graph
        for (int left = reps; left > 0;) {
          const int lg = left >= 8 ? 3 : left >= 4 ? 2 : left >= 2 ? 1 : 0;
          if (!G.graph[lg]) G.graph[lg] = capture(o, G, B.capture_stream, 1 << lg);
          check_hip(hipGraphLaunch(G.graph[lg], st), "hipGraphLaunch");
          left -= 1 << lg;
        }
      } else {
        for (int k = 0; k < reps; ++k) enqueue_iter(o, G, st);
      }
      check_hip(hipMemcpyAsync(B.col_host + g * kBatchMaxCols, G.col, G.M * sizeof(BatchCol),
                               hipMemcpyDeviceToHost, st),
                "hipMemcpyAsync");
    }
    for (hipStream_t st : B.streams) check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
    check_hip(hipGetLastError(), "kernel launch");
    first = false;
    for (size_t g = 0; g < ng; ++g) {
      if (!active[g]) continue;
      const BatchCol* cc = B.col_host + g * kBatchMaxCols;
      bool all = true;
      for (int c = 0; c < B.groups[g].M; ++c) all = all && cc[c].done;
      if (all) {
        active[g] = 0;
        --left;
      }
    }
    if (++total > o.max_iter + 2)
      throw std::runtime_error("batched solve did not settle within max_iter rounds");
  }
  for (size_t g = 0; g < ng; ++g) {
    BatchGroup& G = B.groups[g];
    hipStream_t st = B.streams[G.stream_slot];
    enqueue_finish(G, st);
    check_hip(hipMemcpyAsync(B.col_host + g * kBatchMaxCols, G.col, G.M * sizeof(BatchCol),
                             hipMemcpyDeviceToHost, st),
              "hipMemcpyAsync");
  }
  for (size_t k = 0; k < B.streams.size(); ++k) {
    check_hip(hipEventRecord(B.ev_done[k], B.streams[k]), "hipEventRecord");
    check_hip(hipStreamWaitEvent(s, B.ev_done[k], 0), "hipStreamWaitEvent");
  }
  for (hipStream_t st : B.streams) check_hip(hipStreamSynchronize(st), "hipStreamSynchronize");
  check_hip(hipGetLastError(), "kernel launch");
  int status = MG_OK;
  for (size_t g = 0; g < ng; ++g) {
    BatchGroup& G = B.groups[g];
    const BatchCol* cc = B.col_host + g * kBatchMaxCols;
    int it = 0;
    for (int c = 0; c < G.ncols; ++c) {
      it = std::max(it, int(cc[c].iters));
      if (status == MG_OK && cc[c].status != MG_OK) status = cc[c].status;
      if (res) {
        mg_result& r = res[G.inst[c]];
        r.iterations = cc[c].iters;
        r.status = cc[c].status;
        r.rel_residual = cc[c].bnorm > 0 ? cc[c].true_rnorm / cc[c].bnorm : 0.0;
        r.rel_residual_loop = cc[c].bnorm > 0 ? cc[c].rnorm / cc[c].bnorm : 0.0;
        r.history_len = 0;
        r.fp64_fallback = 0;
      }
    }
    G.last_iters = it;
  }
  return status;
}

std::string batch_signature(const Batch& B) {
  std::map<std::tuple<int, int, int>, int> count;
  for (Hierarchy* h : B.inst_h) count[std::make_tuple(h->lv.back()->nv, h->lv.back()->n, h->bc)]++;
  std::ostringstream os;
  os << "decmg-batch-v1 prec=" << B.opts.precision << " nu=" << B.opts.nu1 << "," << B.opts.nu2
     << " |";
  for (auto& kv : count)
    os << " " << std::get<0>(kv.first) << ":" << std::get<1>(kv.first) << ":"
       << std::get<2>(kv.first) << "x" << kv.second;
  return os.str();
}

bool batch_cache_lookup(const char* path, const std::string& sig, BatchTuning& t) {
  if (!path) return false;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos || line.substr(0, tab) != sig) continue;
    std::istringstream is(line.substr(tab + 1));
    BatchTuning r;
    if (is >> r.max_cols >> r.pad_groups >> r.streams) {
      t = r;
      return true;
    }
  }
  return false;
}

void batch_cache_store(const char* path, const std::string& sig, const BatchTuning& t) {
  if (!path) return;
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line))
      if (line.substr(0, line.find('\t')) != sig && !line.empty()) keep.push_back(line);
  }
  std::ofstream out(path, std::ios::trunc);
  for (const std::string& l : keep) out << l << "\n";
  out << sig << "\t" << t.max_cols << " " << t.pad_groups << " " << t.streams << "\n";
  if (!out) throw std::runtime_error(std::string("cannot write the tuning cache ") + path);
}

double batch_autotune(Batch& B, const double* const* b, double* const* x, int reps,
                      const char* cache_path) {
  std::vector<BatchTuning> cand;
  for (int mc : {8, 16, 32, 64})
    for (int pad : {1, 0})
      for (int st : {1, 2, 4}) cand.push_back(BatchTuning{mc, pad, st});
  double best = 1e300;
  BatchTuning best_t = B.tune;
  hipStream_t s = nullptr;
  check_hip(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  try {
    for (const BatchTuning& t : cand) {
      B.tune = t;
      batch_setup(B);
      (void)batch_solve(B, b, x, nullptr, s);   // warm-up; also learns the iteration counts
      double tmin = 1e300;
      for (int r = 0; r < std::max(1, reps); ++r) {
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        const auto t0 = std::chrono::steady_clock::now();
        (void)batch_solve(B, b, x, nullptr, s);
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        tmin = std::min(tmin, ms);
      }
      if (tmin < best) {
        best = tmin;
        best_t = t;
      }
    }
  } catch (...) {
    (void)hipStreamDestroy(s);
    throw;
  }
  (void)hipStreamDestroy(s);
  B.tune = best_t;
  batch_setup(B);
  batch_cache_store(cache_path, B.signature, best_t);
  return best;
}

}  // namespace decmg
