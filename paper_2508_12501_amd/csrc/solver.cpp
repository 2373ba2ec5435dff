// Host orchestration of the V-cycle and the outer Krylov loops.
//
// The outer loop keeps all its scalars (alpha, beta, norms, the convergence flag) in device
// memory, so one iteration is a fixed sequence of launches with fixed arguments.  It is
// captured once as a hipGraph per (hierarchy, method, cycle shape) and replayed; the host
// enqueues `check_every` replays, then reads the flag.  Replays after convergence cost one
// flag read per kernel.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <stdexcept>

#include "hier.hpp"
#include "solver.hpp"
#include "util.hpp"

namespace decmg {

template <>
LevelVecs<double>& vecs<double>(Level& L) { return L.v64; }
template <>
LevelVecs<float>& vecs<float>(Level& L) { return L.v32; }

template <typename T>
static constexpr int dtype_of() { return sizeof(T) == 8 ? MG_F64 : MG_F32; }

// A weighted-Jacobi sweep, bracketed by probe events when the probe watches this level.
template <typename T>
static void sweep(Hierarchy& H, int l, const T* x, const T* b, T* xo, double omega, const int* done,
                  hipStream_t s) {
  Hierarchy::Probe& P = H.probe;
  const bool timed = P.on && !H.capturing && P.level == l && P.dtype == dtype_of<T>();
  if (!timed) {
    k::jacobi<T>(*H.lv[l], x, b, xo, omega, done, s);
    return;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  check_hip(hipEventCreate(&e0), "hipEventCreate");
  check_hip(hipEventCreate(&e1), "hipEventCreate");
  k::jacobi_timed<T>(*H.lv[l], x, b, xo, omega, done, s, e0, e1);
  P.ev.emplace_back(e0, e1);
  P.stream = s;
}

template <typename T>
static T* mgcycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, int kind,
                  const int* done, hipStream_t s, bool chk = false);

// The coarse-grid correction of level l for a cycle of shape `kind`: level l-1 solved by one
// cycle of the same shape from zero (V), two (W), or an F-cycle then a V-cycle (F).
template <typename T>
static T* coarse_correction(Hierarchy& H, int l, const T* bc, const mg_opts& o, int kind,
                            const int* done, hipStream_t s) {
  T* ec;
  if (kind == MG_CYCLE_W) {
    ec = mgcycle<T>(H, l - 1, bc, nullptr, o, MG_CYCLE_W, done, s);
    ec = mgcycle<T>(H, l - 1, bc, ec, o, MG_CYCLE_W, done, s);
  } else if (kind == MG_CYCLE_F) {
    ec = mgcycle<T>(H, l - 1, bc, nullptr, o, MG_CYCLE_F, done, s);
    ec = mgcycle<T>(H, l - 1, bc, ec, o, MG_CYCLE_V, done, s);
  } else {
    ec = mgcycle<T>(H, l - 1, bc, nullptr, o, MG_CYCLE_V, done, s);
  }
  return ec;
}

// b_c = M(f) (b - A x) as two passes (residual into V.r, then the restriction).  A fused
// coarse-row-centric pass was measured slower even on launch-bound levels: each coarse row
// walks up to seven fine rows, and the dependent index, operator and gather loads of each
// take a fabric round trip in turn (about 17 us against 2 x 4.6 us).
template <typename T>
static void restrict_residual(Level& L, Level& C, LevelVecs<T>& V, const T* x, const T* b,
                              const int* done, hipStream_t s) {
  k::residual<T>(L, x, b, V.r, done, s);
  k::restrict_<T>(L, C, V.r, vecs<T>(C).b, done, s);
}

// `steps` steps of the CG smoother on level l, in place on x (r, p, q in the level's r, t, u).
template <typename T>
static void cg_smooth(Hierarchy& H, int l, T* x, const T* b, int steps, const int* done,
                      hipStream_t s) {
  if (steps <= 0) return;
  Level& L = *H.lv[l];
  LevelVecs<T>& V = vecs<T>(L);
  k::residual<T>(L, x, b, V.r, done, s);
  k::cgs_start<T>(L, V.r, V.t, H.part, done, s);
  k::cgs_fin(L, k::CGS_INIT, H.part, done, s);
  for (int it = 0; it < steps; ++it) {
    k::cgs_spmv_dot<T>(L, V.t, V.u, H.part, done, s);
    k::cgs_fin(L, k::CGS_ALPHA, H.part, done, s);
    k::cgs_update<T>(L, V.t, V.u, x, V.r, H.part, done, s);
    k::cgs_fin(L, k::CGS_BETA, H.part, done, s);
    k::cgs_pupd<T>(L, V.r, V.t, done, s);
  }
}

// A cycle with CG smoothing: in place on the level's x (or on x_init).
template <typename T>
static T* cg_cycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, int kind,
                   const int* done, hipStream_t s) {
  Level& L = *H.lv[l];
  LevelVecs<T>& V = vecs<T>(L);
  if (l == 0) {
    k::coarse<T>(H, b, V.x, done, s);
    return V.x;
  }
  T* cur = x_init ? x_init : V.x;
  if (!x_init) k::fill<T>(cur, L.n, T(0), s);
  cg_smooth<T>(H, l, cur, b, o.nu1, done, s);
  Level& C = *H.lv[l - 1];
  restrict_residual<T>(L, C, V, cur, b, done, s);
  T* ec = coarse_correction<T>(H, l, vecs<T>(C).b, o, kind, done, s);
  k::prolong<T>(L, C, ec, cur, done, s);
  cg_smooth<T>(H, l, cur, b, o.nu2, done, s);
  return cur;
}

// One cycle of shape `kind` on level l (MG_CYCLE_V/W/F): the coarse-grid correction is one
// cycle of the same shape from zero (V), two (W, the second from the first's result), or an
// F-cycle followed by a V-cycle (F).  Returns the buffer holding the result.  chk: the
// opening two sweeps from zero also take the Krylov loop's pending convergence check (only
// where check_fused_ok says the cycle opens with them).
template <typename T>
static T* mgcycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, int kind,
                  const int* done, hipStream_t s, bool chk) {
  Level& L = *H.lv[l];
  LevelVecs<T>& V = vecs<T>(L);
  if (chk && (l == 0 || x_init || o.smoother != MG_SMOOTH_JACOBI ||
              ((o.fuse_levels && L.tiles.ntiles > 0) ? o.nu1 > 2
                                                     : (o.nu1 < 2 || !k::jacobi_two_chk_ok(L))) ||
              (kind == MG_CYCLE_V && l <= coarse_top<T>(H)) ||
              k::coarse_cycle_general_ok<T>(H, l, false)))
    throw std::logic_error("mgcycle: this cycle does not open with a kernel that takes the check");
  if (l == 0) {
    k::coarse<T>(H, b, V.x, done, s);
    return V.x;
  }
  if (o.smoother == MG_SMOOTH_CG) return cg_cycle<T>(H, l, b, x_init, o, kind, done, s);
  const bool gs = o.smoother == MG_SMOOTH_GS;
  if (!x_init && kind == MG_CYCLE_V && !gs && l <= coarse_top<T>(H)) {
    k::coarse_cycle<T>(H, l, b, V.x, o.omega, o.nu1, o.nu2, done, s);
    return V.x;
  }
  if (k::coarse_cycle_general_ok<T>(H, l, gs)) {
    // the whole bottom of a W- or F-cycle, a Gauss-Seidel cycle or a cycle from a given
    // iterate in one launch (in place on x_init)
    T* xo = x_init ? x_init : V.x;
    k::coarse_cycle_general<T>(H, l, b, xo, x_init != nullptr, o.omega, o.nu1, o.nu2, kind, gs,
                               done, s);
    return xo;
  }
  T *cur, *oth;
  int pre = o.nu1;
  if (gs) {
    // multicolour Gauss-Seidel works in place: forward colour order before the coarse-grid
    // correction, backward after it
    cur = x_init ? x_init : V.x;
    if (!x_init) k::fill<T>(cur, L.n, T(0), s);
    const int nc = int(L.gs.size());
    for (int it = 0; it < o.nu1; ++it)
      for (int c = 0; c < nc; ++c) k::gs_color<T>(L, c, cur, b, done, s);
    Level& C = *H.lv[l - 1];
    restrict_residual<T>(L, C, V, cur, b, done, s);
    const T* bc = vecs<T>(C).b;
    T* ec = coarse_correction<T>(H, l, bc, o, kind, done, s);
    k::prolong<T>(L, C, ec, cur, done, s);
    for (int it = 0; it < o.nu2; ++it)
      for (int c = nc - 1; c >= 0; --c) k::gs_color<T>(L, c, cur, b, done, s);
    return cur;
  }
  Level& C = *H.lv[l - 1];
  // launch-bound binary levels with tiles: the down leg from zero (pre-smoothing, residual,
  // restriction) and the up leg (interpolation, post-smoothing) are one launch each
  const bool tiled = o.fuse_levels && L.tiles.ntiles > 0;
  bool restricted = false;
  if (!x_init && tiled && pre <= 2) {
    cur = V.x;
    oth = V.t;
    if (chk)
      k::tile_down<T>(L, b, cur, vecs<T>(C).b, o.omega, pre, done, s, H.scal, H.part,
                      k::red_blocks(L.n));
    else
      k::tile_down<T>(L, b, cur, vecs<T>(C).b, o.omega, pre, done, s);
    pre = 0;
    restricted = true;
  } else if (!x_init) {
    cur = V.x;
    oth = V.t;
    if (pre >= 2) {
      if (chk)
        k::jacobi_two_chk<T>(L, b, cur, o.omega, done, H.scal, H.part, k::red_blocks(L.n), s);
      else
        k::jacobi_two<T>(L, b, cur, o.omega, done, s);
      pre -= 2;
    } else if (pre == 1) {
      k::jacobi_zero<T>(L, b, cur, o.omega, done, s);
      pre = 0;
    } else {
      k::fill<T>(cur, L.n, T(0), s);
    }
  } else {
    cur = x_init;
    oth = (x_init == V.t) ? V.x : V.t;
  }
  for (; pre > 0; --pre) {
    sweep<T>(H, l, cur, b, oth, o.omega, done, s);
    std::swap(cur, oth);
  }
  if (!restricted) restrict_residual<T>(L, C, V, cur, b, done, s);
  const T* bc = vecs<T>(C).b;
  T* ec = coarse_correction<T>(H, l, bc, o, kind, done, s);
  int post = o.nu2;
  if (tiled && (post == 1 || post == 2)) {
    // the tiles read x around their rows, so the result goes to the partner buffer
    k::tile_up<T>(L, ec, cur, b, oth, o.omega, post, done, s);
    std::swap(cur, oth);
    post = 0;
  } else if (post >= 1 && L.n <= kLaunchBoundRows && !L.tr.weighted) {
    // the first post-smoothing sweep reads x + P e_c directly (one launch fewer on levels
    // whose kernels are launch-bound; on large levels the extra dependent gathers cost more
    // than the separate interpolation pass)
    k::prolong_sweep<T>(L, C, ec, cur, b, oth, o.omega, done, s);
    std::swap(cur, oth);
    --post;
  } else {
    k::prolong<T>(L, C, ec, cur, done, s);
  }
  for (; post > 0; --post) {
    sweep<T>(H, l, cur, b, oth, o.omega, done, s);
    std::swap(cur, oth);
  }
  return cur;
}

template <typename T>
T* vcycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, const int* done,
          hipStream_t s, bool chk) {
  return mgcycle<T>(H, l, b, x_init, o, o.cycle, done, s, chk);
}

template double* vcycle<double>(Hierarchy&, int, const double*, double*, const mg_opts&,
                                const int*, hipStream_t, bool);
template float* vcycle<float>(Hierarchy&, int, const float*, float*, const mg_opts&, const int*,
                              hipStream_t, bool);

// Whether a CG/FCG iteration's cycle opens on the finest level with a kernel that takes the
// previous iteration's convergence check in one more workgroup: the fused levels switched on,
// Jacobi smoothing, a finest level with a coarse level below it outside the one-launch
// bottom, and either the tiled down leg (nu1 <= 2) or the two sweeps from zero of a
// row-pattern level (nu1 >= 2).
bool check_fused_ok(const Hierarchy& H, const mg_opts& o) {
  const int top = int(H.lv.size()) - 1;
  if (o.outer == MG_OUTER_IR || !o.fuse_levels) return false;
  if (top < 1 || o.smoother != MG_SMOOTH_JACOBI) return false;
  const Level& L = *H.lv[top];
  if (L.tiles.ntiles > 0 ? o.nu1 > 2 : (o.nu1 < 2 || !k::jacobi_two_chk_ok(L))) return false;
  if (o.precision == MG_F32)
    return !((o.cycle == MG_CYCLE_V && top <= coarse_top<float>(H)) ||
             k::coarse_cycle_general_ok<float>(H, top, false));
  return !((o.cycle == MG_CYCLE_V && top <= coarse_top<double>(H)) ||
           k::coarse_cycle_general_ok<double>(H, top, false));
}

namespace {

// Finalise the partial sums of a streaming reduction over n entries (or, with `tiles`, of a
// one-tile-per-workgroup kernel).  `force` runs it even after convergence (exit bookkeeping).
void fin(Hierarchy& H, int op, int32_t n, bool two, hipStream_t s, bool tiles = false,
         bool force = false) {
  const int nb = tiles ? k::blocks_for(n) : k::red_blocks(n);
  k::finalize(op, nb, H.part, two ? H.part + H.part_cap : nullptr, H.scal, 0.0, force ? 1 : 0, s);
}

// One outer iteration of mg_pcg, enqueued on s (eagerly or under capture).  `parity` selects
// which direction buffer holds p on entry; the iteration leaves the new p in the other one.
// first: the iteration right after a start from p = q = 0 (x = 0, no step pending) of a CG or
// FCG loop on a Dirichlet system: the direction update takes p = z without reading p_old or x
// (so the start need not clear p and q), and FCG, whose beta = -(z.q)/pq is -0 there (set by
// the start), also leaves out that dot and its finalisation.
void enqueue_iteration(Hierarchy& H, const mg_opts& o, int parity, hipStream_t s,
                       bool first = false) {
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  const int top = int(H.lv.size()) - 1;
  const bool natural = H.bc == MG_BC_NATURAL;
  const int* done = &H.scal->done;
  double* P0 = H.part;
  double* P1 = H.part + H.part_cap;
  const double* other = (o.outer == MG_OUTER_FCG) ? H.sq : H.sr;
  // the previous iteration's convergence check rides with the cycle's first kernel
  const bool chk = check_fused_ok(H, o);
  double* z;
  float* z32 = nullptr;
  double* P2 = H.part + 2 * H.part_cap;
  // On singular (natural-boundary) systems the preconditioned vector is projected to zero
  // mean.  CG and FCG take the mean and the projected dot from one pass over z (sum z, z.o,
  // sum o) and subtract the mean inside the p update; IR projects z before using it.
  const bool fused_mean = natural && o.outer != MG_OUTER_IR;
  const bool first_pupd = first && o.outer != MG_OUTER_IR && !natural;
  const bool skip_beta = first_pupd && o.outer == MG_OUTER_FCG;
  if (o.precision == MG_F32) {
    z32 = vcycle<float>(H, top, F.v32.b, nullptr, o, done, s, chk);
    if (H.debug_flags & MG_DEBUG_ZERO_PRECOND32) k::fill<float>(z32, n, 0.0f, s);
    if (fused_mean) {
      k::zsum_dot32(n, H.scal, z32, other, P0, P1, P2, done, s);
    } else {
      if (natural) {
        k::sum32(n, z32, H.scal, P0, done, s);
        fin(H, k::FIN_MEAN, n, false, s);
      }
      if (o.outer == MG_OUTER_IR) {
        k::zconv_dot(n, H.scal, z32, H.sz, other, P0, natural ? 1 : 0, done, s);
      } else if (!skip_beta) {
        // z stays in FP32: the dot and the p update widen it on the fly
        k::zdot32(n, H.scal, z32, other, P0, 0, done, s);
      }
    }
    z = H.sz;
  } else {
    z = vcycle<double>(H, top, H.sr, nullptr, o, done, s, chk);
    if (fused_mean) {
      k::zsum_dot64(n, H.scal, z, other, P0, P1, P2, done, s);
    } else {
      if (natural) {
        k::sum64(n, z, P0, done, s);
        fin(H, k::FIN_MEAN, n, false, s);
      }
      if (!skip_beta) k::zsub_dot(n, H.scal, z, other, P0, natural ? 1 : 0, done, s);
    }
  }
  float* r32 = (o.precision == MG_F32) ? F.v32.b : nullptr;
  if (o.outer == MG_OUTER_IR) {
    k::axpy1(n, z, H.sx, done, s);
    k::residual_norm(F, H.sx, H.sb, H.sr, r32, H.scal, P0, done, s);
    fin(H, k::FIN_CHECK, n, false, s, true);
    return;
  }
  if (fused_mean)
    k::finalize(o.outer == MG_OUTER_CG ? k::FIN_MEAN_BETA_CG : k::FIN_MEAN_BETA_FCG,
                k::red_blocks(n), P0, P1, H.scal, 0.0, 0, s, P2);
  else if (!skip_beta)
    fin(H, o.outer == MG_OUTER_CG ? k::FIN_BETA_CG : k::FIN_BETA_FCG, n, false, s);
  // p = z + beta p formed inside the operator product (z32 carries the mean subtraction on
  // singular systems; an FP64 z has it subtracted already unless the sums were fused)
  const double* p_old = parity ? H.sp2 : H.sp;
  double* p_new = parity ? H.sp : H.sp2;
  // the previous iteration's step x += alpha p_old is taken inside the direction update; this
  // iteration's is left pending (alpha, and the buffer of p_new) for the next one or the exit
  k::pupd_spmv_dot2(F, H.scal, z32, z32 ? nullptr : z, z32 ? (natural ? 1 : 0) : (fused_mean ? 1 : 0),
                    p_old, p_new, H.sq, H.sr, H.sx, P0, P1, done, s, first_pupd);
  k::finalize(o.outer == MG_OUTER_CG ? k::FIN_ALPHA_CG : k::FIN_ALPHA_FCG,
              k::pupd_spmv_partials(F), P0, P1, H.scal, p_new == H.sp2 ? 1.0 : 0.0, 0, s);
  k::update_r(n, H.scal, H.sq, H.sr, r32, P0, done, s);
  // with chk the check waits for the next iteration's first kernel, or for the end of the
  // batch (run_pcg's tail)
  if (!chk) fin(H, k::FIN_CHECK, n, false, s);
}

// One stand-alone V-cycle iteration (mg_solve): x <- V(b, x); r = b - A x; check.
void enqueue_cycle(Hierarchy& H, const mg_opts& o, hipStream_t s) {
  Level& F = *H.lv.back();
  const int top = int(H.lv.size()) - 1;
  const int* done = &H.scal->done;
  // the cycle ends in H.sx or in the finest level's partner buffer (an odd number of Jacobi
  // ping-pongs, or a fused up leg), which is copied back
  const double* xr = vcycle<double>(H, top, H.sb, H.sx, o, done, s);
  if (xr != H.sx) k::copy<double>(xr, H.sx, F.n, done, s);
  k::residual_norm(F, H.sx, H.sb, H.sr, nullptr, H.scal, H.part, done, s);
  fin(H, k::FIN_CHECK, F.n, false, s, true);
}

std::tuple<int, int, int, int, double> graph_key(const mg_opts& o, int kind) {
  return std::make_tuple(kind * 16 + o.outer * 4 + o.precision, o.nu1, o.nu2,
                         o.cycle + 4 * o.smoother + 16 * (o.fuse_levels ? 1 : 0), o.omega);
}

// kind 0 and 2: a Krylov iteration with p in the first or the second buffer; 1: a cycle;
// 3: the first CG/FCG iteration after a start from p = q = 0 (p in the first buffer).  m > 1
// (Krylov kinds, m <= kMaxGraphIters): m iterations in one graph, the later ones alternating
// the buffers (and not first ones): one launch, and one gap between launches, for m
// iterations.
constexpr int kMaxGraphIters = 16;
hipGraphExec_t iteration_graph(Hierarchy& H, const mg_opts& o, int kind, int m = 1) {
  if (m < 1 || m > kMaxGraphIters || (kind == 1 && m != 1))
    throw std::logic_error("iteration_graph: iterations per graph");
  auto key = graph_key(o, kind + 4 * (m - 1));
  auto it = H.graphs.find(key);
  if (it != H.graphs.end()) return it->second;
  hipGraph_t g = nullptr;
  check_hip(hipStreamBeginCapture(H.capture_stream, hipStreamCaptureModeThreadLocal),
            "hipStreamBeginCapture");
  H.capturing = true;
  if (kind == 1) {
    enqueue_cycle(H, o, H.capture_stream);
  } else {
    int parity = kind == 2 ? 1 : 0;
    for (int i = 0; i < m; ++i, parity ^= 1)
      enqueue_iteration(H, o, parity, H.capture_stream, kind == 3 && i == 0);
  }
  H.capturing = false;
  check_hip(hipStreamEndCapture(H.capture_stream, &g), "hipStreamEndCapture");
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  check_hip(e, "hipGraphInstantiate");
  H.graphs[key] = ex;
  return ex;
}

void init_scalars(Hierarchy& H, const mg_opts& o, hipStream_t s) {
  k::init_scalars(H.scal, o.rtol, o.max_iter, double(H.lv.back()->n), H.hist, H.hist_cap, s);
}

void read_scalars(Hierarchy& H, hipStream_t s) {
  check_hip(hipMemcpyAsync(H.scal_host, H.scal, sizeof(DevScalars), hipMemcpyDeviceToHost, s),
            "hipMemcpyAsync");
  check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  check_hip(hipGetLastError(), "kernel launch");
}

// b (natural, nv) -> H.sb (internal); ||b|| with the boundary part; projected for natural.
// With b_nat == nullptr the internal right-hand side is already in H.sb.  check_compat: a
// natural-boundary b whose sum exceeds rounding (|sum b| > kCompatTol sum |b|) ends the solve
// with MG_EINCOMPAT.
void setup_rhs(Hierarchy& H, const double* b_nat, hipStream_t s, bool check_compat = false,
               bool defer_gather = false, const mg_opts* init = nullptr) {
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  // defer_gather (Dirichlet systems only): the caller gathers b into H.sb itself
  if (b_nat && !(defer_gather && H.bc != MG_BC_NATURAL)) k::gather<double>(F.perm, n, b_nat, H.sb, s);
  if (H.bc == MG_BC_NATURAL) {
    if (check_compat) {
      if (init) init_scalars(H, *init, s);
      k::sum_abs64(n, H.sb, H.part, H.part + H.part_cap, s);
      fin(H, k::FIN_MEAN_COMPAT, n, true, s);
    } else {
      // init: the sum's first thread also writes the starting scalars
      if (init)
        k::sum64_init(n, H.sb, H.part, H.scal, init->rtol, init->max_iter, double(n), H.hist,
                      H.hist_cap, s);
      else
        k::sum64(n, H.sb, H.part, nullptr, s);
      fin(H, k::FIN_MEAN, n, false, s);
    }
    k::sub_mean_dot(n, H.scal, H.sb, H.part, s);
    fin(H, k::FIN_BNORM, n, false, s);
  } else if (b_nat) {
    // init: the dot's first thread also writes the starting scalars (no init_scalars launch)
    if (init)
      k::dot_init(F.nv, b_nat, b_nat, H.part, H.scal, init->rtol, init->max_iter, double(n),
                  H.hist, H.hist_cap, s);
    else
      k::dot(F.nv, b_nat, b_nat, H.part, nullptr, s);
    fin(H, k::FIN_BNORM, F.nv, false, s);
  } else {
    if (init)
      k::dot_init(n, H.sb, H.sb, H.part, H.scal, init->rtol, init->max_iter, double(n), H.hist,
                  H.hist_cap, s);
    else
      k::dot(n, H.sb, H.sb, H.part, nullptr, s);
    fin(H, k::FIN_BNORM, n, false, s);
  }
}

// Pending solution step, final projection, true residual, scatter to the caller's numbering
// (kernels only).  Without the projection (Dirichlet systems) it changes x only by the step
// the next iteration would take in the same expression, so it can be enqueued after every
// batch of iterations and simply runs again after more of them; on singular systems it
// projects x in place, which would change the rounding of later iterations, so it runs once at
// the end.
void enqueue_finish(Hierarchy& H, const double* b_nat, double* x_nat, hipStream_t s) {
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  // the solution step of the last CG/FCG iteration (a no-op when none is pending; FIN_RNORM
  // below clears it, so running the finish again takes it only once), with the scatter to the
  // caller's numbering in the same pass on Dirichlet systems
  const bool scatter_now = x_nat && H.bc != MG_BC_NATURAL;
  if (scatter_now)   // with the loop's pending convergence check (a no-op when none is)
    k::finish_scatter(n, H.scal, H.sp, H.sp2, H.sx, F.perm, x_nat, F.bnd_ids,
                      b_nat ? int32_t(F.bnd_h.size()) : 0, b_nat, H.part, k::red_blocks(n), s);
  else if (H.bc != MG_BC_NATURAL)
    k::apply_pending(n, H.scal, H.sp, H.sp2, H.sx, s);
  if (H.bc == MG_BC_NATURAL) {
    k::apply_pending_sum(n, H.scal, H.sp, H.sp2, H.sx, H.part, s);
    fin(H, k::FIN_MEAN, n, false, s, false, true);
    k::sub_mean(n, H.scal, H.sx, s);
  }
  k::true_residual(F, H.sx, H.sb, H.sz, H.part, s);
  k::finalize(k::FIN_RNORM, k::true_residual_partials(F), H.part, nullptr, H.scal, 0.0, 1, s);
  if (x_nat && !scatter_now) {
    k::scatter<double>(F.perm, n, H.sx, x_nat, s);
    k::bnd_copy<double>(F.bnd_ids, int32_t(F.bnd_h.size()), b_nat, x_nat, s);
  }
}

// The caller's result from the host copy of the scalars (read after the last finish), with
// the residual history copied to the caller's host buffer when one is given.
void collect(Hierarchy& H, mg_result* res, hipStream_t s) {
  const DevScalars& h = *H.scal_host;
  if (res) {
    res->iterations = h.iters;
    res->status = h.status;
    res->rel_residual_loop = h.bnorm > 0 ? h.rnorm / h.bnorm : 0.0;
    res->rel_residual = h.bnorm > 0 ? h.true_rnorm / h.bnorm : 0.0;
    res->history_len = 0;
    res->fp64_fallback = 0;
    if (res->history && res->history_cap > 0) {
      const int m = std::min({h.iters, res->history_cap, H.hist_cap});
      if (m > 0) {
        check_hip(hipMemcpyAsync(res->history, H.hist, size_t(m) * sizeof(double),
                                 hipMemcpyDeviceToHost, s),
                  "hipMemcpyAsync");
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
      }
      res->history_len = m;
    }
  }
}

}  // namespace

// Host-side phase timing of a solve, printed to stderr when DECMG_HOST_TIMING is set.
struct HostTimer {
  bool on = std::getenv("DECMG_HOST_TIMING") != nullptr;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now(), last = t0;
  char buf[512] = {0};
  size_t len = 0;
  void mark(const char* what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    const double us = std::chrono::duration<double, std::micro>(now - last).count();
    last = now;
    len += size_t(std::snprintf(buf + len, sizeof(buf) - len, " %s=%.1f", what, us));
  }
  ~HostTimer() {
    if (!on) return;
    const double us = std::chrono::duration<double, std::micro>(last - t0).count();
    std::fprintf(stderr, "[decmg host] total=%.1fus%s\n", us, buf);
  }
};

// Enqueues iterations in batches and checks the device flag between batches.  The first batch
// is the iteration count of the previous solve with the same settings (or check_every); later
// batches are sized from the observed mean residual reduction per iteration, so a solve
// normally needs one or two host round trips and runs few or no no-op iterations.
// `tail` is enqueued after every batch, before the host reads the flag: the exit work (the
// finish of a solve) then follows the last iteration on the device without a host round trip;
// after a batch that did not converge it is simply done again later.  With stall > 0 the loop
// also ends, returning true, once `stall` checks in a row after the first found the loop
// residual no lower than the smallest one seen at an earlier check.
template <typename F, typename G>
bool iterate(Hierarchy& H, const mg_opts& o, int kind, hipStream_t s, F enqueue, G tail,
             HostTimer* T = nullptr, int launched = 0, int stall = 0) {
  const int every = std::max(1, o.check_every);
  auto key = graph_key(o, kind);
  auto it = H.last_iters.find(key);
  // a restarted loop (launched > 0) continues in batches of check_every
  int batch = (it != H.last_iters.end() && launched == 0) ? std::max(1, it->second) : every;
  double best = std::numeric_limits<double>::infinity();
  int flat = 0;
  bool stalled = false;
  while (launched < o.max_iter) {
    batch = std::min(batch, o.max_iter - launched);
    enqueue(batch);
    launched += batch;
    tail();
    if (T) T->mark("enqueue");
    read_scalars(H, s);
    if (T) T->mark("wait");
    const DevScalars& h = *H.scal_host;
    if (h.done) break;
    if (stall > 0) {
      if (h.rnorm < best) {
        best = h.rnorm;
        flat = 0;
      } else if (++flat >= stall) {
        stalled = true;
        break;
      }
    }
    batch = every;
    if (h.iters > 0 && h.rnorm > 0 && h.bnorm > 0) {
      const double rate = std::pow(h.rnorm / h.bnorm, 1.0 / h.iters);
      const double goal = h.rtol * h.bnorm / h.rnorm;
      if (rate > 0 && rate < 1 && goal < 1)
        batch = std::max(1, std::min(4 * every, int(std::ceil(std::log(goal) / std::log(rate)))));
    }
  }
  if (launched == 0) {
    tail();
    read_scalars(H, s);
  }
  if (!stalled) H.last_iters[key] = H.scal_host->iters;
  return stalled;
}

int run_pcg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
            hipStream_t s, bool warm_start, bool check_compat) {
  HostTimer T;
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  // the first reduction over b also writes the starting scalars; a Dirichlet solve from the
  // caller's b gathers b inside the Krylov start below
  const bool gather_in_init = b_nat && H.bc != MG_BC_NATURAL;
  setup_rhs(H, b_nat, s, check_compat, gather_in_init, &o);
  H.p_parity = 0;
  mg_opts cur = o;   // the FP64 fallback switches the cycle's precision
  float* r32 = (o.precision == MG_F32) ? F.v32.b : nullptr;
  if (warm_start && !b_nat) {
    k::residual<double>(F, H.sx, H.sb, H.sr, nullptr, s);
    k::warm_aux(n, H.scal, H.sr, r32, H.sp, H.sq, s);
  } else if (gather_in_init) {
    // a CG or FCG loop's first iteration reads neither p nor q
    const bool keep_pq = o.outer != MG_OUTER_IR;
    k::init_krylov_gather(n, H.scal, F.perm, b_nat, H.sb, H.sr, H.sx, keep_pq ? nullptr : H.sp,
                          keep_pq ? nullptr : H.sq, r32, s);
  } else {
    k::init_krylov(n, H.scal, H.sb, H.sr, H.sx, H.sp, H.sq, r32, s);
  }
  T.mark("setup");
  // CG and FCG on a Dirichlet system: the first iteration after a start from p = q = 0 forms
  // p = z directly (enqueue_iteration's `first`)
  auto first_ok = [&]() { return cur.outer != MG_OUTER_IR && H.bc != MG_BC_NATURAL; };
  // the iteration graphs are captured when a batch of their size and kind first needs them
  T.mark("graph");
  bool fresh = true;   // p = q = 0 and beta = -0: the next iteration is a first one
  // `count` iterations as graphs of up to kMaxGraphIters iterations each (a batch is usually
  // the iteration count of the previous solve, so few graph sizes are ever captured)
  auto step = [&](int count) {
    while (count > 0) {
      const int m = std::min(count, kMaxGraphIters);
      const bool first = fresh && first_ok() && H.p_parity == 0;
      fresh = false;
      if (cur.use_graph) {
        check_hip(hipGraphLaunch(iteration_graph(H, cur, first ? 3 : (H.p_parity ? 2 : 0), m), s),
                  "hipGraphLaunch");
        if (m & 1) H.p_parity ^= 1;
      } else {
        for (int i = 0; i < m; ++i) {
          enqueue_iteration(H, cur, H.p_parity, s, first && i == 0);
          H.p_parity ^= 1;
        }
      }
      count -= m;
    }
  };
  auto tail = [&]() {
    // the last iteration's convergence check when it was left to a next iteration (a no-op
    // otherwise), before the host reads the flag and before the finish reuses the partials;
    // a Dirichlet finish with the caller's x takes it in its first launch
    if (H.bc == MG_BC_NATURAL || !x_nat)
      k::finalize(k::FIN_CHECK, k::red_blocks(n), H.part, nullptr, H.scal, 1.0, 0, s);
    if (H.bc != MG_BC_NATURAL) enqueue_finish(H, b_nat, x_nat, s);
  };
  // the loop from iteration `launched` on; stagnation ends it only while the FP32 cycle runs
  bool fell_back = false;
  const int stall = (o.precision == MG_F32) ? o.stall_checks : 0;
  auto run = [&](int launched) {
    const bool stalled = iterate(H, cur, 0, s, step, tail, &T, launched, fell_back ? 0 : stall);
    if (H.bc == MG_BC_NATURAL) {
      enqueue_finish(H, b_nat, x_nat, s);
      read_scalars(H, s);
    }
    return stalled;
  };
  // restart from x: r = b - A x, p = q = 0, so that the next direction is the preconditioned
  // residual
  auto restart = [&]() {
    k::restart_scalars(H.scal, s);
    k::fill<double>(H.sp, n, 0.0, s);
    k::fill<double>(H.sp2, n, 0.0, s);
    k::fill<double>(H.sq, n, 0.0, s);
    k::residual<double>(F, H.sx, H.sb, H.sr, nullptr, s);
    if (r32) k::to_f32(n, H.scal, H.sr, r32, nullptr, s);
    fresh = true;
  };
  bool stalled = run(0);
  for (;;) {
    const DevScalars& h = *H.scal_host;
    const bool live_rhs = h.bnorm > 0 && std::isfinite(h.bnorm);
    // A stagnating, broken-down or non-finite FP32-preconditioned loop goes on from x with the
    // FP64 cycle (the residual, x and the coarsest solve are FP64 throughout, so x is as good
    // as the last completed iteration left it).
    if (stall > 0 && !fell_back && live_rhs &&
        (stalled || h.status == MG_EBREAKDOWN || h.status == MG_ENONFINITE)) {
      if (h.iters >= o.max_iter) {
        H.scal_host->status = MG_ENOCONV;
        break;
      }
      fell_back = true;
      cur.precision = MG_F64;
      r32 = nullptr;
      const int done_iters = h.iters;
      restart();
      stalled = run(done_iters);
      continue;
    }
    // The solve stops on the true relative residual ||b - A x|| / ||b|| (Sec. 3.1).  CG and
    // FCG loop on the recursively updated residual; when that met rtol and the true one
    // (computed by the finish) did not, the iteration restarts from x.
    if (o.outer != MG_OUTER_IR && h.status == MG_OK && h.bnorm > 0 &&
        h.true_rnorm > o.rtol * h.bnorm) {
      const int done_iters = h.iters;
      if (done_iters >= o.max_iter) {
        H.scal_host->status = MG_ENOCONV;
        break;
      }
      restart();
      stalled = run(done_iters);
      continue;
    }
    break;
  }
  collect(H, res, s);
  if (res) res->fp64_fallback = fell_back ? 1 : 0;
  T.mark("finish");
  return H.scal_host->status;
}

int run_mg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
           hipStream_t s) {
  Level& F = *H.lv.back();
  init_scalars(H, o, s);
  setup_rhs(H, b_nat, s, o.compat_check != 0);
  k::fill<double>(H.sx, F.n, 0.0, s);
  hipGraphExec_t g = o.use_graph ? iteration_graph(H, o, 1) : nullptr;
  iterate(H, o, 1, s, [&](int count) {
    for (int j = 0; j < count; ++j) {
      if (g)
        check_hip(hipGraphLaunch(g, s), "hipGraphLaunch");
      else
        enqueue_cycle(H, o, s);
    }
  }, [&]() {
    if (H.bc != MG_BC_NATURAL) enqueue_finish(H, b_nat, x_nat, s);
  });
  if (H.bc == MG_BC_NATURAL) {
    enqueue_finish(H, b_nat, x_nat, s);
    read_scalars(H, s);
  }
  collect(H, res, s);
  return H.scal_host->status;
}

}  // namespace decmg
