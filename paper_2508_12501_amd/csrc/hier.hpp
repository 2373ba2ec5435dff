// Device-side hierarchy of the DEC multigrid library and the kernel launchers.
//
// Every level keeps its unknowns (interior vertices for zero Dirichlet, all vertices for
// natural boundaries) in an internal order chosen for locality: a Morton (Z-order) sort of
// the vertex coordinates.  Coordinates nest across levels, so parents and children of a
// vertex sit at nearby internal positions on neighbouring levels.  Internal vectors have
// n + 1 entries; entry n is a zero slot that gathers for absent neighbours point at.
#pragma once
#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "decmg.h"
#include "mesh.hpp"

namespace decmg {

constexpr int kSlice = 64;    // SELL slice height: one wavefront, one row per lane
constexpr int kBlock = 256;   // threads per row-parallel workgroup (4 wavefronts)
constexpr int kMaxCoarse = 2048;  // largest coarsest level solved densely
constexpr int kRedBlocks = 4096;  // cap on workgroups (and partial sums) of a reduction

// Operator in sliced ELLPACK (SELL-64): slice s covers internal rows 64s..64s+63 and owns
// columns sptr[s]..sptr[s+1]-1; entry k of lane l sits at [k*64 + l].  The same column
// array serves the FP64 and FP32 weights.  Exact zero couplings (star1 = 0, the diagonals
// of right-triangle grids) are dropped; they contribute nothing to L x.
constexpr int kZeroSlot16 = -32768;  // 16-bit column offset that stands for the zero slot
constexpr int kUnroll = 8;           // rows up to this many entries take the batched-load path

struct DevOperator {
  int32_t nslices = 0, ncols = 0;
  int32_t uw = -1;            // every slice has this width (ELL layout), or -1
  int32_t* sptr = nullptr;
  int32_t* col = nullptr;
  // The same columns as offsets from the row (kZeroSlot16 = zero slot), when every offset of
  // the level fits in 16 bits; the row kernels then read half the index bytes.
  int16_t* col16 = nullptr;
  double* w64 = nullptr;
  float* w32 = nullptr;
  bool w_exact32 = false;     // every FP64 weight equals its FP32 copy: FP64 kernels read w32
  // IEEE binary16 copy of the weights, read by the FP32 and FP64 kernels alike when every
  // weight is exactly a binary16 number (the widened values are then the weights bit for bit)
  uint16_t* w16 = nullptr;
  bool w_exact16 = false;
  // 1 / (sum of the row's weights, in SELL order), 1 in the zero slot: the first Jacobi sweep
  // from zero is x = (omega b) (1/D), a multiplication where a division per coupling cost
  // vector-ALU time in the two-sweeps-from-zero kernels
  double* idiag64 = nullptr;
  float* idiag32 = nullptr;
  // Row patterns (levels of uniform width 1..8 with 16-bit offsets): when the rows take at
  // most kMaxRowPatterns distinct sequences of (offset, weight) entries -- on a grid with a
  // unit coefficient: the interior stencil and the few next to the boundary -- pat[r] names
  // row r's pattern and the two-row kernels read that one byte instead of uw offsets and
  // weights.  poff / pw32 / pw64: npat x uw entries, pattern-major (npat = 0: not used).
  uint8_t* pat = nullptr;
  int16_t* poff = nullptr;
  float* pw32 = nullptr;
  double* pw64 = nullptr;
  int32_t npat = 0;
};
constexpr int kMaxRowPatterns = 256;

struct DevTransfer {          // between level l-1 (coarse) and level l (fine)
  int32_t* pa = nullptr;      // n_f: internal coarse ids (or n_c) of the two parents
  int32_t* pb = nullptr;
  // the same parents packed for the per-step interpolation: per 64-row slice of fine rows a
  // base coarse id, per row the two parents as int16 offsets from it (low half a, high half
  // b; kZeroSlot16 = zero slot), when every offset fits; else null
  int32_t* p_base = nullptr;
  uint32_t* p_ab16 = nullptr;
  int32_t* r_self = nullptr;  // n_c: fine internal id of the kept vertex
  int32_t nslices = 0, ncols = 0;
  int32_t r_uw = -1;          // uniform slice width of the restriction lists, or -1
  int32_t* r_sptr = nullptr;  // SELL over coarse rows of the fine midpoints (weight 1/2)
  int32_t* r_col = nullptr;
  // the same lists as 16-bit offsets from the kept vertex (kZeroSlot16 = zero slot), when the
  // width is uniform and at most 8 and every offset fits; else null
  int16_t* r_col16 = nullptr;
  // Weighted transfers (cubic subdivision, any M(f)): interpolation x_f += sum_k w_k e_{p_k}
  // over three parents per fine unknown; restriction r_c = sum over the coarse row's entries
  // (fine unknown, weight) in SELL-64 (the kept vertex is an entry of weight 1).  The binary
  // fields above are unused then.
  bool weighted = false;
  int32_t* p3 = nullptr;          // (n_f + 1) x 3 coarse parents, zero slot for non-unknowns
  double* pw64 = nullptr;         // (n_f + 1) x 3 weights
  float* pw32 = nullptr;
  int32_t* rw_sptr = nullptr;
  int32_t* rw_col = nullptr;      // fine internal ids (zero slot n_f for padding)
  double* rw64 = nullptr;
  float* rw32 = nullptr;
};

// Workgroup tiles of the fused smoothing kernels of one launch-bound binary level (l >= 1).
// Tile b owns a run of at most kBlock rows of the level's Morton order that lies inside one
// aligned block of 16 x 16 (x 16) lattice cells of the median edge length (F; a 16 x 16 patch
// on a grid) and the coarse rows whose kept vertex lies in F.  Its local rows are F, then the fine rows its coarse rows
// restrict from (R0 = F + those), then the operator neighbours of R0 (R1), then theirs (R2),
// each group in ascending internal order.  Everything a cycle leg needs from those rings is
// recomputed in LDS, so the down leg (Jacobi sweeps from zero, residual, restriction) and the
// up leg (interpolation, sweeps) are one launch each.  Every tile has the same capacity (cap
// local rows, ccap coarse rows; padding repeats a valid id), so a workgroup issues all of its
// index loads at once; local id cap is the zero slot.
struct DevTiles {
  int32_t ntiles = 0;
  int32_t kt = 0;              // local column slots per row (4 or 8)
  int32_t cap = 0, ccap = 0;   // local rows / coarse rows per tile (multiples of 64)
  int64_t rows_total = 0;      // sum of n2 over the tiles
  int32_t* meta = nullptr;     // per tile 8 ints: nF, n0, n1, n2, ncb, 0, 0, 0
  int32_t* row = nullptr;      // [tile][cap]: internal row id
  int32_t* ent = nullptr;      // [tile][cap]: (SELL index of entry 0) << 4 | width; null when
                               // the level's slices are uniform (index computed from the row)
  int16_t* col = nullptr;      // [tile][kt][cap]: local id of entry k (zero slot past the width)
  int32_t* crow = nullptr;     // [tile][ccap]: internal coarse id
  int16_t* cst = nullptr;      // [tile][rws][ccap]: binary levels: local ids of the kept vertex,
                               // then of up to 8 midpoints (zero slot past the row's width);
                               // weighted levels: local ids of the row's entries in SELL order
  int32_t rws = 9;             // slots per owned coarse row in cst
  int32_t* cent = nullptr;     // weighted levels, [tile][ccap]: (SELL index of the coarse row's
                               // first restriction entry) << 6 | its width
};
// One workgroup of kTileThreads threads per tile of up to 256 owned rows, one ring row per
// thread when the rings fit (cap <= kTileThreads, C3: 448), two otherwise (cap <= 2
// kTileThreads, the sphere).  Several wavefronts per SIMD hide each other's dependent chains
// (FP64 divisions above all): 256 threads with four ring rows each left one wavefront per SIMD
// and lost in FP64; 512 threads came out about 1% faster than 1024 on C3.
constexpr int kTileThreads = 512;

// Levels up to this many rows are launch-bound: binary ones run the fused tiles; on the others
// the interpolation is fused into the first post-smoothing sweep (one launch fewer).  On larger
// levels the extra dependent gathers of either cost more than the separate passes.
constexpr int32_t kLaunchBoundRows = 1 << 19;
constexpr int kCoarseThreads = 1024;       // workgroup of the fused coarse cycle
constexpr int kCoarseLdsMax = 160 * 1024;  // LDS budget cap of the fused coarse cycle
// Largest level the fused coarse cycle takes.  It runs in one workgroup, whose memory
// throughput (one CU's outstanding misses) makes it pay only for levels whose operator data is
// a few tens of KB; larger levels run as regular multi-workgroup launches.  (Taking the
// 3969-row level of the 2049^2 grid as well, four rows per thread, saved nothing in FP32 and
// spilled registers in FP64.)
constexpr int32_t kCoarseFuseRows = 2048;
// Iterations whose residual a solve records for mg_result.history.
constexpr int32_t kHistoryCap = 4096;
// Size of the static device work area of porous_integrate_noalloc (one copy per GPU).
constexpr size_t kRkStaticWorkBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;

// Per-level descriptor of the fused coarse cycle (device copy per precision).
template <typename T>
struct CoarseLevel {
  int32_t n = 0, lds = 0;            // unknowns; offset (in T) of x, partner, b in LDS
  int32_t uw = -1, r_uw = -1;        // uniform slice widths of operator / restriction, or -1
  int32_t nslices = 0, r_nslices = 0;
  int32_t lds_sptr = 0, lds_rsptr = 0;  // offsets (in int32) of the preloaded slice bounds
  const int32_t* sptr = nullptr;
  const int32_t* col = nullptr;
  const T* w = nullptr;
  const T* idiag = nullptr;
  const int32_t* pa = nullptr;       // interpolation from level-1
  const int32_t* pb = nullptr;
  const int32_t* r_self = nullptr;   // restriction into level-1
  const int32_t* r_sptr = nullptr;
  const int32_t* r_col = nullptr;
  const int32_t* color = nullptr;    // Gauss-Seidel colour of each row
  int32_t ncolors = 0;
};

template <typename T>
struct LevelVecs {
  T* x = nullptr;
  T* b = nullptr;
  T* r = nullptr;
  T* t = nullptr;
  T* u = nullptr;   // second work vector of the CG smoother
};

// Scalars of the CG smoother on one level (device memory).
struct CgsScalars {
  double rr, pq, alpha, beta;
};

// The rows of one colour class of the level's operator packed in SELL-64 (multicolour
// Gauss-Seidel): packed row p is internal row rowid[p]; entries keep the operator's couplings
// (absolute internal columns, the zero slot for non-unknowns) with their edge ids for weights.
struct GsColor {
  int32_t nrows = 0, nslices = 0, uw = -1;
  std::vector<int32_t> edge_h;     // per entry: edge id, -1 for padding
  int32_t* rowid = nullptr;
  int32_t* sptr = nullptr;
  int32_t* col = nullptr;
  double* w64 = nullptr;
  float* w32 = nullptr;
  bool w_exact32 = false;
};

struct Level {
  Mesh mesh;                       // natural numbering (host)
  int32_t nv = 0, n = 0;
  std::vector<int32_t> perm_h;     // internal -> natural
  std::vector<int32_t> inv_h;      // natural -> internal or -1
  std::vector<int32_t> bnd_h;      // natural ids that are not unknowns
  std::vector<int32_t> entry_edge; // per SELL entry: edge id or -1 (padding)
  std::vector<int32_t> col_h;      // per SELL entry: internal column (host copy)
  std::vector<int32_t> sptr_h;
  int64_t nnz = 0;                 // stored couplings (SELL entries that are not padding)
  int32_t* perm = nullptr;         // device copies
  int32_t* bnd_ids = nullptr;
  double* star0 = nullptr;         // nv, natural numbering
  DevOperator op;
  std::vector<GsColor> gs;         // colour classes, in colour order
  int32_t* row_color = nullptr;    // n + 1: colour class of each internal row (device)
  CgsScalars* cgs = nullptr;
  DevTransfer tr;                  // valid for l >= 1
  DevTiles tiles;                  // fused smoothing tiles (ntiles == 0: none)
  LevelVecs<double> v64;
  LevelVecs<float> v32;
};

struct DevScalars {
  double alpha, beta, rho, pq, rnorm, bnorm, rtol, scale, inv_scale, mean;
  double n_unknowns;
  double true_rnorm;   // ||b - A x|| recomputed at exit
  int32_t done, iters, status, max_iter;
  double* hist;        // relative residual of the loop after each iteration (device), or null
  int32_t hist_cap;
  int32_t pbuf;        // direction buffer (0 first, 1 second) of the pending step x += alpha p
  int32_t check_pending;   // a residual update whose convergence check has not run yet
  int32_t pad_;
};

// Finest-level data of the porous-convection step and of the solve gradients (built on first
// use; edge coefficients refreshed when the vertex coefficient changes).
struct PorousData {
  bool ready = false;
  int64_t kversion = -1;
  double* s1 = nullptr;      // per SELL entry: star1 of the entry's edge (0 for padding)
  double* ke = nullptr;      // per SELL entry: (k_lo + k_hi)/2
  double* y = nullptr;       // per unknown (n + 1): y coordinate
  double* star0 = nullptr;   // per unknown (n + 1)
  double* mask = nullptr;    // per unknown (n + 1): 0 on the walls y = y_min and y = y_max
  int32_t ne = 0;
  int32_t* ea = nullptr;     // per edge: internal id of (lo, hi), or n when not an unknown
  int32_t* eb = nullptr;
  double* s1e = nullptr;     // per edge: star1
  double* ge = nullptr;      // per edge scratch
  int64_t* vptr = nullptr;   // natural vertex -> incident edges
  int32_t* vinc = nullptr;
  double *T = nullptr, *T2 = nullptr, *P = nullptr, *Lm = nullptr, *L2 = nullptr, *M = nullptr,
         *U = nullptr;       // internal work vectors (n + 1)
};

struct Hierarchy {
  int32_t bc = MG_BC_DIRICHLET0;
  bool project = false;
  bool nested_ids = true;   // every level keeps the vertex ids of the level below it
  std::vector<std::unique_ptr<Level>> lv;
  double* coarse_inv = nullptr;    // n0 x n0 FP64 inverse of the coarsest operator
  int32_t n0 = 0;
  std::vector<double> kvert_h;     // vertex coefficient (finest), empty = 1
  double* kvert_d = nullptr;       // device copy of kvert_h (nv of the finest level)
  // edge coefficient per level (natural edge order), empty = none; set instead of kvert_h
  std::vector<std::vector<double>> kedge_h;
  int64_t kversion = 0;            // bumped by every change of the coefficient
  // bumped whenever the form of the weights some row kernel reads changes (binary16, FP32 or
  // FP64 copy); graphs captured before such a change are no longer valid
  int64_t weight_epoch = 0;
  PorousData por;
  // solver workspace (finest level, internal numbering, n+1 entries)
  double *sx = nullptr, *sr = nullptr, *sp = nullptr, *sq = nullptr, *sz = nullptr,
         *sb = nullptr;
  // second direction buffer: iteration k reads p from buf[k % 2] and writes buf[(k + 1) % 2]
  double* sp2 = nullptr;
  int p_parity = 0;
  double* part = nullptr;          // reduction partials, 3 x max blocks
  int32_t part_cap = 0;
  DevScalars* scal = nullptr;
  DevScalars* scal_host = nullptr; // pinned
  double* hist = nullptr;          // residual history of the last solve (device, hist_cap)
  int32_t hist_cap = 0;
  double* aux_host = nullptr;      // pinned, one double (host reads of single device results)
  hipStream_t capture_stream = nullptr;
  std::map<std::tuple<int, int, int, int, double>, hipGraphExec_t> graphs;
  int32_t debug_flags = 0;   // MG_DEBUG_ bits (fault injection for tests)
  std::map<std::tuple<int, int, int, int, double>, int> last_iters;
  // fused coarse cycle: highest level handled by one workgroup, per precision (-1 = none)
  int ctop64 = -1, ctop32 = -1;
  int coarse_width = 0;   // widest operator slice among the levels of the fused cycle
  int coarse_rwidth = 0;  // widest restriction slice among them
  int coarse_rows = 0;    // most unknowns on one of them
  // LDS layout of the fused cycle per precision: vectors, then (8-byte aligned) the dense
  // coarsest inverse, then the slice bounds of every fused level
  size_t cvec64 = 0, cvec32 = 0;        // bytes of the vector region up to each ctop
  size_t cint_off64 = 0, cint_off32 = 0;   // byte offset of the int region
  size_t clds_total64 = 0, clds_total32 = 0;
  int lds_limit = 64 * 1024;
  CoarseLevel<double>* clv64 = nullptr;
  CoarseLevel<float>* clv32 = nullptr;
  std::vector<int32_t> clds64, clds32;   // LDS offsets (in elements) per level
  // in-solve timing probe of the smoothing sweeps (eager launches only)
  struct Probe {
    bool on = false;
    int level = -1, dtype = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    hipStream_t stream = nullptr;
  } probe;
  bool capturing = false;
  ~Hierarchy();
};

// ----------------------------------------------------------------- kernel launchers
// All take internal-order vectors; `done` (nullable) makes a launch a no-op once a solver
// has converged, so speculative iterations cost one flag read.
template <typename T> const CoarseLevel<T>* coarse_levels(const Hierarchy& H);
template <> inline const CoarseLevel<double>* coarse_levels<double>(const Hierarchy& H) { return H.clv64; }
template <> inline const CoarseLevel<float>* coarse_levels<float>(const Hierarchy& H) { return H.clv32; }
template <typename T> int coarse_top(const Hierarchy& H);
template <> inline int coarse_top<double>(const Hierarchy& H) { return H.ctop64; }
template <> inline int coarse_top<float>(const Hierarchy& H) { return H.ctop32; }
template <typename T> size_t coarse_lds_bytes(const Hierarchy& H);
template <> inline size_t coarse_lds_bytes<double>(const Hierarchy& H) { return H.clds_total64; }
template <> inline size_t coarse_lds_bytes<float>(const Hierarchy& H) { return H.clds_total32; }
template <typename T> size_t coarse_int_offset(const Hierarchy& H);
template <> inline size_t coarse_int_offset<double>(const Hierarchy& H) { return H.cint_off64; }
template <> inline size_t coarse_int_offset<float>(const Hierarchy& H) { return H.cint_off32; }

namespace k {
template <typename T> void spmv(const Level& L, const T* x, T* y, const int* done, hipStream_t s);
template <typename T> void residual(const Level& L, const T* x, const T* b, T* r, const int* done, hipStream_t s);
template <typename T> void jacobi(const Level& L, const T* x, const T* b, T* xo, double omega, const int* done, hipStream_t s);
template <typename T> void jacobi_zero(const Level& L, const T* b, T* xo, double omega, const int* done, hipStream_t s);
template <typename T> void jacobi_two(const Level& L, const T* b, T* xo, double omega, const int* done, hipStream_t s);
template <typename T> void jacobi_timed(const Level& L, const T* x, const T* b, T* xo, double omega, const int* done, hipStream_t s, hipEvent_t e0, hipEvent_t e1);
template <typename T> void restrict_(const Level& Lf, const Level& Lc, const T* rf, T* rc, const int* done, hipStream_t s);
template <typename T> void prolong(const Level& Lf, const Level& Lc, const T* ec, T* xf, const int* done, hipStream_t s);
// CG smoother pieces: p = r and rr = r.r; q = A p and p.q; x += alpha p, r -= alpha q and r.r;
// p = r + beta p.  Reductions go through `part` (one partial per workgroup) and cgs_fin.
enum { CGS_INIT = 0, CGS_ALPHA = 1, CGS_BETA = 2 };
template <typename T> void cgs_start(const Level& L, const T* r, T* p, double* part, const int* done, hipStream_t s);
template <typename T> void cgs_spmv_dot(const Level& L, const T* p, T* q, double* part, const int* done, hipStream_t s);
template <typename T> void cgs_update(const Level& L, const T* p, const T* q, T* x, T* r, double* part, const int* done, hipStream_t s);
template <typename T> void cgs_pupd(const Level& L, const T* r, T* p, const int* done, hipStream_t s);
void cgs_fin(const Level& L, int op, const double* part, const int* done, hipStream_t s);
// x_i <- x_i + (b_i - (A x)_i) / A_ii for the rows of colour class c, in place
template <typename T> void gs_color(const Level& L, int c, T* x, const T* b, const int* done, hipStream_t s);
// xo = one weighted-Jacobi sweep of (x + M(f)^T ec), the interpolation fused into the sweep
template <typename T> void prolong_sweep(const Level& Lf, const Level& Lc, const T* ec, const T* x, const T* b, T* xo, double omega, const int* done, hipStream_t s);
template <typename T> void coarse(const Hierarchy& H, const T* b, T* x, const int* done, hipStream_t s);
template <typename T> void coarse_cycle(const Hierarchy& H, int top, const T* b, T* x, double omega, int nu1, int nu2, const int* done, hipStream_t s);
// Fused down leg of a tiled level from x = 0: nu1 (<= 2) Jacobi sweeps into x, and the
// restriction of the residual into bc (the coarse right-hand side)
// chk_part non-null: one more workgroup takes the Krylov loop's pending convergence check from
// its chk_nb (<= 8192) partials, as jacobi_two_chk does
template <typename T> void tile_down(const Level& L, const T* b, T* x, T* bc, double omega, int nu1, const int* done, hipStream_t s,
                                     DevScalars* chk_sc = nullptr, const double* chk_part = nullptr, int32_t chk_nb = 0);
// Fused up leg of a tiled level: xo = nu2 (1 or 2) Jacobi sweeps of x + M(f)^T ec
template <typename T> void tile_up(const Level& L, const T* ec, const T* x, const T* b, T* xo, double omega, int nu2, const int* done, hipStream_t s);
// whether levels top..0 fit the one-workgroup register-resident cycle of any shape and smoother
template <typename T> bool coarse_cycle_general_ok(const Hierarchy& H, int top, bool gs);
// one cycle of shape `kind` on levels top..0 in one launch, from zero or (x_init) from x, in place
template <typename T> void coarse_cycle_general(const Hierarchy& H, int top, const T* b, T* x, bool x_init, double omega, int nu1, int nu2, int kind, bool gs, const int* done, hipStream_t s);
// the same (weighted Jacobi) for ncols right-hand sides stored row-blocked, entry (i, c) at
// i ncols + c: one workgroup per column; requires coarse_cycle_general_ok(H, top, false)
template <typename T> void coarse_cycle_columns(const Hierarchy& H, int top, const T* b, T* x, bool x_init, double omega, int nu1, int nu2, int kind, int ncols, const int* done, hipStream_t s);
template <typename T> void copy(const T* src, T* dst, int32_t n, const int* done, hipStream_t s);
template <typename T> void fill(T* p, int64_t n, T v, hipStream_t s);
template <typename T> void gather(const int32_t* perm, int32_t n, const T* src, T* dst, hipStream_t s);
template <typename T> void scatter(const int32_t* perm, int32_t n, const T* src, T* dst, hipStream_t s);
template <typename T> void bnd_copy(const int32_t* ids, int32_t nb, const T* src, T* dst, hipStream_t s);
template <typename T> void bnd_jacobi(const int32_t* ids, int32_t nb, const T* b, T* x, double omega, hipStream_t s);
template <typename T> void bnd_zero(const int32_t* ids, int32_t nb, T* x, hipStream_t s);
void star0_apply(const Level& L, int bc, const double* f, double* b, hipStream_t s);
void prepare_coarse(const Hierarchy& H);

// Runge-Kutta building blocks (porous.hip): up to 7 vectors with coefficients.
struct RkTerms {
  const double* v[7];
  double c[7];
  int m;
};
// out = y + h * sum_j c_j v_j
void rk_axpy(const double* y, const RkTerms& tm, double h, double* out, int32_t n, hipStream_t s);
// *out = sqrt(mean_i ((scale sum_j c_j v_j)_i / (atol + rtol max(|u_i|, |w_i|)))^2); part holds
// rk_parts(n) doubles of scratch.  Device result.
int rk_parts(int32_t n);
// This GPU's copy of the static work area of the allocation-free integrator
// (kRkStaticWorkBytes, 256-byte aligned): its device address, looked up once per device.
double* rk_static_work();
void rk_wrms(const RkTerms& tm, double scale, const double* u, const double* w, double atol,
             double rtol, double* part, double* out, int32_t n, hipStream_t s);

// out += a * b entrywise, a null meaning 1 (porous.hip)
void mul_acc(int32_t n, const double* a, const double* b, double* out, hipStream_t s);
// porous step and solve gradients (porous.hip)
void por_rhs(const Level& L, const PorousData& D, const double* T, double* rhs, hipStream_t s);
// Tout = (add_T ? T : 0) + dt * dT/dt
void por_update(const Level& L, const PorousData& D, const double* T, const double* P, double* Tout,
                double dt, double phi, double kappa, bool add_T, hipStream_t s);
void por_mu(const Level& L, const PorousData& D, const double* lam, double* mu, hipStream_t s);
void por_adj_rhs(const Level& L, const PorousData& D, const double* T, const double* mu,
                 double* rhs, hipStream_t s);
void por_adj_update(const Level& L, const PorousData& D, const double* T, const double* P,
                    const double* mu, const double* lam, const double* psi, double* lam_out,
                    double dt, double phi, double kappa, hipStream_t s);
void por_grad_k(const Level& L, const PorousData& D, const double* T, const double* P,
                const double* mu, const double* psi, double* gk_nat, double dt, double phi,
                hipStream_t s);
void mg_grad_k(const Level& L, const PorousData& D, const double* lam, const double* u,
               double* gk_nat, hipStream_t s);
// gw_e += -(d0 lam)_e (d0 u)_e per edge (natural edge order); lam, u internal
void mg_grad_w(const Level& L, const PorousData& D, const double* lam, const double* u,
               double* gw_nat, hipStream_t s);

// Krylov building blocks (FP64 outer loop); partial sums land in H.part[0..2][block].
int blocks_for(int32_t n);
int red_blocks(int32_t n);   // grid (= number of partials) of the streaming reductions
// residual_norm runs one 256-row tile per workgroup: blocks_for(n) partials
// p_new = z + beta p_old (z from z32 / scale or from z64, minus the mean when asked), q = A p_new,
// with the block partials of p_new.q (part0) and p_new.r (part1): pupd_spmv_partials(L) of each
int pupd_spmv_partials(const Level& L);
// first: the first iteration after a start from p_old = 0 with no step pending (p = z; p_old
// and x are not read, x is not written)
void pupd_spmv_dot2(const Level& L, const DevScalars* sc, const float* z32, const double* z64,
                    int sub_mean_flag, const double* p_old, double* p_new, double* q,
                    const double* r, double* x, double* part0, double* part1, const int* done,
                    hipStream_t s, bool first = false);
void update_r(int32_t n, const DevScalars* sc, const double* q, double* r, float* r32,
              double* part0, const int* done, hipStream_t s);
void apply_pending(int32_t n, const DevScalars* sc, const double* p0, const double* p1, double* x,
                   hipStream_t s);
// jacobi_two on a row-pattern level with one more workgroup that takes the Krylov loop's
// pending convergence check from the nbp (<= 8192) partials of its residual update (the bits
// of a FIN_CHECK finalisation; a no-op when no check is pending)
bool jacobi_two_chk_ok(const Level& L);
// The exit work's ||b - A x||^2 as true_residual_partials(L) block partials (r_scratch: n
// doubles, used only on levels without row patterns).
bool true_residual_fast(const Level& L);
int true_residual_partials(const Level& L);
void true_residual(const Level& L, const double* x, const double* b, double* r_scratch,
                   double* part0, hipStream_t s);
// Dirichlet exit in one launch: pending step into x, x scattered through perm into x_nat, and
// x_nat[bnd[j]] = b_nat[bnd[j]] for the nbnd boundary vertices.
// part (nullable): also the loop's pending convergence check from its nbp partials, as a
// conditional FIN_CHECK would take it.
void finish_scatter(int32_t n, DevScalars* sc, const double* p0, const double* p1, double* x,
                    const int32_t* perm, double* x_nat, const int32_t* bnd, int32_t nbnd,
                    const double* b_nat, const double* part, int32_t nbp, hipStream_t s);
// sum64 whose partials kernel also writes the solver's starting scalars (init_scalars).
void sum64_init(int32_t n, const double* v, double* part0, DevScalars* sc, double rtol,
                int32_t max_iter, double n_unknowns, double* hist, int32_t hist_cap,
                hipStream_t s);
// sub_mean then dot(v, v) in one pass (same bits).
void sub_mean_dot(int32_t n, const DevScalars* sc, double* v, double* part0, hipStream_t s);
// apply_pending then sum64(x) in one pass (same bits).
void apply_pending_sum(int32_t n, const DevScalars* sc, const double* p0, const double* p1,
                       double* x, double* part0, hipStream_t s);
// p = q = 0 and the scaled FP32 copy of r (r32 nullable), after a warm start's residual.
void warm_aux(int32_t n, const DevScalars* sc, const double* r, float* r32, double* p, double* q,
              hipStream_t s);
// dot() whose partials kernel also writes the solver's starting scalars (init_scalars).
void dot_init(int32_t n, const double* a, const double* b, double* part0, DevScalars* sc,
              double rtol, int32_t max_iter, double n_unknowns, double* hist, int32_t hist_cap,
              hipStream_t s);
// init_krylov with b gathered from the caller's numbering (b[i] = b_nat[perm[i]]) on the way.
// p, q nullable: left as they are (a first iteration that reads neither follows).
void init_krylov_gather(int32_t n, const DevScalars* sc, const int32_t* perm, const double* b_nat,
                        double* b, double* r, double* x, double* p, double* q, float* r32,
                        hipStream_t s);
template <typename T>
void jacobi_two_chk(const Level& L, const T* b, T* xo, double omega, const int* done,
                    DevScalars* sc, const double* part, int32_t nbp, hipStream_t s);
void residual_norm(const Level& L, const double* x, const double* b, double* r, float* r32,
                   const DevScalars* sc, double* part0, const int* done, hipStream_t s);
void sum64(int32_t n, const double* v, double* part0, const int* done, hipStream_t s);
void sum32(int32_t n, const float* v, const DevScalars* sc, double* part0, const int* done, hipStream_t s);
void zconv_dot(int32_t n, const DevScalars* sc, const float* z32, double* z, const double* o,
               double* part0, int sub_mean_flag, const int* done, hipStream_t s);
void zsub_dot(int32_t n, const DevScalars* sc, double* z, const double* o, double* part0,
              int sub_mean_flag, const int* done, hipStream_t s);
void axpy1(int32_t n, const double* z, double* x, const int* done, hipStream_t s);
void zdot32(int32_t n, const DevScalars* sc, const float* z32, const double* o, double* part0,
            int sub_mean_flag, const int* done, hipStream_t s);
void dot(int32_t n, const double* a, const double* b, double* part0, const int* done, hipStream_t s);
void sub_mean(int32_t n, const DevScalars* sc, double* v, hipStream_t s);
void to_f32(int32_t n, const DevScalars* sc, const double* r, float* r32, const int* done, hipStream_t s);
// r = b, x = p = q = 0 and (r32 non-null) r32 = float(b * scale), one pass over n entries
void init_krylov(int32_t n, const DevScalars* sc, const double* b, double* r, double* x,
                 double* p, double* q, float* r32, hipStream_t s);

enum FinOp : int {
  FIN_BNORM = 0,      // bnorm = sqrt(sum0 + boundary part); choose the FP32 scale
  FIN_ALPHA_CG = 1,   // pq = sum0; alpha = rho / pq
  FIN_ALPHA_FCG = 2,  // pq = sum0; alpha = sum1 / pq
  FIN_CHECK = 3,      // rnorm = sqrt(sum0); iters++; convergence / limits
  FIN_BETA_CG = 4,    // beta = sum0 / rho; rho = sum0
  FIN_BETA_FCG = 5,   // beta = -sum0 / pq
  FIN_MEAN = 6,       // mean = sum0 / n
  FIN_RNORM = 7,      // rnorm = sqrt(sum0) (no iteration bookkeeping)
  // singular systems, preconditioned vector z not yet projected: sum0 = z.o, sum1 = sum z,
  // sum2 = sum o; mean = sum1 / n and (z - mean).o = sum0 - mean sum2, then as BETA_CG / FCG
  FIN_MEAN_BETA_CG = 8,
  FIN_MEAN_BETA_FCG = 9,
  // compatibility of a singular system's right-hand side: sum0 = sum b, sum1 = sum |b|;
  // mean = sum0 / n, MG_EINCOMPAT when |sum0| > kCompatTol sum1
  FIN_MEAN_COMPAT = 10,
};
// Relative size of sum b against sum |b| beyond which a natural-boundary right-hand side is
// taken to be outside the operator's range (rounding of a compatible one stays near 1e-16).
constexpr double kCompatTol = 1e-8;
void finalize(int op, int32_t nblocks, const double* part0, const double* part1, DevScalars* sc,
              double extra, int force, hipStream_t s, const double* part2 = nullptr);
// part0 = z.o, part1 = sum z, part2 = sum o (z32 widened by 1/scale), per block
void zsum_dot32(int32_t n, const DevScalars* sc, const float* z32, const double* o, double* part0,
                double* part1, double* part2, const int* done, hipStream_t s);
void zsum_dot64(int32_t n, const DevScalars* sc, const double* z, const double* o, double* part0,
                double* part1, double* part2, const int* done, hipStream_t s);
// starting scalars; hist (nullable) receives the loop's relative residual per iteration, up
// to hist_cap of them
void init_scalars(DevScalars* sc, double rtol, int32_t max_iter, double n_unknowns, double* hist,
                  int32_t hist_cap, hipStream_t s);
// clears the converged flag and status (the loop continues from its current iterate)
void restart_scalars(DevScalars* sc, hipStream_t s);
// block partials of sum v (part0) and of sum |v| (part1)
void sum_abs64(int32_t n, const double* v, double* part0, double* part1, hipStream_t s);
}  // namespace k

}  // namespace decmg
