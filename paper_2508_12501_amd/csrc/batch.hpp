// Batched solves: many right-hand sides over a few hierarchies, solved together.
//
// Instances that share a hierarchy are packed into groups of M columns (M a power of two up
// to 64).  A group's vectors are stored row-blocked, entry (i, c) at [i * M + c], so one
// SELL-64 operator entry, loaded once, serves the M columns of its row, and the gathers of
// x_j are M-wide contiguous loads.  Each column runs its own FCG(1) recurrence with its own
// scalars and convergence flag; a group-wide flag turns every launch of the group into a
// no-op once all its columns are done.  One iteration of a group is captured as a hipGraph;
// groups are spread over a few streams.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "decmg.h"
#include "hier.hpp"

namespace decmg {

constexpr int kBatchMaxCols = 64;

struct BatchCol {
  double alpha, beta, pq, rnorm, bnorm, scale, inv_scale, mean, true_rnorm, rtol, n_unknowns;
  int32_t done, iters, status, max_iter;
};

struct BatchFlag {
  int32_t all_done;   // every column finished: the group's launches return at once
  int32_t n_done;     // finished columns (padding included)
  int32_t pad[62];
};

template <typename T>
struct BatchLevelVecs {
  T *x = nullptr, *t = nullptr, *r = nullptr, *b = nullptr;   // (n_l + 1) * M each
};

struct BatchGroup {
  Hierarchy* H = nullptr;
  int M = 1;                       // columns (power of two)
  int ncols = 0;                   // live columns (the rest are padding, done from the start)
  std::vector<int> inst;           // instance id of each live column
  int stream_slot = 0;
  std::vector<BatchLevelVecs<float>> v32;
  std::vector<BatchLevelVecs<double>> v64;
  double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *B = nullptr, *Z = nullptr;
  double* part = nullptr;          // 2 x red_blocks x M partial sums
  int part_blocks = 0;
  BatchCol* col = nullptr;         // M
  BatchFlag* flag = nullptr;
  const double** bptr = nullptr;   // device table of M input pointers
  double** xptr = nullptr;         // device table of M output pointers
  // graphs of 1, 2, 4 and 8 iterations (graph[k]: 2^k), captured when first used; a batch of
  // iterations launches the binary digits of its count
  hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  int64_t graph_epoch = -1;        // H->weight_epoch when the graphs were captured
  int last_iters = 0;
};

struct BatchTuning {
  int max_cols = 32;
  int pad_groups = 1;
  int streams = 4;
};

struct Batch {
  std::vector<Hierarchy*> inst_h;  // per instance
  mg_opts opts;
  BatchTuning tune;
  std::vector<BatchGroup> groups;
  std::vector<hipStream_t> streams;
  hipStream_t capture_stream = nullptr;
  hipEvent_t ev_start = nullptr;
  std::vector<hipEvent_t> ev_done;
  BatchCol* col_host = nullptr;    // pinned, one block of kBatchMaxCols per group
  void** ptr_host = nullptr;       // pinned staging of pointer tables, 2 x kBatchMaxCols per group
  std::string signature;
  ~Batch();
};

// Build (or rebuild after a tuning change) the groups and their buffers and graphs.
void batch_setup(Batch& B);
void batch_release_groups(Batch& B);
// Solve all instances: b[i], x[i] device pointers (natural order, nv of instance i each).
int batch_solve(Batch& B, const double* const* b, double* const* x, mg_result* res, hipStream_t s);
// Time each candidate tuning on the given inputs and keep the fastest; returns its time (ms).
double batch_autotune(Batch& B, const double* const* b, double* const* x, int reps,
                      const char* cache_path);
std::string batch_signature(const Batch& B);
bool batch_cache_lookup(const char* path, const std::string& sig, BatchTuning& t);
void batch_cache_store(const char* path, const std::string& sig, const BatchTuning& t);

namespace bk {
enum { FIN_BNORM = 0, FIN_ALPHA_FCG, FIN_CHECK, FIN_BETA_FCG, FIN_MEAN, FIN_RNORM, FIN_INIT };
int red_blocks(int32_t n, int M);
void init_cols(BatchCol* col, BatchFlag* flag, int M, int ncols, double rtol, int32_t max_iter,
               double n_unknowns, hipStream_t s);
void finalize(int op, int M, int nb, const double* part0, const double* part1, BatchCol* col,
              BatchFlag* flag, int force, hipStream_t s);
void gather_in(int M, int ncols, const int32_t* perm, int32_t n, const double* const* bptr,
               double* Bv, hipStream_t s);
void scatter_out(int M, int ncols, const int32_t* perm, int32_t n, const int32_t* bnd,
                 int32_t nbnd, const double* Xv, const double* const* bptr, double* const* xptr,
                 hipStream_t s);
void nat_sumsq(int M, int ncols, int32_t nv, const double* const* bptr, double* part, int nb,
               hipStream_t s);
void colsum(int M, int32_t n, const double* v, double* part, int nb, const BatchFlag* flag,
            hipStream_t s);
void colsum32(int M, int32_t n, const float* v, const BatchCol* col, double* part, int nb,
              const BatchFlag* flag, hipStream_t s);
void sub_mean(int M, int32_t n, const BatchCol* col, double* v, hipStream_t s);
void dot(int M, int32_t n, const double* a, const double* b, double* part, int nb,
         const BatchFlag* flag, hipStream_t s);
void start(int M, int32_t n, const BatchCol* col, const double* Bv, double* X, double* R,
           double* P, double* Q, float* r32, hipStream_t s);
template <typename T>
void zdot(int M, int32_t n, const BatchCol* col, const T* z, const double* q, double* part, int nb,
          int sub_mean, const BatchFlag* flag, hipStream_t s);
// p = z + beta p, and the previous iteration's step x += alpha p_old (per live column)
template <typename T>
void pupd(int M, int32_t n, const BatchCol* col, const T* z, double* p, double* x, int sub_mean,
          const BatchFlag* flag, hipStream_t s);
void spmv_dot2(int M, const Level& L, const double* p, double* q, const double* r, double* part0,
               double* part1, int nb, const BatchFlag* flag, hipStream_t s);
// r -= alpha q, its FP32 copy (r32 nullable) and the partials of r.r (per live column)
void update_r(int M, int32_t n, const BatchCol* col, const double* q, double* r, float* r32,
              double* part, int nb, const BatchFlag* flag, hipStream_t s);
// x += alpha p for every column whose last step is still pending (alpha != 0)
void apply_pending(int M, int32_t n, const BatchCol* col, const double* p, double* x,
                   hipStream_t s);
void residual_norm(int M, const Level& L, const double* x, const double* b, double* part, int nb,
                   hipStream_t s);
template <typename T>
void rows(int mode, int M, const Level& L, const T* x, const T* b, T* y, double omega,
          const BatchFlag* flag, hipStream_t s);
template <typename T>
void jacobi_zero(int M, const Level& L, const T* b, T* y, double omega, const BatchFlag* flag,
                 hipStream_t s);
template <typename T>
void restrict_(int M, const Level& Lf, const Level& Lc, const T* rf, T* rc, const BatchFlag* flag,
               hipStream_t s);
template <typename T>
void prolong(int M, const Level& Lf, const Level& Lc, const T* ec, T* xf, const BatchFlag* flag,
             hipStream_t s);
template <typename T>
void prolong_sweep(int M, const Level& Lf, const T* ec, const T* x, const T* b, T* y,
                   double omega, const BatchFlag* flag, hipStream_t s);
template <typename T>
void coarse(int M, const Hierarchy& H, const T* b, T* x, const BatchFlag* flag, hipStream_t s);
void zero(void* p, size_t bytes, hipStream_t s);   // bytes: a multiple of 4
}  // namespace bk

}  // namespace decmg
