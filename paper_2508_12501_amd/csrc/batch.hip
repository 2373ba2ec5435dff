// HIP kernels of the batched (multi right-hand-side) solve.
//
// A group's vectors hold M columns row-blocked: entry (i, c) at [i * M + c], M a power of two
// up to 64.  A 256-thread workgroup covers 256 / M consecutive rows; thread t works on column
// t % M of row t / M.  A wavefront then covers 64 / M consecutive rows that sit in one 64-row
// SELL slice, so the slice width is wave-uniform exactly as in the single-column kernels; the
// M threads of a row load the same column index and weight (one transaction serves them all)
// and gather x_j as one contiguous M-wide segment.
//
// Reductions produce one partial sum per (workgroup, column); a one-workgroup finaliser turns
// them into the per-column scalars of the FCG(1) recurrence and maintains the group flag.
#include <hip/hip_runtime.h>

#include <stdexcept>
#include <type_traits>

#include "batch.hpp"
#include "half16.hpp"
#include "util.hpp"

namespace decmg {
namespace {

constexpr int kThreads = 256;
constexpr int kFin = 256;    // threads of the per-column finaliser
constexpr int kMaxRed = 1024;   // cap on workgroups (partials per column) of a reduction

__device__ __forceinline__ int xcd_blk() {
  const int b = blockIdx.x, g = gridDim.x;
  const int x = b & 7, i = b >> 3, q = g >> 3, r = g & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ void tiles_of(int ntiles, int blk, int& t0, int& t1) {
  const int g = gridDim.x;
  t0 = static_cast<int>(static_cast<int64_t>(ntiles) * blk / g);
  t1 = static_cast<int>(static_cast<int64_t>(ntiles) * (blk + 1) / g);
}

template <bool D16>
__device__ __forceinline__ int colx(const void* __restrict__ col, int idx, int row, int n) {
  if (D16) {
    const int c = static_cast<const int16_t*>(col)[idx];
    return c == kZeroSlot16 ? n : row + c;
  }
  return static_cast<const int32_t*>(col)[idx];
}

// Per-column block reduction of up to two values; threads t < M write part[t * nb + blk]
// (nb = gridDim.x: each column's partials are contiguous, for the per-column finaliser).
template <int M>
__device__ __forceinline__ void block_cols(double v0, double v1, double* part0, double* part1,
                                           int blk) {
  __shared__ double s0[kThreads], s1[kThreads];
  s0[threadIdx.x] = v0;
  if (part1) s1[threadIdx.x] = v1;
  __syncthreads();
  if (threadIdx.x < M) {
    double a = 0.0, b = 0.0;
    for (int j = 0; j < kThreads / M; ++j) {
      a += s0[j * M + threadIdx.x];
      if (part1) b += s1[j * M + threadIdx.x];
    }
    part0[threadIdx.x * gridDim.x + blk] = a;
    if (part1) part1[threadIdx.x * gridDim.x + blk] = b;
  }
}

// Every product of an operator row is accumulated with an explicit fused multiply-add, so that
// the scalar and the vectorised kernels round alike whatever the compiler would contract.
__device__ __forceinline__ float bmac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double bmac(double a, double b, double c) { return __builtin_fma(a, b, c); }

// acc = sum_k w_k (x_i - x_j(k)), d = sum_k w_k over the row's entries, column c.
template <typename T, bool D16, int M, int N, typename WT>
__device__ __forceinline__ void brow_n(const void* __restrict__ col, const WT* __restrict__ w,
                                       const T* __restrict__ x, int beg, int lane, int row, int c,
                                       int n, T xi, T& acc, T& d) {
  int cj[N];
  T wk[N], xj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int idx = (beg + k) * kSlice + lane;
    cj[k] = colx<D16>(col, idx, row, n);
    wk[k] = static_cast<T>(w[idx]);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) xj[k] = x[cj[k] * M + c];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d += wk[k];
    acc = bmac(wk[k], xi - xj[k], acc);
  }
}

template <typename T, bool D16, int M, typename WT>
__device__ __forceinline__ void brow(const int32_t* __restrict__ sptr, const void* __restrict__ col,
                                     const WT* __restrict__ w, const T* __restrict__ x, int row,
                                     int c, int n, T xi, T& acc, T& d) {
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s];
  const int width = sptr[s + 1] - beg;
  const int lane = row & 63;
  acc = T(0);
  d = T(0);
  switch (width) {
    case 0: break;
    case 1: brow_n<T, D16, M, 1>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 2: brow_n<T, D16, M, 2>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 3: brow_n<T, D16, M, 3>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 4: brow_n<T, D16, M, 4>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 5: brow_n<T, D16, M, 5>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 6: brow_n<T, D16, M, 6>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 7: brow_n<T, D16, M, 7>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    case 8: brow_n<T, D16, M, 8>(col, w, x, beg, lane, row, c, n, xi, acc, d); break;
    default:
      for (int k = 0; k < width; ++k) {
        const int idx = (beg + k) * kSlice + lane;
        const T wk = static_cast<T>(w[idx]);
        d += wk;
        acc = bmac(wk, xi - x[colx<D16>(col, idx, row, n) * M + c], acc);
      }
  }
}

#define BK_ROWCOL(M)                                           \
  const int c = threadIdx.x & ((M) - 1);                       \
  const int row = xcd_blk() * (kThreads / (M)) + threadIdx.x / (M);

// MODE 0: y = A x;  1: y = b - A x;  2: y = x + omega (b - A x) / diag
template <typename T, int MODE, bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_rows(const int32_t* __restrict__ sptr,
                                                    const void* __restrict__ col,
                                                    const WT* __restrict__ w,
                                                    const T* __restrict__ x,
                                                    const T* __restrict__ b, T* __restrict__ y,
                                                    int32_t n, T omega,
                                                    const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= n) return;
  const T xi = x[row * M + c];
  const T bi = (MODE == 0) ? T(0) : b[row * M + c];
  T acc, d;
  brow<T, D16, M>(sptr, col, w, x, row, c, n, xi, acc, d);
  if (MODE == 0)
    y[row * M + c] = acc;
  else if (MODE == 1)
    y[row * M + c] = bi - acc;
  else
    y[row * M + c] = xi + omega * (bi - acc) / d;
}

// ----------------------------------------------------------------- vectorised row kernels
// With at least 16 bytes of columns per row (M >= 4 FP32 or M >= 2 FP64 columns), a thread
// takes 16 bytes of consecutive columns of its row: one 16-byte load per vector and per
// neighbour in place of four or two, and a wavefront covers four or two times as many rows,
// so each row's index and weight loads serve more columns.  The arithmetic of every column is
// that of bk_rows (explicit fused multiply-adds in entry order), so the results are the same.
template <typename T>
constexpr int kVW = 16 / static_cast<int>(sizeof(T));

template <typename T, int VW>
struct alignas(sizeof(T) * VW) VecT {
  T v[VW];
};

template <typename T, bool D16, int M, int N, typename WT>
__device__ __forceinline__ void brow_v_n(const void* __restrict__ col, const WT* __restrict__ w,
                                         const T* __restrict__ x, int beg, int lane, int row,
                                         int c0, int n, const VecT<T, kVW<T>>& xi,
                                         T (&acc)[kVW<T>], T& d) {
  constexpr int VW = kVW<T>;
  int cj[N];
  T wk[N];
  VecT<T, VW> xj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int idx = (beg + k) * kSlice + lane;
    cj[k] = colx<D16>(col, idx, row, n);
    wk[k] = static_cast<T>(w[idx]);
  }
#pragma unroll
  for (int k = 0; k < N; ++k)
    xj[k] = *reinterpret_cast<const VecT<T, VW>*>(x + cj[k] * M + c0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d += wk[k];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = bmac(wk[k], xi.v[e] - xj[k].v[e], acc[e]);
  }
}

// bk_rows over 16-byte column vectors (M >= kVW<T>)
template <typename T, int MODE, bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_rows_v(const int32_t* __restrict__ sptr,
                                                      const void* __restrict__ col,
                                                      const WT* __restrict__ w,
                                                      const T* __restrict__ x,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ y, int32_t n, T omega,
                                                      const BatchFlag* __restrict__ flag) {
  constexpr int VW = kVW<T>, TPR = M / VW, RB = kThreads / TPR;
  static_assert(M >= VW && M % VW == 0, "at least one full vector per row");
  using V = VecT<T, VW>;
  if (flag && flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * VW;
  const int row = xcd_blk() * RB + static_cast<int>(threadIdx.x) / TPR;
  if (row >= n) return;
  const V xi = *reinterpret_cast<const V*>(x + row * M + c0);
  V bi;
  if (MODE != 0) bi = *reinterpret_cast<const V*>(b + row * M + c0);
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s];
  const int width = sptr[s + 1] - beg;
  const int lane = row & 63;
  T acc[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) acc[e] = T(0);
  T d = T(0);
  switch (width) {
    case 0: break;
#define BK_ROWV(K)                                                                            \
  case K:                                                                                     \
    brow_v_n<T, D16, M, K>(col, w, x, beg, lane, row, c0, n, xi, acc, d);                     \
    break;
    BK_ROWV(1) BK_ROWV(2) BK_ROWV(3) BK_ROWV(4) BK_ROWV(5) BK_ROWV(6) BK_ROWV(7) BK_ROWV(8)
#undef BK_ROWV
    default:
      for (int k = 0; k < width; ++k) {
        const int idx = (beg + k) * kSlice + lane;
        const T wk = static_cast<T>(w[idx]);
        const V xj = *reinterpret_cast<const V*>(x + colx<D16>(col, idx, row, n) * M + c0);
        d += wk;
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = bmac(wk, xi.v[e] - xj.v[e], acc[e]);
      }
  }
  V out;
#pragma unroll
  for (int e = 0; e < VW; ++e) {
    if (MODE == 0)
      out.v[e] = acc[e];
    else if (MODE == 1)
      out.v[e] = bi.v[e] - acc[e];
    else
      out.v[e] = xi.v[e] + omega * (bi.v[e] - acc[e]) / d;
  }
  *reinterpret_cast<V*>(y + row * M + c0) = out;
}

// bk_jacobi_zero over 16-byte column vectors
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_jacobi_zero_v(const T* __restrict__ idiag,
                                                             const T* __restrict__ b,
                                                             T* __restrict__ y, int32_t n, T omega,
                                                             const BatchFlag* __restrict__ flag) {
  constexpr int VW = kVW<T>, TPR = M / VW, RB = kThreads / TPR;
  using V = VecT<T, VW>;
  if (flag && flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * VW;
  const int row = xcd_blk() * RB + static_cast<int>(threadIdx.x) / TPR;
  if (row >= n) return;
  const V bi = *reinterpret_cast<const V*>(b + row * M + c0);
  const T di = idiag[row];
  V out;
  {
#pragma clang fp contract(off)
#pragma unroll
    for (int e = 0; e < VW; ++e) out.v[e] = omega * bi.v[e] * di;
  }
  *reinterpret_cast<V*>(y + row * M + c0) = out;
}

// restriction over column vectors: rc = rf[kept] + 1/2 (sum of the midpoint entries)
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_restrict_v(const int32_t* __restrict__ self,
                                                          const int32_t* __restrict__ sptr,
                                                          const int32_t* __restrict__ col,
                                                          const T* __restrict__ rf,
                                                          T* __restrict__ rc, int32_t nc,
                                                          const BatchFlag* __restrict__ flag) {
  constexpr int VW = kVW<T>, TPR = M / VW, RB = kThreads / TPR;
  using V = VecT<T, VW>;
  if (flag && flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * VW;
  const int row = xcd_blk() * RB + static_cast<int>(threadIdx.x) / TPR;
  if (row >= nc) return;
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s], width = sptr[s + 1] - beg;
  const int lane = row & 63;
  const V rs = *reinterpret_cast<const V*>(rf + self[row] * M + c0);
  T acc[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) acc[e] = T(0);
  for (int k = 0; k < width; ++k) {
    const V v = *reinterpret_cast<const V*>(rf + col[(beg + k) * kSlice + lane] * M + c0);
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] += v.v[e];
  }
  V out;
#pragma unroll
  for (int e = 0; e < VW; ++e) out.v[e] = rs.v[e] + T(0.5) * acc[e];
  *reinterpret_cast<V*>(rc + row * M + c0) = out;
}

// interpolation over column vectors: xf += 1/2 (ec[pa] + ec[pb])
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_prolong_v(const int32_t* __restrict__ pa,
                                                         const int32_t* __restrict__ pb,
                                                         const T* __restrict__ ec,
                                                         T* __restrict__ xf, int32_t nf,
                                                         const BatchFlag* __restrict__ flag) {
  constexpr int VW = kVW<T>, TPR = M / VW, RB = kThreads / TPR;
  using V = VecT<T, VW>;
  if (flag && flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * VW;
  const int row = xcd_blk() * RB + static_cast<int>(threadIdx.x) / TPR;
  if (row >= nf) return;
  const V ea = *reinterpret_cast<const V*>(ec + pa[row] * M + c0);
  const V eb = *reinterpret_cast<const V*>(ec + pb[row] * M + c0);
  V x = *reinterpret_cast<const V*>(xf + row * M + c0);
#pragma unroll
  for (int e = 0; e < VW; ++e) x.v[e] += T(0.5) * (ea.v[e] + eb.v[e]);
  *reinterpret_cast<V*>(xf + row * M + c0) = x;
}

// bk_prolong_sweep over column vectors
template <typename T, bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_prolong_sweep_v(
    const int32_t* __restrict__ sptr, const void* __restrict__ col, const WT* __restrict__ w,
    const int32_t* __restrict__ pa, const int32_t* __restrict__ pb, const T* __restrict__ ec,
    const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int32_t n, T omega,
    const BatchFlag* __restrict__ flag) {
  constexpr int VW = kVW<T>, TPR = M / VW, RB = kThreads / TPR;
  using V = VecT<T, VW>;
  if (flag && flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * VW;
  const int row = xcd_blk() * RB + static_cast<int>(threadIdx.x) / TPR;
  if (row >= n) return;
  // x0 = x + M(f)^T e_c at one row (the zero slot's parents are the coarse zero slot)
  auto x0 = [&](int j) {
    const V xv = *reinterpret_cast<const V*>(x + j * M + c0);
    const V ea = *reinterpret_cast<const V*>(ec + pa[j] * M + c0);
    const V eb = *reinterpret_cast<const V*>(ec + pb[j] * M + c0);
    V r;
#pragma unroll
    for (int e = 0; e < VW; ++e) r.v[e] = xv.v[e] + T(0.5) * (ea.v[e] + eb.v[e]);
    return r;
  };
  const V xi0 = x0(row);
  const V bi = *reinterpret_cast<const V*>(b + row * M + c0);
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s], width = sptr[s + 1] - beg;
  const int lane = row & 63;
  T acc[VW];
#pragma unroll
  for (int e = 0; e < VW; ++e) acc[e] = T(0);
  T d = T(0);
  for (int k = 0; k < width; ++k) {
    const int idx = (beg + k) * kSlice + lane;
    const V xj = x0(colx<D16>(col, idx, row, n));
    const T wk = static_cast<T>(w[idx]);
    d += wk;
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = bmac(wk, xi0.v[e] - xj.v[e], acc[e]);
  }
  V out;
#pragma unroll
  for (int e = 0; e < VW; ++e) out.v[e] = xi0.v[e] + omega * (bi.v[e] - acc[e]) / d;
  *reinterpret_cast<V*>(y + row * M + c0) = out;
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_jacobi_zero(const T* __restrict__ idiag,
                                                           const T* __restrict__ b,
                                                           T* __restrict__ y, int32_t n, T omega,
                                                           const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= n) return;
  {
#pragma clang fp contract(off)
    y[row * M + c] = omega * b[row * M + c] * idiag[row];
  }
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_restrict(const int32_t* __restrict__ self,
                                                        const int32_t* __restrict__ sptr,
                                                        const int32_t* __restrict__ col,
                                                        const T* __restrict__ rf,
                                                        T* __restrict__ rc, int32_t nc,
                                                        const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= nc) return;
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s], width = sptr[s + 1] - beg;
  const int lane = row & 63;
  T acc = T(0);
  for (int k = 0; k < width; ++k) acc += rf[col[(beg + k) * kSlice + lane] * M + c];
  rc[row * M + c] = rf[self[row] * M + c] + T(0.5) * acc;
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_prolong(const int32_t* __restrict__ pa,
                                                       const int32_t* __restrict__ pb,
                                                       const T* __restrict__ ec,
                                                       T* __restrict__ xf, int32_t nf,
                                                       const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= nf) return;
  xf[row * M + c] += T(0.5) * (ec[pa[row] * M + c] + ec[pb[row] * M + c]);
}

// First post-smoothing sweep with the interpolation fused in: x0 = x + M(f)^T e_c is formed on
// the fly for the row and its neighbours (zero slot included: its parents are the coarse zero
// slot), then y = x0 + omega (b - A x0) / diag.
template <typename T, bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_prolong_sweep(
    const int32_t* __restrict__ sptr, const void* __restrict__ col, const WT* __restrict__ w,
    const int32_t* __restrict__ pa, const int32_t* __restrict__ pb, const T* __restrict__ ec,
    const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int32_t n, T omega,
    const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= n) return;
  const T xi0 = x[row * M + c] + T(0.5) * (ec[pa[row] * M + c] + ec[pb[row] * M + c]);
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  const int beg = sptr[s], width = sptr[s + 1] - beg;
  const int lane = row & 63;
  T acc = T(0), d = T(0);
  for (int k = 0; k < width; ++k) {
    const int idx = (beg + k) * kSlice + lane;
    const int j = colx<D16>(col, idx, row, n);
    const T xj = x[j * M + c] + T(0.5) * (ec[pa[j] * M + c] + ec[pb[j] * M + c]);
    const T wk = static_cast<T>(w[idx]);
    d += wk;
    acc = bmac(wk, xi0 - xj, acc);
  }
  y[row * M + c] = xi0 + omega * (b[row * M + c] - acc) / d;
}

// x = A0^{-1} b on the coarsest level (FP64 dense inverse), one thread per (row, column)
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_coarse(const double* __restrict__ ainv,
                                                      const T* __restrict__ b,
                                                      T* __restrict__ x, int32_t n0,
                                                      const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i >= n0) return;
  const double* a = ainv + static_cast<int64_t>(i) * n0;
  double acc = 0.0;
  for (int j = 0; j < n0; ++j) acc += a[j] * static_cast<double>(b[j * M + c]);
  x[i * M + c] = static_cast<T>(acc);
}

// ----------------------------------------------------------------- Krylov part (FP64)
template <int M>
__global__ __launch_bounds__(kThreads) void bk_gather_in(const int32_t* __restrict__ perm,
                                                         int32_t n,
                                                         const double* const* __restrict__ bptr,
                                                         double* __restrict__ Bv, int ncols) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i >= n) return;
  Bv[i * M + c] = c < ncols ? bptr[c][perm[i]] : 0.0;
}

template <int M>
__global__ __launch_bounds__(kThreads) void bk_scatter_out(const int32_t* __restrict__ perm,
                                                           int32_t n,
                                                           const double* __restrict__ Xv,
                                                           double* const* __restrict__ xptr,
                                                           int ncols) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i >= n || c >= ncols) return;
  xptr[c][perm[i]] = Xv[i * M + c];
}

// x = b at the vertices that are not unknowns (Dirichlet boundary)
template <int M>
__global__ __launch_bounds__(kThreads) void bk_bnd_copy(const int32_t* __restrict__ bnd,
                                                        int32_t nbnd,
                                                        const double* const* __restrict__ bptr,
                                                        double* const* __restrict__ xptr,
                                                        int ncols) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i >= nbnd || c >= ncols) return;
  xptr[c][bnd[i]] = bptr[c][bnd[i]];
}

// sum of squares of each caller vector (natural order, nv entries): block (bx, c)
__global__ __launch_bounds__(kThreads) void bk_nat_sumsq(int M, int ncols, int32_t nv,
                                                         const double* const* __restrict__ bptr,
                                                         double* __restrict__ part) {
  const int c = blockIdx.y;
  double v = 0.0;
  if (c < ncols) {
    const double* b = bptr[c];
    const int ntiles = (nv + kThreads - 1) / kThreads;
    int t0, t1;
    tiles_of(ntiles, blockIdx.x, t0, t1);
    for (int t = t0; t < t1; ++t) {
      const int i = t * kThreads + threadIdx.x;
      if (i < nv) v += b[i] * b[i];
    }
  }
  __shared__ double s[kThreads];
  s[threadIdx.x] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int j = 0; j < kThreads; ++j) a += s[j];
    part[c * gridDim.x + blockIdx.x] = a;
  }
}

// Streaming per-column reductions over a capped grid: logical block b walks a contiguous range
// of (256 / M)-row tiles.
#define BK_TILES(M, n)                                              \
  const int c = threadIdx.x & ((M) - 1);                            \
  const int rb = kThreads / (M);                                    \
  const int blk = blockIdx.x;                                       \
  int t0, t1;                                                       \
  tiles_of(((n) + rb - 1) / rb, blk, t0, t1);

template <int M>
__global__ __launch_bounds__(kThreads) void bk_colsum(int32_t n, const double* __restrict__ v,
                                                      double* __restrict__ part,
                                                      const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_TILES(M, n)
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * rb + threadIdx.x / M;
    if (i < n) a += v[i * M + c];
  }
  block_cols<M>(a, 0.0, part, nullptr, blk);
}

template <int M>
__global__ __launch_bounds__(kThreads) void bk_colsum32(int32_t n, const float* __restrict__ v,
                                                        const BatchCol* __restrict__ col,
                                                        double* __restrict__ part,
                                                        const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_TILES(M, n)
  const double s = col[c].inv_scale;
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * rb + threadIdx.x / M;
    if (i < n) a += static_cast<double>(v[i * M + c]) * s;
  }
  block_cols<M>(a, 0.0, part, nullptr, blk);
}

template <int M>
__global__ __launch_bounds__(kThreads) void bk_sub_mean(int32_t n, const BatchCol* __restrict__ col,
                                                        double* __restrict__ v) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i < n) v[i * M + c] = v[i * M + c] - col[c].mean;
}

template <int M>
__global__ __launch_bounds__(kThreads) void bk_dot(int32_t n, const double* __restrict__ a,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ part,
                                                   const BatchFlag* __restrict__ flag) {
  if (flag && flag->all_done) return;
  BK_TILES(M, n)
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * rb + threadIdx.x / M;
    if (i < n) v += a[i * M + c] * b[i * M + c];
  }
  block_cols<M>(v, 0.0, part, nullptr, blk);
}

// r = b, x = p = q = 0, r32 = scale * r
template <int M>
__global__ __launch_bounds__(kThreads) void bk_start(int32_t n, const BatchCol* __restrict__ col,
                                                     const double* __restrict__ Bv,
                                                     double* __restrict__ X, double* __restrict__ R,
                                                     double* __restrict__ P, double* __restrict__ Q,
                                                     float* __restrict__ r32) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  const int i = gid / M, c = gid & (M - 1);
  if (i >= n) return;
  const int k = i * M + c;
  const double bi = Bv[k];
  R[k] = bi;
  X[k] = 0.0;
  P[k] = 0.0;
  Q[k] = 0.0;
  if (r32) r32[k] = static_cast<float>(bi * col[c].scale);
}

// z widened (FP32: times inv_scale), minus the column mean when projecting
template <typename T>
__device__ __forceinline__ double zval(const T* z, int k, const BatchCol& cc, int sub_mean) {
  double zi = std::is_same<T, float>::value ? static_cast<double>(z[k]) * cc.inv_scale
                                            : static_cast<double>(z[k]);
  if (sub_mean) zi = zi - cc.mean;
  return zi;
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_zdot(int32_t n, const BatchCol* __restrict__ col,
                                                    const T* __restrict__ z,
                                                    const double* __restrict__ q,
                                                    double* __restrict__ part, int sub_mean,
                                                    const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES(M, n)
  const BatchCol cc = col[c];
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * rb + threadIdx.x / M;
    if (i < n) v = bmac(zval<T>(z, i * M + c, cc, sub_mean), q[i * M + c], v);
  }
  block_cols<M>(v, 0.0, part, nullptr, blk);
}

template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_pupd(int32_t n, const BatchCol* __restrict__ col,
                                                    const T* __restrict__ z, double* __restrict__ p,
                                                    double* __restrict__ x, int sub_mean,
                                                    const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_ROWCOL(M)
  if (row >= n) return;
  const BatchCol& cc = col[c];
  if (cc.done) return;
  const int k = row * M + c;
  const double po = p[k];
  x[k] = bmac(cc.alpha, po, x[k]);
  p[k] = bmac(cc.beta, po, zval<T>(z, k, cc, sub_mean));
}

template <bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_spmv_dot2(const int32_t* __restrict__ sptr,
                                                         const void* __restrict__ colv,
                                                         const WT* __restrict__ w,
                                                         const double* __restrict__ p,
                                                         double* __restrict__ q,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ part0,
                                                         double* __restrict__ part1, int32_t n,
                                                         const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES(M, n)
  double v0 = 0.0, v1 = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int row = t * rb + threadIdx.x / M;
    if (row < n) {
      const int k = row * M + c;
      const double pi = p[k];
      double acc, d;
      brow<double, D16, M>(sptr, colv, w, p, row, c, n, pi, acc, d);
      q[k] = acc;
      v0 = bmac(pi, acc, v0);
      v1 = bmac(pi, r[k], v1);
    }
  }
  block_cols<M>(v0, v1, part0, part1, blk);
}

// ----------------------------------------------------------------- Krylov part, vectorised
// Two FP64 columns per thread (M >= 2): tiles of 2 kThreads / M rows; per-column block sums in
// a fixed order (row slots of the workgroup in increasing order).
constexpr int kKV = 2;
using D2 = VecT<double, kKV>;

#define BK_TILES_V(M, n)                                                \
  constexpr int TPR = (M) / kKV, RBV = kThreads / TPR;                  \
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * kKV;           \
  const int slot = static_cast<int>(threadIdx.x) / TPR;                 \
  const int blk = blockIdx.x;                                           \
  int t0, t1;                                                           \
  tiles_of(((n) + RBV - 1) / RBV, blk, t0, t1);

template <int M>
__device__ __forceinline__ void block_cols_v(const double (&v0)[kKV], const double (&v1)[kKV],
                                             double* part0, double* part1, int blk) {
  constexpr int TPR = M / kKV, RBV = kThreads / TPR;
  __shared__ double s0[kThreads * kKV], s1[kThreads * kKV];
#pragma unroll
  for (int e = 0; e < kKV; ++e) {
    s0[threadIdx.x * kKV + e] = v0[e];
    if (part1) s1[threadIdx.x * kKV + e] = v1[e];
  }
  __syncthreads();
  if (static_cast<int>(threadIdx.x) < M) {
    const int c = threadIdx.x, tc = c / kKV, e = c % kKV;
    double a = 0.0, b = 0.0;
    for (int j = 0; j < RBV; ++j) {
      a += s0[(j * TPR + tc) * kKV + e];
      if (part1) b += s1[(j * TPR + tc) * kKV + e];
    }
    part0[c * gridDim.x + blk] = a;
    if (part1) part1[c * gridDim.x + blk] = b;
  }
}

// z.q per column (z widened and, when projecting, minus the column mean)
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_zdot_v(int32_t n, const BatchCol* __restrict__ col,
                                                      const T* __restrict__ z,
                                                      const double* __restrict__ q,
                                                      double* __restrict__ part, int sub_mean,
                                                      const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES_V(M, n)
  const BatchCol ca = col[c0], cb = col[c0 + 1];
  double v[kKV] = {0.0, 0.0}, none[kKV] = {0.0, 0.0};
  for (int t = t0; t < t1; ++t) {
    const int i = t * RBV + slot;
    if (i < n) {
      const int k = i * M + c0;
      const D2 qv = *reinterpret_cast<const D2*>(q + k);
      v[0] = bmac(zval<T>(z, k, ca, sub_mean), qv.v[0], v[0]);
      v[1] = bmac(zval<T>(z, k + 1, cb, sub_mean), qv.v[1], v[1]);
    }
  }
  block_cols_v<M>(v, none, part, nullptr, blk);
}

// p = z + beta p per live column
template <typename T, int M>
__global__ __launch_bounds__(kThreads) void bk_pupd_v(int32_t n, const BatchCol* __restrict__ col,
                                                      const T* __restrict__ z,
                                                      double* __restrict__ p,
                                                      double* __restrict__ x, int sub_mean,
                                                      const BatchFlag* __restrict__ flag) {
  constexpr int TPR = M / kKV, RBV = kThreads / TPR;
  if (flag->all_done) return;
  const int c0 = (static_cast<int>(threadIdx.x) % TPR) * kKV;
  const int row = xcd_blk() * RBV + static_cast<int>(threadIdx.x) / TPR;
  if (row >= n) return;
  const BatchCol& ca = col[c0];
  const BatchCol& cb = col[c0 + 1];
  if (ca.done && cb.done) return;
  const int k = row * M + c0;
  D2 pv = *reinterpret_cast<const D2*>(p + k);
  D2 xv = *reinterpret_cast<const D2*>(x + k);
  if (!ca.done) {
    xv.v[0] = bmac(ca.alpha, pv.v[0], xv.v[0]);
    pv.v[0] = bmac(ca.beta, pv.v[0], zval<T>(z, k, ca, sub_mean));
  }
  if (!cb.done) {
    xv.v[1] = bmac(cb.alpha, pv.v[1], xv.v[1]);
    pv.v[1] = bmac(cb.beta, pv.v[1], zval<T>(z, k + 1, cb, sub_mean));
  }
  *reinterpret_cast<D2*>(x + k) = xv;
  *reinterpret_cast<D2*>(p + k) = pv;
}

// q = A p per column, with the partial sums of p.q and p.r
template <bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_spmv_dot2_v(const int32_t* __restrict__ sptr,
                                                           const void* __restrict__ colv,
                                                           const WT* __restrict__ w,
                                                           const double* __restrict__ p,
                                                           double* __restrict__ q,
                                                           const double* __restrict__ r,
                                                           double* __restrict__ part0,
                                                           double* __restrict__ part1, int32_t n,
                                                           const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES_V(M, n)
  double v0[kKV] = {0.0, 0.0}, v1[kKV] = {0.0, 0.0};
  for (int t = t0; t < t1; ++t) {
    const int row = t * RBV + slot;
    if (row < n) {
      const int k = row * M + c0;
      const D2 pi = *reinterpret_cast<const D2*>(p + k);
      const D2 ri = *reinterpret_cast<const D2*>(r + k);
      const int s = __builtin_amdgcn_readfirstlane(row >> 6);
      const int beg = sptr[s], width = sptr[s + 1] - beg;
      const int lane = row & 63;
      double acc[kKV] = {0.0, 0.0}, d = 0.0;
      switch (width) {
        case 0: break;
#define BK_SPMVV(K)                                                                           \
  case K:                                                                                     \
    brow_v_n<double, D16, M, K>(colv, w, p, beg, lane, row, c0, n, pi, acc, d);               \
    break;
        BK_SPMVV(1) BK_SPMVV(2) BK_SPMVV(3) BK_SPMVV(4) BK_SPMVV(5) BK_SPMVV(6) BK_SPMVV(7)
        BK_SPMVV(8)
#undef BK_SPMVV
        default:
          for (int kk = 0; kk < width; ++kk) {
            const int idx = (beg + kk) * kSlice + lane;
            const double wk = static_cast<double>(w[idx]);
            const D2 pj = *reinterpret_cast<const D2*>(p + colx<D16>(colv, idx, row, n) * M + c0);
            d += wk;
            acc[0] = bmac(wk, pi.v[0] - pj.v[0], acc[0]);
            acc[1] = bmac(wk, pi.v[1] - pj.v[1], acc[1]);
          }
      }
      D2 qv;
      qv.v[0] = acc[0];
      qv.v[1] = acc[1];
      *reinterpret_cast<D2*>(q + k) = qv;
#pragma unroll
      for (int e = 0; e < kKV; ++e) {
        v0[e] = bmac(pi.v[e], acc[e], v0[e]);
        v1[e] = bmac(pi.v[e], ri.v[e], v1[e]);
      }
    }
  }
  block_cols_v<M>(v0, v1, part0, part1, blk);
}

// x += alpha p, r -= alpha q (live columns), the FP32 copy of r, and the partial sums of r.r
template <int M>
__global__ __launch_bounds__(kThreads) void bk_update_r_v(int32_t n, const BatchCol* __restrict__ col,
                                                          const double* __restrict__ q,
                                                          double* __restrict__ r,
                                                          float* __restrict__ r32,
                                                          double* __restrict__ part,
                                                          const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES_V(M, n)
  const BatchCol ca = col[c0], cb = col[c0 + 1];
  const bool la = !ca.done, lb = !cb.done;
  double v[kKV] = {0.0, 0.0}, none[kKV] = {0.0, 0.0};
  if (la || lb) {
    for (int t = t0; t < t1; ++t) {
      const int i = t * RBV + slot;
      if (i < n) {
        const int k = i * M + c0;
        const D2 qv = *reinterpret_cast<const D2*>(q + k);
        D2 rv = *reinterpret_cast<const D2*>(r + k);
        if (la) {
          rv.v[0] = bmac(-ca.alpha, qv.v[0], rv.v[0]);
          v[0] = bmac(rv.v[0], rv.v[0], v[0]);
        }
        if (lb) {
          rv.v[1] = bmac(-cb.alpha, qv.v[1], rv.v[1]);
          v[1] = bmac(rv.v[1], rv.v[1], v[1]);
        }
        *reinterpret_cast<D2*>(r + k) = rv;
        if (r32) {
          if (la) r32[k] = static_cast<float>(rv.v[0] * ca.scale);
          if (lb) r32[k + 1] = static_cast<float>(rv.v[1] * cb.scale);
        }
      }
    }
  }
  block_cols_v<M>(v, none, part, nullptr, blk);
}

template <int M>
__global__ __launch_bounds__(kThreads) void bk_update_r(int32_t n, const BatchCol* __restrict__ col,
                                                        const double* __restrict__ q,
                                                        double* __restrict__ r,
                                                        float* __restrict__ r32,
                                                        double* __restrict__ part,
                                                        const BatchFlag* __restrict__ flag) {
  if (flag->all_done) return;
  BK_TILES(M, n)
  const BatchCol cc = col[c];
  double v = 0.0;
  if (!cc.done) {
    for (int t = t0; t < t1; ++t) {
      const int i = t * rb + threadIdx.x / M;
      if (i < n) {
        const int k = i * M + c;
        const double ri = bmac(-cc.alpha, q[k], r[k]);
        r[k] = ri;
        v = bmac(ri, ri, v);
        if (r32) r32[k] = static_cast<float>(ri * cc.scale);
      }
    }
  }
  block_cols<M>(v, 0.0, part, nullptr, blk);
}

template <bool D16, int M, typename WT>
__global__ __launch_bounds__(kThreads) void bk_residual_norm(const int32_t* __restrict__ sptr,
                                                             const void* __restrict__ colv,
                                                             const WT* __restrict__ w,
                                                             const double* __restrict__ x,
                                                             const double* __restrict__ b,
                                                             double* __restrict__ part,
                                                             int32_t n) {
  BK_TILES(M, n)
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int row = t * rb + threadIdx.x / M;
    if (row < n) {
      const int k = row * M + c;
      double acc, d;
      brow<double, D16, M>(sptr, colv, w, x, row, c, n, x[k], acc, d);
      const double ri = b[k] - acc;
      v += ri * ri;
    }
  }
  block_cols<M>(v, 0.0, part, nullptr, blk);
}

// The solution step each column still has pending when the loop ends: x += alpha p.  The
// direction update takes the previous iteration's step (it reads p_old anyway), so after a
// column's last iteration its step is left for this kernel; alpha = 0 marks none pending
// (the start, a breakdown of the step length, and FIN_RNORM after this kernel).
template <int M>
__global__ __launch_bounds__(kThreads) void bk_apply_pending(int32_t n,
                                                             const BatchCol* __restrict__ col,
                                                             const double* __restrict__ p,
                                                             double* __restrict__ x) {
  BK_ROWCOL(M)
  if (row >= n) return;
  const double a = col[c].alpha;
  if (a == 0.0) return;
  const int k = row * M + c;
  x[k] = bmac(a, p[k], x[k]);
}

__global__ void bk_init(BatchCol* __restrict__ col, BatchFlag* __restrict__ flag, int M, int ncols,
                        double rtol, int32_t max_iter, double n_unknowns) {
  const int c = threadIdx.x;
  if (c < M) {
    BatchCol z = {};
    z.pq = 1.0;
    z.scale = 1.0;
    z.inv_scale = 1.0;
    z.rtol = rtol;
    z.max_iter = max_iter;
    z.n_unknowns = n_unknowns;
    // padding columns carry zeros and are finished from the start
    z.done = c < ncols ? 0 : 1;
    col[c] = z;
  }
  if (c == 0) {
    flag->all_done = ncols > 0 ? 0 : 1;
    flag->n_done = M - ncols;
  }
}

// One workgroup per column c: sum its nb partials part0[c nb ..] (and part1's) in a fixed
// order, then apply `op` to the column.  A column that becomes finished adds itself to
// flag->n_done; the workgroup that completes the count sets flag->all_done, which the later
// launches of the group test (a workgroup of this launch that misses it only finds its column
// finished).
__global__ __launch_bounds__(kFin) void bk_finalize(int op, int M, int nb,
                                                    const double* __restrict__ part0,
                                                    const double* __restrict__ part1,
                                                    BatchCol* __restrict__ col,
                                                    BatchFlag* __restrict__ flag, int force) {
  if (!force && flag->all_done) return;
  const int c = blockIdx.x;
  const double* __restrict__ p0 = part0 + static_cast<size_t>(c) * nb;
  const double* __restrict__ p1 = part1 ? part1 + static_cast<size_t>(c) * nb : nullptr;
  double a = 0.0, b = 0.0;
  // thread t sums partials t, t + kFin, ... in that order, four loads in flight at a time
  for (int base = threadIdx.x; base < nb; base += 4 * kFin) {
    double va[4], vb[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = base + q * kFin;
      const int ic = i < nb ? i : nb - 1;
      va[q] = p0[ic];
      vb[q] = p1 ? p1[ic] : 0.0;
      if (i >= nb) {
        va[q] = 0.0;
        vb[q] = 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      a += va[q];
      b += vb[q];
    }
  }
  __shared__ double sa[kFin], sb[kFin];
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  for (int h = kFin / 2; h > 0; h >>= 1) {
    __syncthreads();
    if (static_cast<int>(threadIdx.x) < h) {
      sa[threadIdx.x] += sa[threadIdx.x + h];
      sb[threadIdx.x] += sb[threadIdx.x + h];
    }
  }
  if (threadIdx.x != 0) return;
  a = sa[0];
  b = sb[0];
  BatchCol& cc = col[c];
  const int was_done = cc.done;
  const bool live = force || !was_done;
  if (live) {
    switch (op) {
      case bk::FIN_BNORM: {
        const double bn = sqrt(a);
        cc.bnorm = bn;
        cc.rnorm = bn;
        if (!isfinite(bn)) {
          cc.status = MG_ENONFINITE;
          cc.done = 1;
        } else if (bn == 0.0) {
          cc.status = MG_OK;
          cc.done = 1;
        } else {
          int e;
          frexp(bn / sqrt(cc.n_unknowns), &e);
          cc.scale = ldexp(1.0, -e);
          cc.inv_scale = ldexp(1.0, e);
        }
        break;
      }
      case bk::FIN_ALPHA_FCG:
        cc.pq = a;
        if (!(a > 0.0) || !isfinite(a) || !isfinite(b)) {
          cc.status = (isfinite(a) && isfinite(b)) ? MG_EBREAKDOWN : MG_ENONFINITE;
          cc.done = 1;
          cc.alpha = 0.0;
        } else {
          cc.alpha = b / a;
        }
        break;
      case bk::FIN_CHECK: {
        const double rn = sqrt(a);
        cc.rnorm = rn;
        cc.iters += 1;
        if (!isfinite(rn)) {
          cc.status = MG_ENONFINITE;
          cc.done = 1;
        } else if (rn <= cc.rtol * cc.bnorm) {
          cc.status = MG_OK;
          cc.done = 1;
        } else if (cc.iters >= cc.max_iter) {
          cc.status = MG_ENOCONV;
          cc.done = 1;
        }
        break;
      }
      case bk::FIN_BETA_FCG:
        cc.beta = -a / cc.pq;
        if (!isfinite(cc.beta)) {
          cc.status = MG_ENONFINITE;
          cc.done = 1;
        }
        break;
      case bk::FIN_MEAN:
        cc.mean = a / cc.n_unknowns;
        break;
      case bk::FIN_RNORM:
        // the exit work took the pending step first
        cc.true_rnorm = sqrt(a);
        cc.alpha = 0.0;
        break;
    }
  }
  if (!was_done && cc.done && atomicAdd(&flag->n_done, 1) == M - 1) flag->all_done = 1;
}

__global__ void bk_fill(uint32_t* __restrict__ p, size_t n) {
  const size_t i = static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) p[i] = 0u;
}

inline unsigned grid_for(int64_t items) {
  return static_cast<unsigned>((items + kThreads - 1) / kThreads);
}
inline unsigned row_blocks(int32_t n, int M) {
  const int rb = kThreads / M;
  return static_cast<unsigned>((n + rb - 1) / rb);
}
inline const void* colp(const Level& L) {
  return L.op.col16 ? static_cast<const void*>(L.op.col16) : static_cast<const void*>(L.op.col);
}

// Calls f(std::integral_constant<int, M>) for a power of two M in [1, 64].
template <typename F>
void with_m(int M, F&& f) {
  switch (M) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    case 32: f(std::integral_constant<int, 32>{}); break;
    case 64: f(std::integral_constant<int, 64>{}); break;
    default: throw std::invalid_argument("batch group width must be a power of two up to 64");
  }
}

// Calls f(w) with the weights T-arithmetic kernels read: the binary16 copy when every weight of
// the level is exactly a binary16 number, else FP32 for FP32 kernels, and for FP64 kernels too
// when every FP64 weight of the level equals its FP32 copy (the same values in every case).
template <typename T, typename F>
void with_wts(const Level& L, F&& f) {
  if (L.op.w_exact16) {
    f(reinterpret_cast<const Half16*>(L.op.w16));
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    f(static_cast<const float*>(L.op.w32));
  } else {
    if (L.op.w_exact32)
      f(static_cast<const float*>(L.op.w32));
    else
      f(static_cast<const double*>(L.op.w64));
  }
}
template <typename P>
using pointee = std::remove_const_t<std::remove_pointer_t<P>>;
template <typename T> const T* idiag_of(const Level& L);
template <> const double* idiag_of<double>(const Level& L) { return L.op.idiag64; }
template <> const float* idiag_of<float>(const Level& L) { return L.op.idiag32; }

}  // namespace

namespace bk {

int red_blocks(int32_t n, int M) {
  const int rb = kThreads / M;
  const int tiles = (n + rb - 1) / rb;
  return std::max(1, std::min(kMaxRed, tiles));
}

void init_cols(BatchCol* col, BatchFlag* flag, int M, int ncols, double rtol, int32_t max_iter,
               double n_unknowns, hipStream_t s) {
  hipLaunchKernelGGL(bk_init, dim3(1), dim3(64), 0, s, col, flag, M, ncols, rtol, max_iter,
                     n_unknowns);
}

void finalize(int op, int M, int nb, const double* part0, const double* part1, BatchCol* col,
              BatchFlag* flag, int force, hipStream_t s) {
  hipLaunchKernelGGL(bk_finalize, dim3(M), dim3(kFin), 0, s, op, M, nb, part0, part1, col, flag,
                     force);
}

void gather_in(int M, int ncols, const int32_t* perm, int32_t n, const double* const* bptr,
               double* Bv, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_gather_in<MM>, dim3(grid_for(int64_t(n) * MM)), dim3(kThreads), 0, s,
                       perm, n, bptr, Bv, ncols);
  });
}

void scatter_out(int M, int ncols, const int32_t* perm, int32_t n, const int32_t* bnd,
                 int32_t nbnd, const double* Xv, const double* const* bptr, double* const* xptr,
                 hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_scatter_out<MM>, dim3(grid_for(int64_t(n) * MM)), dim3(kThreads), 0, s,
                       perm, n, Xv, xptr, ncols);
    if (nbnd > 0)
      hipLaunchKernelGGL(bk_bnd_copy<MM>, dim3(grid_for(int64_t(nbnd) * MM)), dim3(kThreads), 0, s,
                         bnd, nbnd, bptr, xptr, ncols);
  });
}

void nat_sumsq(int M, int ncols, int32_t nv, const double* const* bptr, double* part, int nb,
               hipStream_t s) {
  hipLaunchKernelGGL(bk_nat_sumsq, dim3(nb, M), dim3(kThreads), 0, s, M, ncols, nv, bptr, part);
}

void colsum(int M, int32_t n, const double* v, double* part, int nb, const BatchFlag* flag,
            hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_colsum<MM>, dim3(nb), dim3(kThreads), 0, s, n, v, part, flag);
  });
}

void colsum32(int M, int32_t n, const float* v, const BatchCol* col, double* part, int nb,
              const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_colsum32<MM>, dim3(nb), dim3(kThreads), 0, s, n, v, col, part, flag);
  });
}

void sub_mean(int M, int32_t n, const BatchCol* col, double* v, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_sub_mean<MM>, dim3(grid_for(int64_t(n) * MM)), dim3(kThreads), 0, s, n,
                       col, v);
  });
}

void dot(int M, int32_t n, const double* a, const double* b, double* part, int nb,
         const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_dot<MM>, dim3(nb), dim3(kThreads), 0, s, n, a, b, part, flag);
  });
}

void start(int M, int32_t n, const BatchCol* col, const double* Bv, double* X, double* R,
           double* P, double* Q, float* r32, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_start<MM>, dim3(grid_for(int64_t(n) * MM)), dim3(kThreads), 0, s, n, col,
                       Bv, X, R, P, Q, r32);
  });
}

template <typename T>
void zdot(int M, int32_t n, const BatchCol* col, const T* z, const double* q, double* part, int nb,
          int sub_mean, const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kKV)
      hipLaunchKernelGGL((bk_zdot_v<T, MM>), dim3(nb), dim3(kThreads), 0, s, n, col, z, q, part,
                         sub_mean, flag);
    else
      hipLaunchKernelGGL((bk_zdot<T, MM>), dim3(nb), dim3(kThreads), 0, s, n, col, z, q, part,
                         sub_mean, flag);
  });
}

template <typename T>
void pupd(int M, int32_t n, const BatchCol* col, const T* z, double* p, double* x, int sub_mean,
          const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kKV) {
      constexpr int RBV = kThreads / (MM / kKV);
      hipLaunchKernelGGL((bk_pupd_v<T, MM>), dim3(unsigned((int64_t(n) + RBV - 1) / RBV)),
                         dim3(kThreads), 0, s, n, col, z, p, x, sub_mean, flag);
    } else {
      hipLaunchKernelGGL((bk_pupd<T, MM>), dim3(row_blocks(n, MM)), dim3(kThreads), 0, s, n, col,
                         z, p, x, sub_mean, flag);
    }
  });
}

void spmv_dot2(int M, const Level& L, const double* p, double* q, const double* r, double* part0,
               double* part1, int nb, const BatchFlag* flag, hipStream_t s) {
  if (M >= kKV) {
    with_m(M, [&](auto mc) {
      constexpr int MM = decltype(mc)::value;
      if constexpr (MM >= kKV) {
        with_wts<double>(L, [&](auto w) {
          using WT = pointee<decltype(w)>;
          if (L.op.col16)
            hipLaunchKernelGGL((bk_spmv_dot2_v<true, MM, WT>), dim3(nb), dim3(kThreads), 0, s,
                               L.op.sptr, colp(L), w, p, q, r, part0, part1, L.n, flag);
          else
            hipLaunchKernelGGL((bk_spmv_dot2_v<false, MM, WT>), dim3(nb), dim3(kThreads), 0, s,
                               L.op.sptr, colp(L), w, p, q, r, part0, part1, L.n, flag);
        });
      }
    });
    return;
  }
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    with_wts<double>(L, [&](auto w) {
      using WT = pointee<decltype(w)>;
      if (L.op.col16)
        hipLaunchKernelGGL((bk_spmv_dot2<true, MM, WT>), dim3(nb), dim3(kThreads), 0, s, L.op.sptr,
                           colp(L), w, p, q, r, part0, part1, L.n, flag);
      else
        hipLaunchKernelGGL((bk_spmv_dot2<false, MM, WT>), dim3(nb), dim3(kThreads), 0, s,
                           L.op.sptr, colp(L), w, p, q, r, part0, part1, L.n, flag);
    });
  });
}

void update_r(int M, int32_t n, const BatchCol* col, const double* q, double* r, float* r32,
              double* part, int nb, const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kKV)
      hipLaunchKernelGGL(bk_update_r_v<MM>, dim3(nb), dim3(kThreads), 0, s, n, col, q, r, r32,
                         part, flag);
    else
      hipLaunchKernelGGL(bk_update_r<MM>, dim3(nb), dim3(kThreads), 0, s, n, col, q, r, r32, part,
                         flag);
  });
}

void apply_pending(int M, int32_t n, const BatchCol* col, const double* p, double* x,
                   hipStream_t s) {
  if (n == 0) return;
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL(bk_apply_pending<MM>, dim3(row_blocks(n, MM)), dim3(kThreads), 0, s, n, col,
                       p, x);
  });
}

void residual_norm(int M, const Level& L, const double* x, const double* b, double* part, int nb,
                   hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    with_wts<double>(L, [&](auto w) {
      using WT = pointee<decltype(w)>;
      if (L.op.col16)
        hipLaunchKernelGGL((bk_residual_norm<true, MM, WT>), dim3(nb), dim3(kThreads), 0, s,
                           L.op.sptr, colp(L), w, x, b, part, L.n);
      else
        hipLaunchKernelGGL((bk_residual_norm<false, MM, WT>), dim3(nb), dim3(kThreads), 0, s,
                           L.op.sptr, colp(L), w, x, b, part, L.n);
    });
  });
}

template <typename T>
void rows(int mode, int M, const Level& L, const T* x, const T* b, T* y, double omega,
          const BatchFlag* flag, hipStream_t s) {
  if (M >= kVW<T>) {
    with_m(M, [&](auto mc) {
      constexpr int MM = decltype(mc)::value;
      if constexpr (MM >= kVW<T>) {
        constexpr int RB = kThreads / (MM / kVW<T>);
        const dim3 g(unsigned((int64_t(L.n) + RB - 1) / RB));
        const T om = static_cast<T>(omega);
        const bool d16 = L.op.col16 != nullptr;
        with_wts<T>(L, [&](auto w) {
          using WT = pointee<decltype(w)>;
#define BK_ROWSV_LAUNCH(MODE)                                                                     \
  if (d16)                                                                                        \
    hipLaunchKernelGGL((bk_rows_v<T, MODE, true, MM, WT>), g, dim3(kThreads), 0, s, L.op.sptr,     \
                       colp(L), w, x, b, y, L.n, om, flag);                                       \
  else                                                                                            \
    hipLaunchKernelGGL((bk_rows_v<T, MODE, false, MM, WT>), g, dim3(kThreads), 0, s, L.op.sptr,    \
                       colp(L), w, x, b, y, L.n, om, flag);
          if (mode == 0) {
            BK_ROWSV_LAUNCH(0)
          } else if (mode == 1) {
            BK_ROWSV_LAUNCH(1)
          } else {
            BK_ROWSV_LAUNCH(2)
          }
#undef BK_ROWSV_LAUNCH
        });
      }
    });
    return;
  }
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    const dim3 g(row_blocks(L.n, MM));
    const T om = static_cast<T>(omega);
    const bool d16 = L.op.col16 != nullptr;
    with_wts<T>(L, [&](auto w) {
      using WT = pointee<decltype(w)>;
#define BK_ROWS_LAUNCH(MODE)                                                                     \
  if (d16)                                                                                       \
    hipLaunchKernelGGL((bk_rows<T, MODE, true, MM, WT>), g, dim3(kThreads), 0, s, L.op.sptr,      \
                       colp(L), w, x, b, y, L.n, om, flag);                                      \
  else                                                                                           \
    hipLaunchKernelGGL((bk_rows<T, MODE, false, MM, WT>), g, dim3(kThreads), 0, s, L.op.sptr,     \
                       colp(L), w, x, b, y, L.n, om, flag);
      if (mode == 0) {
        BK_ROWS_LAUNCH(0)
      } else if (mode == 1) {
        BK_ROWS_LAUNCH(1)
      } else {
        BK_ROWS_LAUNCH(2)
      }
#undef BK_ROWS_LAUNCH
    });
  });
}

template <typename T>
void jacobi_zero(int M, const Level& L, const T* b, T* y, double omega, const BatchFlag* flag,
                 hipStream_t s) {
  if (M >= kVW<T>) {
    with_m(M, [&](auto mc) {
      constexpr int MM = decltype(mc)::value;
      if constexpr (MM >= kVW<T>) {
        constexpr int RB = kThreads / (MM / kVW<T>);
        hipLaunchKernelGGL((bk_jacobi_zero_v<T, MM>), dim3(unsigned((int64_t(L.n) + RB - 1) / RB)),
                           dim3(kThreads), 0, s, idiag_of<T>(L), b, y, L.n,
                           static_cast<T>(omega), flag);
      }
    });
    return;
  }
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL((bk_jacobi_zero<T, MM>), dim3(row_blocks(L.n, MM)), dim3(kThreads), 0, s,
                       idiag_of<T>(L), b, y, L.n, static_cast<T>(omega), flag);
  });
}

template <typename T>
void restrict_(int M, const Level& Lf, const Level& Lc, const T* rf, T* rc, const BatchFlag* flag,
               hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kVW<T>) {
      constexpr int RB = kThreads / (MM / kVW<T>);
      hipLaunchKernelGGL((bk_restrict_v<T, MM>), dim3(unsigned((int64_t(Lc.n) + RB - 1) / RB)),
                         dim3(kThreads), 0, s, Lf.tr.r_self, Lf.tr.r_sptr, Lf.tr.r_col, rf, rc,
                         Lc.n, flag);
    } else {
      hipLaunchKernelGGL((bk_restrict<T, MM>), dim3(row_blocks(Lc.n, MM)), dim3(kThreads), 0, s,
                         Lf.tr.r_self, Lf.tr.r_sptr, Lf.tr.r_col, rf, rc, Lc.n, flag);
    }
  });
}

template <typename T>
void prolong(int M, const Level& Lf, const Level& Lc, const T* ec, T* xf, const BatchFlag* flag,
             hipStream_t s) {
  (void)Lc;
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kVW<T>) {
      constexpr int RB = kThreads / (MM / kVW<T>);
      hipLaunchKernelGGL((bk_prolong_v<T, MM>), dim3(unsigned((int64_t(Lf.n) + RB - 1) / RB)),
                         dim3(kThreads), 0, s, Lf.tr.pa, Lf.tr.pb, ec, xf, Lf.n, flag);
    } else {
      hipLaunchKernelGGL((bk_prolong<T, MM>), dim3(row_blocks(Lf.n, MM)), dim3(kThreads), 0, s,
                         Lf.tr.pa, Lf.tr.pb, ec, xf, Lf.n, flag);
    }
  });
}

template <typename T>
void prolong_sweep(int M, const Level& Lf, const T* ec, const T* x, const T* b, T* y,
                   double omega, const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    if constexpr (MM >= kVW<T>) {
      constexpr int RB = kThreads / (MM / kVW<T>);
      const dim3 gv(unsigned((int64_t(Lf.n) + RB - 1) / RB));
      with_wts<T>(Lf, [&](auto w) {
        using WT = pointee<decltype(w)>;
        if (Lf.op.col16)
          hipLaunchKernelGGL((bk_prolong_sweep_v<T, true, MM, WT>), gv, dim3(kThreads), 0, s,
                             Lf.op.sptr, colp(Lf), w, Lf.tr.pa, Lf.tr.pb, ec, x, b, y, Lf.n,
                             static_cast<T>(omega), flag);
        else
          hipLaunchKernelGGL((bk_prolong_sweep_v<T, false, MM, WT>), gv, dim3(kThreads), 0, s,
                             Lf.op.sptr, colp(Lf), w, Lf.tr.pa, Lf.tr.pb, ec, x, b, y, Lf.n,
                             static_cast<T>(omega), flag);
      });
      return;
    }
    const dim3 g(row_blocks(Lf.n, MM));
    with_wts<T>(Lf, [&](auto w) {
      using WT = pointee<decltype(w)>;
      if (Lf.op.col16)
        hipLaunchKernelGGL((bk_prolong_sweep<T, true, MM, WT>), g, dim3(kThreads), 0, s,
                           Lf.op.sptr, colp(Lf), w, Lf.tr.pa, Lf.tr.pb, ec, x, b, y, Lf.n,
                           static_cast<T>(omega), flag);
      else
        hipLaunchKernelGGL((bk_prolong_sweep<T, false, MM, WT>), g, dim3(kThreads), 0, s,
                           Lf.op.sptr, colp(Lf), w, Lf.tr.pa, Lf.tr.pb, ec, x, b, y, Lf.n,
                           static_cast<T>(omega), flag);
    });
  });
}

template <typename T>
void coarse(int M, const Hierarchy& H, const T* b, T* x, const BatchFlag* flag, hipStream_t s) {
  with_m(M, [&](auto mc) {
    constexpr int MM = decltype(mc)::value;
    hipLaunchKernelGGL((bk_coarse<T, MM>), dim3(grid_for(int64_t(H.n0) * MM)), dim3(kThreads), 0,
                       s, H.coarse_inv, b, x, H.n0, flag);
  });
}

void zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / sizeof(uint32_t);
  if (n) hipLaunchKernelGGL(bk_fill, dim3(grid_for(int64_t(n))), dim3(kThreads), 0, s,
                            static_cast<uint32_t*>(p), n);
}

template void zdot<float>(int, int32_t, const BatchCol*, const float*, const double*, double*, int,
                          int, const BatchFlag*, hipStream_t);
template void zdot<double>(int, int32_t, const BatchCol*, const double*, const double*, double*,
                           int, int, const BatchFlag*, hipStream_t);
template void pupd<float>(int, int32_t, const BatchCol*, const float*, double*, double*, int,
                          const BatchFlag*, hipStream_t);
template void pupd<double>(int, int32_t, const BatchCol*, const double*, double*, double*, int,
                           const BatchFlag*, hipStream_t);
template void rows<float>(int, int, const Level&, const float*, const float*, float*, double,
                          const BatchFlag*, hipStream_t);
template void rows<double>(int, int, const Level&, const double*, const double*, double*, double,
                           const BatchFlag*, hipStream_t);
template void jacobi_zero<float>(int, const Level&, const float*, float*, double, const BatchFlag*,
                                 hipStream_t);
template void jacobi_zero<double>(int, const Level&, const double*, double*, double,
                                  const BatchFlag*, hipStream_t);
template void restrict_<float>(int, const Level&, const Level&, const float*, float*,
                               const BatchFlag*, hipStream_t);
template void restrict_<double>(int, const Level&, const Level&, const double*, double*,
                                const BatchFlag*, hipStream_t);
template void prolong<float>(int, const Level&, const Level&, const float*, float*,
                             const BatchFlag*, hipStream_t);
template void prolong<double>(int, const Level&, const Level&, const double*, double*,
                              const BatchFlag*, hipStream_t);
template void prolong_sweep<float>(int, const Level&, const float*, const float*, const float*,
                                   float*, double, const BatchFlag*, hipStream_t);
template void prolong_sweep<double>(int, const Level&, const double*, const double*,
                                    const double*, double*, double, const BatchFlag*, hipStream_t);
template void coarse<float>(int, const Hierarchy&, const float*, float*, const BatchFlag*,
                            hipStream_t);
template void coarse<double>(int, const Hierarchy&, const double*, double*, const BatchFlag*,
                             hipStream_t);

}  // namespace bk
}  // namespace decmg
