// HIP kernels of the DEC multigrid path for CDNA4 (gfx950).
//
// Every stage is a sparse, memory-bound gather, so nothing here uses MFMA.  Rows map one to
// a lane of a 64-wide wavefront; the operator is stored as SELL-64 so that the index and
// weight streams of a wavefront are single coalesced 256/512-byte loads per column.  Row
// blocks are remapped so that each XCD (the hardware hands workgroups to the 8 XCDs in
// turn) walks one contiguous range of rows and its neighbour gathers stay in its own L2.
// Reductions are deterministic: wavefront butterflies, a fixed-order combine of the four
// wavefronts, per-block partials, then one fixed-order finalisation block.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include <algorithm>
#include <cmath>

#include "half16.hpp"
#include "hier.hpp"
#include "util.hpp"

namespace decmg {
namespace {

__device__ __forceinline__ int xcd_block_of(int b, int g) {
  const int x = b & 7, i = b >> 3, q = g >> 3, r = g & 7;
  return x * q + (x < r ? x : r) + i;
}
__device__ __forceinline__ int xcd_block() { return xcd_block_of(blockIdx.x, gridDim.x); }

// Reduction kernels run a capped grid; logical block b walks a contiguous range of 256-row
// tiles so the number of partial sums stays small.
__device__ __forceinline__ void tile_range(int ntiles, int blk, int& t0, int& t1) {
  const int g = gridDim.x;
  t0 = static_cast<int>(static_cast<int64_t>(ntiles) * blk / g);
  t1 = static_cast<int>(static_cast<int64_t>(ntiles) * (blk + 1) / g);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block of kBlock threads: returns the block total in thread 0 (fixed order).
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[kBlock / 64], sb[kBlock / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) {
      ta += sa[i];
      tb += sb[i];
    }
    a = ta;
    b = tb;
  }
}

__device__ __forceinline__ double block_sum1(double a) {
  double b = 0.0;
  block_sum2(a, b);
  return a;
}

// Column of SELL entry idx in row `row`: absolute int32 ids, or (D16) 16-bit offsets from
// the row with kZeroSlot16 marking the zero slot n.
template <bool D16>
__device__ __forceinline__ int col_at(const void* __restrict__ col, int idx, int row, int n) {
  if (D16) {
    const int c = static_cast<const int16_t*>(col)[idx];
    return c == kZeroSlot16 ? n : row + c;
  }
  return static_cast<const int32_t*>(col)[idx];
}

// a * b + c with one rounding.  Every operator row accumulates its entries through this, so a
// row's result does not depend on which products the compiler happens to contract (it leaves
// a product unfused where accumulators of several code paths merge), and the fused cycle legs
// reproduce the per-step kernels bit for bit.
__device__ __forceinline__ double mac(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float mac(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// First Jacobi sweep from zero at one row: omega b (1/D), rounded on its own.  Contraction is
// off here so that the product is never folded into a caller's subtraction: the fused legs
// hold this value in LDS, the per-step kernels recompute it at each neighbour, and both must
// see the same rounded number.
template <typename T>
__device__ __forceinline__ T jacobi_first(T omega, T b, T idiag) {
#pragma clang fp contract(off)
  return omega * b * idiag;
}

// sum_k w_k e_k over the three parents of a weighted interpolation, in parent order with one
// rounding per term
template <typename T>
__device__ __forceinline__ T interp3(T wa, T wb, T wc, T ea, T eb, T ec) {
  return mac(wc, ec, mac(wb, eb, wa * ea));
}

// Column and weight of SELL entry idx of `row`; the weight array is FP64, FP32 or binary16,
// widened to T exactly.
template <typename T, bool D16, typename WT>
__device__ __forceinline__ void entry_at(const void* __restrict__ col, const WT* __restrict__ w,
                                         int idx, int row, int n, int& c, T& wk) {
  c = col_at<D16>(col, idx, row, n);
  wk = static_cast<T>(w[idx]);
}
// The weight of SELL entry idx.
template <typename T, typename WT>
__device__ __forceinline__ T weight_at(const WT* __restrict__ w, int idx) {
  return static_cast<T>(w[idx]);
}

// Launch-bound kernels (n <= kLaunchBoundRows) issue the load of the convergence flag with their
// other first loads and test it only before their stores, which takes a dependent memory round
// trip off their critical path; large launches test it first, so a replay after convergence
// costs one flag read instead of a pass over the data.
#define DECMG_DONE_LOAD(n)                    \
  const int dn_ = done ? *done : 0;           \
  if ((n) > kLaunchBoundRows && dn_) return;
#define DECMG_DONE_CHECK() \
  if (dn_) return;

// Slice bounds of the wavefront holding `row`.  All 64 lanes of a wavefront share one slice,
// so the bounds are scalar loads and the entry loop below has a wave-uniform trip count.  A
// level whose slices all have the same width (uw >= 0) needs no load at all.
__device__ __forceinline__ void slice_bounds(const int32_t* __restrict__ sptr, int uw, int row,
                                             int& beg, int& width) {
  const int s = __builtin_amdgcn_readfirstlane(row >> 6);
  if (uw >= 0) {   // uniform width (ELL): no load
    beg = s * uw;
    width = uw;
  } else {
    beg = sptr[s];
    width = sptr[s + 1] - beg;
  }
}

// acc = sum_k w_k (x_i - x_j(k)) and d = sum_k w_k over the row's SELL entries, in entry
// order.  The entry count is wave-uniform, so a scalar switch picks a fully unrolled body
// that issues all index and weight loads, then all gathers: a wavefront waits on two memory
// round trips instead of two per entry.
template <typename T, bool D16, int N, typename WT>
__device__ __forceinline__ void row_apply_n(const void* __restrict__ col, const WT* __restrict__ w,
                                            const T* __restrict__ x, int beg, int lane, int row,
                                            int n, T xi, T& acc, T& d) {
  int cj[N];
  T wk[N], xj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, cj[k], wk[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) xj[k] = x[cj[k]];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d += wk[k];
    acc = mac(wk[k], xi - xj[k], acc);
  }
}

template <typename T, bool D16, typename WT>
__device__ __forceinline__ void row_apply(const int32_t* __restrict__ sptr, int uw,
                                          const void* __restrict__ col,
                                          const WT* __restrict__ w, const T* __restrict__ x,
                                          int row, int n, T xi, T& acc, T& d) {
  int beg, width;
  slice_bounds(sptr, uw, row, beg, width);
  const int lane = row & 63;
  acc = T(0);
  d = T(0);
  switch (width) {
    case 0: break;
    case 1: row_apply_n<T, D16, 1>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 2: row_apply_n<T, D16, 2>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 3: row_apply_n<T, D16, 3>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 4: row_apply_n<T, D16, 4>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 5: row_apply_n<T, D16, 5>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 6: row_apply_n<T, D16, 6>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 7: row_apply_n<T, D16, 7>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    case 8: row_apply_n<T, D16, 8>(col, w, x, beg, lane, row, n, xi, acc, d); break;
    default:
      for (int k = 0; k < width; ++k) {
        int j;
        T wk;
        entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, j, wk);
        d += wk;
        acc = mac(wk, xi - x[j], acc);
      }
  }
}

// Same batching for the first two sweeps from zero: gathers b and 1/D instead of x.
template <typename T, bool D16, int N, typename WT>
__device__ __forceinline__ void row_two_n(const void* __restrict__ col, const WT* __restrict__ w,
                                          const T* __restrict__ b, const T* __restrict__ idiag,
                                          int beg, int lane, int row, int n, T omega, T xi,
                                          T& acc, T& d) {
  int cj[N];
  T wk[N], bj[N], dj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, cj[k], wk[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    bj[k] = b[cj[k]];
    dj[k] = idiag[cj[k]];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d += wk[k];
    acc = mac(wk[k], xi - jacobi_first(omega, bj[k], dj[k]), acc);
  }
}

// Batched restriction row: sum of the N midpoint values.
template <typename T, int N>
__device__ __forceinline__ T restrict_n(const int32_t* __restrict__ col, const T* __restrict__ rf,
                                        int beg, int lane) {
  int cj[N];
  T v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) cj[k] = col[(beg + k) * kSlice + lane];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = rf[cj[k]];
  T acc = T(0);
#pragma unroll
  for (int k = 0; k < N; ++k) acc += v[k];
  return acc;
}

// The first two smoothing sweeps from x = 0 in one pass: the first sweep is local
// (x1 = omega b (1/D)), so the second reads b and 1/D at the neighbours instead of x1.  The
// expressions are those of k_jacobi_zero and k_rows<T,2>, so the result is the same.  The
// zero slot of 1/D holds 1, making x1 there 0.
template <typename T, bool D16, typename WT = T>
__global__ __launch_bounds__(kBlock) void k_jacobi_two(const int32_t* __restrict__ sptr, int32_t uw,
                                                       const void* __restrict__ col,
                                                       const WT* __restrict__ w,
                                                       const T* __restrict__ idiag,
                                                       const T* __restrict__ b,
                                                       T* __restrict__ y, int32_t n, T omega,
                                                       const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= n) return;
  int beg, width;
  slice_bounds(sptr, uw, row, beg, width);
  const int lane = row & 63;
  const T bi = b[row];
  const T xi = jacobi_first(omega, bi, idiag[row]);
  T acc = T(0), d = T(0);
  switch (width) {
    case 0: break;
    case 1: row_two_n<T, D16, 1>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 2: row_two_n<T, D16, 2>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 3: row_two_n<T, D16, 3>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 4: row_two_n<T, D16, 4>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 5: row_two_n<T, D16, 5>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 6: row_two_n<T, D16, 6>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 7: row_two_n<T, D16, 7>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    case 8: row_two_n<T, D16, 8>(col, w, b, idiag, beg, lane, row, n, omega, xi, acc, d); break;
    default:
      for (int k = 0; k < width; ++k) {
        int j;
        T wk;
        entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, j, wk);
        d += wk;
        acc = mac(wk, xi - jacobi_first(omega, b[j], idiag[j]), acc);
      }
  }
  DECMG_DONE_CHECK()
  y[row] = xi + omega * (bi - acc) / d;
}

// MODE 0: y = A x.  MODE 1: y = b - A x.  MODE 2: y = x + omega (b - A x) / D.
template <typename T, int MODE, bool D16, typename WT = T>
__global__ __launch_bounds__(kBlock) void k_rows(const int32_t* __restrict__ sptr, int32_t uw,
                                                 const void* __restrict__ col,
                                                 const WT* __restrict__ w,
                                                 const T* __restrict__ x,
                                                 const T* __restrict__ b, T* __restrict__ y,
                                                 int32_t n, T omega,
                                                 const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= n) return;
  const T xi = x[row];
  const T bi = (MODE == 0) ? T(0) : b[row];
  T acc, d;
  row_apply<T, D16>(sptr, uw, col, w, x, row, n, xi, acc, d);
  DECMG_DONE_CHECK()
  if (MODE == 0)
    y[row] = acc;
  else if (MODE == 1)
    y[row] = bi - acc;
  else
    y[row] = xi + omega * (bi - acc) / d;
}

// Two rows per thread, kBlock apart, on levels whose slices all have the width uw (ELL): each
// row's index, weight and vector loads are all issued before either row's gathers, so twice
// the bytes are in flight per wavefront (with binary16 weights the finest-level sweeps moved
// 28 B per row and their two dependent memory trips per wavefront were exposed).  Same
// expressions and entry order as the one-row kernels.  The second row of a thread past the end
// is its first row again (computed twice, stored once).
__device__ __forceinline__ int ell_first(int r, int uw) { return (r >> 6) * uw * kSlice + (r & 63); }
// Position of row r's first entry, and the step between its entries: in the SELL-64 arrays, or
// (PAT) in the table of row patterns, where pat[r] names the row's pattern and a pattern's uw
// entries are contiguous.  Pattern entries hold 16-bit offsets from the row and the weights,
// exactly as the SELL entries they replace.
template <bool PAT>
__device__ __forceinline__ int row_first(const uint8_t* __restrict__ pat, int r, int uw) {
  if constexpr (PAT)
    return static_cast<int>(pat[r]) * uw;
  else
    return ell_first(r, uw);
}
// The pattern table of a level in LDS (dynamic shared memory): npat uw 16-bit offsets, then,
// 8-byte aligned, npat uw weights of type WT.  Every thread of the block takes part; call before
// any thread leaves.
__host__ __device__ constexpr int pattern_lds_weights_at(int entries) { return (2 * entries + 7) / 8 * 8; }
template <typename WT>
__device__ __forceinline__ void stage_patterns(const int16_t* __restrict__ off,
                                               const WT* __restrict__ w, int entries,
                                               const int16_t*& soff, const WT*& sw) {
  extern __shared__ double pattern_smem[];
  char* base = reinterpret_cast<char*>(pattern_smem);
  int16_t* o = reinterpret_cast<int16_t*>(base);
  WT* v = reinterpret_cast<WT*>(base + pattern_lds_weights_at(entries));
  for (int i = threadIdx.x; i < entries; i += blockDim.x) {
    o[i] = off[i];
    v[i] = w[i];
  }
  __syncthreads();
  soff = o;
  sw = v;
}

template <typename T, bool D16, int N, bool PAT, typename WT, typename G>
__device__ __forceinline__ void row2_n(const void* __restrict__ col, const WT* __restrict__ w,
                                       int e0, int e1, int r0, int r1, int n, T x0, T x1,
                                       G&& other, T& a0, T& d0, T& a1, T& d1) {
  int c0[N], c1[N];
  T w0[N], w1[N], y0[N], y1[N];
  constexpr int st = PAT ? 1 : kSlice;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    entry_at<T, D16>(col, w, e0 + k * st, r0, n, c0[k], w0[k]);
    entry_at<T, D16>(col, w, e1 + k * st, r1, n, c1[k], w1[k]);
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    y0[k] = other(c0[k]);
    y1[k] = other(c1[k]);
  }
  a0 = d0 = a1 = d1 = T(0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d0 += w0[k];
    a0 = mac(w0[k], x0 - y0[k], a0);
    d1 += w1[k];
    a1 = mac(w1[k], x1 - y1[k], a1);
  }
}
// e0, e1: row_first of r0 and r1
template <typename T, bool D16, bool PAT, typename WT, typename G>
__device__ __forceinline__ void row2(const void* __restrict__ col, const WT* __restrict__ w,
                                     int e0, int e1, int r0, int r1, int uw, int n, T x0, T x1,
                                     G&& other, T& a0, T& d0, T& a1, T& d1) {
#define DECMG_R2(K)                                                                       \
  row2_n<T, D16, K, PAT>(col, w, e0, e1, r0, r1, n, x0, x1, other, a0, d0, a1, d1);         \
  break;
  switch (uw) {
    case 1: DECMG_R2(1)
    case 2: DECMG_R2(2)
    case 3: DECMG_R2(3)
    case 4: DECMG_R2(4)
    case 5: DECMG_R2(5)
    case 6: DECMG_R2(6)
    case 7: DECMG_R2(7)
    default: DECMG_R2(8)
  }
#undef DECMG_R2
}

// k_rows with two rows per thread (uniform widths 1..8 only)
template <typename T, int MODE, bool D16, typename WT, bool PAT>
__device__ __forceinline__ void rows2_body(int32_t uw, const void* __restrict__ col,
                                           const WT* __restrict__ w,
                                           const uint8_t* __restrict__ pat, int npat,
                                           const T* __restrict__ x, const T* __restrict__ b,
                                           T* __restrict__ y, int32_t n, T omega,
                                           const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int r0 = xcd_block() * (2 * kBlock) + threadIdx.x;
  const bool live = r0 < n;
  int r1 = 0, e0 = 0, e1 = 0;
  T x0 = T(0), x1 = T(0), b0 = T(0), b1 = T(0);
  if (live) {
    r1 = (r0 + kBlock < n) ? r0 + kBlock : r0;
    e0 = row_first<PAT>(pat, r0, uw);
    e1 = row_first<PAT>(pat, r1, uw);
    x0 = x[r0];
    x1 = x[r1];
    if (MODE != 0) {
      b0 = b[r0];
      b1 = b[r1];
    }
  }
  if constexpr (PAT) {   // the row loads above are in flight meanwhile
    const int16_t* so;
    const WT* sw;
    stage_patterns(static_cast<const int16_t*>(col), w, npat * uw, so, sw);
    col = so;
    w = sw;
  }
  if (!live) return;
  T a0, d0, a1, d1;
  row2<T, D16, PAT>(col, w, e0, e1, r0, r1, uw, n, x0, x1, [&](int j) { return x[j]; }, a0, d0,
                    a1, d1);
  DECMG_DONE_CHECK()
  if (MODE == 0) {
    y[r0] = a0;
    if (r1 != r0) y[r1] = a1;
  } else if (MODE == 1) {
    y[r0] = b0 - a0;
    if (r1 != r0) y[r1] = b1 - a1;
  } else {
    y[r0] = x0 + omega * (b0 - a0) / d0;
    if (r1 != r0) y[r1] = x1 + omega * (b1 - a1) / d1;
  }
}
template <typename T, int MODE, bool D16, typename WT>
__global__ __launch_bounds__(kBlock) void k_rows2(int32_t uw, const void* __restrict__ col,
                                                  const WT* __restrict__ w,
                                                  const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y,
                                                  int32_t n, T omega,
                                                  const int* __restrict__ done) {
  rows2_body<T, MODE, D16, WT, false>(uw, col, w, nullptr, 0, x, b, y, n, omega, done);
}
// The same over row patterns: pat[r] names row r's pattern, whose offsets and weights are
// entries pat[r] uw .. pat[r] uw + uw - 1 of off and w.  Same values in the same order as the
// SELL entries, so the same results bit for bit, from one byte per row instead of uw offsets
// and weights.
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_rows2p(int32_t uw, const int16_t* __restrict__ off,
                                                   const T* __restrict__ w,
                                                   const uint8_t* __restrict__ pat, int npat,
                                                   const T* __restrict__ x,
                                                   const T* __restrict__ b, T* __restrict__ y,
                                                   int32_t n, T omega,
                                                   const int* __restrict__ done) {
  rows2_body<T, MODE, true, T, true>(uw, off, w, pat, npat, x, b, y, n, omega, done);
}

// k_jacobi_two with two rows per thread (uniform widths 1..8 only)
template <typename T, bool D16, typename WT, bool PAT>
__device__ __forceinline__ void jacobi_two2_body(int32_t uw, const void* __restrict__ col,
                                                 const WT* __restrict__ w,
                                                 const uint8_t* __restrict__ pat, int npat,
                                                 const T* __restrict__ idiag,
                                                 const T* __restrict__ b, T* __restrict__ y,
                                                 int32_t n, T omega,
                                                 const int* __restrict__ done, int blk) {
  DECMG_DONE_LOAD(n)
  const int r0 = blk * (2 * kBlock) + threadIdx.x;
  const bool live = r0 < n;
  int r1 = 0, e0 = 0, e1 = 0;
  T b0 = T(0), b1 = T(0), i0 = T(1), i1 = T(1);
  if (live) {
    r1 = (r0 + kBlock < n) ? r0 + kBlock : r0;
    e0 = row_first<PAT>(pat, r0, uw);
    e1 = row_first<PAT>(pat, r1, uw);
    b0 = b[r0];
    b1 = b[r1];
    i0 = idiag[r0];
    i1 = idiag[r1];
  }
  if constexpr (PAT) {   // the row loads above are in flight meanwhile
    const int16_t* so;
    const WT* sw;
    stage_patterns(static_cast<const int16_t*>(col), w, npat * uw, so, sw);
    col = so;
    w = sw;
  }
  if (!live) return;
  const T x0 = jacobi_first(omega, b0, i0), x1 = jacobi_first(omega, b1, i1);
  T a0, d0, a1, d1;
  row2<T, D16, PAT>(col, w, e0, e1, r0, r1, uw, n, x0, x1,
                    [&](int j) { return jacobi_first(omega, b[j], idiag[j]); }, a0, d0, a1, d1);
  DECMG_DONE_CHECK()
  y[r0] = x0 + omega * (b0 - a0) / d0;
  if (r1 != r0) y[r1] = x1 + omega * (b1 - a1) / d1;
}
template <typename T, bool D16, typename WT>
__global__ __launch_bounds__(kBlock) void k_jacobi_two2(int32_t uw, const void* __restrict__ col,
                                                        const WT* __restrict__ w,
                                                        const T* __restrict__ idiag,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ y, int32_t n, T omega,
                                                        const int* __restrict__ done) {
  jacobi_two2_body<T, D16, WT, false>(uw, col, w, nullptr, 0, idiag, b, y, n, omega, done,
                                      xcd_block());
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_two2p(int32_t uw,
                                                         const int16_t* __restrict__ off,
                                                         const T* __restrict__ w,
                                                         const uint8_t* __restrict__ pat,
                                                         int npat,
                                                         const T* __restrict__ idiag,
                                                         const T* __restrict__ b,
                                                         T* __restrict__ y, int32_t n, T omega,
                                                         const int* __restrict__ done) {
  jacobi_two2_body<T, true, T, true>(uw, off, w, pat, npat, idiag, b, y, n, omega, done,
                                     xcd_block());
}


// First smoothing sweep from x = 0: x = omega b (1/D).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_zero(const T* __restrict__ idiag,
                                                        const T* __restrict__ b,
                                                        T* __restrict__ y, int32_t n, T omega,
                                                        const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= n) return;
  const T v = jacobi_first(omega, b[row], idiag[row]);
  DECMG_DONE_CHECK()
  y[row] = v;
}

// r_c = M(f) r_f: the kept vertex with weight 1, every midpoint of an incident coarse edge
// with weight 1/2.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict(const int32_t* __restrict__ self,
                                                     const int32_t* __restrict__ sptr, int32_t uw,
                                                     const int32_t* __restrict__ col,
                                                     const T* __restrict__ rf,
                                                     T* __restrict__ rc, int32_t nc,
                                                     const int* __restrict__ done) {
  DECMG_DONE_LOAD(nc)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= nc) return;
  int beg, width;
  slice_bounds(sptr, uw, row, beg, width);
  const int lane = row & 63;
  const T rs = rf[self[row]];
  T acc = T(0);
  switch (width) {
    case 0: break;
    case 1: acc = restrict_n<T, 1>(col, rf, beg, lane); break;
    case 2: acc = restrict_n<T, 2>(col, rf, beg, lane); break;
    case 3: acc = restrict_n<T, 3>(col, rf, beg, lane); break;
    case 4: acc = restrict_n<T, 4>(col, rf, beg, lane); break;
    case 5: acc = restrict_n<T, 5>(col, rf, beg, lane); break;
    case 6: acc = restrict_n<T, 6>(col, rf, beg, lane); break;
    case 7: acc = restrict_n<T, 7>(col, rf, beg, lane); break;
    case 8: acc = restrict_n<T, 8>(col, rf, beg, lane); break;
    default:
      for (int k = 0; k < width; ++k) acc += rf[col[(beg + k) * kSlice + lane]];
  }
  DECMG_DONE_CHECK()
  rc[row] = rs + T(0.5) * acc;
}

// k_restrict with two coarse rows per thread, rows r and r + kBlock, over 16-bit column offsets
// from the kept vertex (uniform widths 1..8): all index, kept-value and gather loads of both
// rows go out before either sum.  Same order of summation as k_restrict.
template <typename T, int N>
__device__ __forceinline__ void restrict2_n(const int16_t* __restrict__ col,
                                            const T* __restrict__ rf, int e0, int e1, int s0,
                                            int s1, int nf, T& a0, T& a1) {
  int c0[N], c1[N];
  T v0[N], v1[N];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const int o0 = col[e0 + k * kSlice], o1 = col[e1 + k * kSlice];
    c0[k] = o0 == kZeroSlot16 ? nf : s0 + o0;
    c1[k] = o1 == kZeroSlot16 ? nf : s1 + o1;
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    v0[k] = rf[c0[k]];
    v1[k] = rf[c1[k]];
  }
  a0 = T(0);
  a1 = T(0);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    a0 += v0[k];
    a1 += v1[k];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict2(const int32_t* __restrict__ self,
                                                      int32_t uw,
                                                      const int16_t* __restrict__ col,
                                                      const T* __restrict__ rf,
                                                      T* __restrict__ rc, int32_t nc, int32_t nf,
                                                      const int* __restrict__ done) {
  DECMG_DONE_LOAD(nc)
  const int r0 = xcd_block() * (2 * kBlock) + threadIdx.x;
  if (r0 >= nc) return;
  const int r1 = (r0 + kBlock < nc) ? r0 + kBlock : r0;
  const int s0 = self[r0], s1 = self[r1];
  const int e0 = ell_first(r0, uw), e1 = ell_first(r1, uw);
  const T rs0 = rf[s0], rs1 = rf[s1];
  T a0, a1;
  switch (uw) {
    case 1: restrict2_n<T, 1>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 2: restrict2_n<T, 2>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 3: restrict2_n<T, 3>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 4: restrict2_n<T, 4>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 5: restrict2_n<T, 5>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 6: restrict2_n<T, 6>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    case 7: restrict2_n<T, 7>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
    default: restrict2_n<T, 8>(col, rf, e0, e1, s0, s1, nf, a0, a1); break;
  }
  DECMG_DONE_CHECK()
  rc[r0] = rs0 + T(0.5) * a0;
  if (r1 != r0) rc[r1] = rs1 + T(0.5) * a1;
}

// First post-smoothing sweep fused with the interpolation of the coarse correction.  The
// corrected iterate x0 = x + M(f)^T e_c is formed on the fly, for the row and for each of its
// neighbours, with the rounding of k_prolong; then xo = x0 + omega (b - A x0) / diag.  The
// parent arrays have an entry for the zero slot (pointing at the coarse zero slot), so absent
// neighbours contribute x0 = 0 without a branch.
template <typename T, bool D16, int N, typename WT>
__device__ __forceinline__ void row_prolong_n(const void* __restrict__ col,
                                              const WT* __restrict__ w, const T* __restrict__ x,
                                              const int32_t* __restrict__ pa,
                                              const int32_t* __restrict__ pb,
                                              const T* __restrict__ ec, int beg, int lane,
                                              int row, int n, T xi0, T& acc, T& d) {
  int cj[N], ca[N], cb[N];
  T wk[N], xj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, cj[k], wk[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    xj[k] = x[cj[k]];
    ca[k] = pa[cj[k]];
    cb[k] = pb[cj[k]];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) xj[k] = xj[k] + T(0.5) * (ec[ca[k]] + ec[cb[k]]);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    d += wk[k];
    acc = mac(wk[k], xi0 - xj[k], acc);
  }
}

template <typename T, bool D16, typename WT = T>
__global__ __launch_bounds__(kBlock) void k_prolong_sweep(const int32_t* __restrict__ sptr, int32_t uw,
                                                          const void* __restrict__ col,
                                                          const WT* __restrict__ w,
                                                          const int32_t* __restrict__ pa,
                                                          const int32_t* __restrict__ pb,
                                                          const T* __restrict__ ec,
                                                          const T* __restrict__ x,
                                                          const T* __restrict__ b,
                                                          T* __restrict__ xo, int32_t n, T omega,
                                                          const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= n) return;
  const T xi0 = x[row] + T(0.5) * (ec[pa[row]] + ec[pb[row]]);
  const T bi = b[row];
  int beg, width;
  slice_bounds(sptr, uw, row, beg, width);
  const int lane = row & 63;
  T acc = T(0), d = T(0);
  switch (width) {
    case 0: break;
    case 1: row_prolong_n<T, D16, 1>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 2: row_prolong_n<T, D16, 2>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 3: row_prolong_n<T, D16, 3>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 4: row_prolong_n<T, D16, 4>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 5: row_prolong_n<T, D16, 5>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 6: row_prolong_n<T, D16, 6>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 7: row_prolong_n<T, D16, 7>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    case 8: row_prolong_n<T, D16, 8>(col, w, x, pa, pb, ec, beg, lane, row, n, xi0, acc, d); break;
    default:
      for (int k = 0; k < width; ++k) {
        int j;
        T wk;
        entry_at<T, D16>(col, w, (beg + k) * kSlice + lane, row, n, j, wk);
        const T xj = x[j] + T(0.5) * (ec[pa[j]] + ec[pb[j]]);
        d += wk;
        acc = mac(wk, xi0 - xj, acc);
      }
  }
  DECMG_DONE_CHECK()
  xo[row] = xi0 + omega * (bi - acc) / d;
}

// ------------------------------------------------------------------ fused smoothing tiles
// One workgroup per tile of a binary level (DevTiles): the values a leg of the cycle needs
// around the tile's own rows are recomputed in LDS, so the down leg takes one launch instead of
// three and the up leg one instead of two.  Each value is formed with the expressions and entry
// order of k_jacobi_two, k_rows, k_restrict and k_prolong_sweep, so the results equal theirs
// bit for bit.  A workgroup of TB threads holds rows t + q TB (q < Q) of its tile and up to CQ
// coarse rows per thread: index, weight and right-hand-side loads are all issued before the
// first barrier.  LDS: two vectors of cap + 1 values (dynamic).

// Row data of local row i: global row g, first SELL entry e0 and width, and (rows of R1) the
// weights and local columns of its entries.
template <typename T, typename WT, int KT>
__device__ __forceinline__ void tile_row(int g, int i, int cap, const int32_t* __restrict__ tent,
                                         int uw, const int16_t* __restrict__ tcol,
                                         const WT* __restrict__ w, int& wid, int (&cj)[KT],
                                         T (&wk)[KT]) {
  int e0;
  if (tent) {
    const int e = tent[i];
    e0 = e >> 4;
    wid = e & 15;
  } else {
    e0 = (g >> 6) * uw * kSlice + (g & 63);
    wid = uw;
  }
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    cj[k] = tcol[k * cap + i];
    wk[k] = (k < wid) ? weight_at<T>(w, e0 + k * kSlice) : T(0);
  }
}

template <int NT>
__device__ void fin_check_block(DevScalars* __restrict__ sc, const double* __restrict__ part,
                                int32_t nb);

template <typename T, typename WT, int KT, int TB, int Q, int CQ, bool WTR>
__global__ __launch_bounds__(TB) void k_tile_down(
    const int32_t* __restrict__ meta, const int32_t* __restrict__ trow,
    const int32_t* __restrict__ tent, const int16_t* __restrict__ tcol,
    const int32_t* __restrict__ tcrow, const int16_t* __restrict__ tcst, int32_t cap,
    int32_t ccap, int32_t uw, const WT* __restrict__ w, const T* __restrict__ idiag,
    const T* __restrict__ b, T* __restrict__ x, T* __restrict__ bc, T omega, int nu1,
    const int32_t* __restrict__ tcent, int32_t rws, const T* __restrict__ rw,
    const int* __restrict__ done, DevScalars* __restrict__ chk_sc,
    const double* __restrict__ chk_part, int32_t chk_nb) {
  // with chk_part: block 0 takes the Krylov loop's pending convergence check, the others the
  // tiles
  if (chk_part && blockIdx.x == 0) {
    fin_check_block<TB>(chk_sc, chk_part, chk_nb);
    return;
  }
  extern __shared__ double tile_smem[];
  T* s1 = reinterpret_cast<T*>(tile_smem);
  T* s2 = s1 + (cap + 1);
  const int dn = done ? *done : 0;
  const int tb = chk_part ? xcd_block_of(blockIdx.x - 1, gridDim.x - 1) : xcd_block();
  const int t = threadIdx.x;
  const int32_t* m = meta + 8 * tb;
  const int nF = m[0], n0 = m[1], n1 = m[2], n2 = m[3], ncb = m[4];
  const int nq = (cap + TB - 1) / TB;
  const int32_t* rows = trow + static_cast<int64_t>(tb) * cap;
  const int32_t* ents = tent ? tent + static_cast<int64_t>(tb) * cap : nullptr;
  const int16_t* cols = tcol + static_cast<int64_t>(tb) * KT * cap;
  int g[Q], wid[Q], cj[Q][KT];
  T wk[Q][KT], bq[Q], x1[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < cap) {
      g[q] = rows[i];
      tile_row<T, WT, KT>(g[q], i, cap, ents, uw, cols, w, wid[q], cj[q], wk[q]);
      bq[q] = b[g[q]];
      x1[q] = jacobi_first(omega, bq[q], idiag[g[q]]);
    }
  }
  // restriction rows: CQ per thread at most (ccap <= CQ TB); binary transfers keep their nine
  // local ids in registers, weighted ones read theirs when the residual is ready
  int crow[CQ], cs[CQ][9], ce[CQ];
#pragma unroll
  for (int c = 0; c < CQ; ++c) {
    const int j = min(t + c * TB, ccap - 1);
    crow[c] = tcrow[static_cast<int64_t>(tb) * ccap + j];
    if constexpr (WTR) {
      ce[c] = tcent[static_cast<int64_t>(tb) * ccap + j];
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) cs[c][k] = tcst[(static_cast<int64_t>(tb) * rws + k) * ccap + j];
    }
  }
  // x1 = omega b (1/D) on every local row (the first sweep from zero is local)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < n2) s1[i] = (nu1 >= 1) ? x1[q] : T(0);
  }
  if (t == 0) {
    s1[cap] = T(0);
    s2[cap] = T(0);
  }
  __syncthreads();
  // x2 on R1 (second sweep, k_jacobi_two), or x = 0 / x1 on R1
  if (nu1 == 2) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * TB;
      if (q < nq && i < n1) {
        const T xi = x1[q];
        T acc = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < KT; ++k)
          if (k < wid[q]) {
            d += wk[q][k];
            acc = mac(wk[q][k], xi - s1[cj[q][k]], acc);
          }
        s2[i] = xi + omega * (bq[q] - acc) / d;
      }
    }
    __syncthreads();
  }
  // residual on R0 (k_rows, mode 1) into the vector x no longer needs; own rows of x go out
  const T* xc = (nu1 == 2) ? s2 : s1;
  T* sr = (nu1 == 2) ? s1 : s2;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < n0) {
      const T xi = xc[i];
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < KT; ++k)
        if (k < wid[q]) acc = mac(wk[q][k], xi - xc[cj[q][k]], acc);
      sr[i] = bq[q] - acc;
      if (i < nF && !dn) x[g[q]] = xi;
    }
  }
  __syncthreads();
  // restriction of the residual onto the tile's coarse rows (k_restrict / k_restrict_w)
  if (dn) return;
#pragma unroll
  for (int c = 0; c < CQ; ++c)
    if (t + c * TB < ncb) {
      T acc = T(0);
      if constexpr (WTR) {
        // the coarse row's entries in SELL order: local fine ids here, weights at e0 + k 64
        const int j = t + c * TB, e0 = ce[c] >> 6, wd = ce[c] & 63;
        const int16_t* ids = tcst + static_cast<int64_t>(tb) * rws * ccap + j;
        for (int k = 0; k < wd; ++k) acc = mac(rw[e0 + k * kSlice], sr[ids[k * ccap]], acc);
        bc[crow[c]] = acc;
      } else {
#pragma unroll
        for (int k = 1; k < 9; ++k) acc += sr[cs[c][k]];
        bc[crow[c]] = sr[cs[c][0]] + T(0.5) * acc;
      }
    }
}

template <typename T, typename WT, int KT, int TB, int Q, bool WTR>
__global__ __launch_bounds__(TB) void k_tile_up(
    const int32_t* __restrict__ meta, const int32_t* __restrict__ trow,
    const int32_t* __restrict__ tent, const int16_t* __restrict__ tcol, int32_t cap,
    int32_t uw, const WT* __restrict__ w, const int32_t* __restrict__ pa,
    const int32_t* __restrict__ pb, const T* __restrict__ ec, const T* __restrict__ x,
    const T* __restrict__ b, T* __restrict__ xo, T omega, int nu2,
    const int32_t* __restrict__ p3, const T* __restrict__ pw, const int* __restrict__ done) {
  extern __shared__ double tile_smem[];
  T* s0 = reinterpret_cast<T*>(tile_smem);
  T* s1 = s0 + (cap + 1);
  const int dn = done ? *done : 0;
  const int tb = xcd_block(), t = threadIdx.x;
  const int32_t* m = meta + 8 * tb;
  const int nF = m[0], n1 = m[2], n2 = m[3];
  const int nq = (cap + TB - 1) / TB;
  const int32_t* rows = trow + static_cast<int64_t>(tb) * cap;
  const int32_t* ents = tent ? tent + static_cast<int64_t>(tb) * cap : nullptr;
  const int16_t* cols = tcol + static_cast<int64_t>(tb) * KT * cap;
  int g[Q], wid[Q], cj[Q][KT];
  T wk[Q][KT], bq[Q], xq[Q];
  int ia[Q], ib[Q], ic[Q];
  T wa[Q], wb[Q], wc[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < cap) {
      g[q] = rows[i];
      tile_row<T, WT, KT>(g[q], i, cap, ents, uw, cols, w, wid[q], cj[q], wk[q]);
      bq[q] = b[g[q]];
      xq[q] = x[g[q]];
      if constexpr (WTR) {
        const int64_t o = 3 * static_cast<int64_t>(g[q]);
        ia[q] = p3[o];
        ib[q] = p3[o + 1];
        ic[q] = p3[o + 2];
        wa[q] = pw[o];
        wb[q] = pw[o + 1];
        wc[q] = pw[o + 2];
      } else {
        ia[q] = pa[g[q]];
        ib[q] = pb[g[q]];
      }
    }
  }
  // x0 = x + M(f)^T ec on every local row (k_prolong_sweep's / k_prolong3's rounding)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < n2) {
      if constexpr (WTR)
        xq[q] = xq[q] + interp3(wa[q], wb[q], wc[q], ec[ia[q]], ec[ib[q]], ec[ic[q]]);
      else
        xq[q] = xq[q] + T(0.5) * (ec[ia[q]] + ec[ib[q]]);
      s0[i] = xq[q];
    }
  }
  if (t == 0) {
    s0[cap] = T(0);
    s1[cap] = T(0);
  }
  __syncthreads();
  // first sweep on R1 (k_prolong_sweep)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < n1) {
      const T xi = xq[q];
      T acc = T(0), d = T(0);
#pragma unroll
      for (int k = 0; k < KT; ++k)
        if (k < wid[q]) {
          d += wk[q][k];
          acc = mac(wk[q][k], xi - s0[cj[q][k]], acc);
        }
      xq[q] = xi + omega * (bq[q] - acc) / d;
      s1[i] = xq[q];
    }
  }
  if (nu2 == 2) {
    __syncthreads();
    // second sweep on the tile's own rows (k_rows, mode 2)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = t + q * TB;
      if (q < nq && i < nF) {
        const T xi = xq[q];
        T acc = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < KT; ++k)
          if (k < wid[q]) {
            d += wk[q][k];
            acc = mac(wk[q][k], xi - s1[cj[q][k]], acc);
          }
        xq[q] = xi + omega * (bq[q] - acc) / d;
      }
    }
  }
  if (dn) return;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = t + q * TB;
    if (q < nq && i < nF) xo[g[q]] = xq[q];
  }
}

// ------------------------------------------------------------------ CG smoother
// p = r, partial r.r
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_start(int32_t n, const T* __restrict__ r,
                                                      T* __restrict__ p, double* __restrict__ part,
                                                      const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  const int i = blk * kBlock + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const T ri = r[i];
    p[i] = ri;
    v = static_cast<double>(ri) * static_cast<double>(ri);
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part[blk] = v;
}

// q = A p, partial p.q
template <typename T, bool D16, typename WT>
__global__ __launch_bounds__(kBlock) void k_cgs_spmv_dot(const int32_t* __restrict__ sptr,
                                                         int32_t uw, const void* __restrict__ col,
                                                         const WT* __restrict__ w,
                                                         const T* __restrict__ p,
                                                         T* __restrict__ q,
                                                         double* __restrict__ part, int32_t n,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  const int row = blk * kBlock + threadIdx.x;
  double v = 0.0;
  if (row < n) {
    const T pi = p[row];
    T acc, d;
    row_apply<T, D16>(sptr, uw, col, w, p, row, n, pi, acc, d);
    q[row] = acc;
    v = static_cast<double>(pi) * static_cast<double>(acc);
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part[blk] = v;
}

// x += alpha p, r -= alpha q, partial r.r
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_update(int32_t n, const CgsScalars* __restrict__ sc,
                                                       const T* __restrict__ p,
                                                       const T* __restrict__ q,
                                                       T* __restrict__ x, T* __restrict__ r,
                                                       double* __restrict__ part,
                                                       const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  const int i = blk * kBlock + threadIdx.x;
  const T a = static_cast<T>(sc->alpha);
  double v = 0.0;
  if (i < n) {
    x[i] = x[i] + a * p[i];
    const T ri = r[i] - a * q[i];
    r[i] = ri;
    v = static_cast<double>(ri) * static_cast<double>(ri);
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part[blk] = v;
}

// p = r + beta p
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cgs_pupd(int32_t n, const CgsScalars* __restrict__ sc,
                                                     const T* __restrict__ r, T* __restrict__ p,
                                                     const int* __restrict__ done) {
  if (done && *done) return;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i < n) p[i] = r[i] + static_cast<T>(sc->beta) * p[i];
}

constexpr int kCgsFinThreads = 256;

// Sum of nb partials in a fixed order, then the CG smoother's scalar update.  A step whose
// curvature p.q or residual r.r is not positive gets alpha = 0 and leaves x and r unchanged.
__global__ __launch_bounds__(kCgsFinThreads) void k_cgs_fin(int op, int32_t nb,
                                                         const double* __restrict__ part,
                                                         CgsScalars* __restrict__ sc,
                                                         const int* __restrict__ done) {
  if (done && *done) return;
  double a = 0.0;
  for (int i = threadIdx.x; i < nb; i += kCgsFinThreads) a += part[i];
  __shared__ double sa[kCgsFinThreads / 64];
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sa[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = 0.0;
  for (int i = 0; i < kCgsFinThreads / 64; ++i) a += sa[i];
  if (op == k::CGS_INIT) {
    sc->rr = a;
  } else if (op == k::CGS_ALPHA) {
    sc->pq = a;
    sc->alpha = (sc->rr > 0.0 && a > 0.0 && isfinite(a)) ? sc->rr / a : 0.0;
  } else {
    sc->beta = sc->rr > 0.0 ? a / sc->rr : 0.0;
    sc->rr = a;
  }
}

// One colour class of a multicolour Gauss-Seidel sweep, in place: packed row p (SELL-64 over
// the class) is internal row i = rowid[p], x_i <- x_i + (b_i - (A x)_i) / A_ii with
// (A x)_i = sum_k w_k (x_i - x_j(k)) and A_ii = sum_k w_k.  Rows of one class are not coupled,
// so reading the neighbours while the class is written is race-free.
template <typename T, typename WT>
__global__ __launch_bounds__(kBlock) void k_gs_color(const int32_t* __restrict__ sptr, int32_t uw,
                                                     const int32_t* __restrict__ col,
                                                     const WT* __restrict__ w,
                                                     const int32_t* __restrict__ rowid,
                                                     T* __restrict__ x, const T* __restrict__ b,
                                                     int32_t nrows, int32_t n,
                                                     const int* __restrict__ done) {
  DECMG_DONE_LOAD(nrows)
  const int p = xcd_block() * kBlock + threadIdx.x;
  if (p >= nrows) return;
  const int i = rowid[p];
  const T xi = x[i];
  const T bi = b[i];
  T acc, d;
  row_apply<T, false>(sptr, uw, col, w, x, p, n, xi, acc, d);
  DECMG_DONE_CHECK()
  x[i] = xi + (bi - acc) / d;
}

// x_f += M(f)^T e_c: (e_a + e_b) / 2, with a == b at kept vertices.  Each thread takes
// kProlongRows rows kBlock apart: the parent gathers depend on the parent loads, and with one
// row per thread too few bytes were in flight to cover those two round trips (3.5 TB/s on the
// C3 finest level).  Eight rows per thread were no faster there and slower on the 1M-row
// level (fewer workgroups).
constexpr int kProlongRows = 4;
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong(const int32_t* __restrict__ pa,
                                                    const int32_t* __restrict__ pb,
                                                    const T* __restrict__ ec,
                                                    T* __restrict__ xf, int32_t nf,
                                                    const int* __restrict__ done) {
  DECMG_DONE_LOAD(nf)
  const int base = xcd_block() * (kBlock * kProlongRows) + threadIdx.x;
  int a[kProlongRows], b[kProlongRows];
  T x[kProlongRows];
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r) {
    const int row = base + r * kBlock;
    if (row < nf) {
      a[r] = pa[row];
      b[r] = pb[row];
      x[r] = xf[row];
    }
  }
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r)
    if (base + r * kBlock < nf) x[r] = x[r] + T(0.5) * (ec[a[r]] + ec[b[r]]);
  DECMG_DONE_CHECK()
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r)
    if (base + r * kBlock < nf) xf[base + r * kBlock] = x[r];
}

// k_prolong over packed parents: one 32-bit word per row (two int16 offsets from the slice's
// base coarse id) in place of two int32 ids.  Same arithmetic as k_prolong.
__device__ __forceinline__ int parent16(uint32_t half, int base, int nc) {
  const int o = static_cast<int16_t>(static_cast<uint16_t>(half));
  return o == kZeroSlot16 ? nc : base + o;
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prolong16(const int32_t* __restrict__ pbase,
                                                      const uint32_t* __restrict__ pab,
                                                      const T* __restrict__ ec,
                                                      T* __restrict__ xf, int32_t nf, int32_t nc,
                                                      const int* __restrict__ done) {
  DECMG_DONE_LOAD(nf)
  const int base = xcd_block() * (kBlock * kProlongRows) + threadIdx.x;
  uint32_t ab[kProlongRows];
  int bs[kProlongRows];
  T x[kProlongRows];
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r) {
    const int row = base + r * kBlock;
    if (row < nf) {
      ab[r] = pab[row];
      bs[r] = pbase[row >> 6];
      x[r] = xf[row];
    }
  }
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r)
    if (base + r * kBlock < nf) {
      const int a = parent16(ab[r] & 0xffffu, bs[r], nc);
      const int b = parent16(ab[r] >> 16, bs[r], nc);
      x[r] = x[r] + T(0.5) * (ec[a] + ec[b]);
    }
  DECMG_DONE_CHECK()
#pragma unroll
  for (int r = 0; r < kProlongRows; ++r)
    if (base + r * kBlock < nf) xf[base + r * kBlock] = x[r];
}

// Weighted interpolation xf += M(f)^T ec for any subdivision scheme: three (parent, weight)
// pairs per fine row, stored row-major (12 bytes of ids, 3 weights per row).  Cubic levels
// (Def. 5) put 2/3, 1/3 on the two endpoints of an edge point and 1/3 on each corner of a
// centroid; kept vertices carry weight 1 on themselves.  WT is the stored weight type: FP64
// weights for FP64 cycles, FP32 weights for FP32 cycles.
template <typename T, typename WT>
__global__ __launch_bounds__(kBlock) void k_prolong3(const int32_t* __restrict__ p3,
                                                     const WT* __restrict__ pw,
                                                     const T* __restrict__ ec,
                                                     T* __restrict__ xf, int32_t nf,
                                                     const int* __restrict__ done) {
  DECMG_DONE_LOAD(nf)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= nf) return;
  const size_t o = 3 * size_t(row);
  const int a = p3[o], b = p3[o + 1], c = p3[o + 2];
  const T wa = static_cast<T>(pw[o]), wb = static_cast<T>(pw[o + 1]),
          wc = static_cast<T>(pw[o + 2]);
  const T v = xf[row] + interp3(wa, wb, wc, ec[a], ec[b], ec[c]);
  DECMG_DONE_CHECK()
  xf[row] = v;
}

// Weighted restriction rc = M(f) rf: row r of M(f) lists every fine unknown whose
// interpolation reads coarse unknown r, with that weight, in a 64-row sliced layout (padding
// points at the fine zero slot with weight 0).
template <typename T, typename WT>
__global__ __launch_bounds__(kBlock) void k_restrict_w(const int32_t* __restrict__ sptr,
                                                       const int32_t* __restrict__ col,
                                                       const WT* __restrict__ w,
                                                       const T* __restrict__ rf,
                                                       T* __restrict__ rc, int32_t nc,
                                                       const int* __restrict__ done) {
  DECMG_DONE_LOAD(nc)
  const int row = xcd_block() * kBlock + threadIdx.x;
  if (row >= nc) return;
  const int s = row >> 6, lane = row & 63;
  const int beg = sptr[s], width = sptr[s + 1] - beg;
  T acc = T(0);
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    int cj[4];
    T wk[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = (beg + k + q) * kSlice + lane;
      cj[q] = col[idx];
      wk[q] = static_cast<T>(w[idx]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = rf[cj[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = mac(wk[q], v[q], acc);
  }
  for (; k < width; ++k) {
    const int idx = (beg + k) * kSlice + lane;
    acc = mac(static_cast<T>(w[idx]), rf[col[idx]], acc);
  }
  DECMG_DONE_CHECK()
  rc[row] = acc;
}

// Exact coarsest solve x = A0^{-1} b in FP64 by one workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse(const double* __restrict__ ainv,
                                                const T* __restrict__ b, T* __restrict__ x,
                                                int32_t n0, const int* __restrict__ done) {
  if (done && *done) return;
  __shared__ double sb[kMaxCoarse];
  for (int i = threadIdx.x; i < n0; i += blockDim.x) sb[i] = static_cast<double>(b[i]);
  __syncthreads();
  for (int i = threadIdx.x; i < n0; i += blockDim.x) {
    const double* a = ainv + static_cast<int64_t>(i) * n0;
    double acc = 0.0;
    for (int j = 0; j < n0; ++j) acc += a[j] * sb[j];
    x[i] = static_cast<T>(acc);
  }
}

// The coarse end of a V-cycle (levels top..0) in one workgroup.  Each level keeps x, its
// ping-pong partner and b in LDS (3 (n+1) values, the last of each being the zero slot); the
// residual reuses the partner buffer.  Operator and transfer indices are read from global
// memory (L2 resident at these sizes).  The arithmetic is that of the per-level kernels.
// One sweep or residual pass over a coarse level held in LDS (vectors and slice bounds `sp`
// in LDS, index and weight arrays in global memory).  With KMAX > 0 every thread takes four
// rows per pass and issues all their index and weight loads before any gather: rows are
// clamped to n-1 and entries to the row's last one (the SELL arrays carry one padding column),
// and weights past a row's width are masked to 0, which adds exact zeros.
template <typename T, int KMAX>
__device__ __forceinline__ void cc_sweep(const CoarseLevel<T>& L, const int32_t* sp,
                                         const T* __restrict__ cx, const T* __restrict__ B,
                                         T* __restrict__ out, T omega, int mode) {
  const int n = L.n, nt = blockDim.x;
  if (KMAX == 0) {
    for (int r = threadIdx.x; r < n; r += nt) {
      const int sl = r >> 6, lane = r & 63;
      const int beg = sp[sl], end = sp[sl + 1];
      const T xi = cx[r];
      T acc = T(0), d = T(0);
      for (int k = beg; k < end; ++k) {
        const int idx = k * kSlice + lane;
        const T wk = L.w[idx];
        d += wk;
        acc = mac(wk, xi - cx[L.col[idx]], acc);
      }
      out[r] = (mode == 2) ? xi + omega * (B[r] - acc) / d : B[r] - acc;
    }
    return;
  }
  constexpr int K = KMAX > 0 ? KMAX : 1;
  for (int r0 = threadIdx.x; r0 < n; r0 += 4 * nt) {
    int row[4], beg[4], wid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      row[q] = min(r0 + q * nt, n - 1);
      const int sl = row[q] >> 6;
      beg[q] = sp[sl];
      wid[q] = sp[sl + 1] - beg[q];
    }
    int c[4][K];
    T wv[4][K];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int kk = min(k, max(wid[q] - 1, 0));
        const int idx = (beg[q] + kk) * kSlice + (row[q] & 63);
        c[q][k] = L.col[idx];
        const T wl = L.w[idx];
        wv[q][k] = (k < wid[q]) ? wl : T(0);
      }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const T xi = cx[row[q]];
      T acc = T(0), d = T(0);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        d += wv[q][k];
        acc = mac(wv[q][k], xi - cx[c[q][k]], acc);
      }
      if (r0 + q * nt < n)
        out[row[q]] = (mode == 2) ? xi + omega * (B[row[q]] - acc) / d : B[row[q]] - acc;
    }
  }
}

// The coarse end of a V-cycle (levels top..0) in one workgroup.  LDS holds, per level, x, its
// ping-pong partner and b (3 (n+1) values, the last of each being the zero slot; the residual
// reuses the partner buffer), the dense coarsest inverse, and the slice bounds of the operator
// and restriction of every level.  The arithmetic is that of the per-level kernels.
template <typename T, int KMAX>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_cycle(
    const CoarseLevel<T>* __restrict__ lv, int top, const double* __restrict__ ainv, int32_t n0,
    int32_t inv_off, int32_t int_off, const T* __restrict__ b_in, T* __restrict__ x_out, T omega,
    int nu1, int nu2, const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ double smem_d[];
  T* sm = reinterpret_cast<T*>(smem_d);
  double* sinv = smem_d + inv_off / 8;
  int32_t* sint = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(smem_d) + int_off);
  const int total = lv[top].lds + 3 * (lv[top].n + 1);
  for (int i = threadIdx.x; i < total; i += blockDim.x) sm[i] = T(0);
  for (int i = threadIdx.x; i < n0 * n0; i += blockDim.x) sinv[i] = ainv[i];
  for (int l = 0; l <= top; ++l) {
    const CoarseLevel<T>& L = lv[l];
    for (int i = threadIdx.x; i <= L.nslices; i += blockDim.x) sint[L.lds_sptr + i] = L.sptr[i];
    if (l >= 1)
      for (int i = threadIdx.x; i <= L.r_nslices; i += blockDim.x)
        sint[L.lds_rsptr + i] = L.r_sptr[i];
  }
  __syncthreads();
  {
    const CoarseLevel<T>& L = lv[top];
    T* B = sm + L.lds + 2 * (L.n + 1);
    for (int i = threadIdx.x; i < L.n; i += blockDim.x) B[i] = b_in[i];
  }
  __syncthreads();
  unsigned in_t = 0;   // bit l set: level l's current iterate sits in its partner buffer
  for (int l = top; l >= 1; --l) {
    const CoarseLevel<T>& L = lv[l];
    const int32_t* sp = sint + L.lds_sptr;
    T* X = sm + L.lds;
    T* Tt = X + (L.n + 1);
    T* B = Tt + (L.n + 1);
    T* cx = X;
    T* ox = Tt;
    if (nu1 > 0) {
      for (int r = threadIdx.x; r < L.n; r += blockDim.x) cx[r] = jacobi_first(omega, B[r], L.idiag[r]);
      __syncthreads();
      for (int it = 1; it < nu1; ++it) {
        cc_sweep<T, KMAX>(L, sp, cx, B, ox, omega, 2);
        __syncthreads();
        T* tmp = cx;
        cx = ox;
        ox = tmp;
      }
    } else {
      for (int r = threadIdx.x; r < L.n; r += blockDim.x) cx[r] = T(0);
      __syncthreads();
    }
    cc_sweep<T, KMAX>(L, sp, cx, B, ox, omega, 1);   // residual into the partner buffer
    __syncthreads();
    const CoarseLevel<T>& C = lv[l - 1];
    T* Bc = sm + C.lds + 2 * (C.n + 1);
    const int32_t* rsp = sint + L.lds_rsptr;
    for (int r = threadIdx.x; r < C.n; r += blockDim.x) {
      const int sl = r >> 6, lane = r & 63;
      const int beg = rsp[sl], width = rsp[sl + 1] - beg;
      T acc = T(0);
      for (int k = 0; k < width; ++k) acc += ox[L.r_col[(beg + k) * kSlice + lane]];
      Bc[r] = ox[L.r_self[r]] + T(0.5) * acc;
    }
    __syncthreads();
    if (cx == Tt) in_t |= 1u << l;
  }
  {
    const CoarseLevel<T>& C = lv[0];
    T* X0 = sm + C.lds;
    const T* B0 = X0 + 2 * (C.n + 1);
    for (int i = threadIdx.x; i < n0; i += blockDim.x) {
      const double* a = sinv + static_cast<int64_t>(i) * n0;
      double acc = 0.0;
      for (int j = 0; j < n0; ++j) acc += a[j] * static_cast<double>(B0[j]);
      X0[i] = static_cast<T>(acc);
    }
  }
  __syncthreads();
  for (int l = 1; l <= top; ++l) {
    const CoarseLevel<T>& L = lv[l];
    const CoarseLevel<T>& C = lv[l - 1];
    const int32_t* sp = sint + L.lds_sptr;
    T* X = sm + L.lds;
    T* Tt = X + (L.n + 1);
    T* B = Tt + (L.n + 1);
    T* cx = (in_t >> l & 1u) ? Tt : X;
    T* ox = (cx == X) ? Tt : X;
    const T* ec = sm + C.lds + ((in_t >> (l - 1) & 1u) ? (C.n + 1) : 0);
    for (int r = threadIdx.x; r < L.n; r += blockDim.x) cx[r] += T(0.5) * (ec[L.pa[r]] + ec[L.pb[r]]);
    __syncthreads();
    for (int it = 0; it < nu2; ++it) {
      cc_sweep<T, KMAX>(L, sp, cx, B, ox, omega, 2);
      __syncthreads();
      T* tmp = cx;
      cx = ox;
      ox = tmp;
    }
    if (cx == Tt)
      in_t |= 1u << l;
    else
      in_t &= ~(1u << l);
  }
  const CoarseLevel<T>& L = lv[top];
  const T* xs = sm + L.lds + ((in_t >> top & 1u) ? (L.n + 1) : 0);
  for (int i = threadIdx.x; i < L.n; i += blockDim.x) x_out[i] = xs[i];
}

// The bottom of a cycle (levels NL..0, NL = 1..4) in one workgroup, for V, W and F shapes,
// weighted-Jacobi or multicolour Gauss-Seidel smoothing, from zero or from a given iterate.
// Requirements: the levels below the top have at most one row per thread and the top level
// at most RPT (1 or 2); operator and restriction rows have at most K and 8 entries.  Thread t
// owns row t of every level (and row t + blockDim of the top one) and loads all of their
// index, weight, diagonal, colour and transfer data into registers before the first barrier,
// so the phases that follow touch only registers and LDS: a single workgroup lands on a
// different XCD from one launch to the next, so its L2 is cold, and one round of loads replaces
// a round trip per phase.  LDS holds, per level, x, its ping-pong partner and b (3 (n+1)
// values with a zero slot each) and the dense coarsest inverse.  The recursion of the cycle
// shapes (W: two coarse cycles, the second from the first's result; F: an F-cycle then a
// V-cycle) runs as a loop over a per-level stage kept in bit fields.  GEN = false compiles
// the V-cycle with weighted-Jacobi smoothing from zero alone, as straight-line code with the
// register budget of that case.  The arithmetic, entry order and padding conventions are those
// of the per-level kernels.
template <int L, typename F>
__device__ __forceinline__ void levels_down(F&& f) {   // f(L), f(L - 1), ..., f(1)
  if constexpr (L >= 1) {
    f(std::integral_constant<int, L>{});
    levels_down<L - 1>(f);
  }
}
template <int L, int NL, typename F>
__device__ __forceinline__ void levels_up(F&& f) {     // f(L), f(L + 1), ..., f(NL)
  if constexpr (L <= NL) {
    f(std::integral_constant<int, L>{});
    levels_up<L + 1, NL>(f);
  }
}
template <int NL, typename F>
__device__ __forceinline__ void at_level(int l, F&& f) {
  switch (l) {
    case 1: if constexpr (NL >= 1) f(std::integral_constant<int, 1>{}); break;
    case 2: if constexpr (NL >= 2) f(std::integral_constant<int, 2>{}); break;
    case 3: if constexpr (NL >= 3) f(std::integral_constant<int, 3>{}); break;
    case 4: if constexpr (NL >= 4) f(std::integral_constant<int, 4>{}); break;
    default: break;
  }
}

template <typename T, int K, int NL, int RPT, bool GEN>
__global__ __launch_bounds__(kCoarseThreads) void k_coarse_cycle_reg(
    const CoarseLevel<T>* __restrict__ lv, const double* __restrict__ ainv, int32_t n0,
    int32_t inv_off, const T* __restrict__ b_in, T* __restrict__ x_io, int x_init, T omega,
    int nu1, int nu2, int kind, int gs, const int* __restrict__ done, int stride) {
  constexpr int RW = 8;
  if (done && *done) return;
  // several right-hand sides stored row-blocked (entry (i, c) at i stride + c): workgroup c
  // runs column c
  b_in += blockIdx.x;
  x_io += blockIdx.x;
  const bool use_gs = GEN && gs != 0, use_x = GEN && x_init != 0;
  extern __shared__ double smem_d[];
  T* sm = reinterpret_cast<T*>(smem_d);
  double* sinv = smem_d + inv_off / 8;
  const int t = threadIdx.x, nt = blockDim.x;
  // operator rows: RPT on the top level, one below it; restriction rows (into level l - 1,
  // never the top level): one
  int cj[NL + 1][RPT][K], pa[NL + 1][RPT], pb[NL + 1][RPT], clr[NL + 1][RPT];
  int rc[NL + 1][RW], rs[NL + 1], rwid[NL + 1];
  T wv[NL + 1][RPT][K], dg[NL + 1][RPT];
#pragma unroll
  for (int l = 1; l <= NL; ++l) {
    const CoarseLevel<T>& L = lv[l];
    const int nq = (l == NL) ? RPT : 1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (q >= nq) break;
      const int row = min(t + q * nt, L.n - 1);
      const int sl = row >> 6, lane = row & 63;
      const int beg = L.uw >= 0 ? sl * L.uw : L.sptr[sl];
      const int wid = L.uw >= 0 ? L.uw : L.sptr[sl + 1] - beg;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int idx = (beg + min(k, max(wid - 1, 0))) * kSlice + lane;
        cj[l][q][k] = L.col[idx];
        const T w = L.w[idx];
        wv[l][q][k] = (k < wid) ? w : T(0);
      }
      dg[l][q] = L.idiag[row];
      pa[l][q] = L.pa[row];
      pb[l][q] = L.pb[row];
      clr[l][q] = use_gs ? L.color[row] : 0;
    }
    const int crow = min(t, lv[l - 1].n - 1);
    const int rsl = crow >> 6, rlane = crow & 63;
    const int rbeg = L.r_uw >= 0 ? rsl * L.r_uw : L.r_sptr[rsl];
    rwid[l] = L.r_uw >= 0 ? L.r_uw : L.r_sptr[rsl + 1] - rbeg;
    rs[l] = L.r_self[crow];
#pragma unroll
    for (int k = 0; k < RW; ++k)
      rc[l][k] = L.r_col[(rbeg + min(k, max(rwid[l] - 1, 0))) * kSlice + rlane];
  }
  const int total = lv[NL].lds + 3 * (lv[NL].n + 1);
  for (int i = t; i < total; i += nt) sm[i] = T(0);
  for (int i = t; i < n0 * n0; i += nt) sinv[i] = ainv[i];
  __syncthreads();
  {
    const int n = lv[NL].n;
    for (int i = t; i < n; i += nt) {
      sm[lv[NL].lds + 2 * (n + 1) + i] = b_in[i * stride];
      if (use_x) sm[lv[NL].lds + i] = x_io[i * stride];
    }
  }
  __syncthreads();
  unsigned in_t = 0;   // bit l: level l's current iterate sits in its partner buffer

  // out = sweep of cx (mode 2: Jacobi x + omega (b - A x) / D; mode 1: residual b - A x)
  auto sweep = [&](auto Lc, const T* cx, const T* B, T* out, int mode) {
    constexpr int L = decltype(Lc)::value;
    const int n = lv[L].n;
    constexpr int NQ = (L == NL) ? RPT : 1;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = t + q * nt;
      if (r < n) {
        const T xi = cx[r];
        T acc = T(0), d = T(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          d += wv[L][q][k];
          acc = mac(wv[L][q][k], xi - cx[cj[L][q][k]], acc);
        }
        out[r] = (mode == 2) ? xi + omega * (B[r] - acc) / d : B[r] - acc;
      }
    }
  };
  // one Gauss-Seidel sweep over the colour classes in order (forward) or reversed
  auto gs_sweep = [&](auto Lc, T* cx, const T* B, bool forward) {
    constexpr int L = decltype(Lc)::value;
    const int n = lv[L].n, nc = lv[L].ncolors;
    constexpr int NQ = (L == NL) ? RPT : 1;
    for (int ci = 0; ci < nc; ++ci) {
      const int c = forward ? ci : nc - 1 - ci;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = t + q * nt;
        if (r < n && clr[L][q] == c) {
          const T xi = cx[r];
          T acc = T(0), d = T(0);
#pragma unroll
          for (int k = 0; k < K; ++k) {
            d += wv[L][q][k];
            acc = mac(wv[L][q][k], xi - cx[cj[L][q][k]], acc);
          }
          cx[r] = xi + (B[r] - acc) / d;
        }
      }
      __syncthreads();
    }
  };
  // pre-smoothing, residual and restriction of level L (down leg)
  auto down = [&](auto Lc, bool from_x) {
    constexpr int L = decltype(Lc)::value;
    constexpr int NQ = (L == NL) ? RPT : 1;
    const int n = lv[L].n;
    T* X = sm + lv[L].lds;
    T* Tt = X + (n + 1);
    T* B = Tt + (n + 1);
    T* cx = from_x ? ((in_t >> L & 1u) ? Tt : X) : X;
    T* ox = (cx == X) ? Tt : X;
    if (use_gs) {
      if (!from_x) {
        for (int i = t; i < n; i += nt) cx[i] = T(0);
        __syncthreads();
      }
      for (int it = 0; it < nu1; ++it) gs_sweep(Lc, cx, B, true);
    } else {
      int pre = nu1;
      if (!from_x) {
        if (pre > 0) {
#pragma unroll
          for (int q = 0; q < NQ; ++q)
            if (t + q * nt < n) cx[t + q * nt] = jacobi_first(omega, B[t + q * nt], dg[L][q]);
          --pre;
        } else {
          for (int i = t; i < n; i += nt) cx[i] = T(0);
        }
        __syncthreads();
      }
      for (; pre > 0; --pre) {
        sweep(Lc, cx, B, ox, 2);
        __syncthreads();
        T* tmp = cx;
        cx = ox;
        ox = tmp;
      }
    }
    sweep(Lc, cx, B, ox, 1);   // residual into the partner buffer
    __syncthreads();
    const int nc = lv[L - 1].n;
    if (t < nc) {
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < RW; ++k)
        if (k < rwid[L]) acc += ox[rc[L][k]];
      sm[lv[L - 1].lds + 2 * (nc + 1) + t] = ox[rs[L]] + T(0.5) * acc;
    }
    __syncthreads();
    if (cx == Tt)
      in_t |= 1u << L;
    else
      in_t &= ~(1u << L);
  };
  // interpolation of the coarse correction and post-smoothing of level L (up leg)
  auto up = [&](auto Lc) {
    constexpr int L = decltype(Lc)::value;
    constexpr int NQ = (L == NL) ? RPT : 1;
    const int n = lv[L].n, nc = lv[L - 1].n;
    T* X = sm + lv[L].lds;
    T* Tt = X + (n + 1);
    T* B = Tt + (n + 1);
    T* cx = (in_t >> L & 1u) ? Tt : X;
    T* ox = (cx == X) ? Tt : X;
    const T* ec = sm + lv[L - 1].lds + ((in_t >> (L - 1) & 1u) ? (nc + 1) : 0);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (t + q * nt < n) cx[t + q * nt] += T(0.5) * (ec[pa[L][q]] + ec[pb[L][q]]);
    __syncthreads();
    if (use_gs) {
      for (int it = 0; it < nu2; ++it) gs_sweep(Lc, cx, B, false);
    } else {
      for (int it = 0; it < nu2; ++it) {
        sweep(Lc, cx, B, ox, 2);
        __syncthreads();
        T* tmp = cx;
        cx = ox;
        ox = tmp;
      }
    }
    if (cx == Tt)
      in_t |= 1u << L;
    else
      in_t &= ~(1u << L);
  };

  // the coarsest level: x_0 = A_0^+ b_0 with the dense inverse
  auto solve0 = [&]() {
    T* X0 = sm + lv[0].lds;
    const T* B0 = X0 + 2 * (lv[0].n + 1);
    for (int i = t; i < n0; i += nt) {
      const double* a = sinv + static_cast<int64_t>(i) * n0;
      double acc = 0.0;
      for (int j = 0; j < n0; ++j) acc += a[j] * static_cast<double>(B0[j]);
      X0[i] = static_cast<T>(acc);
    }
    in_t &= ~1u;
    __syncthreads();
  };

  if constexpr (!GEN) {
    levels_down<NL>([&](auto Lc) { down(Lc, false); });
    solve0();
    levels_up<1, NL>([&](auto Lc) { up(Lc); });
    const T* xs = sm + lv[NL].lds + ((in_t >> NL & 1u) ? (lv[NL].n + 1) : 0);
    for (int i = t; i < lv[NL].n; i += nt) x_io[i * stride] = xs[i];
    return;
  }
  // the recursion as a loop: per level a 2-bit stage (0 enter, 1 after the first coarse
  // cycle, 2 after the second), a 2-bit shape and a start-from-x bit
  unsigned stage = 0, shape = unsigned(kind) << (2 * NL), from = unsigned(use_x ? 1 : 0) << NL;
  int level = NL;
  for (;;) {
    if (level == 0) {
      solve0();
      level = 1;
      continue;
    }
    const unsigned st = (stage >> (2 * level)) & 3u;
    const unsigned sh = (shape >> (2 * level)) & 3u;
    if (st == 0) {
      at_level<NL>(level, [&](auto Lc) { down(Lc, (from >> level) & 1u); });
      const unsigned child = sh;   // V -> V, W -> W, F -> F for the first coarse cycle
      stage = (stage & ~(3u << (2 * level))) | (1u << (2 * level));
      const int c = level - 1;
      stage &= ~(3u << (2 * c));
      shape = (shape & ~(3u << (2 * c))) | (child << (2 * c));
      from &= ~(1u << c);
      level = c;
      continue;
    }
    if (st == 1 && (sh == MG_CYCLE_W || sh == MG_CYCLE_F)) {
      const unsigned child = (sh == MG_CYCLE_F) ? unsigned(MG_CYCLE_V) : unsigned(MG_CYCLE_W);
      stage = (stage & ~(3u << (2 * level))) | (2u << (2 * level));
      const int c = level - 1;
      stage &= ~(3u << (2 * c));
      shape = (shape & ~(3u << (2 * c))) | (child << (2 * c));
      from |= 1u << c;
      level = c;
      continue;
    }
    at_level<NL>(level, [&](auto Lc) { up(Lc); });
    if (level == NL) break;
    ++level;
  }
  const T* xs = sm + lv[NL].lds + ((in_t >> NL & 1u) ? (lv[NL].n + 1) : 0);
  for (int i = t; i < lv[NL].n; i += nt) x_io[i * stride] = xs[i];
}

// dst = src (a no-op once `done` is set, like the kernels that produced src)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_copy(const T* __restrict__ src, T* __restrict__ dst,
                                                 int32_t n, const int* __restrict__ done) {
  DECMG_DONE_LOAD(n)
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i >= n) return;
  const T v = src[i];
  DECMG_DONE_CHECK()
  dst[i] = v;
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t n, T v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
__global__ void k_gather(const int32_t* __restrict__ perm, int32_t n, const T* __restrict__ src,
                         T* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

template <typename T>
__global__ void k_scatter(const int32_t* __restrict__ perm, int32_t n, const T* __restrict__ src,
                          T* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[perm[i]] = src[i];
}

template <typename T>
__global__ void k_bnd_copy(const int32_t* __restrict__ ids, int32_t nb, const T* __restrict__ src,
                           T* __restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) dst[ids[i]] = src[ids[i]];
}

template <typename T>
__global__ void k_bnd_jacobi(const int32_t* __restrict__ ids, int32_t nb, const T* __restrict__ b,
                             T* __restrict__ x, T omega) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) {
    const int v = ids[i];
    x[v] = x[v] + omega * (b[v] - x[v]);
  }
}

template <typename T>
__global__ void k_bnd_zero(const int32_t* __restrict__ ids, int32_t nb, T* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) x[ids[i]] = T(0);
}

__global__ void k_star0(const double* __restrict__ s0, const double* __restrict__ f,
                        double* __restrict__ b, int32_t nv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nv) b[i] = s0[i] * f[i];
}

// ------------------------------------------------------------------ Krylov kernels (FP64)
// The preconditioned vector widened to FP64 at one row: z32 / scale for an FP32 cycle output
// (the scale is a power of two, so this is exact), z itself for an FP64 one; minus the mean on
// singular systems.  Contraction is off so every row and neighbour gets the same rounding.
template <typename ZT>
__device__ __forceinline__ double z_val(ZT zraw, double s, double m, bool sub_mean) {
#pragma clang fp contract(off)
  double zj = static_cast<double>(zraw);
  if constexpr (std::is_same<ZT, float>::value) zj = zj * s;
  if (sub_mean) zj = zj - m;
  return zj;
}

template <typename ZT, bool D16, int N, bool FIRST, typename WT>
__device__ __forceinline__ void row_pnew_n(const void* __restrict__ col, const WT* __restrict__ w,
                                           const ZT* __restrict__ z, const double* __restrict__ po,
                                           int beg, int lane, int row, int n, double s, double m,
                                           bool sub_mean, double beta, double pi, double& acc) {
  int cj[N];
  ZT zj[N];
  double wk[N], pj[N];
#pragma unroll
  for (int k = 0; k < N; ++k) entry_at<double, D16>(col, w, (beg + k) * kSlice + lane, row, n, cj[k], wk[k]);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    zj[k] = z[cj[k]];
    pj[k] = FIRST ? 0.0 : po[cj[k]];
  }
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const double zv = z_val(zj[k], s, m, sub_mean);
    const double xj = FIRST ? zv : mac(beta, pj[k], zv);
    acc = mac(wk[k], pi - xj, acc);
  }
}

// The direction update of (flexible) CG folded into its operator product: p = z + beta p_old
// is formed at the row and again at each neighbour, q = A p, and the block partials of p.q and
// p.r.  p goes to a second buffer (neighbours still read p_old) and is never read back here,
// which saves the separate update pass and one write-then-read of p.  The previous
// iteration's solution step x += alpha p_old is taken here too, where p_old is read anyway
// (alpha still holds that iteration's step length; it is 0 when no step is pending).
// FIRST: the first iteration after a start from p_old = 0 with no solution step pending,
// where p = z exactly (beta p_old = -0 adds nothing): p_old and x are not read.
template <typename ZT, bool D16, typename WT, bool FIRST = false>
__global__ __launch_bounds__(kBlock) void k_pupd_spmv_dot2(
    const int32_t* __restrict__ sptr, int32_t uw, const void* __restrict__ col,
    const WT* __restrict__ w, const DevScalars* __restrict__ sc, const ZT* __restrict__ z,
    int sub_mean, const double* __restrict__ po, double* __restrict__ pn,
    double* __restrict__ q, const double* __restrict__ r, double* __restrict__ x,
    double* __restrict__ part0, double* __restrict__ part1, int32_t n,
    const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  const int row = blk * kBlock + threadIdx.x;
  double v0 = 0.0, v1 = 0.0;
  if (row < n) {
    const double s = sc->inv_scale, m = sub_mean ? sc->mean : 0.0, beta = sc->beta;
    double pi;
    if constexpr (FIRST) {
      pi = z_val(z[row], s, m, sub_mean != 0);
    } else {
      const double ax = sc->alpha;
      const double pold = po[row], xi = x[row];
      pi = mac(beta, pold, z_val(z[row], s, m, sub_mean != 0));
      x[row] = mac(ax, pold, xi);
    }
    const double ri = r[row];
    int beg, width;
    slice_bounds(sptr, uw, row, beg, width);
    const int lane = row & 63;
    double acc = 0.0;
    switch (width) {
      case 0: break;
#define DECMG_PN(K)                                                                          \
  case K:                                                                                    \
    row_pnew_n<ZT, D16, K, FIRST>(col, w, z, po, beg, lane, row, n, s, m, sub_mean != 0, beta, \
                                  pi, acc);                                                  \
    break;
      DECMG_PN(1) DECMG_PN(2) DECMG_PN(3) DECMG_PN(4) DECMG_PN(5) DECMG_PN(6) DECMG_PN(7)
      DECMG_PN(8)
#undef DECMG_PN
      default:
        for (int k = 0; k < width; ++k) {
          int j;
          double wk;
          entry_at<double, D16>(col, w, (beg + k) * kSlice + lane, row, n, j, wk);
          const double zj = z_val(z[j], s, m, sub_mean != 0);
          const double xj = FIRST ? zj : mac(beta, po[j], zj);
          acc = mac(wk, pi - xj, acc);
        }
    }
    pn[row] = pi;
    q[row] = acc;
    v0 = pi * acc;
    v1 = pi * ri;
  }
  block_sum2(v0, v1);
  if (threadIdx.x == 0) {
    part0[blk] = v0;
    part1[blk] = v1;
  }
}

// k_pupd_spmv_dot2 with two rows per thread (uniform widths 1..8 only): one partial per
// 2 kBlock rows
template <typename ZT, bool D16, typename WT, bool PAT, bool FIRST = false>
__device__ __forceinline__ void pupd_spmv_dot2_2_body(
    int32_t uw, const void* __restrict__ col, const WT* __restrict__ w,
    const uint8_t* __restrict__ pat, int npat, const DevScalars* __restrict__ sc,
    const ZT* __restrict__ z, int sub_mean, const double* __restrict__ po,
    double* __restrict__ pn, double* __restrict__ q, const double* __restrict__ r,
    double* __restrict__ x, double* __restrict__ part0, double* __restrict__ part1, int32_t n,
    const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  const int r0 = blk * (2 * kBlock) + threadIdx.x;
  const bool live = r0 < n;
  const double s = sc->inv_scale, m = sub_mean ? sc->mean : 0.0, beta = sc->beta;
  const double ax = sc->alpha;
  const bool sm = sub_mean != 0;
  int r1 = 0, e0 = 0, e1 = 0;
  ZT z0 = ZT(0), z1 = ZT(0);
  double o0 = 0.0, o1 = 0.0, q0r = 0.0, q1r = 0.0, x0 = 0.0, x1 = 0.0;
  if (live) {
    r1 = (r0 + kBlock < n) ? r0 + kBlock : r0;
    e0 = row_first<PAT>(pat, r0, uw);
    e1 = row_first<PAT>(pat, r1, uw);
    if constexpr (!FIRST) {
      o0 = po[r0];
      o1 = po[r1];
      x0 = x[r0];
      x1 = x[r1];
    }
    z0 = z[r0];
    z1 = z[r1];
    q0r = r[r0];
    q1r = r[r1];
  }
  if constexpr (PAT) {   // the row loads above are in flight meanwhile
    const int16_t* so;
    const WT* sw;
    stage_patterns(static_cast<const int16_t*>(col), w, npat * uw, so, sw);
    col = so;
    w = sw;
  }
  double v0 = 0.0, v1 = 0.0;
  if (live) {
    const double p0 = FIRST ? z_val(z0, s, m, sm) : mac(beta, o0, z_val(z0, s, m, sm));
    const double p1 = FIRST ? z_val(z1, s, m, sm) : mac(beta, o1, z_val(z1, s, m, sm));
    double a0, d0, a1, d1;
    row2<double, D16, PAT>(col, w, e0, e1, r0, r1, uw, n, p0, p1,
                           [&](int j) {
                             if constexpr (FIRST) return z_val(z[j], s, m, sm);
                             else return mac(beta, po[j], z_val(z[j], s, m, sm));
                           },
                           a0, d0, a1, d1);
    pn[r0] = p0;
    q[r0] = a0;
    if constexpr (!FIRST) x[r0] = mac(ax, o0, x0);
    v0 = p0 * a0;
    v1 = p0 * q0r;
    if (r1 != r0) {
      pn[r1] = p1;
      q[r1] = a1;
      if constexpr (!FIRST) x[r1] = mac(ax, o1, x1);
      v0 += p1 * a1;
      v1 += p1 * q1r;
    }
  }
  block_sum2(v0, v1);
  if (threadIdx.x == 0) {
    part0[blk] = v0;
    part1[blk] = v1;
  }
}
template <typename ZT, bool D16, typename WT, bool FIRST = false>
__global__ __launch_bounds__(kBlock) void k_pupd_spmv_dot2_2(
    int32_t uw, const void* __restrict__ col, const WT* __restrict__ w,
    const DevScalars* __restrict__ sc, const ZT* __restrict__ z, int sub_mean,
    const double* __restrict__ po, double* __restrict__ pn, double* __restrict__ q,
    const double* __restrict__ r, double* __restrict__ x, double* __restrict__ part0,
    double* __restrict__ part1, int32_t n, const int* __restrict__ done) {
  pupd_spmv_dot2_2_body<ZT, D16, WT, false, FIRST>(uw, col, w, nullptr, 0, sc, z, sub_mean, po,
                                                   pn, q, r, x, part0, part1, n, done);
}
// over row patterns (see k_rows2p)
template <typename ZT, bool FIRST = false>
__global__ __launch_bounds__(kBlock) void k_pupd_spmv_dot2_2p(
    int32_t uw, const int16_t* __restrict__ off, const double* __restrict__ w,
    const uint8_t* __restrict__ pat, int npat, const DevScalars* __restrict__ sc,
    const ZT* __restrict__ z, int sub_mean, const double* __restrict__ po,
    double* __restrict__ pn, double* __restrict__ q, const double* __restrict__ r,
    double* __restrict__ x, double* __restrict__ part0, double* __restrict__ part1, int32_t n,
    const int* __restrict__ done) {
  pupd_spmv_dot2_2_body<ZT, true, double, true, FIRST>(uw, off, w, pat, npat, sc, z, sub_mean, po,
                                                       pn, q, r, x, part0, part1, n, done);
}

// r -= alpha q, its FP32 copy for the next cycle and the block partials of r.r (x takes the
// step in the next direction update, or in k_apply_pending when the loop ends first)
__global__ __launch_bounds__(kBlock) void k_update_r(int32_t n, const DevScalars* __restrict__ sc,
                                                     const double* __restrict__ q,
                                                     double* __restrict__ r,
                                                     float* __restrict__ r32,
                                                     double* __restrict__ part0,
                                                     const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double a = sc->alpha, scale = sc->scale;
  double v = 0.0;
  int t = t0;
  // four tiles' loads in flight before any of them is used (same order of summation)
  for (; t + 4 <= t1; t += 4) {
    double rv[4], qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = min((t + u) * kBlock + static_cast<int>(threadIdx.x), n - 1);
      rv[u] = r[i];
      qv[u] = q[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = (t + u) * kBlock + threadIdx.x;
      if (i < n) {
        const double ri = rv[u] - a * qv[u];
        r[i] = ri;
        v += ri * ri;
        if (r32) r32[i] = static_cast<float>(ri * scale);
      }
    }
  }
  for (; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      const double ri = r[i] - a * q[i];
      r[i] = ri;
      v += ri * ri;
      if (r32) r32[i] = static_cast<float>(ri * scale);
    }
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

// The solution step still pending when the loop ends: x += alpha p with p the direction
// buffer the last direction update wrote (sc->pbuf).  alpha = 0 means none is pending (set so
// by the start, by a breakdown of the step length, and by the end-of-solve finalisation once
// the step is taken), which also keeps a direction left non-finite by a breakdown out of x.
__global__ __launch_bounds__(kBlock) void k_apply_pending(int32_t n,
                                                          const DevScalars* __restrict__ sc,
                                                          const double* __restrict__ p0,
                                                          const double* __restrict__ p1,
                                                          double* __restrict__ x) {
  const double a = sc->alpha;
  if (a == 0.0) return;
  const double* __restrict__ p = sc->pbuf ? p1 : p0;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i < n) x[i] = mac(a, p[i], x[i]);
}

template <bool D16, typename WT = double>
__global__ __launch_bounds__(kBlock) void k_residual_norm(const int32_t* __restrict__ sptr, int32_t uw,
                                                          const void* __restrict__ col,
                                                          const WT* __restrict__ w,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ b,
                                                          double* __restrict__ r,
                                                          float* __restrict__ r32,
                                                          const DevScalars* __restrict__ sc,
                                                          double* __restrict__ part0, int32_t n,
                                                          const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  const int row = blk * kBlock + threadIdx.x;
  double v = 0.0;
  if (row < n) {
    const double bi = b[row];
    double acc, d;
    row_apply<double, D16>(sptr, uw, col, w, x, row, n, x[row], acc, d);
    const double ri = bi - acc;
    r[row] = ri;
    v = ri * ri;
    if (r32) r32[row] = static_cast<float>(ri * sc->scale);
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

// ||b - A x||^2 block partials with two rows per thread (one partial per 2 kBlock rows; over
// row patterns or the uniform-width SELL arrays, which hold the same entries in the same
// order, so both give the same bits), r itself not stored: the true residual of the exit work.
template <bool D16, typename WT, bool PAT>
__device__ __forceinline__ void true_residual2_body(int32_t uw, const void* __restrict__ col,
                                                    const WT* __restrict__ w,
                                                    const uint8_t* __restrict__ pat, int npat,
                                                    const double* __restrict__ x,
                                                    const double* __restrict__ b,
                                                    double* __restrict__ part0, int32_t n) {
  const int blk = xcd_block();
  const int r0 = blk * (2 * kBlock) + threadIdx.x;
  const bool live = r0 < n;
  int r1 = 0, e0 = 0, e1 = 0;
  double x0 = 0.0, x1 = 0.0, b0 = 0.0, b1 = 0.0;
  if (live) {
    r1 = (r0 + kBlock < n) ? r0 + kBlock : r0;
    e0 = row_first<PAT>(pat, r0, uw);
    e1 = row_first<PAT>(pat, r1, uw);
    x0 = x[r0];
    x1 = x[r1];
    b0 = b[r0];
    b1 = b[r1];
  }
  if constexpr (PAT) {   // the row loads above are in flight meanwhile
    const int16_t* so;
    const WT* sw;
    stage_patterns(static_cast<const int16_t*>(col), w, npat * uw, so, sw);
    col = so;
    w = sw;
  }
  double v = 0.0;
  if (live) {
    double a0, d0, a1, d1;
    row2<double, D16, PAT>(col, w, e0, e1, r0, r1, uw, n, x0, x1, [&](int j) { return x[j]; },
                           a0, d0, a1, d1);
    const double q0 = b0 - a0;
    v = q0 * q0;
    if (r1 != r0) {
      const double q1 = b1 - a1;
      v = mac(q1, q1, v);
    }
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}
__global__ __launch_bounds__(kBlock) void k_true_residual2p(int32_t uw,
                                                            const int16_t* __restrict__ off,
                                                            const double* __restrict__ w,
                                                            const uint8_t* __restrict__ pat,
                                                            int npat,
                                                            const double* __restrict__ x,
                                                            const double* __restrict__ b,
                                                            double* __restrict__ part0,
                                                            int32_t n) {
  true_residual2_body<true, double, true>(uw, off, w, pat, npat, x, b, part0, n);
}
template <bool D16, typename WT>
__global__ __launch_bounds__(kBlock) void k_true_residual2(int32_t uw,
                                                           const void* __restrict__ col,
                                                           const WT* __restrict__ w,
                                                           const double* __restrict__ x,
                                                           const double* __restrict__ b,
                                                           double* __restrict__ part0,
                                                           int32_t n) {
  true_residual2_body<D16, WT, false>(uw, col, w, nullptr, 0, x, b, part0, n);
}

template <int NT>
__device__ void fin_check_block(DevScalars* __restrict__ sc, const double* __restrict__ part,
                                int32_t nb);

// The exit of a Dirichlet solve in one pass: the pending solution step x += alpha p (alpha = 0:
// none), x scattered to the caller's numbering, and (blocks past the interior rows) the
// boundary vertices' values copied from b.
__global__ __launch_bounds__(kBlock) void k_finish_scatter(
    int32_t n, DevScalars* __restrict__ sc, const double* __restrict__ p0,
    const double* __restrict__ p1, double* __restrict__ x, const int32_t* __restrict__ perm,
    double* __restrict__ x_nat, const int32_t* __restrict__ bnd, int32_t nbnd,
    const double* __restrict__ b_nat, const double* __restrict__ part, int32_t nbp) {
  // block 0: the loop's pending convergence check (fin_check_block), which reads neither
  // alpha nor the direction the others use
  if (blockIdx.x == 0) {
    if (part) fin_check_block<kBlock>(sc, part, nbp);
    return;
  }
  const int b = blockIdx.x - 1;
  const int nbi = (n + kBlock - 1) / kBlock;
  if (b >= nbi) {
    const int j = (b - nbi) * kBlock + threadIdx.x;
    if (j < nbnd) x_nat[bnd[j]] = b_nat[bnd[j]];
    return;
  }
  const int i = b * kBlock + threadIdx.x;
  if (i >= n) return;
  const double a = sc->alpha;
  const double* __restrict__ p = sc->pbuf ? p1 : p0;
  double xi = x[i];
  if (a != 0.0) {
    xi = mac(a, p[i], xi);
    x[i] = xi;
  }
  x_nat[perm[i]] = xi;
}

// The start of a solve from x = 0 on a Dirichlet system: b gathered from the caller's
// numbering into the internal right-hand side, r = b, x = 0, p = q = 0 (unless p, q are null:
// a first FCG iteration that reads neither), and the scaled FP32 copy of r.
__global__ __launch_bounds__(kBlock) void k_init_krylov_gather(
    int32_t n, const DevScalars* __restrict__ sc, const int32_t* __restrict__ perm,
    const double* __restrict__ b_nat, double* __restrict__ b, double* __restrict__ r,
    double* __restrict__ x, double* __restrict__ p, double* __restrict__ q,
    float* __restrict__ r32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = b_nat[perm[i]];
  b[i] = v;
  r[i] = v;
  x[i] = 0.0;
  if (p) p[i] = 0.0;
  if (q) q[i] = 0.0;
  if (r32) r32[i] = static_cast<float>(v * sc->scale);
}

// part0 = z.o, part1 = sum z, part2 = sum o per block (z widened by 1/scale when ZT is float):
// the sums from which the mean projection of z and the projected dot follow in one pass.
template <typename ZT>
__global__ __launch_bounds__(kBlock) void k_zsum_dot(int32_t n, const DevScalars* __restrict__ sc,
                                                     const ZT* __restrict__ z,
                                                     const double* __restrict__ o,
                                                     double* __restrict__ part0,
                                                     double* __restrict__ part1,
                                                     double* __restrict__ part2,
                                                     const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double s = std::is_same_v<ZT, float> ? sc->inv_scale : 1.0;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      const double zi = std::is_same_v<ZT, float> ? static_cast<double>(z[i]) * s
                                                  : static_cast<double>(z[i]);
      const double oi = o[i];
      v0 += zi * oi;
      v1 += zi;
      v2 += oi;
    }
  }
  block_sum2(v0, v1);
  __syncthreads();   // block_sum2's LDS slots are reused by the next reduction
  v2 = block_sum1(v2);
  if (threadIdx.x == 0) {
    part0[blk] = v0;
    part1[blk] = v1;
    part2[blk] = v2;
  }
}

__global__ __launch_bounds__(kBlock) void k_sum64(int32_t n, const double* __restrict__ v,
                                                  double* __restrict__ part0,
                                                  const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) a += v[i];
  }
  a = block_sum1(a);
  if (threadIdx.x == 0) part0[blk] = a;
}

// Block partials of sum v and of sum |v| (the compatibility test of a singular system's
// right-hand side).
__global__ __launch_bounds__(kBlock) void k_sum_abs64(int32_t n, const double* __restrict__ v,
                                                      double* __restrict__ part0,
                                                      double* __restrict__ part1) {
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  double a = 0.0, b = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      const double x = v[i];
      a += x;
      b += fabs(x);
    }
  }
  a = block_sum1(a);
  b = block_sum1(b);
  if (threadIdx.x == 0) {
    part0[blk] = a;
    part1[blk] = b;
  }
}

__global__ __launch_bounds__(kBlock) void k_sum32(int32_t n, const float* __restrict__ v,
                                                  const DevScalars* __restrict__ sc,
                                                  double* __restrict__ part0,
                                                  const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double s = sc->inv_scale;
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) a += static_cast<double>(v[i]) * s;
  }
  a = block_sum1(a);
  if (threadIdx.x == 0) part0[blk] = a;
}

// z = z32 / scale - mean (mean only when sub_mean), part0 = z . o
__global__ __launch_bounds__(kBlock) void k_zconv_dot(int32_t n, const DevScalars* __restrict__ sc,
                                                      const float* __restrict__ z32,
                                                      double* __restrict__ z,
                                                      const double* __restrict__ o,
                                                      double* __restrict__ part0, int sub_mean,
                                                      const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double s = sc->inv_scale, m = sub_mean ? sc->mean : 0.0;
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      double zi = static_cast<double>(z32[i]) * s;
      if (sub_mean) zi = zi - m;
      z[i] = zi;
      v += zi * o[i];
    }
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

// part0 = z . o with z = z32 / scale - mean, without storing z
__global__ __launch_bounds__(kBlock) void k_zdot32(int32_t n, const DevScalars* __restrict__ sc,
                                                   const float* __restrict__ z32,
                                                   const double* __restrict__ o,
                                                   double* __restrict__ part0, int sub_mean,
                                                   const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double s = sc->inv_scale, m = sub_mean ? sc->mean : 0.0;
  double v = 0.0;
  int t = t0;
  // four tiles' loads in flight before their products are summed (same order of summation)
  for (; t + 4 <= t1; t += 4) {
    float zf[4];
    double ov[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = min((t + q) * kBlock + static_cast<int>(threadIdx.x), n - 1);
      zf[q] = z32[i];
      ov[q] = o[i];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if ((t + q) * kBlock + static_cast<int>(threadIdx.x) < n) {
        double zi = static_cast<double>(zf[q]) * s;
        if (sub_mean) zi = zi - m;
        v += zi * ov[q];
      }
    }
  }
  for (; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      double zi = static_cast<double>(z32[i]) * s;
      if (sub_mean) zi = zi - m;
      v += zi * o[i];
    }
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

// z -= mean (when sub_mean), part0 = z . o
__global__ __launch_bounds__(kBlock) void k_zsub_dot(int32_t n, const DevScalars* __restrict__ sc,
                                                     double* __restrict__ z,
                                                     const double* __restrict__ o,
                                                     double* __restrict__ part0, int sub_mean,
                                                     const int* __restrict__ done) {
  if (*done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double m = sub_mean ? sc->mean : 0.0;
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      double zi = z[i];
      if (sub_mean) {
        zi = zi - m;
        z[i] = zi;
      }
      v += zi * o[i];
    }
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

__global__ __launch_bounds__(kBlock) void k_axpy1(int32_t n, const double* __restrict__ z,
                                                  double* __restrict__ x,
                                                  const int* __restrict__ done) {
  if (*done) return;
  const int i = xcd_block() * kBlock + threadIdx.x;
  if (i < n) x[i] = x[i] + z[i];
}

__global__ __launch_bounds__(kBlock) void k_dot(int32_t n, const double* __restrict__ a,
                                                const double* __restrict__ b,
                                                double* __restrict__ part0,
                                                const int* __restrict__ done) {
  if (done && *done) return;
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) v += a[i] * b[i];
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

// The solver's starting scalars (as k_init_scalars writes them)
__device__ __forceinline__ void write_start_scalars(DevScalars* __restrict__ sc, double rtol,
                                                    int32_t max_iter, double n_unknowns,
                                                    double* hist, int32_t hist_cap) {
  DevScalars z = {};
  z.hist = hist;
  z.hist_cap = hist_cap;
  z.rho = 1.0;
  z.pq = 1.0;
  z.beta = -0.0;
  z.scale = 1.0;
  z.inv_scale = 1.0;
  z.rtol = rtol;
  z.max_iter = max_iter;
  z.n_unknowns = n_unknowns;
  *sc = z;
}

// k_sum64 (block partials of sum v) whose first thread also writes the starting scalars, for
// the start of a solve on a singular system
__global__ __launch_bounds__(kBlock) void k_sum64_init(int32_t n, const double* __restrict__ v,
                                                       double* __restrict__ part0,
                                                       DevScalars* __restrict__ sc, double rtol,
                                                       int32_t max_iter, double n_unknowns,
                                                       double* hist, int32_t hist_cap) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    write_start_scalars(sc, rtol, max_iter, n_unknowns, hist, hist_cap);
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) a += v[i];
  }
  a = block_sum1(a);
  if (threadIdx.x == 0) part0[blk] = a;
}

// v -= mean and the block partials of v.v in one pass (k_sub_mean then k_dot, the same values
// and order of summation)
__global__ __launch_bounds__(kBlock) void k_sub_mean_dot(int32_t n,
                                                         const DevScalars* __restrict__ sc,
                                                         double* __restrict__ v,
                                                         double* __restrict__ part0) {
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double m = sc->mean;
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      const double vi = v[i] - m;
      v[i] = vi;
      a += vi * vi;
    }
  }
  a = block_sum1(a);
  if (threadIdx.x == 0) part0[blk] = a;
}

// The pending solution step x += alpha p (none when alpha = 0) and the block partials of
// sum x in one pass (k_apply_pending then k_sum64), for the exit of a singular system's solve
__global__ __launch_bounds__(kBlock) void k_apply_pending_sum(int32_t n,
                                                              const DevScalars* __restrict__ sc,
                                                              const double* __restrict__ p0,
                                                              const double* __restrict__ p1,
                                                              double* __restrict__ x,
                                                              double* __restrict__ part0) {
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  const double al = sc->alpha;
  const double* __restrict__ p = sc->pbuf ? p1 : p0;
  double a = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) {
      double xi = x[i];
      if (al != 0.0) {
        xi = mac(al, p[i], xi);
        x[i] = xi;
      }
      a += xi;
    }
  }
  a = block_sum1(a);
  if (threadIdx.x == 0) part0[blk] = a;
}

// A warm start's remaining set-up after r = b - A x: p = q = 0 and the scaled FP32 copy of r
// (r32 nullable)
__global__ __launch_bounds__(kBlock) void k_warm_aux(int32_t n, const DevScalars* __restrict__ sc,
                                                     const double* __restrict__ r,
                                                     float* __restrict__ r32,
                                                     double* __restrict__ p,
                                                     double* __restrict__ q) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = 0.0;
  q[i] = 0.0;
  if (r32) r32[i] = static_cast<float>(r[i] * sc->scale);
}

// k_dot whose first thread also writes the solver's starting scalars (k_init_scalars), for
// the start of a solve: the finalisation after it reads both
__global__ __launch_bounds__(kBlock) void k_dot_init(int32_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ part0,
                                                     DevScalars* __restrict__ sc, double rtol,
                                                     int32_t max_iter, double n_unknowns,
                                                     double* hist, int32_t hist_cap) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    write_start_scalars(sc, rtol, max_iter, n_unknowns, hist, hist_cap);
  const int blk = xcd_block();
  int t0, t1;
  tile_range((n + kBlock - 1) / kBlock, blk, t0, t1);
  double v = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int i = t * kBlock + threadIdx.x;
    if (i < n) v += a[i] * b[i];
  }
  v = block_sum1(v);
  if (threadIdx.x == 0) part0[blk] = v;
}

__global__ void k_sub_mean(int32_t n, const DevScalars* __restrict__ sc, double* __restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = v[i] - sc->mean;
}

// Start of a solve from x = 0 in one pass: r = b, x = p = q = 0, and the scaled FP32 copy of
// r when the cycle runs in FP32 (r32 non-null).
__global__ __launch_bounds__(kBlock) void k_init_krylov(int32_t n, const DevScalars* __restrict__ sc,
                                                        const double* __restrict__ b,
                                                        double* __restrict__ r,
                                                        double* __restrict__ x,
                                                        double* __restrict__ p,
                                                        double* __restrict__ q,
                                                        float* __restrict__ r32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = b[i];
  r[i] = v;
  x[i] = 0.0;
  p[i] = 0.0;
  q[i] = 0.0;
  if (r32) r32[i] = static_cast<float>(v * sc->scale);
}

__global__ void k_to_f32(int32_t n, const DevScalars* __restrict__ sc, const double* __restrict__ r,
                         float* __restrict__ r32, const int* __restrict__ done) {
  if (done && *done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r32[i] = static_cast<float>(r[i] * sc->scale);
}

// One workgroup: fixed-order sum of the partials, then the scalar step `op`.
// Starting values of the solver scalars (a kernel, so no host copy is in flight).
__global__ void k_init_scalars(DevScalars* __restrict__ sc, double rtol, int32_t max_iter,
                               double n_unknowns, double* hist, int32_t hist_cap) {
  DevScalars z = {};
  z.hist = hist;
  z.hist_cap = hist_cap;
  z.rho = 1.0;
  z.pq = 1.0;
  // what FCG's first beta = -(z.q)/pq is with q = 0 and pq = 1, for a first iteration that
  // skips that dot
  z.beta = -0.0;
  z.scale = 1.0;
  z.inv_scale = 1.0;
  z.rtol = rtol;
  z.max_iter = max_iter;
  z.n_unknowns = n_unknowns;
  *sc = z;
}

constexpr int kFinThreads = 1024;

// The convergence check of the Krylov loop from sum(r_i^2) = a: the loop residual, the
// iteration count, the history entry, and the end of the loop on convergence, a non-finite
// residual or the iteration limit.  Clears the pending-check mark.
__device__ __forceinline__ void fin_check_apply(DevScalars* __restrict__ sc, double a, int iters,
                                                int max_iter, double rtol, double bnorm,
                                                double* hist, int hist_cap) {
  const double rn = sqrt(a);
  sc->check_pending = 0;
  sc->rnorm = rn;
  sc->iters = iters + 1;
  if (hist && iters < hist_cap) hist[iters] = rn / bnorm;
  if (!isfinite(rn)) {
    sc->status = MG_ENONFINITE;
    sc->done = 1;
  } else if (rn <= rtol * bnorm) {
    sc->status = MG_OK;
    sc->done = 1;
  } else if (iters + 1 >= max_iter) {
    sc->status = MG_ENOCONV;
    sc->done = 1;
  }
}

// The pending convergence check taken by one workgroup (NT = 256 or 512 threads) of another
// kernel: the sum of the nb <= 8 kFinThreads partials in exactly k_finalize's order (its
// thread v adds part[v], part[v + 1024], ... and pads with zeros to eight terms; each 64-thread
// wave sums with the same butterfly; thread 0 adds the sixteen wave sums in order), so the
// check gives the same bits as a separate FIN_CHECK launch.  Thread t stands for k_finalize's
// threads t + NT j, j < 1024 / NT.
template <int NT = 256>
__device__ void fin_check_block(DevScalars* __restrict__ sc, const double* __restrict__ part,
                                int32_t nb) {
  const int done0 = sc->done, pending = sc->check_pending;
  const double rtol = sc->rtol, bnorm = sc->bnorm;
  const int iters = sc->iters, max_iter = sc->max_iter;
  double* const hist = sc->hist;
  const int hist_cap = sc->hist_cap;
  if (done0 || !pending) return;
  const int t = threadIdx.x;
  __shared__ double sw[kFinThreads / 64];
  // one stand-in thread at a time keeps the register need of the host kernel low; this
  // workgroup runs beside the others, so its round trips are not on their path
  static_assert(NT == 256 || NT == 512, "fin_check_block: 256 or 512 threads");
#pragma unroll 1
  for (int j = 0; j < kFinThreads / NT; ++j) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = t + NT * j + q * kFinThreads;
      v[q] = i < nb ? part[i] : 0.0;
    }
    double a = 0.0;
#pragma unroll
    for (int q = 0; q < 8; ++q) a += v[q];
    a = wave_sum(a);
    if ((t & 63) == 0) sw[(t >> 6) + (NT / 64) * j] = a;
  }
  __syncthreads();
  if (t != 0) return;
  double a = 0.0;
  for (int i = 0; i < kFinThreads / 64; ++i) a += sw[i];
  fin_check_apply(sc, a, iters, max_iter, rtol, bnorm, hist, hist_cap);
}

// k_jacobi_two2p with one extra workgroup (block 0) that takes the Krylov loop's pending
// convergence check, which the sweeps do not wait for: it runs beside them instead of as a
// launch of its own between the residual update and the cycle
template <typename T>
__global__ __launch_bounds__(kBlock) void k_jacobi_two2p_chk(
    int32_t uw, const int16_t* __restrict__ off, const T* __restrict__ w,
    const uint8_t* __restrict__ pat, int npat, const T* __restrict__ idiag,
    const T* __restrict__ b, T* __restrict__ y, int32_t n, T omega,
    const int* __restrict__ done, DevScalars* __restrict__ sc,
    const double* __restrict__ part, int32_t nbp) {
  if (blockIdx.x == 0) {
    fin_check_block<kBlock>(sc, part, nbp);
    return;
  }
  jacobi_two2_body<T, true, T, true>(uw, off, w, pat, npat, idiag, b, y, n, omega, done,
                                     xcd_block_of(blockIdx.x - 1, gridDim.x - 1));
}

// Per-thread part of the finaliser's fixed-order sum: thread t adds part[t + k * kFinThreads]
// for k = 0, 1, ... in that order, B loads of each array in flight at a time.
template <int B>
__device__ __forceinline__ void fin_accumulate(int32_t nb, const double* __restrict__ part0,
                                               const double* __restrict__ part1,
                                               const double* __restrict__ part2, double& a,
                                               double& b, double& c) {
  for (int base = 0; nb > 0 && base < nb; base += B * kFinThreads) {
    double va[B], vb[B], vc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int i = base + j * kFinThreads + threadIdx.x;
      const int ic = i < nb ? i : nb - 1;
      va[j] = part0[ic];
      vb[j] = part1 ? part1[ic] : 0.0;
      vc[j] = part2 ? part2[ic] : 0.0;
      if (i >= nb) {
        va[j] = 0.0;
        vb[j] = 0.0;
        vc[j] = 0.0;
      }
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      a += va[j];
      b += vb[j];
      c += vc[j];
    }
  }
}

__global__ __launch_bounds__(kFinThreads) void k_finalize(int op, int32_t nb,
                                                          const double* __restrict__ part0,
                                                          const double* __restrict__ part1,
                                                          const double* __restrict__ part2,
                                                          DevScalars* __restrict__ sc,
                                                          double extra, int force) {
  // The flag and the scalars the step reads are loaded with the partial sums, not in round
  // trips of their own before and after them; the flag is tested before the first store.
  const int done0 = sc->done;
  const double rho = sc->rho, pq = sc->pq, rtol = sc->rtol, bnorm = sc->bnorm;
  const double nun = sc->n_unknowns;
  const int iters = sc->iters, max_iter = sc->max_iter;
  double* const hist = sc->hist;
  const int hist_cap = sc->hist_cap, pending = sc->check_pending;
  // thread t sums part[t], part[t + 1024], ... in that order; loads go out in batches of 8, or
  // of 16 when there are more than 8 per thread (the one-partial-per-256-rows kernels on the
  // finest level), so that a single round trip fetches them all
  double a = 0.0, b = 0.0, c = 0.0;
  if (nb > 8 * kFinThreads)
    fin_accumulate<16>(nb, part0, part1, part2, a, b, c);
  else
    fin_accumulate<8>(nb, part0, part1, part2, a, b, c);
  __shared__ double sa[kFinThreads / 64], sb[kFinThreads / 64], scc[kFinThreads / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if ((threadIdx.x & 63) == 0) {
    sa[threadIdx.x >> 6] = a;
    sb[threadIdx.x >> 6] = b;
    scc[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x != 0 || (!force && done0)) return;
  a = 0.0;
  b = 0.0;
  c = 0.0;
  for (int i = 0; i < kFinThreads / 64; ++i) {
    a += sa[i];
    b += sb[i];
    c += scc[i];
  }
  if (op == k::FIN_MEAN_BETA_CG || op == k::FIN_MEAN_BETA_FCG) {
    // the projected vector's dot from the unprojected sums, then the plain beta update
    const double mean = b / nun;
    sc->mean = mean;
    a = a - mean * c;
    op = (op == k::FIN_MEAN_BETA_CG) ? k::FIN_BETA_CG : k::FIN_BETA_FCG;
  }
  switch (op) {
    case k::FIN_BNORM: {
      const double bn = sqrt(a + extra);
      sc->bnorm = bn;
      sc->rnorm = bn;
      if (!isfinite(bn)) {
        sc->status = MG_ENONFINITE;
        sc->done = 1;
      } else if (bn == 0.0) {
        sc->status = MG_OK;
        sc->done = 1;
      } else {
        // power-of-two scale that brings the residual to O(1) for the FP32 copy
        int e;
        frexp(bn / sqrt(nun), &e);
        sc->scale = ldexp(1.0, -e);
        sc->inv_scale = ldexp(1.0, e);
      }
      break;
    }
    // extra: the direction buffer (0 or 1) that holds this iteration's p, which the pending
    // solution step x += alpha p reads; on a breakdown no step is pending (alpha = 0)
    case k::FIN_ALPHA_CG:
      sc->pq = a;
      if (!(a > 0.0) || !isfinite(a)) {
        sc->status = isfinite(a) ? MG_EBREAKDOWN : MG_ENONFINITE;
        sc->done = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = rho / a;
        sc->pbuf = extra != 0.0 ? 1 : 0;
        sc->check_pending = 1;
      }
      break;
    case k::FIN_ALPHA_FCG:
      sc->pq = a;
      if (!(a > 0.0) || !isfinite(a) || !isfinite(b)) {
        sc->status = (isfinite(a) && isfinite(b)) ? MG_EBREAKDOWN : MG_ENONFINITE;
        sc->done = 1;
        sc->alpha = 0.0;
      } else {
        sc->alpha = b / a;
        sc->pbuf = extra != 0.0 ? 1 : 0;
        sc->check_pending = 1;
      }
      break;
    case k::FIN_CHECK:
      // extra != 0: only when a residual update is waiting for its check (the end of a batch
      // of iterations whose checks run inside the next iteration's first kernel)
      if (extra != 0.0 && !pending) break;
      fin_check_apply(sc, a, iters, max_iter, rtol, bnorm, hist, hist_cap);
      break;
    case k::FIN_BETA_CG:
      if (!(a > 0.0) || !isfinite(a)) {
        sc->status = isfinite(a) ? MG_EBREAKDOWN : MG_ENONFINITE;
        sc->done = 1;
      } else {
        sc->beta = a / rho;
        sc->rho = a;
      }
      break;
    case k::FIN_BETA_FCG:
      sc->beta = -a / pq;
      if (!isfinite(-a / pq)) {
        sc->status = MG_ENONFINITE;
        sc->done = 1;
      }
      break;
    case k::FIN_MEAN:
      sc->mean = a / nun;
      break;
    case k::FIN_MEAN_COMPAT:
      // a = sum b, b = sum |b|: a right-hand side of a singular (natural-boundary) system is
      // in the range of the operator when sum b = 0; beyond rounding it has no solution
      sc->mean = a / nun;
      if (!isfinite(a) || !isfinite(b)) {
        sc->status = MG_ENONFINITE;
        sc->done = 1;
      } else if (fabs(a) > k::kCompatTol * b) {
        sc->status = MG_EINCOMPAT;
        sc->done = 1;
      }
      break;
    case k::FIN_RNORM:
      // ends the exit work, which took the pending solution step first
      sc->true_rnorm = sqrt(a);
      sc->alpha = 0.0;
      break;
  }
}

inline unsigned grid_for(int64_t n) { return static_cast<unsigned>((n + kBlock - 1) / kBlock); }

inline void check_hip_k(hipError_t e) {
  if (e != hipSuccess) throw DeviceError(std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
}

}  // namespace

// ------------------------------------------------------------------ launchers
namespace k {

int blocks_for(int32_t n) { return static_cast<int>(grid_for(n)); }
int red_blocks(int32_t n) { return std::max(1, std::min(static_cast<int>(grid_for(n)), kRedBlocks)); }

template <typename T>
static const T* weights(const Level& L);
template <>
const double* weights<double>(const Level& L) { return L.op.w64; }
template <>
const float* weights<float>(const Level& L) { return L.op.w32; }
template <typename T>
static const T* diagonal(const Level& L);
template <>
const double* diagonal<double>(const Level& L) { return L.op.idiag64; }
template <>
const float* diagonal<float>(const Level& L) { return L.op.idiag32; }

// Calls f(w) with the weight array the T-arithmetic row kernels read: the binary16 copy when
// every weight of the level is exactly a binary16 number, else the FP32 copy for FP32 kernels,
// and for FP64 kernels too when every FP64 weight is exactly an FP32 number.  The widened
// values are the weights bit for bit in every case; only the bytes read change.
template <typename T, typename F>
static void with_weights(const Level& L, F&& f) {
  if (L.op.w_exact16) {
    f(reinterpret_cast<const Half16*>(L.op.w16));
    return;
  }
  if constexpr (std::is_same<T, float>::value) {
    f(L.op.w32);
  } else {
    if (L.op.w_exact32)
      f(static_cast<const float*>(L.op.w32));
    else
      f(static_cast<const double*>(L.op.w64));
  }
}
template <typename P>
using pointee_t = std::remove_const_t<std::remove_pointer_t<P>>;

// Levels whose slices all have one width of 1..8 entries take the two-rows-per-thread kernels.
static bool two_rows(const Level& L) { return L.op.uw >= 1 && L.op.uw <= 8; }
static unsigned grid2_for(int32_t n) { return unsigned((int64_t(n) + 2 * kBlock - 1) / (2 * kBlock)); }
// those of them whose rows take few distinct patterns read one byte per row (k_*2p kernels)
static bool row_patterns(const Level& L) { return two_rows(L) && L.op.npat > 0; }
template <typename T>
static size_t pattern_lds(const Level& L) {
  const int entries = L.op.npat * L.op.uw;
  return size_t(pattern_lds_weights_at(entries)) + size_t(entries) * sizeof(T);
}
template <typename T>
static const T* pattern_weights(const Level& L);
template <>
const double* pattern_weights<double>(const Level& L) { return L.op.pw64; }
template <>
const float* pattern_weights<float>(const Level& L) { return L.op.pw32; }

template <typename T, int MODE>
static void rows(const Level& L, const T* x, const T* b, T* y, double omega, const int* done,
                 hipStream_t s) {
  if (L.n == 0) return;
  if (row_patterns(L)) {
    hipLaunchKernelGGL((k_rows2p<T, MODE>), dim3(grid2_for(L.n)), dim3(kBlock),
                       pattern_lds<T>(L), s, L.op.uw, L.op.poff, pattern_weights<T>(L), L.op.pat,
                       L.op.npat, x, b, y, L.n, static_cast<T>(omega), done);
    return;
  }
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (two_rows(L)) {
      if (L.op.col16)
        hipLaunchKernelGGL((k_rows2<T, MODE, true, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                           L.op.uw, static_cast<const void*>(L.op.col16), w, x, b, y, L.n,
                           static_cast<T>(omega), done);
      else
        hipLaunchKernelGGL((k_rows2<T, MODE, false, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                           L.op.uw, static_cast<const void*>(L.op.col), w, x, b, y, L.n,
                           static_cast<T>(omega), done);
      return;
    }
    if (L.op.col16)
      hipLaunchKernelGGL((k_rows<T, MODE, true, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col16), w, x, b, y, L.n,
                         static_cast<T>(omega), done);
    else
      hipLaunchKernelGGL((k_rows<T, MODE, false, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col), w, x, b, y, L.n,
                         static_cast<T>(omega), done);
  });
}
// A weighted-Jacobi sweep whose start and stop are stamped into e0/e1 by the dispatch
// itself (kernel execution time only, no queueing between the two events).
template <typename T>
void jacobi_timed(const Level& L, const T* x, const T* b, T* xo, double omega, const int* done,
                  hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (L.n == 0) return;
  if (row_patterns(L)) {
    hipExtLaunchKernelGGL((k_rows2p<T, 2>), dim3(grid2_for(L.n)), dim3(kBlock),
                          pattern_lds<T>(L), s, e0, e1, 0, L.op.uw, L.op.poff,
                          pattern_weights<T>(L), L.op.pat, L.op.npat, x, b, xo, L.n,
                          static_cast<T>(omega), done);
    return;
  }
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (two_rows(L)) {
      if (L.op.col16)
        hipExtLaunchKernelGGL((k_rows2<T, 2, true, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                              e0, e1, 0, L.op.uw, static_cast<const void*>(L.op.col16), w, x, b,
                              xo, L.n, static_cast<T>(omega), done);
      else
        hipExtLaunchKernelGGL((k_rows2<T, 2, false, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0,
                              s, e0, e1, 0, L.op.uw, static_cast<const void*>(L.op.col), w, x, b,
                              xo, L.n, static_cast<T>(omega), done);
      return;
    }
    if (L.op.col16)
      hipExtLaunchKernelGGL((k_rows<T, 2, true, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, e0,
                            e1, 0, L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col16), w, x, b, xo,
                            L.n, static_cast<T>(omega), done);
    else
      hipExtLaunchKernelGGL((k_rows<T, 2, false, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, e0,
                            e1, 0, L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col), w, x, b, xo, L.n,
                            static_cast<T>(omega), done);
  });
}

template <typename T>
void spmv(const Level& L, const T* x, T* y, const int* done, hipStream_t s) {
  rows<T, 0>(L, x, static_cast<const T*>(nullptr), y, 0.0, done, s);
}
template <typename T>
void residual(const Level& L, const T* x, const T* b, T* r, const int* done, hipStream_t s) {
  rows<T, 1>(L, x, b, r, 0.0, done, s);
}
template <typename T>
void jacobi(const Level& L, const T* x, const T* b, T* xo, double omega, const int* done,
            hipStream_t s) {
  rows<T, 2>(L, x, b, xo, omega, done, s);
}
template <typename T>
void jacobi_two(const Level& L, const T* b, T* xo, double omega, const int* done, hipStream_t s) {
  if (L.n == 0) return;
  if (row_patterns(L)) {
    hipLaunchKernelGGL((k_jacobi_two2p<T>), dim3(grid2_for(L.n)), dim3(kBlock),
                       pattern_lds<T>(L), s, L.op.uw, L.op.poff, pattern_weights<T>(L), L.op.pat,
                       L.op.npat, diagonal<T>(L), b, xo, L.n, static_cast<T>(omega), done);
    return;
  }
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (two_rows(L)) {
      if (L.op.col16)
        hipLaunchKernelGGL((k_jacobi_two2<T, true, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                           L.op.uw, static_cast<const void*>(L.op.col16), w, diagonal<T>(L), b, xo,
                           L.n, static_cast<T>(omega), done);
      else
        hipLaunchKernelGGL((k_jacobi_two2<T, false, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                           L.op.uw, static_cast<const void*>(L.op.col), w, diagonal<T>(L), b, xo,
                           L.n, static_cast<T>(omega), done);
      return;
    }
    if (L.op.col16)
      hipLaunchKernelGGL((k_jacobi_two<T, true, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col16), w, diagonal<T>(L), b, xo,
                         L.n, static_cast<T>(omega), done);
    else
      hipLaunchKernelGGL((k_jacobi_two<T, false, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col), w, diagonal<T>(L), b, xo,
                         L.n, static_cast<T>(omega), done);
  });
}
bool jacobi_two_chk_ok(const Level& L) { return L.n > 0 && row_patterns(L); }
template <typename T>
void jacobi_two_chk(const Level& L, const T* b, T* xo, double omega, const int* done,
                    DevScalars* sc, const double* part, int32_t nbp, hipStream_t s) {
  if (!jacobi_two_chk_ok(L)) throw std::logic_error("jacobi_two_chk: level without row patterns");
  if (nbp < 1 || nbp > 8 * kFinThreads) throw std::logic_error("jacobi_two_chk: partial count");
  hipLaunchKernelGGL((k_jacobi_two2p_chk<T>), dim3(grid2_for(L.n) + 1), dim3(kBlock),
                     pattern_lds<T>(L), s, L.op.uw, L.op.poff, pattern_weights<T>(L), L.op.pat,
                     L.op.npat, diagonal<T>(L), b, xo, L.n, static_cast<T>(omega), done, sc, part,
                     nbp);
}
template <typename T>
void jacobi_zero(const Level& L, const T* b, T* xo, double omega, const int* done, hipStream_t s) {
  if (L.n == 0) return;
  hipLaunchKernelGGL((k_jacobi_zero<T>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, diagonal<T>(L), b,
                     xo, L.n, static_cast<T>(omega), done);
}
template <typename T>
void restrict_(const Level& Lf, const Level& Lc, const T* rf, T* rc, const int* done,
               hipStream_t s) {
  if (Lc.n == 0) return;
  if (Lf.tr.weighted) {
    if constexpr (std::is_same_v<T, double>)
      hipLaunchKernelGGL((k_restrict_w<T, double>), dim3(grid_for(Lc.n)), dim3(kBlock), 0, s,
                         Lf.tr.rw_sptr, Lf.tr.rw_col, Lf.tr.rw64, rf, rc, Lc.n, done);
    else
      hipLaunchKernelGGL((k_restrict_w<T, float>), dim3(grid_for(Lc.n)), dim3(kBlock), 0, s,
                         Lf.tr.rw_sptr, Lf.tr.rw_col, Lf.tr.rw32, rf, rc, Lc.n, done);
    return;
  }
  if (Lf.tr.r_col16) {
    hipLaunchKernelGGL((k_restrict2<T>), dim3(grid2_for(Lc.n)), dim3(kBlock), 0, s, Lf.tr.r_self,
                       Lf.tr.r_uw, Lf.tr.r_col16, rf, rc, Lc.n, Lf.n, done);
    return;
  }
  hipLaunchKernelGGL((k_restrict<T>), dim3(grid_for(Lc.n)), dim3(kBlock), 0, s, Lf.tr.r_self,
                     Lf.tr.r_sptr, Lf.tr.r_uw, Lf.tr.r_col, rf, rc, Lc.n, done);
}
template <typename T>
void prolong(const Level& Lf, const Level& Lc, const T* ec, T* xf, const int* done,
             hipStream_t s) {
  if (Lf.n == 0) return;
  if (Lf.tr.weighted) {
    if constexpr (std::is_same_v<T, double>)
      hipLaunchKernelGGL((k_prolong3<T, double>), dim3(grid_for(Lf.n)), dim3(kBlock), 0, s,
                         Lf.tr.p3, Lf.tr.pw64, ec, xf, Lf.n, done);
    else
      hipLaunchKernelGGL((k_prolong3<T, float>), dim3(grid_for(Lf.n)), dim3(kBlock), 0, s,
                         Lf.tr.p3, Lf.tr.pw32, ec, xf, Lf.n, done);
    return;
  }
  const int64_t groups = (int64_t(Lf.n) + kBlock * kProlongRows - 1) / (kBlock * kProlongRows);
  if (Lf.tr.p_ab16) {
    hipLaunchKernelGGL((k_prolong16<T>), dim3(groups), dim3(kBlock), 0, s, Lf.tr.p_base,
                       Lf.tr.p_ab16, ec, xf, Lf.n, Lc.n, done);
    return;
  }
  hipLaunchKernelGGL((k_prolong<T>), dim3(groups), dim3(kBlock), 0, s, Lf.tr.pa, Lf.tr.pb, ec,
                     xf, Lf.n, done);
}
template <typename T>
void prolong_sweep(const Level& Lf, const Level& /*Lc*/, const T* ec, const T* x, const T* b,
                   T* xo, double omega, const int* done, hipStream_t s) {
  if (Lf.n == 0) return;
  with_weights<T>(Lf, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (Lf.op.col16)
      hipLaunchKernelGGL((k_prolong_sweep<T, true, WT>), dim3(grid_for(Lf.n)), dim3(kBlock), 0, s,
                         Lf.op.sptr, Lf.op.uw, static_cast<const void*>(Lf.op.col16), w, Lf.tr.pa, Lf.tr.pb,
                         ec, x, b, xo, Lf.n, static_cast<T>(omega), done);
    else
      hipLaunchKernelGGL((k_prolong_sweep<T, false, WT>), dim3(grid_for(Lf.n)), dim3(kBlock), 0, s,
                         Lf.op.sptr, Lf.op.uw, static_cast<const void*>(Lf.op.col), w, Lf.tr.pa, Lf.tr.pb,
                         ec, x, b, xo, Lf.n, static_cast<T>(omega), done);
  });
}
template <typename T>
static size_t tile_lds(const DevTiles& D) { return 2 * size_t(D.cap + 1) * sizeof(T); }
// weights of the weighted transfers in the arithmetic type (as k_restrict_w / k_prolong3 read)
template <typename T>
static const T* transfer_weights(const Level& L) {
  if constexpr (std::is_same<T, float>::value) return L.tr.rw32; else return L.tr.rw64;
}
template <typename T>
static const T* interp_weights(const Level& L) {
  if constexpr (std::is_same<T, float>::value) return L.tr.pw32; else return L.tr.pw64;
}

template <typename T>
void tile_down(const Level& L, const T* b, T* x, T* bc, double omega, int nu1, const int* done,
               hipStream_t s, DevScalars* chk_sc, const double* chk_part, int32_t chk_nb) {
  const DevTiles& D = L.tiles;
  if (D.ntiles == 0) throw std::logic_error("tile_down on a level without tiles");
  if (chk_part && (!chk_sc || chk_nb < 1 || chk_nb > 8 * kFinThreads))
    throw std::logic_error("tile_down: convergence check arguments");
  const size_t lds = tile_lds<T>(D);
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    const T* rw = transfer_weights<T>(L);
    auto go = [&](auto kern, int tbk) {
      hipLaunchKernelGGL(kern, dim3(D.ntiles + (chk_part ? 1 : 0)), dim3(tbk), lds, s, D.meta,
                         D.row, D.ent, D.col, D.crow, D.cst, D.cap, D.ccap, L.op.uw, w,
                         diagonal<T>(L), b, x, bc, static_cast<T>(omega), nu1, D.cent, D.rws, rw,
                         done, chk_sc, chk_part, chk_nb);
    };
    const bool one = D.cap <= kTileThreads;
    if (L.tr.weighted) {
      if (D.kt == 4)
        one ? go(k_tile_down<T, WT, 4, kTileThreads, 1, 1, true>, kTileThreads)
            : go(k_tile_down<T, WT, 4, kTileThreads, 2, 1, true>, kTileThreads);
      else
        one ? go(k_tile_down<T, WT, 8, kTileThreads, 1, 1, true>, kTileThreads)
            : go(k_tile_down<T, WT, 8, kTileThreads, 2, 1, true>, kTileThreads);
    } else if (D.kt == 4) {
      one ? go(k_tile_down<T, WT, 4, kTileThreads, 1, 1, false>, kTileThreads)
          : go(k_tile_down<T, WT, 4, kTileThreads, 2, 1, false>, kTileThreads);
    } else {
      one ? go(k_tile_down<T, WT, 8, kTileThreads, 1, 1, false>, kTileThreads)
          : go(k_tile_down<T, WT, 8, kTileThreads, 2, 1, false>, kTileThreads);
    }
  });
}
template <typename T>
void tile_up(const Level& L, const T* ec, const T* x, const T* b, T* xo, double omega, int nu2,
             const int* done, hipStream_t s) {
  const DevTiles& D = L.tiles;
  if (D.ntiles == 0) throw std::logic_error("tile_up on a level without tiles");
  const size_t lds = tile_lds<T>(D);
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    const T* pw = interp_weights<T>(L);
    auto go = [&](auto kern, int tbk) {
      hipLaunchKernelGGL(kern, dim3(D.ntiles), dim3(tbk), lds, s, D.meta, D.row, D.ent, D.col,
                         D.cap, L.op.uw, w, L.tr.pa, L.tr.pb, ec, x, b, xo,
                         static_cast<T>(omega), nu2, L.tr.p3, pw, done);
    };
    const bool one = D.cap <= kTileThreads;
    if (L.tr.weighted) {
      if (D.kt == 4)
        one ? go(k_tile_up<T, WT, 4, kTileThreads, 1, true>, kTileThreads)
            : go(k_tile_up<T, WT, 4, kTileThreads, 2, true>, kTileThreads);
      else
        one ? go(k_tile_up<T, WT, 8, kTileThreads, 1, true>, kTileThreads)
            : go(k_tile_up<T, WT, 8, kTileThreads, 2, true>, kTileThreads);
    } else if (D.kt == 4) {
      one ? go(k_tile_up<T, WT, 4, kTileThreads, 1, false>, kTileThreads)
          : go(k_tile_up<T, WT, 4, kTileThreads, 2, false>, kTileThreads);
    } else {
      one ? go(k_tile_up<T, WT, 8, kTileThreads, 1, false>, kTileThreads)
          : go(k_tile_up<T, WT, 8, kTileThreads, 2, false>, kTileThreads);
    }
  });
}

template <typename T>
void cgs_start(const Level& L, const T* r, T* p, double* part, const int* done, hipStream_t s) {
  if (L.n == 0) return;
  hipLaunchKernelGGL((k_cgs_start<T>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, r, p, part,
                     done);
}
template <typename T>
void cgs_spmv_dot(const Level& L, const T* p, T* q, double* part, const int* done, hipStream_t s) {
  if (L.n == 0) return;
  with_weights<T>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (L.op.col16)
      hipLaunchKernelGGL((k_cgs_spmv_dot<T, true, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col16), w, p, q, part,
                         L.n, done);
    else
      hipLaunchKernelGGL((k_cgs_spmv_dot<T, false, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col), w, p, q, part,
                         L.n, done);
  });
}
template <typename T>
void cgs_update(const Level& L, const T* p, const T* q, T* x, T* r, double* part, const int* done,
                hipStream_t s) {
  if (L.n == 0) return;
  hipLaunchKernelGGL((k_cgs_update<T>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.cgs, p, q,
                     x, r, part, done);
}
template <typename T>
void cgs_pupd(const Level& L, const T* r, T* p, const int* done, hipStream_t s) {
  if (L.n == 0) return;
  hipLaunchKernelGGL((k_cgs_pupd<T>), dim3(grid_for(L.n)), dim3(kBlock), 0, s, L.n, L.cgs, r, p,
                     done);
}
void cgs_fin(const Level& L, int op, const double* part, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_cgs_fin, dim3(1), dim3(kCgsFinThreads), 0, s, op, int32_t(grid_for(L.n)),
                     part, L.cgs, done);
}
template <typename T>
void gs_color(const Level& L, int c, T* x, const T* b, const int* done, hipStream_t s) {
  const GsColor& G = L.gs[c];
  if (G.nrows == 0) return;
  auto launch = [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    hipLaunchKernelGGL((k_gs_color<T, WT>), dim3(grid_for(G.nrows)), dim3(kBlock), 0, s, G.sptr,
                       G.uw, G.col, w, G.rowid, x, b, G.nrows, L.n, done);
  };
  if constexpr (std::is_same<T, float>::value)
    launch(static_cast<const float*>(G.w32));
  else if (G.w_exact32)
    launch(static_cast<const float*>(G.w32));
  else
    launch(static_cast<const double*>(G.w64));
}
template <typename T>
void coarse(const Hierarchy& H, const T* b, T* x, const int* done, hipStream_t s) {
  if (H.n0 == 0) return;
  hipLaunchKernelGGL((k_coarse<T>), dim3(1), dim3(256), 0, s, H.coarse_inv, b, x, H.n0, done);
}
template <typename T, int K>
static void launch_coarse_cycle(const Hierarchy& H, int top, const T* b, T* x, double omega,
                                int nu1, int nu2, const int* done, hipStream_t s) {
  const size_t bytes = coarse_lds_bytes<T>(H);
  const size_t int_off = coarse_int_offset<T>(H);
  const size_t inv_off = int_off - size_t(H.n0) * H.n0 * sizeof(double);
  hipLaunchKernelGGL((k_coarse_cycle<T, K>), dim3(1), dim3(kCoarseThreads), bytes, s,
                     coarse_levels<T>(H), top, H.coarse_inv, H.n0, int32_t(inv_off),
                     int32_t(int_off), b, x, static_cast<T>(omega), nu1, nu2, done);
}

template <typename T, int K, int NL, int RPT, bool GEN>
static void allow_lds(int bytes) {
  if (bytes > 64 * 1024)
    check_hip_k(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_coarse_cycle_reg<T, K, NL, RPT, GEN>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
}
template <typename T, int K>
static void allow_reg(int bytes) {
  allow_lds<T, K, 1, 1, false>(bytes); allow_lds<T, K, 1, 2, false>(bytes);
  allow_lds<T, K, 2, 1, false>(bytes); allow_lds<T, K, 2, 2, false>(bytes);
  allow_lds<T, K, 3, 1, false>(bytes); allow_lds<T, K, 3, 2, false>(bytes);
  allow_lds<T, K, 4, 1, false>(bytes); allow_lds<T, K, 4, 2, false>(bytes);
  allow_lds<T, K, 1, 1, true>(bytes);  allow_lds<T, K, 1, 2, true>(bytes);
  allow_lds<T, K, 2, 1, true>(bytes);  allow_lds<T, K, 2, 2, true>(bytes);
  allow_lds<T, K, 3, 1, true>(bytes);  allow_lds<T, K, 3, 2, true>(bytes);
  allow_lds<T, K, 4, 1, true>(bytes);  allow_lds<T, K, 4, 2, true>(bytes);
}

// Allows the fused coarse cycles their dynamic LDS (above the default 64 KiB); called once when
// a hierarchy is built, outside any stream capture.
void prepare_coarse(const Hierarchy& H) {
  const int b64 = int(coarse_lds_bytes<double>(H)), b32 = int(coarse_lds_bytes<float>(H));
  auto allow = [](const void* f, int bytes) {
    if (bytes > 64 * 1024)
      check_hip_k(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  };
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<double, 4>), b64);
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<double, 8>), b64);
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<double, 0>), b64);
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<float, 4>), b32);
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<float, 8>), b32);
  allow(reinterpret_cast<const void*>(&k_coarse_cycle<float, 0>), b32);
  allow_reg<double, 4>(b64);
  allow_reg<double, 8>(b64);
  allow_reg<float, 4>(b32);
  allow_reg<float, 8>(b32);
}

template <typename T, int K, int NL, int RPT, bool GEN>
static void launch_coarse_cycle_reg(const Hierarchy& H, const T* b, T* x, bool x_init,
                                    double omega, int nu1, int nu2, int kind, bool gs,
                                    const int* done, int ncols, hipStream_t s) {
  const size_t bytes = coarse_lds_bytes<T>(H);
  const size_t int_off = coarse_int_offset<T>(H);
  const size_t inv_off = int_off - size_t(H.n0) * H.n0 * sizeof(double);
  hipLaunchKernelGGL((k_coarse_cycle_reg<T, K, NL, RPT, GEN>), dim3(ncols), dim3(kCoarseThreads),
                     bytes, s, coarse_levels<T>(H), H.coarse_inv, H.n0, int32_t(inv_off), b, x,
                     x_init ? 1 : 0, static_cast<T>(omega), nu1, nu2, kind, gs ? 1 : 0, done,
                     ncols);
}
template <typename T, int K, int RPT, bool GEN>
static void coarse_cycle_reg(const Hierarchy& H, int top, const T* b, T* x, bool x_init,
                             double omega, int nu1, int nu2, int kind, bool gs, const int* done,
                             int ncols, hipStream_t s) {
  switch (top) {
    case 1: launch_coarse_cycle_reg<T, K, 1, RPT, GEN>(H, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s); break;
    case 2: launch_coarse_cycle_reg<T, K, 2, RPT, GEN>(H, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s); break;
    case 3: launch_coarse_cycle_reg<T, K, 3, RPT, GEN>(H, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s); break;
    default: launch_coarse_cycle_reg<T, K, 4, RPT, GEN>(H, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s); break;
  }
}
template <typename T, bool GEN>
static void coarse_cycle_regs(const Hierarchy& H, int top, const T* b, T* x, bool x_init,
                              double omega, int nu1, int nu2, int kind, bool gs, const int* done,
                              hipStream_t s, int ncols = 1) {
  const bool one = H.lv[top]->n <= kCoarseThreads;
  if (H.coarse_width <= 4) {
    if (one)
      coarse_cycle_reg<T, 4, 1, GEN>(H, top, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s);
    else
      coarse_cycle_reg<T, 4, 2, GEN>(H, top, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s);
  } else {
    if (one)
      coarse_cycle_reg<T, 8, 1, GEN>(H, top, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s);
    else
      coarse_cycle_reg<T, 8, 2, GEN>(H, top, b, x, x_init, omega, nu1, nu2, kind, gs, done, ncols, s);
  }
}

template <typename T>
bool coarse_cycle_general_ok(const Hierarchy& H, int top, bool gs) {
  // levels below `top` at most one row per thread, `top` itself at most two; narrow rows; a
  // colouring with few classes for Gauss-Seidel
  if (top < 1 || top > 4 || top > coarse_top<T>(H)) return false;
  int below = 0;
  for (int l = 0; l < top; ++l) below = std::max(below, H.lv[l]->n);
  if (below > kCoarseThreads || H.lv[top]->n > 2 * kCoarseThreads) return false;
  if (H.coarse_rwidth > 8 || H.coarse_width > 8) return false;
  if (gs)
    for (int l = 1; l <= top; ++l)
      if (H.lv[l]->gs.empty() || H.lv[l]->gs.size() > 16) return false;
  return true;
}

template <typename T>
void coarse_cycle_general(const Hierarchy& H, int top, const T* b, T* x, bool x_init,
                          double omega, int nu1, int nu2, int kind, bool gs, const int* done,
                          hipStream_t s) {
  coarse_cycle_regs<T, true>(H, top, b, x, x_init, omega, nu1, nu2, kind, gs, done, s);
}

template <typename T>
void coarse_cycle_columns(const Hierarchy& H, int top, const T* b, T* x, bool x_init,
                          double omega, int nu1, int nu2, int kind, int ncols, const int* done,
                          hipStream_t s) {
  if (!coarse_cycle_general_ok<T>(H, top, false))
    throw std::logic_error("coarse_cycle_columns: levels do not fit the fused bottom");
  if (!x_init && kind == MG_CYCLE_V)
    coarse_cycle_regs<T, false>(H, top, b, x, false, omega, nu1, nu2, MG_CYCLE_V, false, done, s,
                                ncols);
  else
    coarse_cycle_regs<T, true>(H, top, b, x, x_init, omega, nu1, nu2, kind, false, done, s, ncols);
}

template <typename T>
void coarse_cycle(const Hierarchy& H, int top, const T* b, T* x, double omega, int nu1, int nu2,
                  const int* done, hipStream_t s) {
  const int kmax = H.coarse_width;
  if (coarse_cycle_general_ok<T>(H, top, false)) {
    coarse_cycle_regs<T, false>(H, top, b, x, false, omega, nu1, nu2, MG_CYCLE_V, false, done, s);
    return;
  }
  if (kmax <= 4)
    launch_coarse_cycle<T, 4>(H, top, b, x, omega, nu1, nu2, done, s);
  else if (kmax <= 8)
    launch_coarse_cycle<T, 8>(H, top, b, x, omega, nu1, nu2, done, s);
  else
    launch_coarse_cycle<T, 0>(H, top, b, x, omega, nu1, nu2, done, s);
}
template <typename T>
void copy(const T* src, T* dst, int32_t n, const int* done, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_copy<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, src, dst, n, done);
}
template <typename T>
void fill(T* p, int64_t n, T v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
}
template <typename T>
void gather(const int32_t* perm, int32_t n, const T* src, T* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_gather<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, src, dst);
}
template <typename T>
void scatter(const int32_t* perm, int32_t n, const T* src, T* dst, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_scatter<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, perm, n, src, dst);
}
template <typename T>
void bnd_copy(const int32_t* ids, int32_t nb, const T* src, T* dst, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_bnd_copy<T>), dim3(grid_for(nb)), dim3(kBlock), 0, s, ids, nb, src, dst);
}
template <typename T>
void bnd_jacobi(const int32_t* ids, int32_t nb, const T* b, T* x, double omega, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_bnd_jacobi<T>), dim3(grid_for(nb)), dim3(kBlock), 0, s, ids, nb, b, x,
                     static_cast<T>(omega));
}
template <typename T>
void bnd_zero(const int32_t* ids, int32_t nb, T* x, hipStream_t s) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_bnd_zero<T>), dim3(grid_for(nb)), dim3(kBlock), 0, s, ids, nb, x);
}
void star0_apply(const Level& L, int bc, const double* f, double* b, hipStream_t s) {
  hipLaunchKernelGGL(k_star0, dim3(grid_for(L.nv)), dim3(kBlock), 0, s, L.star0, f, b, L.nv);
  if (bc == MG_BC_DIRICHLET0) bnd_zero<double>(L.bnd_ids, static_cast<int32_t>(L.bnd_h.size()), b, s);
}

int pupd_spmv_partials(const Level& L) {
  return two_rows(L) ? static_cast<int>(grid2_for(L.n)) : blocks_for(L.n);
}
void pupd_spmv_dot2(const Level& L, const DevScalars* sc, const float* z32, const double* z64,
                    int sub_mean_flag, const double* p_old, double* p_new, double* q,
                    const double* r, double* x, double* part0, double* part1, const int* done,
                    hipStream_t s, bool first) {
  auto launch = [&](auto fc) {
    constexpr bool FIRST = decltype(fc)::value;
    if (row_patterns(L)) {
      if (z32)
        hipLaunchKernelGGL((k_pupd_spmv_dot2_2p<float, FIRST>), dim3(grid2_for(L.n)),
                           dim3(kBlock), pattern_lds<double>(L), s, L.op.uw, L.op.poff, L.op.pw64,
                           L.op.pat, L.op.npat, sc, z32, sub_mean_flag, p_old, p_new, q, r, x,
                           part0, part1, L.n, done);
      else
        hipLaunchKernelGGL((k_pupd_spmv_dot2_2p<double, FIRST>), dim3(grid2_for(L.n)),
                           dim3(kBlock), pattern_lds<double>(L), s, L.op.uw, L.op.poff, L.op.pw64,
                           L.op.pat, L.op.npat, sc, z64, sub_mean_flag, p_old, p_new, q, r, x,
                           part0, part1, L.n, done);
      return;
    }
    with_weights<double>(L, [&](auto w) {
      using WT = pointee_t<decltype(w)>;
      auto go = [&](auto zp) {
        using ZT = pointee_t<decltype(zp)>;
        if (two_rows(L)) {
          if (L.op.col16)
            hipLaunchKernelGGL((k_pupd_spmv_dot2_2<ZT, true, WT, FIRST>), dim3(grid2_for(L.n)),
                               dim3(kBlock), 0, s, L.op.uw, static_cast<const void*>(L.op.col16),
                               w, sc, zp, sub_mean_flag, p_old, p_new, q, r, x, part0, part1,
                               L.n, done);
          else
            hipLaunchKernelGGL((k_pupd_spmv_dot2_2<ZT, false, WT, FIRST>), dim3(grid2_for(L.n)),
                               dim3(kBlock), 0, s, L.op.uw, static_cast<const void*>(L.op.col), w,
                               sc, zp, sub_mean_flag, p_old, p_new, q, r, x, part0, part1, L.n,
                               done);
          return;
        }
        if (L.op.col16)
          hipLaunchKernelGGL((k_pupd_spmv_dot2<ZT, true, WT, FIRST>), dim3(grid_for(L.n)),
                             dim3(kBlock), 0, s, L.op.sptr, L.op.uw,
                             static_cast<const void*>(L.op.col16), w, sc, zp, sub_mean_flag, p_old,
                             p_new, q, r, x, part0, part1, L.n, done);
        else
          hipLaunchKernelGGL((k_pupd_spmv_dot2<ZT, false, WT, FIRST>), dim3(grid_for(L.n)),
                             dim3(kBlock), 0, s, L.op.sptr, L.op.uw,
                             static_cast<const void*>(L.op.col), w, sc, zp, sub_mean_flag, p_old,
                             p_new, q, r, x, part0, part1, L.n, done);
      };
      if (z32)
        go(z32);
      else
        go(z64);
    });
  };
  if (first)
    launch(std::true_type{});
  else
    launch(std::false_type{});
}
void update_r(int32_t n, const DevScalars* sc, const double* q, double* r, float* r32,
              double* part0, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_update_r, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, q, r, r32, part0,
                     done);
}
void apply_pending(int32_t n, const DevScalars* sc, const double* p0, const double* p1, double* x,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_apply_pending, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, p0, p1, x);
}
void residual_norm(const Level& L, const double* x, const double* b, double* r, float* r32,
                   const DevScalars* sc, double* part0, const int* done, hipStream_t s) {
  with_weights<double>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (L.op.col16)
      hipLaunchKernelGGL((k_residual_norm<true, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col16), w, x, b, r, r32, sc,
                         part0, L.n, done);
    else
      hipLaunchKernelGGL((k_residual_norm<false, WT>), dim3(grid_for(L.n)), dim3(kBlock), 0, s,
                         L.op.sptr, L.op.uw, static_cast<const void*>(L.op.col), w, x, b, r, r32, sc, part0,
                         L.n, done);
  });
}
void zsum_dot32(int32_t n, const DevScalars* sc, const float* z32, const double* o, double* part0,
                double* part1, double* part2, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_zsum_dot<float>, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, z32, o,
                     part0, part1, part2, done);
}
void zsum_dot64(int32_t n, const DevScalars* sc, const double* z, const double* o, double* part0,
                double* part1, double* part2, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_zsum_dot<double>, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, z, o,
                     part0, part1, part2, done);
}
void sum64(int32_t n, const double* v, double* part0, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_sum64, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, v, part0, done);
}
void sum32(int32_t n, const float* v, const DevScalars* sc, double* part0, const int* done,
           hipStream_t s) {
  hipLaunchKernelGGL(k_sum32, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, v, sc, part0, done);
}
void zconv_dot(int32_t n, const DevScalars* sc, const float* z32, double* z, const double* o,
               double* part0, int sub_mean_flag, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_zconv_dot, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, z32, z, o, part0,
                     sub_mean_flag, done);
}
void zsub_dot(int32_t n, const DevScalars* sc, double* z, const double* o, double* part0,
              int sub_mean_flag, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_zsub_dot, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, z, o, part0,
                     sub_mean_flag, done);
}
void zdot32(int32_t n, const DevScalars* sc, const float* z32, const double* o, double* part0,
            int sub_mean_flag, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_zdot32, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, z32, o, part0,
                     sub_mean_flag, done);
}
void axpy1(int32_t n, const double* z, double* x, const int* done, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy1, dim3(grid_for(n)), dim3(kBlock), 0, s, n, z, x, done);
}
void dot(int32_t n, const double* a, const double* b, double* part0, const int* done,
         hipStream_t s) {
  hipLaunchKernelGGL(k_dot, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, a, b, part0, done);
}
void dot_init(int32_t n, const double* a, const double* b, double* part0, DevScalars* sc,
              double rtol, int32_t max_iter, double n_unknowns, double* hist, int32_t hist_cap,
              hipStream_t s) {
  hipLaunchKernelGGL(k_dot_init, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, a, b, part0, sc, rtol,
                     max_iter, n_unknowns, hist, hist_cap);
}
void sum64_init(int32_t n, const double* v, double* part0, DevScalars* sc, double rtol,
                int32_t max_iter, double n_unknowns, double* hist, int32_t hist_cap,
                hipStream_t s) {
  hipLaunchKernelGGL(k_sum64_init, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, v, part0, sc, rtol,
                     max_iter, n_unknowns, hist, hist_cap);
}
void sub_mean_dot(int32_t n, const DevScalars* sc, double* v, double* part0, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mean_dot, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, v, part0);
}
void apply_pending_sum(int32_t n, const DevScalars* sc, const double* p0, const double* p1,
                       double* x, double* part0, hipStream_t s) {
  hipLaunchKernelGGL(k_apply_pending_sum, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, sc, p0, p1,
                     x, part0);
}
void warm_aux(int32_t n, const DevScalars* sc, const double* r, float* r32, double* p, double* q,
              hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_warm_aux, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, r, r32, p, q);
}
void sub_mean(int32_t n, const DevScalars* sc, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, v);
}
bool true_residual_fast(const Level& L) { return L.n > 0 && two_rows(L); }
int true_residual_partials(const Level& L) {
  return true_residual_fast(L) ? static_cast<int>(grid2_for(L.n)) : blocks_for(L.n);
}
void true_residual(const Level& L, const double* x, const double* b, double* r_scratch,
                   double* part0, hipStream_t s) {
  if (L.n == 0) return;
  if (!true_residual_fast(L)) {
    residual_norm(L, x, b, r_scratch, nullptr, nullptr, part0, nullptr, s);
    return;
  }
  if (row_patterns(L)) {
    hipLaunchKernelGGL(k_true_residual2p, dim3(grid2_for(L.n)), dim3(kBlock), pattern_lds<double>(L),
                       s, L.op.uw, L.op.poff, L.op.pw64, L.op.pat, L.op.npat, x, b, part0, L.n);
    return;
  }
  with_weights<double>(L, [&](auto w) {
    using WT = pointee_t<decltype(w)>;
    if (L.op.col16)
      hipLaunchKernelGGL((k_true_residual2<true, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                         L.op.uw, static_cast<const void*>(L.op.col16), w, x, b, part0, L.n);
    else
      hipLaunchKernelGGL((k_true_residual2<false, WT>), dim3(grid2_for(L.n)), dim3(kBlock), 0, s,
                         L.op.uw, static_cast<const void*>(L.op.col), w, x, b, part0, L.n);
  });
}
void finish_scatter(int32_t n, DevScalars* sc, const double* p0, const double* p1, double* x,
                    const int32_t* perm, double* x_nat, const int32_t* bnd, int32_t nbnd,
                    const double* b_nat, const double* part, int32_t nbp, hipStream_t s) {
  if (part && (nbp < 1 || nbp > 8 * kFinThreads))
    throw std::logic_error("finish_scatter: partial count");
  const unsigned g = 1 + grid_for(n) + grid_for(nbnd);
  hipLaunchKernelGGL(k_finish_scatter, dim3(g), dim3(kBlock), 0, s, n, sc, p0, p1, x, perm, x_nat,
                     bnd, nbnd, b_nat, part, nbp);
}
void init_krylov_gather(int32_t n, const DevScalars* sc, const int32_t* perm, const double* b_nat,
                        double* b, double* r, double* x, double* p, double* q, float* r32,
                        hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_krylov_gather, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, perm,
                     b_nat, b, r, x, p, q, r32);
}
void init_krylov(int32_t n, const DevScalars* sc, const double* b, double* r, double* x,
                 double* p, double* q, float* r32, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_init_krylov, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, b, r, x, p, q,
                     r32);
}
void to_f32(int32_t n, const DevScalars* sc, const double* r, float* r32, const int* done,
            hipStream_t s) {
  hipLaunchKernelGGL(k_to_f32, dim3(grid_for(n)), dim3(kBlock), 0, s, n, sc, r, r32, done);
}
void finalize(int op, int32_t nblocks, const double* part0, const double* part1, DevScalars* sc,
              double extra, int force, hipStream_t s, const double* part2) {
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kFinThreads), 0, s, op, nblocks, part0, part1,
                     part2, sc, extra, force);
}

void init_scalars(DevScalars* sc, double rtol, int32_t max_iter, double n_unknowns, double* hist,
                  int32_t hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(1), 0, s, sc, rtol, max_iter, n_unknowns, hist,
                     hist_cap);
}

// A loop restarted from x with p = q = 0: the direction scalars start as at k_init_scalars
// (their values then do not enter the first new direction, only keep it finite).
__global__ void k_restart_scalars(DevScalars* __restrict__ sc) {
  sc->done = 0;
  sc->status = MG_OK;
  sc->rho = 1.0;
  sc->pq = 1.0;
  sc->beta = -0.0;
  sc->check_pending = 0;
}

void restart_scalars(DevScalars* sc, hipStream_t s) {
  hipLaunchKernelGGL(k_restart_scalars, dim3(1), dim3(1), 0, s, sc);
}

void sum_abs64(int32_t n, const double* v, double* part0, double* part1, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_abs64, dim3(red_blocks(n)), dim3(kBlock), 0, s, n, v, part0, part1);
}

#define DECMG_INST(T)                                                                          \
  template void spmv<T>(const Level&, const T*, T*, const int*, hipStream_t);                   \
  template void residual<T>(const Level&, const T*, const T*, T*, const int*, hipStream_t);     \
  template void jacobi<T>(const Level&, const T*, const T*, T*, double, const int*, hipStream_t); \
  template void jacobi_zero<T>(const Level&, const T*, T*, double, const int*, hipStream_t);    \
  template void jacobi_two<T>(const Level&, const T*, T*, double, const int*, hipStream_t);     \
  template void jacobi_two_chk<T>(const Level&, const T*, T*, double, const int*, DevScalars*,   \
                                  const double*, int32_t, hipStream_t);                          \
  template void jacobi_timed<T>(const Level&, const T*, const T*, T*, double, const int*,        \
                                hipStream_t, hipEvent_t, hipEvent_t);                           \
  template void restrict_<T>(const Level&, const Level&, const T*, T*, const int*, hipStream_t); \
  template void prolong<T>(const Level&, const Level&, const T*, T*, const int*, hipStream_t);  \
  template void prolong_sweep<T>(const Level&, const Level&, const T*, const T*, const T*, T*,  \
                                 double, const int*, hipStream_t);                              \
  template void gs_color<T>(const Level&, int, T*, const T*, const int*, hipStream_t);         \
  template void cgs_start<T>(const Level&, const T*, T*, double*, const int*, hipStream_t);    \
  template void cgs_spmv_dot<T>(const Level&, const T*, T*, double*, const int*, hipStream_t); \
  template void cgs_update<T>(const Level&, const T*, const T*, T*, T*, double*, const int*,   \
                              hipStream_t);                                                     \
  template void cgs_pupd<T>(const Level&, const T*, T*, const int*, hipStream_t);             \
  template void coarse<T>(const Hierarchy&, const T*, T*, const int*, hipStream_t);             \
  template void coarse_cycle<T>(const Hierarchy&, int, const T*, T*, double, int, int, const int*, \
                                hipStream_t);                                                  \
  template bool coarse_cycle_general_ok<T>(const Hierarchy&, int, bool);                         \
  template void coarse_cycle_columns<T>(const Hierarchy&, int, const T*, T*, bool, double, int,    \
                                        int, int, int, const int*, hipStream_t);                 \
  template void tile_down<T>(const Level&, const T*, T*, T*, double, int, const int*,         \
                             hipStream_t, DevScalars*, const double*, int32_t);                 \
  template void tile_up<T>(const Level&, const T*, const T*, const T*, T*, double, int,       \
                           const int*, hipStream_t);                                           \
  template void coarse_cycle_general<T>(const Hierarchy&, int, const T*, T*, bool, double, int,  \
                                        int, int, bool, const int*, hipStream_t);                \
  template void copy<T>(const T*, T*, int32_t, const int*, hipStream_t);                        \
  template void fill<T>(T*, int64_t, T, hipStream_t);                                          \
  template void gather<T>(const int32_t*, int32_t, const T*, T*, hipStream_t);                 \
  template void scatter<T>(const int32_t*, int32_t, const T*, T*, hipStream_t);                \
  template void bnd_copy<T>(const int32_t*, int32_t, const T*, T*, hipStream_t);               \
  template void bnd_jacobi<T>(const int32_t*, int32_t, const T*, T*, double, hipStream_t);     \
  template void bnd_zero<T>(const int32_t*, int32_t, T*, hipStream_t);
DECMG_INST(double)
DECMG_INST(float)
#undef DECMG_INST

}  // namespace k
}  // namespace decmg
