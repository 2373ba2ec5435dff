// HIP kernels of the porous-convection step (Sec. 3.2 of arXiv 2508.12501) and of the
// gradients of the multigrid solve.
//
// Vertex-centric kernels walk a vertex's couplings in the operator's SELL-64 layout; every
// edge term is written from the row vertex v's side with its neighbour u, in a form that does
// not depend on the edge orientation:
//   (y_hi - y_lo)(T_lo + T_hi)/2 * s_e  = (y_v - y_u)(T_v + T_u)/2   (b1_e times the sign s_e)
//   q_e (d0 T)_e                        = Q_vu (T_v - T_u),
//   Q_vu = -k_e ((p_v - p_u) - (y_v - y_u)(T_v + T_u)/2)
// where s_e = +1 if v is the edge's head.  Couplings with star1 = 0 are absent from the
// layout; every term here carries star1 or star1 k, so they contribute nothing.
// Gradients with respect to vertex coefficients are computed per edge, then summed into the
// vertices through a vertex -> incident-edge list (all vertices, natural numbering).
#include <hip/hip_runtime.h>

#include <mutex>

#include "hier.hpp"
#include "util.hpp"

namespace decmg {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int pcol(const void* col, bool d16, int idx, int row, int n) {
  if (d16) {
    const int c = static_cast<const int16_t*>(col)[idx];
    return c == kZeroSlot16 ? n : row + c;
  }
  return static_cast<const int32_t*>(col)[idx];
}

struct RowIter {
  int beg, end, lane;
  __device__ RowIter(const int32_t* sptr, int row) {
    const int s = row >> 6;
    beg = sptr[s];
    end = sptr[s + 1];
    lane = row & 63;
  }
};

// rhs_v = sum_e w_e (y_v - y_u)(T_v + T_u)/2   (d0^T W b1)
__global__ __launch_bounds__(kThreads) void k_por_rhs(const int32_t* __restrict__ sptr,
                                                      const void* __restrict__ col, int d16,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ T,
                                                      double* __restrict__ rhs, int32_t n) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const RowIter it(sptr, v);
  const double yv = y[v], Tv = T[v];
  double acc = 0.0;
  for (int k = it.beg; k < it.end; ++k) {
    const int idx = k * kSlice + it.lane;
    const int u = pcol(col, d16, idx, v, n);
    acc += w[idx] * ((yv - y[u]) * (0.5 * (Tv + T[u])));
  }
  rhs[v] = acc;
}

// T' = T + dt mask / star0 * ( -(1/phi) sum_e star1_e Q_vu (T_v - T_u) / 2
//                              - kappa sum_e star1_e (T_v - T_u) ),  or only the rate
// (the bracket times mask / star0) when add_T is 0
__global__ __launch_bounds__(kThreads) void k_por_update(
    const int32_t* __restrict__ sptr, const void* __restrict__ col, int d16,
    const double* __restrict__ s1, const double* __restrict__ ke, const double* __restrict__ y,
    const double* __restrict__ T, const double* __restrict__ P, const double* __restrict__ star0,
    const double* __restrict__ mask, double* __restrict__ Tout, int32_t n, double dt,
    double inv_phi, double kappa, int add_T) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const RowIter it(sptr, v);
  const double yv = y[v], Tv = T[v], Pv = P[v];
  double adv = 0.0, diff = 0.0;
  for (int k = it.beg; k < it.end; ++k) {
    const int idx = k * kSlice + it.lane;
    const int u = pcol(col, d16, idx, v, n);
    const double Tu = T[u];
    const double q = -ke[idx] * ((Pv - P[u]) - (yv - y[u]) * (0.5 * (Tv + Tu)));
    adv += 0.5 * s1[idx] * (q * (Tv - Tu));
    diff += s1[idx] * (Tv - Tu);
  }
  const double rate = mask[v] * (-inv_phi * adv - kappa * diff) / star0[v];
  Tout[v] = add_T ? Tv + dt * rate : rate;
}

__global__ void k_por_mu(const double* __restrict__ lam, const double* __restrict__ mask,
                         const double* __restrict__ star0, double* __restrict__ mu, int32_t n) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v < n) mu[v] = mask[v] * lam[v] / star0[v];
}

// adjoint pressure right-hand side: sum_e k_e c_e (T_v - T_u), c_e = star1_e (mu_v + mu_u)/2
__global__ __launch_bounds__(kThreads) void k_por_adj_rhs(const int32_t* __restrict__ sptr,
                                                          const void* __restrict__ col, int d16,
                                                          const double* __restrict__ s1,
                                                          const double* __restrict__ ke,
                                                          const double* __restrict__ T,
                                                          const double* __restrict__ mu,
                                                          double* __restrict__ rhs, int32_t n) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const RowIter it(sptr, v);
  const double Tv = T[v], mv = mu[v];
  double acc = 0.0;
  for (int k = it.beg; k < it.end; ++k) {
    const int idx = k * kSlice + it.lane;
    const int u = pcol(col, d16, idx, v, n);
    const double c = 0.5 * s1[idx] * (mv + mu[u]);
    acc += ke[idx] * (c * (Tv - T[u]));
  }
  rhs[v] = acc;
}

// lambda_n = lambda + dt * ( -(1/phi) [ sum c Q_vu + sum (k c (T_v-T_u) - w (psi_v-psi_u))
//                                        (y_v - y_u)/2 ] - kappa sum star1 (mu_v - mu_u) )
__global__ __launch_bounds__(kThreads) void k_por_adj_update(
    const int32_t* __restrict__ sptr, const void* __restrict__ col, int d16,
    const double* __restrict__ s1, const double* __restrict__ ke, const double* __restrict__ y,
    const double* __restrict__ T, const double* __restrict__ P, const double* __restrict__ mu,
    const double* __restrict__ lam, const double* __restrict__ psi, double* __restrict__ lam_out,
    int32_t n, double dt, double inv_phi, double kappa) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  const RowIter it(sptr, v);
  const double yv = y[v], Tv = T[v], Pv = P[v], mv = mu[v], psv = psi[v];
  double ta = 0.0, tb = 0.0, lm = 0.0;
  for (int k = it.beg; k < it.end; ++k) {
    const int idx = k * kSlice + it.lane;
    const int u = pcol(col, d16, idx, v, n);
    const double Tu = T[u], dyv = yv - y[u], sv = s1[idx], kv = ke[idx];
    const double c = 0.5 * sv * (mv + mu[u]);
    const double q = -kv * ((Pv - P[u]) - dyv * (0.5 * (Tv + Tu)));
    ta += c * q;
    tb += 0.5 * ((kv * (c * (Tv - Tu)) - (sv * kv) * (psv - psi[u])) * dyv);
    lm += sv * (mv - mu[u]);
  }
  lam_out[v] = lam[v] + dt * (-inv_phi * (ta + tb) - kappa * lm);
}

// per-edge dJ/dk_e of one porous step:
//   dt (-1/phi) (b1 - d0 p)_e (c_e (d0 T)_e - star1_e (d0 psi)_e)
__global__ void k_por_grad_edges(const int32_t* __restrict__ ea, const int32_t* __restrict__ eb,
                                 const double* __restrict__ s1e, const double* __restrict__ y,
                                 const double* __restrict__ T, const double* __restrict__ P,
                                 const double* __restrict__ mu, const double* __restrict__ psi,
                                 double* __restrict__ ge, int32_t ne, double dt, double inv_phi) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= ne) return;
  const int a = ea[e], b = eb[e];
  const double b1 = (y[b] - y[a]) * (0.5 * (T[a] + T[b]));
  const double c = 0.5 * s1e[e] * (mu[a] + mu[b]);
  ge[e] = dt * (-inv_phi) * ((b1 - (P[b] - P[a])) * (c * (T[b] - T[a]) - s1e[e] * (psi[b] - psi[a])));
}

// per-edge dJ/dk_e of the solve L u = b: -star1_e (d0 lambda)_e (d0 u)_e
__global__ void k_mg_grad_edges(const int32_t* __restrict__ ea, const int32_t* __restrict__ eb,
                                const double* __restrict__ s1e, const double* __restrict__ lam,
                                const double* __restrict__ u, double* __restrict__ ge, int32_t ne) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= ne) return;
  const int a = ea[e], b = eb[e];
  ge[e] = -s1e[e] * ((lam[b] - lam[a]) * (u[b] - u[a]));
}

// gw_e += -(lam_hi - lam_lo)(u_hi - u_lo): the derivative with respect to the edge weight
__global__ void k_mg_grad_w(const int32_t* __restrict__ ea, const int32_t* __restrict__ eb,
                            const double* __restrict__ lam, const double* __restrict__ u,
                            double* __restrict__ gw, int32_t ne) {
  const int e = blockIdx.x * kThreads + threadIdx.x;
  if (e >= ne) return;
  const int a = ea[e], b = eb[e];
  gw[e] += -((lam[b] - lam[a]) * (u[b] - u[a]));
}

// g_v += (1/2) sum over the edges at v of ge_e   (k_e = (k_lo + k_hi)/2), natural numbering
__global__ void k_edges_to_vertices(const int64_t* __restrict__ vptr,
                                    const int32_t* __restrict__ vinc, const double* __restrict__ ge,
                                    double* __restrict__ g, int32_t nv) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= nv) return;
  double acc = 0.0;
  for (int64_t q = vptr[v]; q < vptr[v + 1]; ++q) acc += ge[vinc[q]];
  g[v] += 0.5 * acc;
}

// ---- Runge-Kutta stage combinations and weighted RMS norms (internal order, n rows)

// out = y + h * sum_j c_j v_j over the m terms, summed in term order.
__global__ __launch_bounds__(kThreads) void k_rk_axpy(const double* __restrict__ y, k::RkTerms tm,
                                                      double h, double* __restrict__ out,
                                                      int32_t n) {
  const int v = blockIdx.x * kThreads + threadIdx.x;
  if (v >= n) return;
  double acc = 0.0;
  for (int j = 0; j < tm.m; ++j) acc += tm.c[j] * tm.v[j][v];
  out[v] = y[v] + h * acc;
}

// part[block] = sum over the block's rows of (scale * sum_j c_j v_j / sc)^2 with
// sc = atol + rtol * max(|u|, |w|).
__global__ __launch_bounds__(kThreads) void k_rk_wsq(k::RkTerms tm, double scale,
                                                     const double* __restrict__ u,
                                                     const double* __restrict__ w, double atol,
                                                     double rtol, double* __restrict__ part,
                                                     int32_t n) {
  __shared__ double red[kThreads / 64];
  const int v = blockIdx.x * kThreads + threadIdx.x;
  double s = 0.0;
  if (v < n) {
    double acc = 0.0;
    for (int j = 0; j < tm.m; ++j) acc += tm.c[j] * tm.v[j][v];
    const double sc = atol + rtol * fmax(fabs(u[v]), fabs(w[v]));
    const double e = scale * acc / sc;
    s = e * e;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) b += red[q];
    part[blockIdx.x] = b;
  }
}

// out[0] = sqrt(sum(part) / n), one workgroup.
__global__ __launch_bounds__(kThreads) void k_rk_rms_fin(const double* __restrict__ part,
                                                         int32_t nparts, int32_t n,
                                                         double* __restrict__ out) {
  __shared__ double red[kThreads / 64];
  double s = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kThreads) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int q = 0; q < kThreads / 64; ++q) b += red[q];
    out[0] = sqrt(b / double(n));
  }
}

inline unsigned blocks(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

// out += a * b entrywise (a null: a = 1) -- the chain rule of k = exp(g): dJ/dg = k dJ/dk
__global__ __launch_bounds__(kThreads) void k_mul_acc(int32_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     double* __restrict__ out) {
  const int32_t i = blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  out[i] += a ? a[i] * b[i] : b[i];
}

const void* colp(const Level& L) {
  return L.op.col16 ? static_cast<const void*>(L.op.col16) : static_cast<const void*>(L.op.col);
}

}  // namespace

// Work area of the allocation-free integrator: one copy on every GPU the library runs on, held
// until the process ends.  In host code this name is not a device address; host code uses the
// address rk_static_work() looks up for the current device.
static __device__ __align__(256) double scratch[kRkStaticWorkBytes / sizeof(double)];

namespace k {

double* rk_static_work() {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = -1;
  check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) throw DeviceError("device ordinal out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress");
    addr[dev] = p;
  }
  return static_cast<double*>(addr[dev]);
}

void mul_acc(int32_t n, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mul_acc, dim3(blocks(n)), dim3(kThreads), 0, s, n, a, b, out);
}

void rk_axpy(const double* y, const RkTerms& tm, double h, double* out, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_rk_axpy, dim3(blocks(n)), dim3(kThreads), 0, s, y, tm, h, out, n);
}
int rk_parts(int32_t n) { return int(blocks(n)); }
void rk_wrms(const RkTerms& tm, double scale, const double* u, const double* w, double atol,
             double rtol, double* part, double* out, int32_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_rk_wsq, dim3(blocks(n)), dim3(kThreads), 0, s, tm, scale, u, w, atol, rtol,
                     part, n);
  hipLaunchKernelGGL(k_rk_rms_fin, dim3(1), dim3(kThreads), 0, s, part, int32_t(blocks(n)), n, out);
}

void por_rhs(const Level& L, const PorousData& D, const double* T, double* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_por_rhs, dim3(blocks(L.n)), dim3(kThreads), 0, s, L.op.sptr, colp(L),
                     L.op.col16 ? 1 : 0, L.op.w64, D.y, T, rhs, L.n);
}
void por_update(const Level& L, const PorousData& D, const double* T, const double* P, double* Tout,
                double dt, double phi, double kappa, bool add_T, hipStream_t s) {
  hipLaunchKernelGGL(k_por_update, dim3(blocks(L.n)), dim3(kThreads), 0, s, L.op.sptr, colp(L),
                     L.op.col16 ? 1 : 0, D.s1, D.ke, D.y, T, P, D.star0, D.mask, Tout, L.n, dt,
                     1.0 / phi, kappa, add_T ? 1 : 0);
}
void por_mu(const Level& L, const PorousData& D, const double* lam, double* mu, hipStream_t s) {
  hipLaunchKernelGGL(k_por_mu, dim3(blocks(L.n)), dim3(kThreads), 0, s, lam, D.mask, D.star0, mu, L.n);
}
void por_adj_rhs(const Level& L, const PorousData& D, const double* T, const double* mu,
                 double* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_por_adj_rhs, dim3(blocks(L.n)), dim3(kThreads), 0, s, L.op.sptr, colp(L),
                     L.op.col16 ? 1 : 0, D.s1, D.ke, T, mu, rhs, L.n);
}
void por_adj_update(const Level& L, const PorousData& D, const double* T, const double* P,
                    const double* mu, const double* lam, const double* psi, double* lam_out,
                    double dt, double phi, double kappa, hipStream_t s) {
  hipLaunchKernelGGL(k_por_adj_update, dim3(blocks(L.n)), dim3(kThreads), 0, s, L.op.sptr, colp(L),
                     L.op.col16 ? 1 : 0, D.s1, D.ke, D.y, T, P, mu, lam, psi, lam_out, L.n, dt,
                     1.0 / phi, kappa);
}
void por_grad_k(const Level& L, const PorousData& D, const double* T, const double* P,
                const double* mu, const double* psi, double* gk_nat, double dt, double phi,
                hipStream_t s) {
  hipLaunchKernelGGL(k_por_grad_edges, dim3(blocks(D.ne)), dim3(kThreads), 0, s, D.ea, D.eb, D.s1e,
                     D.y, T, P, mu, psi, D.ge, D.ne, dt, 1.0 / phi);
  hipLaunchKernelGGL(k_edges_to_vertices, dim3(blocks(L.nv)), dim3(kThreads), 0, s, D.vptr, D.vinc,
                     D.ge, gk_nat, L.nv);
}
void mg_grad_w(const Level& L, const PorousData& D, const double* lam, const double* u,
               double* gw_nat, hipStream_t s) {
  (void)L;
  hipLaunchKernelGGL(k_mg_grad_w, dim3(blocks(D.ne)), dim3(kThreads), 0, s, D.ea, D.eb, lam, u,
                     gw_nat, D.ne);
}
void mg_grad_k(const Level& L, const PorousData& D, const double* lam, const double* u,
               double* gk_nat, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_grad_edges, dim3(blocks(D.ne)), dim3(kThreads), 0, s, D.ea, D.eb, D.s1e,
                     lam, u, D.ge, D.ne);
  hipLaunchKernelGGL(k_edges_to_vertices, dim3(blocks(L.nv)), dim3(kThreads), 0, s, D.vptr, D.vinc,
                     D.ge, gk_nat, L.nv);
}

}  // namespace k
}  // namespace decmg
