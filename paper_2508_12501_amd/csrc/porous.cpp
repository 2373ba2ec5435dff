// Host orchestration of the porous-convection step (Sec. 3.2 of arXiv 2508.12501), its
// discrete adjoint, and the adjoint of the multigrid-preconditioned solve.  The pressure and
// adjoint-pressure solves run the same MG-PCG as mg_pcg, on internal-order vectors.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>

#include "hier.hpp"
#include "solver.hpp"
#include "util.hpp"

namespace decmg {

namespace {

template <typename T>
T* dev_upload(const std::vector<T>& h) {
  T* d = nullptr;
  check_hip(hipMalloc(&d, std::max<size_t>(h.size(), 1) * sizeof(T)), "hipMalloc");
  if (!h.empty())
    check_hip(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
  return d;
}

double* dev_zeros(int64_t n) {
  double* d = nullptr;
  check_hip(hipMalloc(&d, std::max<int64_t>(n, 1) * sizeof(double)), "hipMalloc");
  check_hip(hipMemset(d, 0, std::max<int64_t>(n, 1) * sizeof(double)), "hipMemset");
  return d;
}

void ensure(Hierarchy& H) {
  PorousData& D = H.por;
  Level& F = *H.lv.back();
  const Mesh& m = F.mesh;
  const int32_t n = F.n;
  if (!D.ready) {
    std::vector<double> y(n + 1, 0.0), s0(n + 1, 1.0), mask(n + 1, 1.0);
    double ymin = 1e300, ymax = -1e300;
    for (int64_t v = 0; v < m.nv; ++v) {
      ymin = std::min(ymin, m.xyz[3 * v + 1]);
      ymax = std::max(ymax, m.xyz[3 * v + 1]);
    }
    for (int32_t k = 0; k < n; ++k) {
      const int32_t v = F.perm_h[k];
      y[k] = m.xyz[3 * v + 1];
      s0[k] = m.star0[v];
      mask[k] = (y[k] == ymin || y[k] == ymax) ? 0.0 : 1.0;
    }
    D.y = dev_upload(y);
    D.star0 = dev_upload(s0);
    D.mask = dev_upload(mask);
    std::vector<double> s1(F.entry_edge.size(), 0.0);
    for (size_t i = 0; i < s1.size(); ++i)
      if (F.entry_edge[i] >= 0) s1[i] = m.star1[F.entry_edge[i]];
    D.s1 = dev_upload(s1);
    D.ne = int32_t(m.ne);
    std::vector<int32_t> ea(m.ne), eb(m.ne);
    for (int64_t e = 0; e < m.ne; ++e) {
      const int32_t a = F.inv_h[m.edge[2 * e]], b = F.inv_h[m.edge[2 * e + 1]];
      ea[e] = a >= 0 ? a : n;
      eb[e] = b >= 0 ? b : n;
    }
    D.ea = dev_upload(ea);
    D.eb = dev_upload(eb);
    D.s1e = dev_upload(m.star1);
    D.ge = dev_zeros(m.ne);
    std::vector<int64_t> vptr(m.nv + 1, 0);
    for (int64_t e = 0; e < m.ne; ++e) {
      vptr[m.edge[2 * e] + 1]++;
      vptr[m.edge[2 * e + 1] + 1]++;
    }
    for (int64_t v = 0; v < m.nv; ++v) vptr[v + 1] += vptr[v];
    std::vector<int32_t> vinc(vptr[m.nv]);
    std::vector<int64_t> pos(vptr.begin(), vptr.end() - 1);
    for (int64_t e = 0; e < m.ne; ++e) {
      vinc[pos[m.edge[2 * e]]++] = int32_t(e);
      vinc[pos[m.edge[2 * e + 1]]++] = int32_t(e);
    }
    D.vptr = dev_upload(vptr);
    D.vinc = dev_upload(vinc);
    for (double** p : {&D.T, &D.T2, &D.P, &D.Lm, &D.L2, &D.M, &D.U}) *p = dev_zeros(n + 1);
    D.ready = true;
  }
  if (D.kversion != H.kversion) {
    const std::vector<double> kedge = level_edge_coeff(H, H.lv.size() - 1);
    std::vector<double> ke(F.entry_edge.size(), 0.0);
    for (size_t i = 0; i < ke.size(); ++i) {
      const int32_t e = F.entry_edge[i];
      if (e < 0) continue;
      ke[i] = kedge.empty() ? 1.0 : kedge[e];
    }
    if (!D.ke) check_hip(hipMalloc(&D.ke, std::max<size_t>(ke.size(), 1) * sizeof(double)), "hipMalloc");
    if (!ke.empty())
      check_hip(hipMemcpy(D.ke, ke.data(), ke.size() * sizeof(double), hipMemcpyHostToDevice),
                "hipMemcpy");
    D.kversion = H.kversion;
  }
}

void check_params(const Hierarchy& H, const PorousParams& p) {
  if (H.bc != MG_BC_NATURAL)
    throw std::invalid_argument("the porous step needs a hierarchy with natural boundaries");
  if (!(p.Ra > 0) || !(p.phi > 0) || !std::isfinite(p.Ra) || !std::isfinite(p.phi) ||
      !(p.delta_T > 0) || !(p.y_len > 0) || !std::isfinite(p.delta_T) || !std::isfinite(p.y_len))
    throw std::invalid_argument("Ra, phi, delta_T and y_len must be finite and positive");
}

}  // namespace

void porous_prepare(Hierarchy& H) { ensure(H); }
void porous_check(const Hierarchy& H, const PorousParams& p) { check_params(H, p); }
PorousParams porous_params_of(const porous_params& p) {
  PorousParams q{p.Ra, p.phi, p.dt, p.solve};
  q.delta_T = p.delta_T;
  q.y_len = p.y_len;
  return q;
}

namespace {

// Pressure (or adjoint pressure) solve of the right-hand side already in H.sb; result in H.sx.
int solve_internal(Hierarchy& H, const mg_opts& o, mg_result* res, hipStream_t s) {
  return run_pcg(H, o, nullptr, nullptr, res, s);
}

}  // namespace

int run_porous_step(Hierarchy& H, const PorousParams& p, const double* T_nat, double* Tout_nat,
                    double* p_nat, mg_result* res, hipStream_t s) {
  check_params(H, p);
  ensure(H);
  PorousData& D = H.por;
  Level& F = *H.lv.back();
  k::gather<double>(F.perm, F.n, T_nat, D.T, s);
  k::por_rhs(F, D, D.T, H.sb, s);
  const int st = solve_internal(H, p.solve, res, s);
  k::por_update(F, D, D.T, H.sx, D.T2, p.dt, p.phi, p.kappa(), true, s);
  k::scatter<double>(F.perm, F.n, D.T2, Tout_nat, s);
  if (p_nat) k::scatter<double>(F.perm, F.n, H.sx, p_nat, s);
  check_hip(hipGetLastError(), "kernel launch");
  return st;
}

int run_porous_rhs(Hierarchy& H, const PorousParams& p, const double* T_nat, double* rhs_nat,
                   double* p_nat, mg_result* res, hipStream_t s) {
  check_params(H, p);
  ensure(H);
  PorousData& D = H.por;
  Level& F = *H.lv.back();
  k::gather<double>(F.perm, F.n, T_nat, D.T, s);
  k::por_rhs(F, D, D.T, H.sb, s);
  const int st = solve_internal(H, p.solve, res, s);
  k::por_update(F, D, D.T, H.sx, D.T2, 1.0, p.phi, p.kappa(), false, s);
  k::scatter<double>(F.perm, F.n, D.T2, rhs_nat, s);
  if (p_nat) k::scatter<double>(F.perm, F.n, H.sx, p_nat, s);
  check_hip(hipGetLastError(), "kernel launch");
  return st;
}

int run_porous_adjoint(Hierarchy& H, const PorousParams& p, const double* T_nat,
                       const double* p_nat, const double* lam_nat, double* lam_out_nat,
                       double* gk_nat, double* psi_nat, hipStream_t s) {
  check_params(H, p);
  ensure(H);
  PorousData& D = H.por;
  Level& F = *H.lv.back();
  const int32_t n = F.n;
  k::gather<double>(F.perm, n, T_nat, D.T, s);
  int st = MG_OK;
  if (p_nat) {
    k::gather<double>(F.perm, n, p_nat, D.P, s);
  } else {
    k::por_rhs(F, D, D.T, H.sb, s);
    st = solve_internal(H, p.solve, nullptr, s);
    check_hip(hipMemcpyAsync(D.P, H.sx, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s),
              "hipMemcpyAsync");
    if (st != MG_OK) return st;
  }
  k::gather<double>(F.perm, n, lam_nat, D.Lm, s);
  k::por_mu(F, D, D.Lm, D.M, s);
  k::por_adj_rhs(F, D, D.T, D.M, H.sb, s);
  st = solve_internal(H, p.solve, nullptr, s);
  k::por_adj_update(F, D, D.T, D.P, D.M, D.Lm, H.sx, D.L2, p.dt, p.phi, p.kappa(), s);
  if (gk_nat) k::por_grad_k(F, D, D.T, D.P, D.M, H.sx, gk_nat, p.dt, p.phi, s);
  k::scatter<double>(F.perm, n, D.L2, lam_out_nat, s);
  if (psi_nat) k::scatter<double>(F.perm, n, H.sx, psi_nat, s);
  check_hip(hipGetLastError(), "kernel launch");
  return st;
}

int run_pcg_adjoint(Hierarchy& H, const mg_opts& o, const double* u_nat, const double* gu_nat,
                    double* gb_nat, double* gk_nat, double* gw_nat, mg_result* res,
                    hipStream_t s) {
  const int st = run_pcg(H, o, gu_nat, gb_nat, res, s);
  if (gw_nat) {
    ensure(H);
    PorousData& D = H.por;
    Level& F = *H.lv.back();
    k::gather<double>(F.perm, F.n, u_nat, D.U, s);
    k::mg_grad_w(F, D, H.sx, D.U, gw_nat, s);
    check_hip(hipGetLastError(), "kernel launch");
  }
  if (gk_nat) {
    ensure(H);
    PorousData& D = H.por;
    Level& F = *H.lv.back();
    // u enters only through d0 u, so its mean (natural boundary) does not matter
    k::gather<double>(F.perm, F.n, u_nat, D.U, s);
    k::mg_grad_k(F, D, H.sx, D.U, gk_nat, s);
    check_hip(hipGetLastError(), "kernel launch");
  }
  return st;
}

void free_porous(Hierarchy& H) {
  PorousData& D = H.por;
  for (void* p : {(void*)D.s1, (void*)D.ke, (void*)D.y, (void*)D.star0, (void*)D.mask, (void*)D.ea,
                  (void*)D.eb, (void*)D.s1e, (void*)D.ge, (void*)D.vptr, (void*)D.vinc, (void*)D.T,
                  (void*)D.T2, (void*)D.P, (void*)D.Lm, (void*)D.L2, (void*)D.M, (void*)D.U})
    if (p) (void)hipFree(p);
  D = PorousData();
}

}  // namespace decmg
