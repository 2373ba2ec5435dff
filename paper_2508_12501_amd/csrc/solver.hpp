// Host entry points shared by the C-ABI layer.
#pragma once
#include "hier.hpp"

namespace decmg {

template <typename T>
LevelVecs<T>& vecs(Level& L);

// One V(nu1, nu2) cycle on level l for A_l x = b.  x_init == nullptr means x = 0 (the first
// pre-sweep then reads only b and the diagonal); otherwise x_init is the initial guess and
// one of its buffers.  Returns the buffer that holds the result.  chk: the finest level's
// opening sweeps also take the Krylov loop's pending convergence check.
template <typename T>
T* vcycle(Hierarchy& H, int l, const T* b, T* x_init, const mg_opts& o, const int* done,
          hipStream_t s, bool chk = false);
// Whether a CG/FCG iteration with these options leaves its convergence check to the first
// kernel of the next iteration's cycle (see jacobi_two_chk).
bool check_fused_ok(const Hierarchy& H, const mg_opts& o);

Hierarchy* build_hierarchy(const Mesh& base, const mg_hier_opts& o);
// Levels over given meshes whose interpolation rows are already set (set_interp_from_geomap).
Hierarchy* build_hierarchy_maps(std::vector<Mesh> meshes, bool nested_ids, const mg_hier_opts& o);
void upload_weights(Hierarchy& H);
// Edge coefficient of level l (natural edge order): the edge field when one is set, else
// (k_lo + k_hi)/2 from the vertex field at the level's own ids; empty when k = 1.
std::vector<double> level_edge_coeff(const Hierarchy& H, size_t l);
// Every level's edge coefficient from the finest level's: a coarse edge takes the mean of the
// fine edges it was split into (two halves, or three thirds on a cubic subdivision).
std::vector<std::vector<double>> coarsen_edge_coeff(const Hierarchy& H, std::vector<double> ke);
// warm_start (internal right-hand side only, b_nat == nullptr): start from the iterate left in
// H.sx by the previous solve instead of zero.  check_compat: a natural-boundary b_nat outside
// the operator's range ends the solve with MG_EINCOMPAT (the caller's right-hand sides; the
// adjoint's upstream gradient is projected instead).
int run_pcg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
            hipStream_t s, bool warm_start = false, bool check_compat = false);
int run_mg(Hierarchy& H, const mg_opts& o, const double* b_nat, double* x_nat, mg_result* res,
           hipStream_t s);

// porous step, its adjoint and the adjoint of mg_pcg (porous.cpp)
struct PorousParams {
  double Ra, phi, dt;
  mg_opts solve;
  double delta_T = 1.0, y_len = 1.0;
  double kappa() const { return delta_T * y_len / (phi * Ra); }
};
int run_porous_step(Hierarchy& H, const PorousParams& p, const double* T_nat, double* Tout_nat,
                    double* p_nat, mg_result* res, hipStream_t s);
// Dormand-Prince 5(4) integration of dT/dt = rhs (porous_rk.cpp).
int run_porous_integrate(Hierarchy& H, const porous_rk_opts& o, const double* T0_nat,
                         int32_t n_save, const double* t_save, double* Tsave_nat,
                         double* Tend_nat, porous_rk_stats* stats, hipStream_t s);
// The same integration with its work in this GPU's static work area (no device or pinned
// allocation; the pressure solves run eagerly).
int run_porous_integrate_noalloc(Hierarchy& H, const porous_rk_opts& o, const double* T0_nat,
                                 int32_t n_save, const double* t_save, double* Tsave_nat,
                                 double* Tend_nat, porous_rk_stats* stats, hipStream_t s);
// bytes of static work area the allocation-free integration needs for n unknowns
size_t porous_integrate_static_bytes(int32_t n);
// Porous data of the finest level (built on first use, refreshed when k changes).
void porous_prepare(Hierarchy& H);
void porous_check(const Hierarchy& H, const PorousParams& p);
PorousParams porous_params_of(const porous_params& p);
// dT/dt of the step (no time step): porous_step = T + dt * rhs.
int run_porous_rhs(Hierarchy& H, const PorousParams& p, const double* T_nat, double* rhs_nat,
                   double* p_nat, mg_result* res, hipStream_t s);
int run_porous_adjoint(Hierarchy& H, const PorousParams& p, const double* T_nat,
                       const double* p_nat, const double* lam_nat, double* lam_out_nat,
                       double* gk_nat, double* psi_nat, hipStream_t s);
int run_pcg_adjoint(Hierarchy& H, const mg_opts& o, const double* u_nat, const double* gu_nat,
                    double* gb_nat, double* gk_nat, double* gw_nat, mg_result* res,
                    hipStream_t s);
void free_porous(Hierarchy& H);

}  // namespace decmg
