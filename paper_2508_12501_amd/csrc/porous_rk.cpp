// Adaptive explicit Runge-Kutta integration of the porous-convection model (Sec. 3.2: the
// method of lines, dT/dt = rhs(T) with one pressure solve per right-hand side).  The pair is
// Dormand and Prince's 5(4) (Dormand & Prince 1980, "A family of embedded Runge-Kutta
// formulae"): seven stages whose last is the next step's first, the 5th-order result kept and
// the embedded 4th-order one used for the error.  The step-size rule and the starting step
// follow Hairer, Norsett and Wanner, Solving ODEs I, Sec. II.4.  Host control flow; every
// vector operation is a kernel on the stream, with one host read of the error norm per step.
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "hier.hpp"
#include "solver.hpp"
#include "util.hpp"

namespace decmg {

namespace {

// Butcher tableau: stage s (1..6) is y + h sum_{j<s} A[s][j] k_j; row 6 is the 5th-order
// weights (the stage-7 input is the new solution).  E = b5 - b4.
constexpr double A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};
constexpr double B4[7] = {5179.0 / 57600, 0, 7571.0 / 16695, 393.0 / 640, -92097.0 / 339200,
                          187.0 / 2100, 1.0 / 40};
constexpr double C[7] = {0, 1.0 / 5, 3.0 / 10, 4.0 / 5, 8.0 / 9, 1, 1};   // stage times / h

constexpr double kSafety = 0.9, kFacMin = 0.2, kFacMax = 10.0;

struct DevBuf {
  double* p = nullptr;
  explicit DevBuf(int64_t n) {
    check_hip(hipMalloc(&p, std::max<int64_t>(n, 1) * sizeof(double)), "hipMalloc");
    check_hip(hipMemset(p, 0, std::max<int64_t>(n, 1) * sizeof(double)), "hipMemset");
  }
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

struct HostScalar {
  double* p = nullptr;
  HostScalar() { check_hip(hipHostMalloc(reinterpret_cast<void**>(&p), sizeof(double), 0), "hipHostMalloc"); }
  ~HostScalar() {
    if (p) (void)hipHostFree(p);
  }
  HostScalar(const HostScalar&) = delete;
  HostScalar& operator=(const HostScalar&) = delete;
};

// terms sum_j c_j v_j with the zero coefficients left out (adding 0 * v_j changes nothing)
k::RkTerms terms(std::initializer_list<std::pair<const double*, double>> list) {
  k::RkTerms t{};
  t.m = 0;
  for (const auto& [v, c] : list)
    if (c != 0.0) {
      t.v[t.m] = v;
      t.c[t.m] = c;
      ++t.m;
    }
  return t;
}

// Device vectors of one integration (twelve of n + 1 doubles, the error norm and its reduction
// partials) and a pinned host double for reading the norm.
struct Work {
  double *y, *yn, *ys, *dscal, *part, *p0, *p1;
  double* kv[7];
  double* host;
};

// The work of porous_integrate: allocated for the call, freed at its end.
struct OwnedWork {
  DevBuf y, yn, ys, dscal, part, p0, p1;
  std::vector<std::unique_ptr<DevBuf>> kb;
  HostScalar hs;
  Work w{};
  explicit OwnedWork(int32_t n)
      : y(n + 1), yn(n + 1), ys(n + 1), dscal(1), part(k::rk_parts(n)), p0(n + 1), p1(n + 1) {
    w = Work{y.p, yn.p, ys.p, dscal.p, part.p, p0.p, p1.p, {}, hs.p};
    for (int j = 0; j < 7; ++j) {
      kb.emplace_back(std::make_unique<DevBuf>(n + 1));
      w.kv[j] = kb.back()->p;
    }
  }
};

// Layout of the same work in the static area of porous_integrate_noalloc: every vector starts
// on a 256-byte boundary.  Returns the doubles used; with base == nullptr it only counts.
size_t static_layout(int32_t n, double* base, Work* w) {
  const size_t vec = (size_t(n) + 1 + 31) / 32 * 32;
  const size_t parts = (size_t(k::rk_parts(n)) + 31) / 32 * 32;
  size_t off = 0;
  auto take = [&](size_t len) {
    double* p = base ? base + off : nullptr;
    off += len;
    return p;
  };
  Work v{};
  v.y = take(vec);
  v.yn = take(vec);
  v.ys = take(vec);
  v.p0 = take(vec);
  v.p1 = take(vec);
  for (double*& q : v.kv) q = take(vec);
  v.dscal = take(32);
  v.part = take(parts);
  if (w) *w = v;
  return off;
}

struct Integrator {
  Hierarchy& H;
  const porous_rk_opts& o;
  PorousParams prm;
  hipStream_t s;
  int32_t n;
  porous_rk_stats st{};
  Work w;
  double* kv[7];
  // Initial guesses of the pressure solves: the first starts from zero, the second from the
  // first's result, every later one from the linear extrapolation in time of the last two
  // pressures (p1 at time t1, p0 at t0) to the time of the new right-hand side.
  int npres = 0;
  double t0p = 0.0, t1p = 0.0;

  Integrator(Hierarchy& H_, const porous_rk_opts& o_, hipStream_t s_, const Work& w_)
      : H(H_), o(o_), prm(porous_params_of(o_.model)), s(s_), n(H_.lv.back()->n), w(w_) {
    for (int j = 0; j < 7; ++j) kv[j] = w.kv[j];
  }

  // kout = rhs(yin) for the state at time t_eval; returns the pressure solve's status
  int rhs(const double* yin, double* kout, double t_eval) {
    Level& F = *H.lv.back();
    PorousData& D = H.por;
    k::por_rhs(F, D, yin, H.sb, s);
    if (npres >= 2 && t1p != t0p) {
      const double theta = std::min(2.0, std::max(-2.0, (t_eval - t1p) / (t1p - t0p)));
      k::rk_axpy(w.p1, terms({{w.p1, 1.0}, {w.p0, -1.0}}), theta, H.sx, n, s);
    } else if (npres == 1) {
      check_hip(hipMemcpyAsync(H.sx, w.p1, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s),
                "hipMemcpyAsync");
    }
    mg_result r{};
    const int code = run_pcg(H, prm.solve, nullptr, nullptr, &r, s, npres >= 1);
    std::swap(w.p0, w.p1);
    check_hip(hipMemcpyAsync(w.p1, H.sx, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s),
              "hipMemcpyAsync");
    t0p = t1p;
    t1p = t_eval;
    npres = std::min(npres + 1, 2);
    k::por_update(F, D, yin, H.sx, kout, 1.0, prm.phi, prm.kappa(), false, s);
    st.rhs_evals += 1;
    st.pressure_iterations += r.iterations;
    return code;
  }

  double read_norm() {
    check_hip(hipMemcpyAsync(w.host, w.dscal, sizeof(double), hipMemcpyDeviceToHost, s),
              "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    return *w.host;
  }

  double wrms(const k::RkTerms& t, double scale, const double* u, const double* u2) {
    k::rk_wrms(t, scale, u, u2, o.atol, o.rtol, w.part, w.dscal, n, s);
    return read_norm();
  }

  // Hairer-Norsett-Wanner starting step from f0 = kv[0] (one more right-hand side)
  int start_step(double& h) {
    const double d0 = wrms(terms({{w.y, 1.0}}), 1.0, w.y, w.y);
    const double d1 = wrms(terms({{kv[0], 1.0}}), 1.0, w.y, w.y);
    double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 : 0.01 * d0 / d1;
    h0 = std::min(h0, o.t_end);
    k::rk_axpy(w.y, terms({{kv[0], 1.0}}), h0, w.ys, n, s);
    if (int code = rhs(w.ys, kv[1], h0); code != MG_OK) return code;
    const double d2 = wrms(terms({{kv[1], 1.0}, {kv[0], -1.0}}), 1.0 / h0, w.y, w.y);
    const double dm = std::max(d1, d2);
    const double h1 = dm <= 1e-15 ? std::max(1e-6, h0 * 1e-3) : std::pow(0.01 / dm, 1.0 / 5.0);
    h = std::min({100.0 * h0, h1, o.t_end});
    return MG_OK;
  }

  // stages 2..7 of a step of size h from (y, kv[0]) at time t; the new solution lands in yn,
  // its right-hand side in kv[6]
  int stages(double t, double h) {
    for (int si = 1; si <= 6; ++si) {
      const double* a = A[si];
      const k::RkTerms tm = terms({{kv[0], a[0]}, {kv[1], a[1]}, {kv[2], a[2]}, {kv[3], a[3]},
                                   {kv[4], a[4]}, {kv[5], a[5]}});
      double* dst = si == 6 ? w.yn : w.ys;
      k::rk_axpy(w.y, tm, h, dst, n, s);
      if (int code = rhs(dst, kv[si], t + C[si] * h); code != MG_OK) return code;
    }
    return MG_OK;
  }

  double step_error(double h) {
    const double* b5 = A[6];
    const k::RkTerms t = terms({{kv[0], b5[0] - B4[0]}, {kv[1], b5[1] - B4[1]},
                                {kv[2], b5[2] - B4[2]}, {kv[3], b5[3] - B4[3]},
                                {kv[4], b5[4] - B4[4]}, {kv[5], b5[5] - B4[5]},
                                {kv[6], 0.0 - B4[6]}});
    return wrms(t, h, w.y, w.yn);
  }

  int run(const double* T0_nat, int32_t n_save, const double* t_save, double* Tsave_nat,
          double* Tend_nat) {
    Level& F = *H.lv.back();
    const int32_t nv = F.nv;
    k::gather<double>(F.perm, n, T0_nat, w.y, s);
    st.h_min = HUGE_VAL;
    st.h_max = 0.0;
    int code = rhs(w.y, kv[0], 0.0);
    if (code != MG_OK) return code;
    double h = o.h0;
    if (!o.fixed_step && !(h > 0)) {
      if ((code = start_step(h)) != MG_OK) return code;
    }
    double t = 0.0, facmax = kFacMax;
    int32_t next_save = 0;
    while (t < o.t_end) {
      if (st.accepted + st.rejected >= o.max_steps) break;
      if (h < 1e-14 * o.t_end) break;
      const double t_stop = next_save < n_save ? t_save[next_save] : o.t_end;
      bool hit = false;
      if (t + 1.01 * h >= t_stop) {
        h = t_stop - t;
        hit = true;
      }
      if ((code = stages(t, h)) != MG_OK) return code;
      double err = 0.0;
      if (!o.fixed_step) err = step_error(h);
      if (o.fixed_step || err <= 1.0) {
        t = hit ? t_stop : t + h;
        std::swap(w.y, w.yn);
        std::swap(kv[0], kv[6]);
        st.accepted += 1;
        st.h_min = std::min(st.h_min, h);
        st.h_max = std::max(st.h_max, h);
        if (hit && next_save < n_save) {
          k::scatter<double>(F.perm, n, w.y, Tsave_nat + int64_t(next_save) * nv, s);
          ++next_save;
        }
        if (o.fixed_step) {
          h = o.h0;
        } else {
          const double fac = err == 0.0 ? facmax : kSafety * std::pow(err, -1.0 / 5.0);
          h *= std::min(facmax, std::max(kFacMin, fac));
          facmax = kFacMax;
        }
      } else {
        st.rejected += 1;
        const double fac = std::isfinite(err) ? kSafety * std::pow(err, -1.0 / 5.0) : kFacMin;
        h *= std::max(kFacMin, fac);
        facmax = 1.0;
      }
    }
    st.t = t;
    if (st.accepted == 0) st.h_min = 0.0;
    k::scatter<double>(F.perm, n, w.y, Tend_nat, s);
    check_hip(hipGetLastError(), "kernel launch");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    return t >= o.t_end ? MG_OK : MG_ENOCONV;
  }
};

}  // namespace

int run_porous_integrate(Hierarchy& H, const porous_rk_opts& o, const double* T0_nat,
                         int32_t n_save, const double* t_save, double* Tsave_nat,
                         double* Tend_nat, porous_rk_stats* stats, hipStream_t s) {
  porous_check(H, porous_params_of(o.model));
  porous_prepare(H);
  OwnedWork ow(H.lv.back()->n);
  Integrator I(H, o, s, ow.w);
  const int code = I.run(T0_nat, n_save, t_save, Tsave_nat, Tend_nat);
  if (stats) *stats = I.st;
  return code;
}

size_t porous_integrate_static_bytes(int32_t n) { return static_layout(n, nullptr, nullptr) * sizeof(double); }

int run_porous_integrate_noalloc(Hierarchy& H, const porous_rk_opts& o, const double* T0_nat,
                                 int32_t n_save, const double* t_save, double* Tsave_nat,
                                 double* Tend_nat, porous_rk_stats* stats, hipStream_t s) {
  porous_check(H, porous_params_of(o.model));
  const int32_t n = H.lv.back()->n;
  const size_t need = porous_integrate_static_bytes(n);
  if (need > kRkStaticWorkBytes)
    throw std::invalid_argument("porous_integrate_noalloc: " + std::to_string(n) +
                                " unknowns need " + std::to_string(need) +
                                " bytes of work area; the static area holds " +
                                std::to_string(kRkStaticWorkBytes));
  if (!H.por.ready)
    throw std::invalid_argument(
        "the porous data of this hierarchy is not set up: one porous_step, porous_rhs or "
        "porous_integrate call on it sets it up");
  // refreshes the edge coefficients after a coefficient change (host-to-device copy only:
  // set-up has allocated every porous buffer)
  porous_prepare(H);
  Work w{};
  double* base = k::rk_static_work();
  static_layout(n, base, &w);
  w.host = H.aux_host;
  // the area keeps the previous call's contents: start from zeros, as freshly allocated work
  // does (every vector's last entry is the zero slot that couplings to non-unknowns read)
  k::fill<double>(base, int64_t(need / sizeof(double)), 0.0, s);
  porous_rk_opts oe = o;
  oe.model.solve.use_graph = 0;   // capturing a graph allocates
  Integrator I(H, oe, s, w);
  const int code = I.run(T0_nat, n_save, t_save, Tsave_nat, Tend_nat);
  if (stats) *stats = I.st;
  return code;
}

}  // namespace decmg
