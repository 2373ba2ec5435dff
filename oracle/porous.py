"""Darcy-Boussinesq porous convection on the DEC and its discrete adjoint -- FP64 reference.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The model is Sec. 3.2 (Eq. poisson,
Eqs. dec_darcy .. dec_pconv_heat_up and the diagram Fig. pc_decapode) with alpha rho0 |g| = 1
and k/eta scale 1 (the paper sets alpha rho0 = 1/g and k_etaf = 1), which leaves the advection
factor 1/phi and the diffusivity kappa = Delta T y_max / (phi Ra), the paper's product for
lambda / (rho0 c_p); the scaled form takes Delta T = y_max = 1.  Readings:

* Q13 edge permeability k_e = (k_lo + k_hi) / 2 from a vertex field k = exp(g);
* Q14 buoyancy 1-form b1 = yhat^flat wedge T, the wedge of a 1-form and a 0-form being the
  endpoint average: b1_e = (y_hi - y_lo) (T_lo + T_hi) / 2; hot fluid rises;
* Darcy flux q = -K (d0 p - b1);  delta q = 0 gives d0^T W d0 p = d0^T W b1, W = star1 K;
* advection L_q T as star0^{-1} (q wedge star1 d0 T): sum over edges at a vertex of
  star1_e q_e (d0 T)_e / 2; diffusion -star0^{-1} L T with L = d0^T star1 d0;
* bc: dT/dt = 0 on the walls, the vertices of smallest and of largest y (y = 0 and y = 1 on
  the unit square); natural boundary elsewhere;
* Q16 forward Euler with a fixed dt (a parameter of the step, not differentiated);
* Q17 the pressure has natural boundaries (kernel = constants); it is the zero-mean solution.

The adjoint is the exact transpose of the discrete step (implicit-function form for the
pressure solve), derived in closed form; it is pinned against central finite differences.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dec
from . import multigrid as omg


class PorousModel:
    """One square mesh (natural-BC hierarchy) with permeability k = exp(g) at its vertices."""

    def __init__(self, h: omg.Hierarchy, g: np.ndarray, Ra: float = 1000.0, phi: float = 0.1,
                 dt: float | None = None, solver: str = "direct", rtol: float = 1e-10,
                 delta_T: float = 1.0, y_len: float = 1.0):
        assert h.bc == "natural"
        self.h = h
        lv = h.fine
        self.lv = lv
        self.Ra, self.phi = Ra, phi
        self.kappa = delta_T * y_len / (phi * Ra)
        self.solver, self.rtol = solver, rtol
        self.d0 = sp.csr_matrix(lv.d0, dtype=np.float64)
        self.absd0 = abs(self.d0)
        self.y = lv.xyz[:, 1].copy()
        self.dy = self.d0 @ self.y                       # yhat^flat: y_hi - y_lo per edge
        self.star1, self.star0 = lv.star1, lv.star0
        self.L1 = dec.laplacian(lv.d0, lv.star1)         # unit-k Laplacian (diffusion)
        self.wall = (self.y == self.y.min()) | (self.y == self.y.max())
        self.mask = (~self.wall).astype(np.float64)
        self.set_g(g)
        if dt is None:
            dt = stable_dt(lv, self.kv, Ra, phi)
        self.dt = dt

    def set_g(self, g):
        self.g = np.asarray(g, dtype=np.float64)
        self.kv = np.exp(self.g)
        self.h.set_vertex_coeff(self.kv)
        e = self.lv.edges
        self.ke = 0.5 * (self.kv[e[:, 0]] + self.kv[e[:, 1]])
        self.W = self.star1 * self.ke
        self.LK = self.lv.A                             # d0^T diag(W) d0 (set_vertex_coeff)
        self._lu = None

    # -- pieces of one step
    def buoyancy(self, T):
        return self.dy * (0.5 * (self.absd0 @ T))       # b1_e = dy_e (T_lo + T_hi)/2

    def solve(self, rhs):
        """Zero-mean solution of L_K p = rhs."""
        if self.solver == "direct":
            # the definition of multigrid.direct_solve (ground vertex 0, solve, remove the
            # mean) with the sparse LU factor kept while k does not change
            if self._lu is None:
                import scipy.sparse.linalg as spla
                self._lu = spla.splu(sp.csc_matrix(self.LK)[1:, 1:])
            b = rhs - rhs.mean()
            x = np.zeros_like(b)
            x[1:] = self._lu.solve(b[1:])
            return x - x.mean()
        x, k, _ = omg.mg_pcg(self.h, rhs, rtol=self.rtol)
        self.last_iterations = k
        return x

    def pressure(self, T):
        b1 = self.buoyancy(T)
        rhs = self.d0.T @ (self.W * b1)
        return self.solve(rhs), b1

    def tdot(self, T, p=None):
        if p is None:
            p, b1 = self.pressure(T)
        else:
            b1 = self.buoyancy(T)
        q = -self.ke * (self.d0 @ p - b1)
        adv = 0.5 * (self.absd0.T @ (self.star1 * q * (self.d0 @ T)))
        diff = self.L1 @ T
        return self.mask * (-(1.0 / self.phi) * adv - self.kappa * diff) / self.star0, p

    def rhs(self, T):
        """dT/dt of the method of lines (the bracket of the step without dt)."""
        return self.tdot(T)[0]

    def step(self, T):
        Td, p = self.tdot(T)
        return T + self.dt * Td, p

    def rollout(self, T0, steps):
        T = T0.copy()
        for _ in range(steps):
            T, _ = self.step(T)
        return T

    # -- adjoint of one step: returns lambda_n and the increment of dJ/dk_v.  The pressure p
    # and the adjoint pressure psi are solved for unless given.
    def step_adjoint(self, T, lam, p=None, psi=None):
        if p is None:
            p, b1 = self.pressure(T)
        else:
            b1 = self.buoyancy(T)
        mu = self.mask * lam / self.star0
        d0T = self.d0 @ T
        q = -self.ke * (self.d0 @ p - b1)
        c = 0.5 * self.star1 * (self.absd0 @ mu)        # c_e = star1_e (mu_lo + mu_hi)/2
        g = c * d0T
        if psi is None:
            psi = self.solve(self.d0.T @ (self.ke * g))  # adjoint pressure
        d0psi = self.d0 @ psi
        h = self.ke * g - self.W * d0psi
        jac_t = (-(1.0 / self.phi) * (self.d0.T @ (c * q) + 0.5 * (self.absd0.T @ (h * self.dy)))
                 - self.kappa * (self.L1 @ mu))
        lam_prev = lam + self.dt * jac_t
        gk_e = self.dt * (-(1.0 / self.phi)) * (b1 - self.d0 @ p) * (g - self.star1 * d0psi)
        gk_v = 0.5 * (self.absd0.T @ gk_e)
        return lam_prev, gk_v

    def loss_and_grad(self, T0, w, steps, ckpt=None):
        """J = w . T_N and (dJ/dg, dJ/dT0) by the discrete adjoint, storing T every `ckpt`
        steps and recomputing each segment in the backward sweep."""
        ckpt = ckpt or steps
        saved = {0: T0.copy()}
        T = T0.copy()
        for n in range(steps):
            T, _ = self.step(T)
            if (n + 1) % ckpt == 0 and n + 1 < steps:
                saved[n + 1] = T.copy()
        J = float(w @ T)
        lam = w.copy()
        gk = np.zeros_like(T0)
        starts = sorted(saved)
        for s0 in reversed(starts):
            s1 = min(s0 + ckpt, steps)
            seg = [saved[s0]]
            for _ in range(s0, s1 - 1):
                seg.append(self.step(seg[-1])[0])
            for n in range(s1 - 1, s0 - 1, -1):
                lam, dk = self.step_adjoint(seg[n - s0], lam)
                gk += dk
        return J, gk * self.kv, lam


def stable_dt(lv, kv, Ra, phi):
    """dt = 1/2 min(h^2 phi Ra / 4, 2 phi / (Ra k_max^2)) with h the shortest edge (Q16)."""
    e = lv.edges
    h = np.min(np.linalg.norm(lv.xyz[e[:, 1]] - lv.xyz[e[:, 0]], axis=1))
    return 0.5 * min(h * h * phi * Ra / 4.0, 2.0 * phi / (Ra * float(np.max(kv)) ** 2))


def smooth_logk(h: omg.Hierarchy, noise: np.ndarray, sweeps: int = 20, omega: float = 0.8):
    """g from white noise by `sweeps` weighted-Jacobi sweeps on the unit-k natural-BC
    Laplacian with zero right-hand side (the C5 recipe)."""
    L = dec.laplacian(h.fine.d0, h.fine.star1)
    return omg.jacobi(L, np.zeros_like(noise), noise, omega, sweeps)
