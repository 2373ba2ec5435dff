"""Pins of the oracle's Dormand-Prince 5(4) integrator (oracle/rk.py) and of the porous model
on the paper's porous-convection setup (workloads.E4).

* The tableau satisfies the order conditions it is built on: row sums equal the nodes, the
  5th-order weights integrate polynomials of degree < 5 exactly and meet the coupled order
  3 and 4 conditions, the embedded weights integrate degree < 4, and the last stage row equals
  the 5th-order weights (first same as last).
* Fixed steps converge at order 5 on a nonlinear problem (the pendulum).
* Adaptive runs reproduce the matrix exponential of a linear system within their tolerance,
  and tighter tolerances give smaller errors; save times are met exactly.
* Porous model on E4: kappa = Delta T y_max / (phi Ra) = 40, initial peak 400/pi, the
  conductive state between the walls is steady, and the walls do not move.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import dec
from oracle import multigrid as omg
from oracle import porous as op
from oracle import rk
import workloads as W


def test_tableau_order_conditions():
    c = np.array(rk.C)
    A = np.zeros((7, 7))
    for i, row in enumerate(rk.A):
        A[i, :len(row)] = row
    b5, b4 = np.array(rk.B5), np.array(rk.B4)
    assert np.abs(A.sum(axis=1) - c).max() <= 1e-15
    for k in range(1, 6):
        assert abs(b5 @ c ** (k - 1) - 1.0 / k) <= 1e-15, k
    for k in range(1, 5):
        assert abs(b4 @ c ** (k - 1) - 1.0 / k) <= 1e-15, k
    assert abs(b5 @ (A @ c) - 1 / 6) <= 1e-15
    assert abs(b5 @ (c * (A @ c)) - 1 / 8) <= 1e-15
    assert abs(b5 @ (A @ c ** 2) - 1 / 12) <= 1e-15
    assert abs(b5 @ (A @ (A @ c)) - 1 / 24) <= 1e-15
    assert abs(b4 @ (A @ (A @ c)) - 1 / 24) <= 1e-15
    assert np.array_equal(A[6, :6], b5[:6]) and b5[6] == 0.0
    # the embedded pair differs at 5th order: its error constant is not zero
    assert abs(b4 @ c ** 4 - 1 / 5) > 1e-4


def test_fixed_step_order_five():
    def f(y):
        return np.array([y[1], -np.sin(y[0])])
    ref, _, _ = rk.integrate(f, np.array([1.0, 0.0]), 2.0, h0=2.0 / 2048, fixed_step=True)
    errs = []
    for n in (8, 16, 32):
        y, _, st = rk.integrate(f, np.array([1.0, 0.0]), 2.0, h0=2.0 / n, fixed_step=True)
        assert st["accepted"] == n and st["rhs_evals"] == 6 * n + 1
        errs.append(np.abs(y - ref).max())
    for a, b in zip(errs, errs[1:]):
        assert 28.0 < a / b < 40.0


def test_adaptive_linear_system_against_expm():
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((6, 6))
    M = -(Q @ Q.T) / 6.0 + 0.5 * (Q - Q.T)
    y0 = rng.standard_normal(6)
    ts = [0.3, 1.0, 1.7]
    errs = {}
    for rtol in (1e-6, 1e-10):
        y, saved, st = rk.integrate(lambda v: M @ v, y0, 2.0, rtol=rtol, atol=rtol * 1e-3,
                                    t_save=ts)
        assert st["t"] == 2.0 and len(saved) == 3
        exact = [sla.expm(M * t) @ y0 for t in ts + [2.0]]
        e = max(np.abs(s - x).max() / np.abs(x).max() for s, x in zip(saved + [y], exact))
        errs[rtol] = e
        assert e <= 50 * rtol
    assert errs[1e-6] > 100 * errs[1e-10]


def _e4(nsub=3):
    E = W.E4
    xyz, tri = dec.square_grid(E["base_cells"])
    h = omg.Hierarchy(W.e4_coords(xyz), tri, nsub, bc="natural")
    m = op.PorousModel(h, np.zeros(h.fine.nv), Ra=E["Ra"], phi=E["phi"], delta_T=E["delta_T"],
                       y_len=E["y_range"][1] - E["y_range"][0])
    return h, m


def test_e4_setup():
    h, m = _e4()
    assert m.kappa == 40.0
    T0 = W.e4_initial_temperature(h.fine.xyz)
    assert abs(T0.max() - 400.0 / math.pi) < 1e-12 and abs(T0.max() - 127.3) < 0.05
    n = 4 * 2 ** 3
    assert m.wall.sum() == 2 * (n + 1)
    assert np.all(T0[h.fine.xyz[:, 1] == -20.0] == 100.0)
    assert np.all(T0[h.fine.xyz[:, 1] == 0.0] == -100.0)


def test_e4_conductive_state_and_walls():
    h, m = _e4()
    y = h.fine.xyz[:, 1]
    T = 100.0 - 200.0 * (y + 20.0) / 20.0
    scale = m.kappa * np.max(abs(m.L1) @ np.abs(T) / m.star0)
    assert np.abs(m.rhs(T)).max() <= 1e-13 * scale
    T0 = W.e4_initial_temperature(h.fine.xyz)
    yT, _, st = rk.integrate(m.rhs, T0, 0.02, rtol=1e-9, atol=1e-6)
    assert st["t"] == 0.02 and st["rejected"] <= st["accepted"]
    assert np.array_equal(yT[m.wall], T0[m.wall])
    # heat leaves the hot blob: its peak decays
    assert yT[~m.wall].max() < T0[~m.wall].max()


# ---------------------------------------------------------------------------------------------
# Independent pin of the starting step and the step-size controller: SciPy's RK45 implements
# the same Dormand-Prince pair with the Hairer-Norsett-Wanner starting-step rule and the same
# controller (safety 0.9, factors in [0.2, 10], exponent -1/5, a factor of at most 1 on the step
# after a rejection, RMS error norm with scale atol + rtol max(|y|, |y_new|)).  It was written
# independently of this oracle, so a mistake shared by the oracle and the library copy of the
# controller (an exponent, a swapped norm, a missed clamp) shows up here.  The two differ only
# in how they land on t_end (SciPy clamps the step that would pass it, the oracle also cuts a
# step that would end within 1% of it), so the comparison covers every step before the last
# and the state at the last common time.  The starting step is compared on its own (to
# rounding).  The step sequences then start from the same given first step, four times the
# automatic one: the automatic step has err ~ 1e-5, formed from stage sums that cancel to
# 1e-7 .. 1e-11 of their size, so the two codes' summation orders would move the next step by up
# to 1e-6 relative; a first step with err ~ 0.1 keeps every estimate well conditioned.  A
# controller mistake (a constant, the exponent, a clamp, the norm) moves h by 1e-2 or more.

def _scipy_steps(f, y0, t_end, rtol, atol, first_step=None):
    from scipy.integrate import RK45
    s = RK45(lambda t, y: f(y), 0.0, np.array(y0, dtype=np.float64), t_end, rtol=rtol,
             atol=atol, first_step=first_step)
    h_first = s.h_abs
    steps = []  # (t_start, h, rejections before acceptance, y_after)
    while s.status == "running":
        t0, nfev0 = s.t, s.nfev
        msg = s.step()
        assert msg is None, msg
        attempts = (s.nfev - nfev0) // 6
        steps.append((t0, s.t - t0, attempts - 1, s.y.copy()))
    return h_first, steps


def _oracle_steps(f, y0, t_end, rtol, atol, first_step=0.0):
    log = []
    rej = [0]

    def tr(t0, h, err, acc, y):
        if acc:
            log.append((t0, h, rej[0], y.copy()))
            rej[0] = 0
        else:
            rej[0] += 1

    y0 = np.array(y0, dtype=np.float64)
    h_first = rk.start_step(f, y0, f(y0), t_end, atol, rtol)
    _, _, st = rk.integrate(f, y0, t_end, rtol=rtol, atol=atol, h0=first_step, trace=tr)
    return h_first, log, st


def _van_der_pol(mu):
    return lambda y: np.array([y[1], mu * (1.0 - y[0] ** 2) * y[1] - y[0]])


def _linear6():
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((6, 6))
    M = -(Q @ Q.T) / 6.0 + 0.5 * (Q - Q.T)
    return (lambda v: M @ v), rng.standard_normal(6)


@pytest.mark.parametrize("case", ["linear6", "vdp5"])
@pytest.mark.parametrize("rtol", [1e-6, 1e-9])
def test_controller_against_scipy_rk45(case, rtol):
    if case == "linear6":
        f, y0 = _linear6()
        t_end = 3.0
    else:
        f, y0 = _van_der_pol(5.0), np.array([2.0, 0.0])
        t_end = 12.0
    atol = 1e-3 * rtol
    hs, _ = _scipy_steps(f, y0, t_end, rtol, atol)
    ho = rk.start_step(f, y0, f(y0), t_end, atol, rtol)
    assert abs(ho - hs) <= 1e-14 * hs
    _, ss = _scipy_steps(f, y0, t_end, rtol, atol, first_step=4.0 * hs)
    _, so, st = _oracle_steps(f, y0, t_end, rtol, atol, first_step=4.0 * hs)
    # every accepted step before the one that lands on t_end: same start, size and rejections
    n = min(len(ss), len(so)) - 1
    assert n >= 20 and abs(len(ss) - len(so)) <= 1
    total_rej = 0
    for k in range(n):
        (ts, h_s, r_s, _), (to, h_o, r_o, _) = ss[k], so[k]
        assert r_s == r_o, (k, r_s, r_o)
        assert abs(h_o - h_s) <= 1e-6 * h_s, (k, h_o, h_s)
        assert abs(to - ts) <= 1e-7 * max(ts, 1.0), (k, to, ts)
        total_rej += r_o
    ys, yo = ss[n - 1][3], so[n - 1][3]
    assert np.abs(yo - ys).max() <= 1e-6 * max(1.0, np.abs(ys).max())
    if case == "vdp5":
        # the relaxation oscillation forces rejections: the comparison covers that branch
        assert total_rej >= 3
    assert st["t"] == t_end
