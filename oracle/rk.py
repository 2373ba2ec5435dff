"""Adaptive explicit Runge-Kutta 5(4) integration -- plain FP64 reference.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  The paper integrates its porous
model (Sec. 3.2, method of lines) with an explicit adaptive 5(4) Runge-Kutta pair.  This is
the Dormand-Prince 5(4) pair (J. R. Dormand and P. J. Prince, 1980): seven stages, the last
evaluated at the new solution and reused as the next step's first; the 5th-order solution is
kept, the embedded 4th-order one only measures the error.  Step-size control and the starting
step follow Hairer, Norsett and Wanner, Solving ODEs I, Sec. II.4.  Readings (not fixed by the
paper): error norm sqrt(mean((y5 - y4)_i / (atol + rtol max(|y_i|, |y5_i|)))^2); accept when
<= 1; next step h min(fmax, max(0.2, 0.9 err^(-1/5))), fmax = 10, or 1 after a rejection; a
step that would end within 1% of a save time or of t_end is cut to land on it.
"""
from __future__ import annotations

import numpy as np

# stage i input = y + h sum_j A[i][j] k_j; A[6] holds the 5th-order weights
C = (0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0)
A = ((),
     (1 / 5,),
     (3 / 40, 9 / 40),
     (44 / 45, -56 / 15, 32 / 9),
     (19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729),
     (9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656),
     (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84))
B5 = A[6] + (0.0,)
B4 = (5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40)


def combo(coefs, ks):
    """sum_j c_j k_j over the nonzero coefficients, in order."""
    acc = None
    for c, k in zip(coefs, ks):
        if c != 0.0:
            acc = c * k if acc is None else acc + c * k
    return acc


def wrms(v, u, w, atol, rtol):
    sc = atol + rtol * np.maximum(np.abs(u), np.abs(w))
    return float(np.sqrt(np.mean((v / sc) ** 2)))


def start_step(f, y0, f0, t_end, atol, rtol):
    """Hairer-Norsett-Wanner starting step (one extra evaluation of f)."""
    d0 = wrms(y0, y0, y0, atol, rtol)
    d1 = wrms(f0, y0, y0, atol, rtol)
    h0 = 1e-6 if (d0 < 1e-5 or d1 < 1e-5) else 0.01 * d0 / d1
    h0 = min(h0, t_end)
    f1 = f(y0 + h0 * f0)
    d2 = wrms((1.0 / h0) * (f1 - f0), y0, y0, atol, rtol)
    dm = max(d1, d2)
    h1 = max(1e-6, h0 * 1e-3) if dm <= 1e-15 else (0.01 / dm) ** (1.0 / 5.0)
    return min(100.0 * h0, h1, t_end)


def integrate(f, y0, t_end, rtol=1e-9, atol=1e-6, h0=0.0, t_save=(), fixed_step=False,
              max_steps=100000, trace=None):
    """Integrate y' = f(y) from t = 0 to t_end.  Returns (y(t_end), [y(t) for t in t_save],
    stats) with stats = accepted, rejected, rhs_evals, t, h_min, h_max.  trace (optional) is
    called after every attempted step as trace(t_start, h, err, accepted, y_after)."""
    y = np.array(y0, dtype=np.float64)
    st = dict(accepted=0, rejected=0, rhs_evals=0, t=0.0, h_min=np.inf, h_max=0.0)

    def F(v):
        st["rhs_evals"] += 1
        return f(v)

    k0 = F(y)
    h = float(h0)
    if not fixed_step and not h > 0:
        h = start_step(F, y, k0, t_end, atol, rtol)
    t, facmax, saved = 0.0, 10.0, []
    t_save = list(t_save)
    while t < t_end:
        if st["accepted"] + st["rejected"] >= max_steps or h < 1e-14 * t_end:
            break
        t_stop = t_save[len(saved)] if len(saved) < len(t_save) else t_end
        hit = t + 1.01 * h >= t_stop
        if hit:
            h = t_stop - t
        ks = [k0]
        for i in range(1, 7):
            yi = y + h * combo(A[i], ks)
            ks.append(F(yi))
        y5 = yi
        err = 0.0
        if not fixed_step:
            err = wrms(h * combo([b - e for b, e in zip(B5, B4)], ks), y, y5, atol, rtol)
        if fixed_step or err <= 1.0:
            t0 = t
            t = t_stop if hit else t + h
            y, k0 = y5, ks[6]
            st["accepted"] += 1
            st["h_min"], st["h_max"] = min(st["h_min"], h), max(st["h_max"], h)
            if hit and len(saved) < len(t_save):
                saved.append(y.copy())
            if trace is not None:
                trace(t0, h, err, True, y)
            if fixed_step:
                h = float(h0)
            else:
                fac = facmax if err == 0.0 else 0.9 * err ** (-1.0 / 5.0)
                h *= min(facmax, max(0.2, fac))
                facmax = 10.0
        else:
            if trace is not None:
                trace(t, h, err, False, y)
            st["rejected"] += 1
            fac = 0.9 * err ** (-1.0 / 5.0) if np.isfinite(err) else 0.2
            h *= max(0.2, fac)
            facmax = 1.0
    st["t"] = t
    return y, saved, st
