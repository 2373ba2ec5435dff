"""Pins of the porous-convection oracle (Sec. 3.2): exact conductive state, compatibility and
zero divergence of the Darcy flux, and the discrete adjoint against central differences."""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg
from oracle import porous as op
import workloads as W


def _model(n=4, nsub=2, noise=0.5, seed=1, **kw):
    xyz, tri = dec.square_grid(n)
    h = omg.Hierarchy(xyz, tri, nsub, bc="natural")
    g = noise * W.normal(h.fine.nv, seed)
    return op.PorousModel(h, g, **kw)


def test_conductive_state_is_exact():
    """T = 1 - y with any permeability: p = y - y^2/2 (+ const) makes q = 0 exactly, and T
    does not move (linear precision of L on the side walls, masked walls)."""
    m = _model(noise=1.0)
    T = 1.0 - m.y
    p, b1 = m.pressure(T)
    ref = m.y - 0.5 * m.y ** 2
    ref -= ref.mean()
    assert np.abs(p - ref).max() < 1e-12
    q = -m.ke * (m.d0 @ p - b1)
    assert np.abs(q).max() < 1e-12
    T2 = m.rollout(T, 10)
    assert np.abs(T2 - T).max() < 1e-13


def test_pressure_rhs_compatible_and_flux_divergence_free():
    m = _model(noise=1.0)
    T = 1.0 - m.y + 0.1 * W.normal(m.lv.nv, 3)
    b1 = m.buoyancy(T)
    rhs = m.d0.T @ (m.W * b1)
    assert abs(rhs.sum()) <= 1e-14 * np.abs(rhs).sum()
    p, _ = m.pressure(T)
    q = -m.ke * (m.d0 @ p - b1)
    div = m.d0.T @ (m.star1 * q)
    assert np.abs(div).max() <= 1e-12 * np.abs(rhs).max()


def _fd_check(m, T0, w, steps, ckpt, eps=1e-6, ndir=4):
    J, gg, gT = m.loss_and_grad(T0, w, steps, ckpt)
    rng = np.random.default_rng(17)
    g0 = m.g.copy()
    for _ in range(ndir):
        v = rng.standard_normal(len(T0))
        Jp = w @ m.rollout(T0 + eps * v, steps)
        Jm = w @ m.rollout(T0 - eps * v, steps)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - gT @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, gT @ v)
    for _ in range(ndir):
        v = rng.standard_normal(len(g0))
        m.set_g(g0 + eps * v)
        Jp = w @ m.rollout(T0, steps)
        m.set_g(g0 - eps * v)
        Jm = w @ m.rollout(T0, steps)
        m.set_g(g0)
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - gg @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, gg @ v)
    return J, gg, gT


def test_adjoint_matches_central_differences():
    m = _model(noise=0.8, dt=2e-4)
    T0 = 1.0 - m.y + 0.2 * W.normal(m.lv.nv, 4)
    T0[m.wall] = 1.0 - m.y[m.wall]
    w = W.normal(m.lv.nv, 5)
    _fd_check(m, T0, w, steps=6, ckpt=2)


def test_adjoint_single_components():
    m = _model(noise=0.8, dt=2e-4)
    T0 = 1.0 - m.y + 0.2 * W.normal(m.lv.nv, 6)
    w = W.normal(m.lv.nv, 7)
    J, gg, gT = m.loss_and_grad(T0, w, 4, 2)
    eps = 1e-6
    g0 = m.g.copy()
    for i in (0, 7, m.lv.nv // 2, m.lv.nv - 3):
        e = np.zeros_like(T0)
        e[i] = 1.0
        fd = (w @ m.rollout(T0 + eps * e, 4) - w @ m.rollout(T0 - eps * e, 4)) / (2 * eps)
        assert abs(fd - gT[i]) <= 1e-6 * max(1.0, abs(fd))
        m.set_g(g0 + eps * e)
        Jp = w @ m.rollout(T0, 4)
        m.set_g(g0 - eps * e)
        Jm = w @ m.rollout(T0, 4)
        m.set_g(g0)
        assert abs((Jp - Jm) / (2 * eps) - gg[i]) <= 1e-6 * max(1.0, abs(gg[i]))


def test_checkpointing_does_not_change_the_gradient():
    m = _model(noise=0.5, dt=2e-4)
    T0 = 1.0 - m.y + 0.2 * W.normal(m.lv.nv, 8)
    w = W.normal(m.lv.nv, 9)
    a = m.loss_and_grad(T0, w, 6, 6)
    b = m.loss_and_grad(T0, w, 6, 2)
    c = m.loss_and_grad(T0, w, 6, 4)
    for x, y in ((a, b), (a, c)):
        assert x[0] == y[0]
        assert np.array_equal(x[1], y[1]) and np.array_equal(x[2], y[2])


def test_mg_pcg_pressure_matches_direct():
    md = _model(noise=0.7)
    mp = _model(noise=0.7, solver="mg_pcg", rtol=1e-13)
    T = 1.0 - md.y + 0.1 * W.normal(md.lv.nv, 10)
    pd, _ = md.pressure(T)
    pp, _ = mp.pressure(T)
    assert np.linalg.norm(pp - pd) <= 1e-11 * np.linalg.norm(pd)


def test_smoothed_logk_and_dt():
    xyz, tri = dec.square_grid(4)
    h = omg.Hierarchy(xyz, tri, 3, bc="natural")
    noise = W.normal(h.fine.nv, 5)
    g = op.smooth_logk(h, noise)
    # each sweep changes x by -omega D^{-1} L x and 1^T L = 0, so sum_i D_i x_i is kept;
    # the high-frequency part (the variance) is damped
    D = dec.laplacian(h.fine.d0, h.fine.star1).diagonal()
    assert abs(D @ g - D @ noise) < 1e-12 * (D @ np.abs(noise))
    assert g.std() < 0.6 * noise.std()
    dt = op.stable_dt(h.fine, np.exp(g), 1000.0, 0.1)
    hh = 1 / 32
    assert dt == 0.5 * min(hh * hh * 0.1 * 1000 / 4, 2 * 0.1 / (1000 * np.exp(g).max() ** 2))
