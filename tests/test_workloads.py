"""The seeded input generators: determinism and the spherical-harmonic evaluator."""
import math

import numpy as np
import scipy.special as ss

import workloads as W


def test_seeded_draws_are_deterministic():
    assert np.array_equal(W.normal(1000, 3), W.normal(1000, 3))
    assert not np.array_equal(W.normal(1000, 3), W.normal(1000, 4))
    assert len(W.sh_coefficients()) == 80
    inst = W.c4_instances()
    assert len(inst) == 256 and inst == W.c4_instances()


def _gauss_sphere(nt=40, nphi=80):
    x, wt = np.polynomial.legendre.leggauss(nt)
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    X, P = np.meshgrid(x, ph, indexing="ij")
    s = np.sqrt(1 - X ** 2)
    xyz = np.stack([s * np.cos(P), s * np.sin(P), X], axis=-1).reshape(-1, 3)
    w = (wt[:, None] * np.full(nphi, 2 * math.pi / nphi)[None, :]).ravel()
    return xyz, w


def test_real_sph_harm_orthonormal():
    xyz, w = _gauss_sphere()
    Y = W.real_sph_harm(8, xyz)
    keys = sorted(Y)
    G = np.array([[np.sum(w * Y[a] * Y[b]) for b in keys] for a in keys])
    assert np.abs(G - np.eye(len(keys))).max() < 1e-12


def test_real_sph_harm_matches_scipy():
    xyz, _ = _gauss_sphere(9, 13)
    theta = np.arccos(xyz[:, 2])
    phi = np.arctan2(xyz[:, 1], xyz[:, 0])
    Y = W.real_sph_harm(8, xyz)
    for l in range(9):
        for m in range(-l, l + 1):
            c = ss.sph_harm_y(l, abs(m), theta, phi)
            ref = c.real if m == 0 else math.sqrt(2) * (c.real if m > 0 else c.imag)
            # scipy carries the Condon-Shortley phase (-1)^m
            assert np.allclose(Y[(l, m)], (-1) ** abs(m) * ref, atol=1e-12)


def test_sphere_exact_solves_laplace_beltrami():
    """-lap_S Y_lm = l(l+1) Y_lm, checked with the spherical Laplacian by finite differences
    in (theta, phi) at interior points."""
    coeffs = W.sh_coefficients()
    th, ph, d = 1.1, 0.7, 1e-4

    def u(t, p):
        x = np.array([[math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)]])
        return W.sphere_exact(x, coeffs)[0]

    lap = ((u(th + d, ph) - 2 * u(th, ph) + u(th - d, ph)) / d ** 2
           + math.cos(th) / math.sin(th) * (u(th + d, ph) - u(th - d, ph)) / (2 * d)
           + (u(th, ph + d) - 2 * u(th, ph) + u(th, ph - d)) / (d * math.sin(th)) ** 2)
    x = np.array([[math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]])
    assert abs(-lap - W.sphere_rhs(x, coeffs)[0]) < 1e-5
