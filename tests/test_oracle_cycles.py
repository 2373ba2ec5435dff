"""Pins of the oracle's cycle shapes (multigrid.mgcycle).

* On two levels the coarse-grid correction is exact whatever the shape: V, W and F give the
  same iterate bit for bit.
* On more levels the cycle from x = 0 equals (I - E_l) A_l^{-1} b with the error propagation
  matrices of the textbook recursion, built here densely and independently of the cycle code:
  S = I - omega D^{-1} A (Jacobi), E_0 = 0 and
      E_l = S^nu2 (I - P (I - K_{l-1}) A_{l-1}^{-1} R A_l) S^nu1,
  with K = E_V (V), E_W^2 (W: two cycles, the second from the first's result), and
  E_V E_F (F: an F-cycle, then a V-cycle from its result).
* With the solver in a Krylov loop, W needs no more iterations than V on the 65 x 65 grid.
"""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg
import workloads as W


def _square(nsub, base=4):
    xyz, tri = dec.square_grid(base)
    return omg.Hierarchy(xyz, tri, nsub)


def test_two_levels_all_shapes_equal():
    h = _square(1)
    b = h.rhs(W.normal(h.fine.nv, 21))
    xv = omg.mgcycle(h, b, kind="V")
    assert np.array_equal(xv, omg.mgcycle(h, b, kind="W"))
    assert np.array_equal(xv, omg.mgcycle(h, b, kind="F"))


def _error_matrices(h, nu1=2, nu2=2, omega=0.8):
    E = {k: [None] * (h.top + 1) for k in "VWF"}
    for k in "VWF":
        E[k][0] = np.zeros((h.levels[0].nv, h.levels[0].nv))
    for l in range(1, h.top + 1):
        A = h.levels[l].A.toarray()
        Ac = h.levels[l - 1].A.toarray()
        n, nc = A.shape[0], Ac.shape[0]
        P = np.column_stack([h.prolong(l, e) for e in np.eye(nc)])
        R = np.column_stack([h.restrict(l, e) for e in np.eye(n)])
        S = np.eye(n) - omega * np.diag(1.0 / np.diag(A)) @ A
        S1 = np.linalg.matrix_power(S, nu1)
        S2 = np.linalg.matrix_power(S, nu2)
        Aci = np.linalg.inv(Ac)
        K = {"V": E["V"][l - 1],
             "W": E["W"][l - 1] @ E["W"][l - 1],
             "F": E["V"][l - 1] @ E["F"][l - 1]}
        for k in "VWF":
            E[k][l] = S2 @ (np.eye(n) - P @ (np.eye(nc) - K[k]) @ Aci @ R @ A) @ S1
    return E


@pytest.mark.parametrize("kind", ["V", "W", "F"])
def test_cycle_matches_error_propagation(kind):
    h = _square(3, base=2)          # 4 levels, 17 x 17 finest
    E = _error_matrices(h)
    A = h.fine.A.toarray()
    b = h.rhs(W.normal(h.fine.nv, 22))
    ref = (np.eye(A.shape[0]) - E[kind][h.top]) @ np.linalg.solve(A, b)
    x = omg.mgcycle(h, b, kind=kind)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    if kind != "V":   # the shapes differ once there are three or more levels
        assert not np.allclose(x, omg.mgcycle(h, b, kind="V"), rtol=1e-10, atol=0)


def test_w_cycle_not_slower_than_v():
    h = _square(4)
    b = h.rhs(W.manufactured_c1(h.fine.xyz))
    _, kv, _ = omg.mg_pcg(h, b, cycle="V")
    _, kw, _ = omg.mg_pcg(h, b, cycle="W")
    _, kf, _ = omg.mg_pcg(h, b, cycle="F")
    assert kw <= kv and kf <= kv
