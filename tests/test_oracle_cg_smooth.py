"""Pins of the oracle's CG smoother (multigrid.cg_smooth): k CG steps from x0 give the A-norm
best approximation x0 + V (V^T A V)^{-1} V^T r0 over the Krylov space spanned by
r0, A r0, ..., A^{k-1} r0 (built here by dense orthogonalisation, not by the CG recurrences);
n steps on an n x n system reach the exact solution; the cycle with CG smoothing, used inside
FCG, converges."""
import numpy as np
import pytest

from oracle import dec
from oracle import multigrid as omg
import workloads as W


def _level(nsub=2):
    xyz, tri = dec.square_grid(2)
    h = omg.Hierarchy(xyz, tri, nsub)
    return h, h.fine.A.toarray()


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cg_steps_are_krylov_minimisers(k):
    h, A = _level()
    n = A.shape[0]
    b = W.normal(n, 51)
    x0 = W.normal(n, 52)
    r0 = b - A @ x0
    K = np.column_stack([np.linalg.matrix_power(A, j) @ r0 for j in range(k)])
    V, _ = np.linalg.qr(K)
    ref = x0 + V @ np.linalg.solve(V.T @ A @ V, V.T @ r0)
    x = omg.cg_smooth(h.fine.A, b, x0, k)
    assert np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)


def test_cg_exact_after_n_steps():
    xyz, tri = dec.square_grid(2)
    h = omg.Hierarchy(xyz, tri, 0)     # 9 vertices, 1 interior
    A = h.fine.A
    b = W.normal(A.shape[0], 53)
    x = omg.cg_smooth(A, b, np.zeros_like(b), A.shape[0])
    assert np.linalg.norm(A @ x - b) <= 1e-12 * np.linalg.norm(b)


def test_cg_smoothed_cycle_in_fcg():
    xyz, tri = dec.square_grid(4)
    h = omg.Hierarchy(xyz, tri, 4)
    b = h.rhs(W.manufactured_c1(h.fine.xyz))
    x, k, hist = omg.mg_fcg(h, b, nu1=3, nu2=3, smoother="cg")
    assert hist[-1] <= 1e-10 and k <= 20
    assert omg.rel_residual(h, b, x) <= 1e-10
