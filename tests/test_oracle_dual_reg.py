"""Pins of the oracle's K1 with dual regularization delta_c > 0 (Remark 1).

* the sparse K1 solve with -delta_c I equals the dense solve of the
  augmented system K2 with delta_c (a different formulation: slacks kept,
  condensation with C = (I + delta_c D_s)^-1 done by the test), and its
  refinement history reaches rounding (so the residual with the delta_c
  term is right);
* omega_k1 with delta_c equals the componentwise backward error computed
  row by row with loops over the dense data;
* delta_c = 0 reproduces the hot path's K1 functions exactly.
"""
import numpy as np
import pytest

from oracle import dense as od
from oracle import sparse as osp
from paper_2405_14236_amd import workloads


@pytest.mark.parametrize("delta_c", [1e-8, 1e-4, 1.0])
def test_sparse_k1_with_delta_c_equals_k2(delta_c):
    p = workloads.tiny_grid(11, nx=4, ny=3, sigma_range=(-1, 1))
    W, G, H = od.problem_dense(p)
    Ds = p.sigma_s_ineq
    n, me, mi = p.n, p.m_eq, p.m_ineq
    rng = np.random.default_rng(11)
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    M = od.augmented_k2(W, p.sigma_x, G, H, Ds, delta_c=delta_c)
    sol = np.linalg.solve(M, -np.concatenate([r1, r2, r3, r4]))
    dx2, dy2 = sol[:n], sol[n + mi:n + mi + me]
    # condensation of the slack block with delta_c (Sec. 2.2): D_H = D_s C
    C = 1.0 / (1.0 + delta_c * Ds)
    DH = Ds * C
    rb1 = -(r1 + H.T @ (DH * r4 - C * r2))
    rb2 = -r3
    P = osp.Problem(p)
    dx, dy, hist = osp.solve_k1(P, p.sigma_x, DH, rb1, rb2, delta_c=delta_c)
    assert hist[-1] <= 1e-14
    assert np.abs(dx - dx2).max() <= 1e-9 * np.abs(dx2).max()
    assert np.abs(dy - dy2).max() <= 1e-9 * np.abs(dy2).max()
    # the primal Schur complement of eqn:primal gives the same point
    K = od.condensed_matrix(W, p.sigma_x, H, DH)
    dxs, dys = od.primal_schur_delta_c(K, G, rb1, rb2, delta_c)
    assert np.abs(dxs - dx2).max() <= 1e-8 * np.abs(dx2).max()


def test_omega_k1_delta_c_row_by_row():
    p = workloads.tiny_grid(12, nx=3, ny=3)
    W, G, H = od.problem_dense(p)
    sh = p.sigma_s_ineq
    rng = np.random.default_rng(12)
    dx, dy = rng.standard_normal(p.n), rng.standard_normal(p.m_eq)
    dc = 0.37
    P = osp.Problem(p)
    got = osp.omega_k1(P.W, p.sigma_x, P.H, sh, P.G, dx, dy, p.r1bar, p.r2bar, delta_c=dc)
    worst = 0.0
    for i in range(p.n):
        num, den = p.r1bar[i], abs(p.r1bar[i])
        for j in range(p.n):
            num -= W[i, j] * dx[j]
            den += abs(W[i, j] * dx[j])
        num -= p.sigma_x[i] * dx[i]
        den += abs(p.sigma_x[i] * dx[i])
        for r in range(p.m_ineq):
            hx = sum(H[r, j] * dx[j] for j in range(p.n))
            ahx = sum(abs(H[r, j] * dx[j]) for j in range(p.n))
            num -= H[r, i] * sh[r] * hx
            den += abs(H[r, i] * sh[r]) * ahx
        for r in range(p.m_eq):
            num -= G[r, i] * dy[r]
            den += abs(G[r, i] * dy[r])
        worst = max(worst, abs(num) / den)
    for r in range(p.m_eq):
        num, den = p.r2bar[r], abs(p.r2bar[r])
        for j in range(p.n):
            num -= G[r, j] * dx[j]
            den += abs(G[r, j] * dx[j])
        num += dc * dy[r]
        den += dc * abs(dy[r])
        worst = max(worst, abs(num) / den)
    assert np.isclose(got, worst, rtol=1e-10)


def test_delta_c_zero_is_the_hot_path_k1():
    p = workloads.tiny_grid(13, nx=3, ny=3)
    P = osp.Problem(p)
    rng = np.random.default_rng(13)
    dx, dy = rng.standard_normal(p.n), rng.standard_normal(p.m_eq)
    args = (P.W, p.sigma_x, P.H, p.sigma_s_ineq, P.G, dx, dy, p.r1bar, p.r2bar)
    a1, a2 = osp.k1_residual(*args)
    b1, b2 = osp.k1_residual(*args, delta_c=0.0)
    assert np.array_equal(a1, b1) and np.array_equal(a2, b2)
    G = P.G.toarray()
    assert np.allclose(a2, p.r2bar - G @ dx, rtol=1e-14, atol=1e-14)
