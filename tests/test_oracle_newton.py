"""Pins of the Newton-step oracle (oracle/newton.py).

* the condensed route (rbar, K1 solve, slack recovery) equals a dense solve
  of the augmented system K2, for LiftedKKT's shape (every row with a
  slack) and HyKKT's (equality rows without);
* with E = S^-1 V, the four blocks and the bound-multiplier step d_v equal
  the dense solve of the unreduced system K3 (eq:kkt:unreduced), whose
  right-hand side is written from the iterate (z, v, s, mu) and not from r2;
* omega_k2 equals the backward error computed row by row with loops.
"""
import numpy as np
import pytest

from oracle import dense as od
from oracle import newton as on
from paper_2405_14236_amd import workloads


def _data(seed, lifted):
    p = workloads.tiny_grid(seed, nx=4, ny=3, sigma_range=(-1, 1))
    W, G, H = od.problem_dense(p)
    if lifted:
        G, H, E = np.zeros((0, p.n)), np.vstack([G, H]), p.sigma_s
    else:
        E = p.sigma_s_ineq
    return p, W, G, H, E


@pytest.mark.parametrize("lifted", [True, False])
def test_condensed_route_equals_k2(lifted):
    p, W, G, H, E = _data(21, lifted)
    rng = np.random.default_rng(21)
    r = [rng.standard_normal(k) for k in (p.n, H.shape[0], G.shape[0], H.shape[0])]
    dx, ds, dy, dz = on.solve_augmented(W, p.sigma_x, G, H, E, *r)
    sol = np.linalg.solve(od.augmented_k2(W, p.sigma_x, G, H, E), -np.concatenate(r))
    n, mi, me = p.n, H.shape[0], G.shape[0]
    ref = (sol[:n], sol[n:n + mi], sol[n + mi:n + mi + me], sol[n + mi + me:])
    for a, b in zip((dx, ds, dy, dz), ref):
        if b.size:
            assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()
    assert on.omega_k2(W, p.sigma_x, G, H, E, *r, dx, ds, dy, dz) < 1e-13


@pytest.mark.parametrize("lifted", [True, False])
def test_recovery_and_bound_step_equal_k3(lifted):
    p, W, G, H, _ = _data(22, lifted)
    rng = np.random.default_rng(22)
    n, mi, me = p.n, H.shape[0], G.shape[0]
    s = 10.0 ** rng.uniform(-2, 1, mi)
    v = 10.0 ** rng.uniform(-2, 1, mi)
    z = rng.standard_normal(mi)
    mu = 0.03
    gradL, g, hs = rng.standard_normal(n), rng.standard_normal(me), rng.standard_normal(mi)
    K3 = on.unreduced_k3(W, p.sigma_x, G, H, s, v)
    sol = np.linalg.solve(K3, -np.concatenate([gradL, z - v, g, hs, s * v - mu]))
    E = v / s
    r2 = z - mu / s  # r2 of K2 (Sec. 2.2)
    dx, ds, dy, dz = on.solve_augmented(W, p.sigma_x, G, H, E, gradL, r2, g, hs)
    dv = on.bound_dual_step(s, v, mu, ds)
    ref = np.split(sol, np.cumsum([n, mi, me, mi]))
    for a, b in zip((dx, ds, dy, dz, dv), ref):
        if b.size:
            assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max()


def test_omega_k2_row_by_row():
    p, W, G, H, E = _data(23, False)
    rng = np.random.default_rng(23)
    n, mi, me = p.n, H.shape[0], G.shape[0]
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    dx, ds, dy, dz = (rng.standard_normal(k) for k in (n, mi, me, mi))
    got = on.omega_k2(W, p.sigma_x, G, H, E, r1, r2, r3, r4, dx, ds, dy, dz)
    worst = 0.0
    for i in range(n):
        num, den = -r1[i], abs(r1[i])
        for j in range(n):
            num -= W[i, j] * dx[j]
            den += abs(W[i, j] * dx[j])
        num -= p.sigma_x[i] * dx[i]
        den += abs(p.sigma_x[i] * dx[i])
        for r in range(me):
            num -= G[r, i] * dy[r]
            den += abs(G[r, i] * dy[r])
        for r in range(mi):
            num -= H[r, i] * dz[r]
            den += abs(H[r, i] * dz[r])
        worst = max(worst, abs(num) / den)
    for r in range(mi):
        num = -r2[r] - E[r] * ds[r] - dz[r]
        worst = max(worst, abs(num) / (abs(E[r] * ds[r]) + abs(dz[r]) + abs(r2[r])))
        num, den = -r4[r] - ds[r], abs(ds[r]) + abs(r4[r])
        for j in range(n):
            num -= H[r, j] * dx[j]
            den += abs(H[r, j] * dx[j])
        worst = max(worst, abs(num) / den)
    for r in range(me):
        num, den = -r3[r], abs(r3[r])
        for j in range(n):
            num -= G[r, j] * dx[j]
            den += abs(G[r, j] * dx[j])
        worst = max(worst, abs(num) / den)
    assert np.isclose(got, worst, rtol=1e-10)
