"""Randomized sweeps of the oracle over tiny shapes (n in [2, 40]), against
solves of formulations it does not use: the condensed LiftedKKT solve and
HyKKT's three steps against dense K2 / K1 solves; and the growth of
cond(K_gamma) with gamma once gamma dominates (Sec. 4, linear in gamma)."""
import numpy as np
from hypothesis import given, settings, strategies as st

from oracle import dense as od


def _inst(seed, n, me, mi):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n))
    W = A @ A.T / n + np.eye(n)
    G = rng.standard_normal((me, n))
    H = rng.standard_normal((mi, n))
    sx = 10.0 ** rng.uniform(-2, 2, n)
    sh = 10.0 ** rng.uniform(-2, 2, mi)
    return rng, W, G, H, sx, sh


@settings(max_examples=40, deadline=None)
@given(seed=st.integers(0, 10_000), n=st.integers(2, 40), mi=st.integers(0, 20), frac=st.floats(0.0, 0.9))
def test_condensed_equals_augmented_random(seed, n, mi, frac):
    me = int(frac * (n - 1))
    rng, W, G, H, sx, sh = _inst(seed, n, me, mi)
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    sol = np.linalg.solve(od.augmented_k2(W, sx, G, H, sh), -np.concatenate([r1, r2, r3, r4]))
    rb1, rb2 = od.condensed_rhs(r1, r2, r3, r4, H, sh)
    K = od.condensed_matrix(W, sx, H, sh)
    dx, dy = od.solve_k1(K, G, rb1, rb2)
    assert np.allclose(dx, sol[:n], rtol=1e-7, atol=1e-9 * np.abs(sol[:n]).max())
    if me:
        dx2, dy2, _, ok = od.hykkt_steps(K, G, rb1, rb2, 1e4)
        assert ok
        assert np.allclose(dx2, dx, rtol=1e-5, atol=1e-7 * np.abs(dx).max())
        assert np.allclose(dy2, dy, rtol=1e-5, atol=1e-7 * np.abs(dy).max())


def test_cond_k_gamma_grows_linearly_in_gamma():
    rng, W, G, H, sx, sh = _inst(7, 20, 6, 8)
    K = od.condensed_matrix(W, sx, H, sh)
    c = [np.linalg.cond(od.k_gamma(W, sx, H, sh, G, g)) for g in (1e4, 1e5, 1e6)]
    assert 8.0 < c[1] / c[0] < 12.0 and 8.0 < c[2] / c[1] < 12.0
