"""Pins of the inertia-correction oracle (oracle/inertia.py).

* the delta_w rule on scalar predicates, against sequences derived by hand
  from Waechter & Biegler (2006), Sec. 3.1;
* eigenvalue brute force: every rejected trial leaves a non-positive
  eigenvalue in the condensed matrix, the accepted one none (checks the
  Cholesky test independently of Cholesky);
* Sylvester's law (eq:ipm:inertia): at every trial the augmented system K2
  with delta_w on its primal and slack blocks has the inertia
  (n + m_i, m_i + m_e, 0) exactly when the condensed matrix was accepted;
* the regularized condensed solve equals the solve of K2 with the same
  delta_w (pins that delta_w also enters the slack weights).
"""
import numpy as np
import pytest

from oracle import dense as od
from oracle import inertia as oi
from paper_2405_14236_amd import workloads
from tests._common import plant_negative_curvature


def test_rule_by_hand():
    # negative eigenvalue -0.3, no earlier correction: delta_w_0 = 1e-4, then x100
    d, tried, last = oi.correct(lambda x: x > 0.3, 0.0)
    assert tried == [0.0, 1e-4, 1e-2, 1.0] and d == 1.0 and last == 1.0
    # earlier correction 0.5: first trial 0.5/3, then x8
    d, tried, last = oi.correct(lambda x: x > 0.3, 0.5)
    assert tried == pytest.approx([0.0, 0.5 / 3, 4.0 / 3], rel=1e-15) and d == tried[-1] and last == d
    # positive definite at delta_w = 0: one trial, delta_w_last kept
    d, tried, last = oi.correct(lambda x: True, 0.7)
    assert (d, tried, last) == (0.0, [0.0], 0.7)
    # tiny delta_w_last: the first trial is floored at delta_w_min
    d, tried, last = oi.correct(lambda x: x > 0.0, 3e-21)
    assert tried == [0.0, 1e-20] and d == 1e-20
    # a singular matrix (zero eigenvalue) is rejected at delta_w = 0 like an indefinite one
    d, tried, _ = oi.correct(lambda x: oi.cholesky_ok(np.array([[x]])), 0.0)
    assert tried == [0.0, 1e-4] and d == 1e-4
    # every trial up to delta_w_max fails: no delta_w, delta_w_last unchanged
    d, tried, last = oi.correct(lambda x: False, 0.0, dict(delta_w_max=0.5))
    assert d is None and tried == [0.0, 1e-4, 1e-2] and last == 0.0


def _small(seed):
    return workloads.tiny_grid(seed, nx=4, ny=3, vpn=3, sigma_range=(-1, 1))


CASES = [(0, 0.5, 0.0), (1, 5.0, 0.0), (2, 0.5, 0.3), (3, 40.0, 2.0)]


def _setup(form, seed, theta, gamma=1e7):
    p = plant_negative_curvature(_small(seed), form, theta, gamma)
    W, G, H = od.problem_dense(p)
    return p, W, G, H


@pytest.mark.parametrize("seed,theta,last", CASES)
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_accepted_trial_is_first_with_positive_spectrum(form, seed, theta, last):
    gamma = 1e7
    p, W, G, H = _setup(form, seed, theta, gamma)
    if form == "lifted":
        J = np.vstack([G, H])
        mat = lambda d: oi.lifted_matrix(W, p.sigma_x, J, p.sigma_s, d)
        d, tried, new_last = oi.lifted_correction(W, p.sigma_x, J, p.sigma_s, last)
    else:
        mat = lambda d: oi.hykkt_matrix(W, p.sigma_x, H, p.sigma_s_ineq, G, gamma, d)
        d, tried, new_last = oi.hykkt_correction(W, p.sigma_x, H, p.sigma_s_ineq, G, gamma, last)
    assert d is not None and len(tried) >= 2 and d == tried[-1] == new_last
    for t in tried[:-1]:
        assert np.linalg.eigvalsh(mat(t))[0] < 0.0, t
    assert np.linalg.eigvalsh(mat(d))[0] > 0.0


@pytest.mark.parametrize("seed,theta,last", CASES)
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_trials_agree_with_k2_inertia(form, seed, theta, last):
    gamma = 1e7
    p, W, G, H = _setup(form, seed, theta, gamma)
    n = p.n
    if form == "lifted":
        # all rows carry slacks (relaxed equalities, Sec. 3.2): K2 has no equality block
        J = np.vstack([G, H])
        d, tried, _ = oi.lifted_correction(W, p.sigma_x, J, p.sigma_s, last)
        Ge, Hi, Ds = np.zeros((0, n)), J, p.sigma_s
    else:
        d, tried, _ = oi.hykkt_correction(W, p.sigma_x, H, p.sigma_s_ineq, G, gamma, last)
        Ge, Hi, Ds = G, H, p.sigma_s_ineq
        K_acc = oi.lifted_matrix(W, p.sigma_x, H, p.sigma_s_ineq, d)
        assert gamma > od.gamma_threshold(K_acc, G)
    me, mi = Ge.shape[0], Hi.shape[0]
    want = (n + mi, mi + me, 0)
    for t in tried:
        got = od.inertia(od.augmented_k2(W, p.sigma_x, Ge, Hi, Ds, delta_w=t))
        assert (got == want) == (t == d), (t, got, want)


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_regularized_solve_equals_k2_solve(form):
    p, W, G, H = _setup(form, 5, 2.0)
    rng = np.random.default_rng(5)
    n = p.n
    if form == "lifted":
        J = np.vstack([G, H])
        d, _, _ = oi.lifted_correction(W, p.sigma_x, J, p.sigma_s)
        Ge, Hi, Ds = np.zeros((0, n)), J, p.sigma_s
    else:
        d, _, _ = oi.hykkt_correction(W, p.sigma_x, H, p.sigma_s_ineq, G, 1e7)
        Ge, Hi, Ds = G, H, p.sigma_s_ineq
    assert d > 0.0
    me, mi = Ge.shape[0], Hi.shape[0]
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    M = od.augmented_k2(W, p.sigma_x, Ge, Hi, Ds, delta_w=d)
    sol = np.linalg.solve(M, -np.concatenate([r1, r2, r3, r4]))
    dx_k2, dy_k2 = sol[:n], sol[n + mi:n + mi + me]
    rb1, rb2 = od.condensed_rhs(r1, r2, r3, r4, Hi, Ds, delta_w=d)
    sx, ss = oi.regularized_diagonals(p.sigma_x, Ds, d)
    K = od.condensed_matrix(W, sx, Hi, ss)
    dx, dy = od.solve_k1(K, Ge, rb1, rb2)
    assert np.abs(dx - dx_k2).max() <= 1e-9 * np.abs(dx_k2).max()
    if me:
        assert np.abs(dy - dy_k2).max() <= 1e-9 * np.abs(dy_k2).max()
    # leaving the slack weights unshifted solves a different system
    K_wrong = od.condensed_matrix(W, sx, Hi, Ds)
    dx_w, _ = od.solve_k1(K_wrong, Ge, rb1, rb2)
    assert np.abs(dx_w - dx_k2).max() > 1e-6 * np.abs(dx_k2).max()
