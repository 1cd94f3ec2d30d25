"""GPU parity of the inertia-corrected factorization (ckkt_factorize_inertia).

* small and mid-size planted cases (negative eigenvalue -theta of the
  condensed matrix, exact by dense eigenvalues): the device search makes the
  oracle's trials (oracle/inertia.py, LAPACK Cholesky as the test) and the
  following ckkt_solve meets omega <= 1e-10 on the REGULARIZED system, the
  solution matching the oracle's dense solve;
* the 66,000-variable network-flow workload with W's diagonal lowered by s:
  every rejected trial is certified by a negative diagonal entry of K(delta_w)
  and the accepted one is the first trial >= s (then K(delta_w) - K is
  positive semidefinite), computed by the oracle from diagonals only;
* delta_w_last carried from one call to the next, a positive definite input
  (one trial, bitwise the plain factorization) and the give-up path.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as od
from oracle import inertia as oi
from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import omega_of, plant_negative_curvature, rhs_of
from tests.test_host_inertia import CASES, GAMMA, oracle_trials

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def regularized(p, form, delta):
    """The problem whose condensed matrix is K(delta_w): delta_w on sigma_x and
    on the slack weights (all rows for LiftedKKT, the inequality rows for HyKKT)."""
    ss = p.sigma_s + delta if form == "lifted" else np.concatenate([p.sigma_s[:p.m_eq], p.sigma_s[p.m_eq:] + delta])
    return dataclasses.replace(p, sigma_x=p.sigma_x + delta, sigma_s=ss)


def device_search(p, form, last=0.0, **params):
    s = Solver(p, form).bind(DEV)
    vals = device_values(p, DEV, form)
    st, res = s.factorize_inertia(*vals, gamma=GAMMA, delta_w_last=last, raise_on_error=False, **params)
    return s, vals, st, res


def solve(s, p, form):
    rhs = torch.as_tensor(rhs_of(p, form), device=DEV)
    sol, info = s.solve(rhs, raise_on_error=False)
    torch.cuda.synchronize()
    return sol.cpu().numpy(), info


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_device_search_matches_oracle(form, case):
    make, theta, last = CASES[case]
    p = plant_negative_curvature(make(), form, theta, GAMMA)
    print_case("device_search", form=form, case=case, n=p.n, theta=theta, last=last)
    d, tried, new_last, K = oracle_trials(p, form, last)
    s, _, st, res = device_search(p, form, last)
    assert st == 0
    assert res == {"delta_w": d, "attempts": len(tried), "delta_w_last": new_last}
    x, info = solve(s, p, form)
    assert info["status"] == 0, info
    pr = regularized(p, form, d)
    om = omega_of(pr, form, x, GAMMA)
    assert om <= 1e-10, (om, info)
    # the oracle's solve of the regularized system (dense)
    W, G, H = od.problem_dense(pr)
    if form == "lifted":
        xo = od.solve_lifted(W, pr.sigma_x, np.vstack([G, H]), pr.sigma_s, pr.b)
    else:
        Kr = od.condensed_matrix(W, pr.sigma_x, H, pr.sigma_s_ineq)
        xo = np.concatenate(od.solve_k1(Kr, G, pr.r1bar, pr.r2bar))
    fe = np.abs(x - xo).max() / np.abs(xo).max()
    print("forward error", fe, info)
    if case < 4:  # diagonals in [0.1, 10]: well conditioned
        assert fe <= 1e-8


def full_size_plant(p, form, margin=0.5):
    """W diagonal lowered by s = min_j K_jj + margin; the expected trials from
    delta_w_last = 0 with a proof for each (diagonals only)."""
    P = osp.Problem(p)
    if form == "lifted":
        J, wts = P.J, p.sigma_s
    else:
        J, wts = P.H, p.sigma_s_ineq
    K = osp.assemble_condensed(P.W, p.sigma_x, J, wts)
    kdiag = K.diagonal()
    if form == "hykkt":
        kdiag = kdiag + GAMMA * np.asarray(P.G.multiply(P.G).sum(axis=0)).ravel()
    s = kdiag.min() + margin
    jsq = np.asarray(J.multiply(J).sum(axis=0)).ravel()
    w = p.w_val.copy()
    for i in range(p.n):
        for k in range(p.w_ptr[i], p.w_ptr[i + 1]):
            if p.w_idx[k] == i:
                w[k] -= s
    pp = dataclasses.replace(p, w_val=w)
    expect, delta = [], 0.0
    while True:
        expect.append(delta)
        if delta >= s:
            break  # K(delta) - K = (delta - s) I + delta J^T J is PSD and K is SPD
        # a negative diagonal entry certifies that K(delta) is not positive definite
        assert (kdiag - s + delta * (1.0 + jsq)).min() < 0.0, ("no certificate at", delta)
        delta = oi.DEFAULTS["delta_w_0"] if delta == 0.0 else delta * oi.DEFAULTS["kappa_plus_bar"]
    return pp, s, expect


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_device_search_full_size(form):
    p = workloads.network_flow(10_000, seed=0)
    # K_gamma's smallest diagonal entry (~570) belongs to a variable with no
    # inequality row: a margin of 200 keeps the trials up to 100 certified
    pp, s, expect = full_size_plant(p, form, margin=0.5 if form == "lifted" else 200.0)
    print_case("device_search_full", form=form, n=p.n, shift=s, expect=expect)
    sv, _, st, res = device_search(pp, form)
    assert st == 0
    assert res == {"delta_w": expect[-1], "attempts": len(expect), "delta_w_last": expect[-1]}
    x, info = solve(sv, pp, form)
    assert info["status"] == 0, info
    om = omega_of(regularized(pp, form, expect[-1]), form, x, GAMMA)
    print("omega", om, info)
    assert om <= 1e-10


def test_delta_w_last_carried_between_calls():
    base = workloads.tiny_grid(8, nx=6, ny=5, sigma_range=(-1, 1))
    p1 = plant_negative_curvature(base, "lifted", 0.5)
    p2 = plant_negative_curvature(base, "lifted", 3.0)
    print_case("delta_w_last_carried", n=p1.n)
    d1, t1, last1, _ = oracle_trials(p1, "lifted", 0.0)
    d2, t2, last2, _ = oracle_trials(p2, "lifted", last1)
    s = Solver(p1, "lifted").bind(DEV)  # same pattern for both systems
    assert np.array_equal(p1.w_idx, p2.w_idx) and np.array_equal(p1.h_idx, p2.h_idx)
    st, r1 = s.factorize_inertia(*device_values(p1, DEV, "lifted"), delta_w_last=0.0)
    assert r1 == {"delta_w": d1, "attempts": len(t1), "delta_w_last": last1}
    st, r2 = s.factorize_inertia(*device_values(p2, DEV, "lifted"), delta_w_last=r1["delta_w_last"])
    assert r2 == {"delta_w": d2, "attempts": len(t2), "delta_w_last": last2}
    x, info = solve(s, p2, "lifted")
    assert omega_of(regularized(p2, "lifted", d2), "lifted", x) <= 1e-10


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_positive_definite_input_one_trial_bitwise(form):
    p = workloads.tiny_grid(10, nx=8, ny=8)
    print_case("spd_one_trial", form=form, n=p.n)
    s, vals, st, res = device_search(p, form, last=0.25)
    assert st == 0 and res == {"delta_w": 0.0, "attempts": 1, "delta_w_last": 0.25}
    x, info = solve(s, p, form)
    s0 = Solver(p, form).bind(DEV)
    s0.factorize(*vals, gamma=GAMMA)
    x0, info0 = solve(s0, p, form)
    assert np.array_equal(x, x0) and info == info0


def test_gives_up_above_delta_w_max():
    p = plant_negative_curvature(workloads.tiny_grid(7, nx=4, ny=3, sigma_range=(-1, 1)), "lifted", 5.0)
    print_case("gives_up", n=p.n)
    s, _, st, res = device_search(p, "lifted", delta_w_max=0.5)
    assert st == -3 and res == {"delta_w": 1e-2, "attempts": 3, "delta_w_last": 0.0}
    _, info = solve(s, p, "lifted")
    assert info["status"] == -3
