"""CPU tests of the inertia-corrected factorization through the C-ABI.

ckkt_host_factor_solve_inertia runs the library's delta_w search over the
sequential host factorization of the same plan; its trials, accepted delta_w
and delta_w_last must equal those of the oracle (oracle/inertia.py, dense
LAPACK Cholesky as the test), and its solution must solve the regularized
system.  The argument checks of both inertia entry points need no GPU.
"""
import ctypes

import numpy as np
import pytest

from oracle import dense as od
from oracle import inertia as oi
from paper_2405_14236_amd import _lib, workloads
from paper_2405_14236_amd.solver import Solver, inertia_params
from tests._common import plant_negative_curvature

GAMMA = 1e7


def oracle_trials(p, form, last, **params):
    W, G, H = od.problem_dense(p)
    if form == "lifted":
        J = np.vstack([G, H])
        d, tried, new_last = oi.lifted_correction(W, p.sigma_x, J, p.sigma_s, last, params)
        K = oi.lifted_matrix(W, p.sigma_x, J, p.sigma_s, d) if d is not None else None
    else:
        d, tried, new_last = oi.hykkt_correction(W, p.sigma_x, H, p.sigma_s_ineq, G, GAMMA, last, params)
        K = oi.hykkt_matrix(W, p.sigma_x, H, p.sigma_s_ineq, G, GAMMA, d) if d is not None else None
    return d, tried, new_last, K


CASES = [
    # (problem, theta, delta_w_last)
    (lambda: workloads.tiny_grid(0, nx=4, ny=3, sigma_range=(-1, 1)), 0.5, 0.0),
    (lambda: workloads.tiny_grid(1, nx=4, ny=3, sigma_range=(-1, 1)), 5.0, 0.0),
    (lambda: workloads.tiny_grid(2, nx=6, ny=5, sigma_range=(-1, 1)), 0.5, 0.3),
    (lambda: workloads.tiny_grid(3, nx=6, ny=5, sigma_range=(-1, 1)), 40.0, 2.0),
    (lambda: workloads.tiny_grid(4), 0.5, 0.0),
    (lambda: workloads.tiny_grid(5), 3.0, 1e-3),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_host_search_matches_oracle(form, case):
    make, theta, last = CASES[case]
    p = plant_negative_curvature(make(), form, theta, GAMMA)
    d, tried, new_last, K = oracle_trials(p, form, last)
    assert d is not None and len(tried) >= 2
    s = Solver(p, form)
    ss = p.sigma_s if form == "lifted" else p.sigma_s_ineq
    rhs = p.b if form == "lifted" else p.r1bar
    x, st, res = s.host_factor_solve_inertia(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, GAMMA, rhs,
                                             delta_w_last=last)
    assert st == 0
    assert res == {"delta_w": d, "attempts": len(tried), "delta_w_last": new_last}
    xo = np.linalg.solve(K, rhs)
    assert np.abs(x - xo).max() <= 1e-6 * np.abs(xo).max()


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_host_search_spd_needs_one_trial(form):
    p = workloads.tiny_grid(6, nx=4, ny=4)
    s = Solver(p, form)
    ss = p.sigma_s if form == "lifted" else p.sigma_s_ineq
    rhs = p.b if form == "lifted" else p.r1bar
    x, st, res = s.host_factor_solve_inertia(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, GAMMA, rhs,
                                             delta_w_last=0.25)
    assert st == 0 and res == {"delta_w": 0.0, "attempts": 1, "delta_w_last": 0.25}
    x0, st0, _ = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, GAMMA, rhs)
    assert st0 == 0 and np.array_equal(x, x0)


def test_host_search_gives_up_at_delta_w_max():
    p = plant_negative_curvature(workloads.tiny_grid(7, nx=4, ny=3, sigma_range=(-1, 1)), "lifted", 5.0)
    d, tried, new_last, _ = oracle_trials(p, "lifted", 0.0, delta_w_max=0.5)
    assert d is None and tried == [0.0, 1e-4, 1e-2]
    s = Solver(p, "lifted")
    _, st, res = s.host_factor_solve_inertia(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s, 0.0, p.b,
                                             delta_w_last=0.0, delta_w_max=0.5)
    assert st == -3  # CKKT_ERR_NOT_SPD
    assert res == {"delta_w": 1e-2, "attempts": 3, "delta_w_last": 0.0}


@pytest.mark.parametrize("bad", [dict(kappa_minus=1.5), dict(kappa_minus=0.0), dict(kappa_plus=1.0),
                                 dict(kappa_plus_bar=0.5), dict(delta_w_min=0.0), dict(delta_w_0=-1.0),
                                 dict(delta_w_max=float("inf")), dict(delta_w_0=float("nan"))])
def test_inertia_parameters_out_of_range_rejected(bad):
    p = workloads.tiny_grid(0, nx=3, ny=3)
    s = Solver(p, "lifted")
    _, st, _ = s.host_factor_solve_inertia(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s, 0.0, p.b, **bad)
    assert st == -1
    lib = _lib.load()
    ic = inertia_params(0.0, **bad)
    assert lib.ckkt_factorize_inertia(s.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1
    ic = inertia_params(-1.0)
    assert lib.ckkt_factorize_inertia(s.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1


def test_inertia_entry_point_needs_fp64_single_system():
    p = workloads.tiny_grid(0, nx=3, ny=3)
    lib = _lib.load()
    ic = inertia_params()
    s32 = Solver(p, "lifted", "fp32_ir")
    assert lib.ckkt_factorize_inertia(s32.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1
    sb = Solver(None, "lifted", batch=[p, workloads.tiny_grid(1, nx=3, ny=3)])
    assert lib.ckkt_factorize_inertia(sb.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1
    s = Solver(p, "lifted")  # no workspace bound yet
    assert lib.ckkt_factorize_inertia(s.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -6
    assert lib.ckkt_factorize_inertia(s.h, None, None, None, None, None, 0.0, None, None) == -1
    assert lib.ckkt_factorize_inertia(None, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1
