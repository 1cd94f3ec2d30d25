"""Dense Jacobian rows split off the condensed matrix (opt.dense_row_min),
checked on the CPU through the host run of the plan: the analysis keeps the
rows out of K's pattern, and the host factor-solve with its Woodbury step
solves the FULL system, certified by the oracle (which knows nothing of the
split).  Argument checks of the option need no GPU."""
import ctypes

import numpy as np
import pytest

from oracle import sparse as osp
from paper_2405_14236_amd import _lib, workloads
from paper_2405_14236_amd.solver import Solver
from tests._common import omega_kgamma


def _prob(seed, count=3, frac=0.6, **kw):
    return workloads.with_dense_rows(workloads.tiny_grid(seed, **kw), count=count, frac=frac, seed=seed)


def test_split_rows_leave_the_pattern():
    p = _prob(40)
    full = Solver(p, "lifted").info()
    split = Solver(p, "lifted", dense_row_min=50).info()
    assert full["n_dense_rows"] == 0 and split["n_dense_rows"] == 3
    assert split["nnz_k"] < full["nnz_k"] / 3
    base = Solver(workloads.tiny_grid(40), "lifted").info()
    assert split["nnz_k"] == base["nnz_k"]  # the same pattern as without the dense rows


@pytest.mark.parametrize("seed", [41, 42])
@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_host_woodbury_solves_the_full_system(seed, formulation):
    p = _prob(seed, sigma_range=(-3, 3))
    gamma = 1e7
    s = Solver(p, formulation, dense_row_min=50)
    assert s.info()["n_dense_rows"] == 3
    ss = p.sigma_s if formulation == "lifted" else p.sigma_s_ineq
    x, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, gamma, p.b)
    assert st == 0 and fc == -1
    if formulation == "lifted":
        P = osp.Problem(p)
        om = osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, x, p.b)
    else:
        om = omega_kgamma(p, x, p.b, gamma)
    assert om < 1e-11, om
    # and the same point as the unsplit factorization
    x0, st0, _ = Solver(p, formulation).host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, gamma, p.b)
    assert st0 == 0
    assert np.abs(x - x0).max() <= 1e-6 * np.abs(x0).max()


def test_dense_row_option_arguments():
    p = _prob(43)
    lib = _lib.load()
    with pytest.raises(_lib.CkktError):
        Solver(p, "lifted", "fp32_ir", dense_row_min=50)
    with pytest.raises(_lib.CkktError):
        Solver(p, "lifted", dense_row_min=-1)
    with pytest.raises(_lib.CkktError):
        Solver(None, "lifted", batch=[p, p], dense_row_min=50)
    many = workloads.with_dense_rows(workloads.tiny_grid(44), count=65, frac=0.4, seed=44)
    with pytest.raises(_lib.CkktError):
        Solver(many, "lifted", dense_row_min=50)
    s = Solver(p, "lifted", dense_row_min=50)
    from paper_2405_14236_amd.solver import inertia_params
    ic = inertia_params()
    assert lib.ckkt_factorize_inertia(s.h, None, None, None, None, None, 0.0, ctypes.byref(ic), None) == -1


@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_host_woodbury_dense_equality_row(formulation):
    """A dense row of G: split with weight gamma (HyKKT) or its relaxed sigma_s (LiftedKKT)."""
    p = workloads.with_dense_rows(workloads.tiny_grid(49, sigma_range=(-2, 2)), count=1, frac=0.7, seed=49,
                                  equality=True)
    gamma = 1e7
    s = Solver(p, formulation, dense_row_min=50)
    assert s.info()["n_dense_rows"] == 1
    ss = p.sigma_s if formulation == "lifted" else p.sigma_s_ineq
    x, st, _ = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, gamma, p.b)
    assert st == 0
    if formulation == "lifted":
        P = osp.Problem(p)
        om = osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, x, p.b)
    else:
        om = omega_kgamma(p, x, p.b, gamma)
    assert om < 1e-11, om


def test_host_gamma_below_threshold_is_not_spd():
    """Sec. 3.1 / eq:ipm:inertia: with K indefinite but positive definite on
    Ker(G), K_gamma fails for small gamma and factors above the threshold."""
    from oracle import dense as od
    import dataclasses
    base = workloads.tiny_grid(57, nx=4, ny=3, vpn=3, sigma_range=(-1, 1))
    W, G, H = od.problem_dense(base)
    K = od.condensed_matrix(W, base.sigma_x, H, base.sigma_s_ineq)
    Y, Z, _ = od.null_range_bases(G)
    lo, hi = np.linalg.eigvalsh(K)[0], np.linalg.eigvalsh(Z.T @ K @ Z)[0]
    assert hi > lo + 0.1
    shift = 0.5 * (lo + hi) + 0.5 * (hi - lo) * 0.5  # between the two smallest eigenvalues
    w = base.w_val.copy()
    for i in range(base.n):
        for k in range(base.w_ptr[i], base.w_ptr[i + 1]):
            if base.w_idx[k] == i:
                w[k] -= shift
    p = dataclasses.replace(base, w_val=w)
    Kp = K - shift * np.eye(base.n)
    assert np.linalg.eigvalsh(Kp)[0] < 0 < np.linalg.eigvalsh(Z.T @ Kp @ Z)[0]
    thr = od.gamma_threshold(Kp, G)
    s = Solver(p, "hykkt")
    _, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s_ineq, 1e-6, p.r1bar)
    assert st == -3 and fc >= 0
    _, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s_ineq, 10 * thr, p.r1bar)
    assert st == 0 and fc == -1
