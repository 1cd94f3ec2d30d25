"""Edge cases of the entry points around the hot path, on the GPU against the
oracle: inertia correction without constraint rows, dual regularization
without equality rows, the K2 step without constraints, and a dense
equality row split with weight gamma inside HyKKT's CG."""
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

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def test_inertia_without_constraints():
    base = workloads.tiny_grid(50, nx=5, ny=4, m_eq=0, m_ineq=0, sigma_range=(-1, 1))
    p = plant_negative_curvature(base, "lifted", 2.0)
    print_case("inertia_no_rows", n=p.n)
    W, _, _ = od.problem_dense(p)
    d, tried, last = oi.lifted_correction(W, p.sigma_x, np.zeros((0, p.n)), np.zeros(0), 0.0)
    s = Solver(p, "lifted").bind(DEV)
    st, res = s.factorize_inertia(*device_values(p, DEV, "lifted"))
    assert st == 0 and res == {"delta_w": d, "attempts": len(tried), "delta_w_last": last}
    x, info = s.solve(torch.as_tensor(p.b, device=DEV))
    torch.cuda.synchronize()
    xo = np.linalg.solve(oi.lifted_matrix(W, p.sigma_x, np.zeros((0, p.n)), np.zeros(0), d), p.b)
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-10 * np.abs(xo).max()


def test_dual_reg_without_equalities():
    p = workloads.tiny_grid(51, m_eq=0, sigma_range=(-1, 1))
    print_case("dual_reg_no_eq", n=p.n, m_ineq=p.m_ineq)
    s = Solver(p, "hykkt").bind(DEV)
    s.factorize_dual_reg(*device_values(p, DEV, "hykkt"), 1e-5)
    z, info = s.solve(torch.as_tensor(p.r1bar, device=DEV))
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["cg_iters"] == 0
    P = osp.Problem(p)
    om = osp.omega_k1(P.W, p.sigma_x, P.H, p.sigma_s_ineq, P.G, z.cpu().numpy(), np.zeros(0), p.r1bar,
                      np.zeros(0), 1e-5)
    assert om <= 1e-10


def test_k2_step_without_constraints():
    p = workloads.tiny_grid(52, m_eq=0, m_ineq=0, sigma_range=(-1, 1))
    print_case("k2_no_rows", n=p.n)
    s = Solver(p, "lifted").bind(DEV)
    s.factorize(*device_values(p, DEV, "lifted"))
    r1 = torch.as_tensor(np.random.default_rng(52).standard_normal(p.n), device=DEV)
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    dx, ds, _, dz, info = s.solve_augmented(r1, e, None, e)
    torch.cuda.synchronize()
    assert info["status"] == 0 and ds.numel() == 0 and dz.numel() == 0
    W, _, _ = od.problem_dense(p)
    xo = np.linalg.solve(W + np.diag(p.sigma_x), -r1.cpu().numpy())
    assert np.abs(dx.cpu().numpy() - xo).max() <= 1e-10 * np.abs(xo).max()


def test_dense_equality_row_hykkt_cg():
    p = workloads.with_dense_rows(workloads.tiny_grid(53, sigma_range=(-1, 1)), count=2, frac=0.7, seed=53,
                                  equality=True)
    print_case("dense_eq_row", n=p.n, m_eq=p.m_eq)
    s = Solver(p, "hykkt", dense_row_min=60).bind(DEV)
    assert s.info()["n_dense_rows"] == 2
    s.factorize(*device_values(p, DEV, "hykkt"), gamma=1e7)
    z, info = s.solve(torch.as_tensor(rhs_of(p, "hykkt"), device=DEV))
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["cg_iters"] > 0, info
    assert omega_of(p, "hykkt", z.cpu().numpy()) <= 1e-10
