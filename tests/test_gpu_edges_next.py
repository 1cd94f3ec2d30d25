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


def _nan_at(a, k=3, val=float("nan")):
    b = np.array(a, dtype=np.float64, copy=True)
    b[k] = val
    return b


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_nonfinite_inputs_reported(form, precision):
    p = workloads.tiny_grid(54)
    print_case("nonfinite", form=form, precision=precision, n=p.n)
    s = Solver(p, form, precision).bind(DEV)
    rhs = torch.as_tensor(rhs_of(p, form), device=DEV)
    for bad in (dataclasses.replace(p, sigma_x=_nan_at(p.sigma_x)),
                dataclasses.replace(p, w_val=_nan_at(p.w_val, val=float("inf")))):
        s.factorize(*device_values(bad, DEV, form), gamma=1e7)
        assert s.factor_status() == -9
        _, info = s.solve(rhs, raise_on_error=False)
        assert info["status"] == -9, info
    # a clean system afterwards: the flag is cleared; a NaN right-hand side is reported
    s.factorize(*device_values(p, DEV, form), gamma=1e7)
    assert s.factor_status() == 0
    _, info = s.solve(rhs, raise_on_error=False)
    assert info["status"] == 0
    bad_rhs = torch.as_tensor(_nan_at(rhs_of(p, form)), device=DEV)
    _, info = s.solve(bad_rhs, raise_on_error=False)
    assert info["status"] == -9, info


def test_nonfinite_k2_right_hand_side():
    p = workloads.tiny_grid(55)
    print_case("nonfinite_k2", n=p.n)
    s = Solver(p, "lifted").bind(DEV)
    s.factorize(*device_values(p, DEV, "lifted"))
    rng = np.random.default_rng(55)
    r = [torch.as_tensor(_nan_at(rng.standard_normal(k)) if i == 3 else rng.standard_normal(k), device=DEV)
         for i, k in enumerate((p.n, p.m, 0, p.m))]
    *_, info = s.solve_augmented(r[0], r[1], None, r[3], raise_on_error=False)
    assert info["status"] == -9


def test_cg_limit_and_refinement_limit():
    """One CG iteration per outer step: the outer FP64 refinement on K1 still
    reaches the gate (a stationary iteration around an inexact inner solve);
    with the refinement also limited to one step it reports
    CKKT_ERR_NO_CONVERGENCE and leaves its best iterate."""
    p = workloads.tiny_grid(56)
    print_case("cg_maxit_1", n=p.n)
    rhs = torch.as_tensor(rhs_of(p, "hykkt"), device=DEV)
    s = Solver(p, "hykkt", cg_maxit=1).bind(DEV)
    s.factorize(*device_values(p, DEV, "hykkt"), gamma=1e7)
    z, info = s.solve(rhs, raise_on_error=False)
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["refine_steps"] > 0 and info["cg_iters"] == info["refine_steps"] + 1, info
    assert omega_of(p, "hykkt", z.cpu().numpy()) <= 1e-10
    s1 = Solver(p, "hykkt", cg_maxit=1, ir_maxit=1).bind(DEV)
    s1.factorize(*device_values(p, DEV, "hykkt"), gamma=1e7)
    z1, info1 = s1.solve(rhs, raise_on_error=False)
    torch.cuda.synchronize()
    assert info1["status"] == -4, info1
    assert 1e-10 < info1["omega"] < np.inf and np.all(np.isfinite(z1.cpu().numpy()))


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_loaded_plan_solves_bitwise(form):
    p = workloads.network_flow(2_000, seed=62)
    print_case("plan_load", form=form, n=p.n)
    s = Solver(p, form).bind(DEV)
    t = Solver.from_plan(s.save_plan()).bind(DEV)
    vals = device_values(p, DEV, form)
    rhs = torch.as_tensor(rhs_of(p, form), device=DEV)
    out = []
    for sv in (s, t):
        sv.factorize(*vals, gamma=1e7)
        z, info = sv.solve(rhs)
        torch.cuda.synchronize()
        out.append((z.cpu().numpy(), info))
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1] == out[1][1]
    assert omega_of(p, form, out[1][0]) <= 1e-10


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_k2_step_fp32_factor(form):
    """The K2 Newton step on an FP32 + FP64-refinement handle meets the 1e-8
    gate (refining on K2, falling back to the FP64 factor when it stalls)."""
    from oracle import newton as on
    import scipy.sparse as sp
    p = workloads.tiny_grid(63, nx=12, ny=12)
    print_case("k2_fp32", form=form, n=p.n)
    s = Solver(p, form, "fp32_ir", tol=1e-8).bind(DEV)
    s.factorize(*device_values(p, DEV, form), gamma=1e7)
    ms = p.m if form == "lifted" else p.m_ineq
    me = 0 if form == "lifted" else p.m_eq
    rng = np.random.default_rng(63)
    r = [rng.standard_normal(k) for k in (p.n, ms, me, ms)]
    t = [torch.as_tensor(a, device=DEV) for a in r]
    dx, ds, dy, dz, info = s.solve_augmented(t[0], t[1], t[2] if me else None, t[3])
    torch.cuda.synchronize()
    assert info["status"] == 0, info
    P = osp.Problem(p)
    if form == "lifted":
        G, H, E = sp.csr_matrix((0, p.n)), P.J, p.sigma_s
    else:
        G, H, E = P.G, P.H, p.sigma_s_ineq
    yv = dy.cpu().numpy() if dy is not None else np.zeros(0)
    om = on.omega_k2(P.W, p.sigma_x, G, H, E, *r, dx.cpu().numpy(), ds.cpu().numpy(), yv, dz.cpu().numpy())
    print("omega", om, info)
    assert om <= 1e-8


def test_dual_reg_fp32_factor():
    p = workloads.tiny_grid(64, nx=12, ny=12)
    print_case("dual_reg_fp32", n=p.n)
    s = Solver(p, "hykkt", "fp32_ir", tol=1e-8).bind(DEV)
    s.factorize_dual_reg(*device_values(p, DEV, "hykkt"), 1e-6)
    z, info = s.solve(torch.as_tensor(rhs_of(p, "hykkt"), device=DEV), raise_on_error=False)
    torch.cuda.synchronize()
    assert info["status"] == 0 and info["cg_iters"] == 0, info
    P = osp.Problem(p)
    zz = z.cpu().numpy()
    om = osp.omega_k1(P.W, p.sigma_x, P.H, p.sigma_s_ineq, P.G, zz[:p.n], zz[p.n:], p.r1bar, p.r2bar, 1e-6)
    print("omega", om, info)
    assert om <= 1e-8
