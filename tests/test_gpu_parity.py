"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Gates (the residual reading is the componentwise relative backward error
omega, computed by the oracle on the GPU's output):
  * FP64 LiftedKKT and HyKKT: omega <= 1e-10 (and the library's own omega
    agrees with the oracle's to within rounding);
  * assembled K: every entry within 8 u (|W_ij| + sum_r |d_r J_ri J_rj|) of
    the oracle's brute-force assembly;
  * one factor application: identical (to rounding) to the host run of the
    same plan, and omega of K^{-1} b small;
  * forward error vs the oracle's solution reported, and gated only on
    well-conditioned inputs.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as od
from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import omega_kgamma, omega_of, rhs_of, sigma_rows

pytestmark = pytest.mark.gpu

DEV = "cuda"
U64 = np.finfo(np.float64).eps / 2


def run(p, formulation, precision="fp64", gamma=1e7, **opts):
    s = Solver(p, formulation, precision, **opts).bind(DEV)
    vals = device_values(p, DEV, formulation)
    s.factorize(*vals, gamma=gamma)
    rhs = torch.as_tensor(rhs_of(p, formulation), device=DEV)
    sol, info = s.solve(rhs)
    torch.cuda.synchronize()
    return s, vals, sol.cpu().numpy(), info


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tiny_lifted_fp64(seed):
    p = workloads.tiny_grid(seed)
    print_case("tiny_lifted_fp64", seed=seed, n=p.n)
    s, vals, x, info = run(p, "lifted")
    om = omega_of(p, "lifted", x)
    assert om <= 1e-10, (om, info)
    assert info["omega"] <= 1e-10
    # the library's omega is the oracle's up to rounding of the residual
    assert abs(info["omega"] - om) <= 1e-14 + 0.1 * om
    P = osp.Problem(p)
    xo, _ = osp.solve_lifted(P, p.sigma_x, p.sigma_s, p.b)
    fe = np.abs(x - xo).max() / np.abs(xo).max()
    print("forward error vs oracle", fe, info)
    assert fe < 1e-4  # kappa ~ 1e8 on this input


@pytest.mark.parametrize("seed", [0, 3])
def test_tiny_hykkt_fp64(seed):
    p = workloads.tiny_grid(seed)
    print_case("tiny_hykkt_fp64", seed=seed, n=p.n)
    s, vals, z, info = run(p, "hykkt")
    om = omega_of(p, "hykkt", z)
    assert om <= 1e-10, (om, info)
    assert info["cg_iters"] > 0
    P = osp.Problem(p)
    dx, dy, _ = osp.solve_k1(P, p.sigma_x, p.sigma_s_ineq, p.r1bar, p.r2bar)
    fe = np.abs(z[:p.n] - dx).max() / np.abs(dx).max()
    print("forward error vs oracle", fe, info)


def test_well_conditioned_forward_error():
    """Diagonals in [0.1, 10]: the solution itself must match the oracle."""
    p = workloads.tiny_grid(4, sigma_range=(-1, 1))
    print_case("tiny_wellcond", n=p.n)
    for form in ("lifted", "hykkt"):
        s, vals, z, info = run(p, form)
        P = osp.Problem(p)
        if form == "lifted":
            xo, _ = osp.solve_lifted(P, p.sigma_x, p.sigma_s, p.b)
            assert np.abs(z - xo).max() <= 1e-10 * np.abs(xo).max()
        else:
            dx, dy, _ = osp.solve_k1(P, p.sigma_x, p.sigma_s_ineq, p.r1bar, p.r2bar)
            assert np.abs(z[:p.n] - dx).max() <= 1e-9 * np.abs(dx).max()
            assert np.abs(z[p.n:] - dy).max() <= 1e-9 * np.abs(dy).max()


@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_assembled_k_matches_oracle(formulation):
    p = workloads.tiny_grid(5)
    print_case("assembly", formulation=formulation)
    gamma = 1e7
    s = Solver(p, formulation).bind(DEV)
    s.factorize(*device_values(p, DEV, formulation), gamma=gamma)
    rows, cols, vals = s.export_k()
    kv = vals.cpu().numpy()
    W, G, H = od.problem_dense(p)
    J = np.vstack([G, H])
    d = sigma_rows(p, formulation, gamma)
    K = od.assemble_bruteforce(W, p.sigma_x, J, d)
    mag = np.abs(W) + np.diag(p.sigma_x) + np.abs(J).T @ np.diag(np.abs(d)) @ np.abs(J)
    err = np.abs(kv - K[rows, cols])
    assert np.all(err <= 8 * U64 * mag[rows, cols] + 1e-300), err.max()
    # every structural entry of K is present exactly once
    assert len(set(zip(rows.tolist(), cols.tolist()))) == len(rows)
    nz = np.argwhere(np.tril(mag) > 0)
    assert len(nz) == len(rows)


@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_factor_application_matches_host_run(formulation):
    """Device sweeps/factor == host run of the same plan (same arithmetic up to
    FMA contraction), on a size that uses both front paths."""
    p = workloads.network_flow(4000, seed=4)
    print_case("apply_inverse_vs_host", formulation=formulation, n=p.n)
    gamma = 1e7
    s = Solver(p, formulation, lds_front_max=64).bind(DEV)
    assert s.info()["n_big_fronts"] > 0
    vals = device_values(p, DEV, formulation)
    s.factorize(*vals, gamma=gamma)
    b = torch.as_tensor(p.b, device=DEV)
    x = s.apply_inverse(b).cpu().numpy()
    ss = p.sigma_s if formulation == "lifted" else p.sigma_s_ineq
    xh, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, gamma, p.b)
    assert st == 0
    scale = np.abs(xh).max()
    assert np.abs(x - xh).max() <= 1e-6 * scale, np.abs(x - xh).max() / scale
    assert omega_kgamma(p, x, p.b, gamma if formulation == "hykkt" else 0.0) < 1e-9 if formulation == "hykkt" \
        else osp.omega_condensed(osp.Problem(p).W, p.sigma_x, osp.Problem(p).J, p.sigma_s, x, p.b) < 1e-9


@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_network_flow_10k_fp64(formulation):
    """The n = 66,000 network-flow workload (10k nodes, 13k edges)."""
    p = workloads.network_flow(10_000, seed=0)
    print_case("netflow10k_fp64", formulation=formulation, n=p.n)
    s, vals, z, info = run(p, formulation)
    om = omega_of(p, formulation, z)
    print(info, "oracle omega", om)
    assert om <= 1e-10


def test_deterministic():
    p = workloads.network_flow(3000, seed=1)
    print_case("determinism", n=p.n)
    outs = []
    for _ in range(2):
        s, vals, x, info = run(p, "lifted")
        outs.append(x)
    assert np.array_equal(outs[0], outs[1])


def test_not_spd_status():
    p = workloads.tiny_grid(0, nx=3, ny=3, sigma_range=(-1, 1))
    print_case("not_spd", n=p.n)
    w = p.w_val.copy()
    i = 7
    w[p.w_ptr[i + 1] - 1] = -1e6
    q = workloads.KKTProblem(**{**p.__dict__, "w_val": w})
    s = Solver(q, "lifted").bind(DEV)
    s.factorize(*device_values(q, DEV, "lifted"))
    assert s.factor_status() == -3
    rhs = torch.as_tensor(q.b, device=DEV)
    _, info = s.solve(rhs, raise_on_error=False)
    assert info["status"] == -3
    assert s.info()["failed_column"] >= 0


@pytest.mark.parametrize("shift", [1e-2, 1.0, 1e3])
def test_not_spd_column_matches_host_run_large_fronts(shift):
    """A matrix that is not positive definite (W's diagonal lowered), factorized
    with most fronts forced onto the large-front path (panel and trailing-update
    launches): the device reports the same outcome and the same first failing
    column as the host run of the same plan (a failure in a later front can only
    raise the column, and the device keeps the smallest)."""
    p = workloads.network_flow(2000, seed=5)
    rows = np.repeat(np.arange(p.n), np.diff(p.w_ptr))
    wv = p.w_val.copy()
    wv[rows == p.w_idx] -= shift
    q = workloads.KKTProblem(**{**p.__dict__, "w_val": wv})
    print_case("not_spd_large_fronts", n=q.n, shift=shift)
    s = Solver(q, "lifted", lds_front_max=32).bind(DEV)
    assert s.info()["n_big_fronts"] > 0
    s.factorize(*device_values(q, DEV, "lifted"))
    st_dev, fc_dev = s.factor_status(), s.info()["failed_column"]
    _, st, fc = s.host_factor_solve(q.w_val, q.g_val, q.h_val, q.sigma_x, q.sigma_s, 0.0, q.b)
    print("device", st_dev, fc_dev, "host", st, fc, flush=True)
    assert (st_dev == 0) == (st == 0), (st_dev, st)
    assert (st != 0) == (shift >= 1.0)  # the two larger shifts make K indefinite
    if st != 0:
        assert st_dev == -3
        assert fc_dev == fc, (fc_dev, fc)


def test_edge_no_constraints_and_single_variable():
    # m_eq = m_ineq = 0 and n = 1
    for nx, ny in ((1, 1), (2, 1)):
        p = workloads.tiny_grid(1, nx=nx, ny=ny, vpn=1, m_eq=0, m_ineq=0, sigma_range=(-2, 2))
        print_case("edge_empty_J", n=p.n)
        s, vals, x, info = run(p, "lifted")
        W, G, H = od.problem_dense(p)
        xo = np.linalg.solve(W + np.diag(p.sigma_x), p.b)
        assert np.allclose(x, xo, rtol=1e-12, atol=1e-14)


def test_edge_hykkt_without_equalities():
    p = workloads.tiny_grid(2, nx=4, ny=3, m_eq=0, m_ineq=20, sigma_range=(-4, 4))
    print_case("edge_hykkt_no_eq", n=p.n)
    s, vals, z, info = run(p, "hykkt")
    assert omega_of(p, "hykkt", z) <= 1e-10


def test_graph_replay_matches_direct_launches(monkeypatch):
    """Captured launch sequences (hipGraph) give bitwise the direct-launch
    result, on several replays with eager work in between."""
    p = workloads.network_flow(2500, seed=7)
    print_case("graph_vs_direct", n=p.n)
    res = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("CKKT_NO_GRAPH", mode)
        s = Solver(p, "hykkt").bind(DEV)
        outs = []
        for k in range(3):
            q = p.with_sigma(p.sigma_x * (1 + k), p.sigma_s * (1 + 0.5 * k))
            s.factorize(*device_values(q, DEV, "hykkt"), gamma=1e7)
            z, info = s.solve(torch.as_tensor(rhs_of(q, "hykkt"), device=DEV))
            torch.cuda.synchronize()
            outs.append(z.cpu().numpy())
            _ = torch.randn(1000, device=DEV).sum().item()  # unrelated eager work
        res[mode] = outs
    for a, b in zip(res["0"], res["1"]):
        assert np.array_equal(a, b)


def test_large_network_flow_fronts_at_lds_limit():
    """The n = 528,000 network-flow workload (80k nodes): its fronts reach the
    LDS capacity of one workgroup; every launch must fit and the FP64 solve
    must meet the gate."""
    p = workloads.network_flow(80_000, seed=0)
    print_case("netflow80k_fp64", n=p.n)
    s, vals, x, info = run(p, "lifted")
    om = omega_of(p, "lifted", x)
    print(info, "oracle omega", om, s.info()["max_front"])
    assert om <= 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_dependency_driven_sweeps_match_level_sweeps(monkeypatch, precision):
    """The dependency-driven sweeps (wave and workgroup workers taking
    supernodes from ticket counters) and the level-by-level sweeps apply the
    same factor: solutions agree to rounding, both meet the gate, and
    repeated applications of the dependency-driven sweeps are bitwise
    identical (the arithmetic order does not depend on the schedule)."""
    p = workloads.network_flow(6000, seed=11, sigma_range=(-2, 2))  # moderate conditioning
    print_case("sweep_schedules", n=p.n, precision=precision)
    tol = 1e-10 if precision == "fp64" else 1e-8
    out = {}
    for mode in ("0", "1", "2"):  # level by level; dependency-driven; hybrid (the default)
        monkeypatch.setenv("CKKT_DEP_SWEEPS", mode)
        s = Solver(p, "lifted", precision, tol=tol).bind(DEV)
        s.factorize(*device_values(p, DEV, "lifted"))
        b = torch.as_tensor(p.b, device=DEV)
        x1 = s.apply_inverse(b)
        x2 = s.apply_inverse(b)
        z, info = s.solve(b)
        torch.cuda.synchronize()
        assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
        assert omega_of(p, "lifted", z.cpu().numpy()) <= tol
        out[mode] = x1.cpu().numpy()
    a = out["0"]
    for mode in ("1", "2"):
        assert np.abs(a - out[mode]).max() <= 1e-8 * np.abs(a).max(), mode


@pytest.mark.parametrize("case,precision,tiled", [
    ("pde20", "fp64", "1024"),
    ("pde20", "fp64", "141"),
    ("netflow4000_lds64", "fp64", "65"),
    ("netflow4000_lds64", "fp32_ir", "65"),
    ("netflow40k", "fp32_ir", "141"),
])
def test_tiled_sweeps_match_workgroup_sweeps(monkeypatch, case, precision, tiled):
    """Fronts swept by the tiled kernels (many workgroups, one launch per
    64-column block) and by one workgroup each apply the same factor: both
    meet the gate, repeated applications are bitwise identical, and the two
    agree to rounding.  pde20 has fronts up to 1507 rows (ragged last
    blocks, rows below the own columns; with 141 every front above the LDS
    limit is tiled); netflow4000 with a 64-row LDS limit tiles every front
    from 65 rows on (one or two column blocks); netflow40k covers the FP32
    factor on fronts up to 328 rows."""
    if case == "pde20":
        p, opts = workloads.pde_control(20), {}
    elif case == "netflow40k":
        p, opts = workloads.network_flow(40_000, seed=3, sigma_range=(-2, 2)), {}
    else:
        p, opts = workloads.network_flow(4000, seed=4, sigma_range=(-2, 2)), {"lds_front_max": 64}
    print_case("tiled_sweeps", case=case, n=p.n, precision=precision, tiled=tiled)
    tol = 1e-10 if precision == "fp64" else 1e-8
    out = {}
    for mode in (tiled, "16000"):
        monkeypatch.setenv("CKKT_TILED_SWEEP_FRONT", mode)
        s = Solver(p, "lifted", precision, tol=tol, **opts).bind(DEV)
        s.factorize(*device_values(p, DEV, "lifted"))
        b = torch.as_tensor(p.b, device=DEV)
        x1 = s.apply_inverse(b)
        x2 = s.apply_inverse(b)
        z, info = s.solve(b)
        torch.cuda.synchronize()
        assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
        om = omega_of(p, "lifted", z.cpu().numpy())
        print(mode, info, "oracle omega", om)
        assert om <= tol
        out[mode] = x1.cpu().numpy()
    # different summation orders, amplified by the conditioning of K
    a, c = out[tiled], out["16000"]
    assert np.all(np.isfinite(a)) and np.abs(a - c).max() <= 1e-6 * np.abs(a).max()


def test_fp32_factor_overflow_falls_back_to_fp64():
    """pde12's lifted matrix is beyond FP32 (its FP32 factor overflows to
    non-finite values): the solve must see a non-finite residual, refactor
    in FP64 and meet the gate, never report the non-finite iterate as
    converged."""
    p = workloads.pde_control(12)
    print_case("fp32_overflow_fallback", n=p.n)
    z, info = None, None
    s = Solver(p, "lifted", "fp32_ir", tol=1e-8).bind(DEV)
    s.factorize(*device_values(p, DEV, "lifted"))
    z, info = s.solve(torch.as_tensor(p.b, device=DEV))
    torch.cuda.synchronize()
    z = z.cpu().numpy()
    print(info)
    assert info["fallback"] == 2
    assert np.all(np.isfinite(z))
    assert omega_of(p, "lifted", z) <= 1e-8


@pytest.mark.parametrize("case,wide", [("pde20", "141"), ("pde20", "2048"), ("netflow4000_lds64", "65")])
def test_wide_panels_match_narrow_panels(monkeypatch, case, wide):
    """FP64 levels factored with wide panels (kPanelNB-column panels whose
    updates stop at the wide panel's end, then one rank-128 MFMA update of
    the trailing matrix) give the factor of the rank-32 schedule: both meet
    the gate and their solutions agree to rounding.  pde20 with 141 puts
    every level with a front above the LDS limit on wide panels (fronts
    whose own columns end inside a wide panel, several row chunks); with
    2048 no level qualifies (the two runs must then be bitwise equal);
    netflow4000 with a 64-row LDS limit has fronts narrower than one wide
    panel."""
    if case == "pde20":
        p, opts = workloads.pde_control(20), {}
    else:
        p, opts = workloads.network_flow(4000, seed=4, sigma_range=(-2, 2)), {"lds_front_max": 64}
    print_case("wide_panels", case=case, n=p.n, wide=wide)
    out = {}
    for mode in (wide, "100000"):
        monkeypatch.setenv("CKKT_WIDE_FRONT", mode)
        s = Solver(p, "lifted", "fp64").bind(DEV)
        s.factorize(*device_values(p, DEV, "lifted"))
        assert s.factor_status() == 0
        b = torch.as_tensor(p.b, device=DEV)
        x = s.apply_inverse(b)
        z, info = s.solve(b)
        torch.cuda.synchronize()
        om = omega_of(p, "lifted", z.cpu().numpy())
        print(mode, info, "oracle omega", om)
        assert om <= 1e-10
        out[mode] = x.cpu().numpy()
    a, c = out[wide], out["100000"]
    if wide == "2048":
        assert np.array_equal(a, c)
    else:
        assert np.all(np.isfinite(a)) and np.abs(a - c).max() <= 1e-6 * np.abs(a).max()



@pytest.mark.parametrize("case,precision,tiled", [
    ("pde20", "fp64", "1024"),
    ("pde20", "fp64", "141"),
    ("netflow4000_lds64", "fp32_ir", "65"),
])
def test_tiled_level_launch_bitwise(monkeypatch, case, precision, tiled):
    """Tiled fronts swept in one launch per level (workgroups waiting on
    per-block flags) apply exactly the arithmetic of one launch per column
    block: bitwise equal results, over several applications (the flags'
    epoch advances), in a captured graph and with direct launches."""
    if case == "pde20":
        p, opts = workloads.pde_control(20), {}
    else:
        p, opts = workloads.network_flow(4000, seed=4, sigma_range=(-2, 2)), {"lds_front_max": 64}
    print_case("tiled_level", case=case, precision=precision, tiled=tiled)
    monkeypatch.setenv("CKKT_TILED_SWEEP_FRONT", tiled)
    out = {}
    for graph in ("0", "1"):
        monkeypatch.setenv("CKKT_NO_GRAPH", graph)
        for mode in ("0", "1"):
            monkeypatch.setenv("CKKT_TILED_LEVEL", mode)
            s = Solver(p, "lifted", precision, **opts).bind(DEV)
            s.factorize(*device_values(p, DEV, "lifted"))
            b = torch.as_tensor(p.b, device=DEV)
            xs = [s.apply_inverse(b).cpu().numpy() for _ in range(3)]
            _, info = s.solve(b)
            assert info["status"] == 0
            for x in xs[1:]:
                assert np.array_equal(x, xs[0])
            out[(graph, mode)] = xs[0]
    ref = out[("1", "0")]
    assert np.all(np.isfinite(ref))
    for k, v in out.items():
        assert np.array_equal(v, ref), k


def test_hykkt_cg_graph_follows_new_value_arrays():
    """The captured CG iteration reads the G values of the current system:
    after the caller moves its value arrays (new allocations, old ones freed
    and overwritten), a solve gives the same result as before."""
    p = workloads.network_flow(2000, seed=12)
    print_case("cg_graph_new_arrays", n=p.n)
    s = Solver(p, "hykkt").bind(DEV)
    rhs = torch.as_tensor(rhs_of(p, "hykkt"), device=DEV)
    vals = device_values(p, DEV, "hykkt")
    s.factorize(*vals, gamma=1e7)
    z1, _ = s.solve(rhs)
    z1 = z1.cpu().numpy()
    del vals
    torch.cuda.synchronize()
    junk = [torch.full((p.g_val.size,), float("nan"), dtype=torch.float64, device=DEV) for _ in range(4)]
    vals2 = device_values(p, DEV, "hykkt")
    s.factorize(*vals2, gamma=1e7)
    z2, info = s.solve(rhs)
    torch.cuda.synchronize()
    del junk
    assert info["cg_iters"] > 0
    assert np.array_equal(z1, z2.cpu().numpy())
