"""GPU tests of the FP32 + FP64-refinement form and of the batched form.

Gate for both: componentwise relative backward error omega <= 1e-8 on every
system (every instance of a batch), certified by the CPU oracle on the
returned solution.  The path each solve took (Richardson on the FP32
factor, FP64 PCG preconditioned by it, FP64 refactorization) is reported.
"""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import omega_of, rhs_of

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def solve_once(p, formulation, precision, tol, gamma=1e7, **opts):
    s = Solver(p, formulation, precision, tol=tol, **opts).bind(DEV)
    s.factorize(*device_values(p, DEV, formulation), gamma=gamma)
    z, info = s.solve(torch.as_tensor(rhs_of(p, formulation), device=DEV))
    torch.cuda.synchronize()
    return z.cpu().numpy(), info


@pytest.mark.parametrize("srange", [(-2, 2), (-8, 8)])
@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_fp32_ir_tiny(formulation, srange):
    p = workloads.tiny_grid(1, sigma_range=srange)
    print_case("fp32_ir_tiny", formulation=formulation, srange=srange)
    z, info = solve_once(p, formulation, "fp32_ir", 1e-8)
    om = omega_of(p, formulation, z)
    print(info, "oracle omega", om)
    assert om <= 1e-8


def test_fp32_ir_moderate_needs_no_fallback():
    """Diagonals in [1e-2, 1e2]: the FP32 factor is a good enough
    preconditioner for plain Richardson (no fallback)."""
    p = workloads.network_flow(3000, seed=2, sigma_range=(-2, 2))
    print_case("fp32_ir_moderate", n=p.n)
    z, info = solve_once(p, "lifted", "fp32_ir", 1e-10)
    assert info["fallback"] == 0 and info["refine_steps"] >= 1
    assert omega_of(p, "lifted", z) <= 1e-10


@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_fp32_ir_network_flow_10k(formulation):
    p = workloads.network_flow(10_000, seed=0)
    print_case("fp32_ir_nf10k", formulation=formulation, n=p.n)
    z, info = solve_once(p, formulation, "fp32_ir", 1e-8)
    om = omega_of(p, formulation, z)
    print(info, "oracle omega", om)
    assert om <= 1e-8


def test_fp32_factor_tiled_path():
    p = workloads.network_flow(4000, seed=5)
    print_case("fp32_tiled", n=p.n)
    z, info = solve_once(p, "lifted", "fp32_ir", 1e-10, lds_front_max=64)
    assert omega_of(p, "lifted", z) <= 1e-10


def _batch_values(probs, formulation):
    cat = lambda xs: torch.as_tensor(np.concatenate(xs), device=DEV)
    w = cat([q.w_val for q in probs])
    g = cat([q.g_val for q in probs])
    h = cat([q.h_val for q in probs])
    sx = cat([q.sigma_x for q in probs])
    if formulation == "lifted":
        ss = cat([q.sigma_s[:q.m_eq] for q in probs] + [q.sigma_s[q.m_eq:] for q in probs])
        rhs = cat([q.b for q in probs])
    else:
        ss = cat([q.sigma_s[q.m_eq:] for q in probs])
        rhs = cat([q.r1bar for q in probs] + [q.r2bar for q in probs])
    return (w, g, h, sx, ss), rhs


def _split(probs, z, formulation):
    out, off = [], 0
    if formulation == "lifted":
        for q in probs:
            out.append(z[off:off + q.n]); off += q.n
        return out
    n_tot = sum(q.n for q in probs)
    offy = n_tot
    for q in probs:
        out.append(np.concatenate([z[off:off + q.n], z[offy:offy + q.m_eq]]))
        off += q.n; offy += q.m_eq
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_batched_every_instance_meets_gate(formulation, precision):
    rng = np.random.default_rng(3)
    probs = [workloads.network_flow(int(N), seed=50 + i) for i, N in enumerate(rng.integers(500, 2001, 12))]
    print_case("batched", formulation=formulation, precision=precision, count=len(probs))
    tol = 1e-10 if precision == "fp64" else 1e-8
    s = Solver(None, formulation, precision, batch=probs, tol=tol).bind(DEV)
    vals, rhs = _batch_values(probs, formulation)
    s.factorize(*vals, gamma=1e7)
    z, info = s.solve(rhs)
    torch.cuda.synchronize()
    parts = _split(probs, z.cpu().numpy(), formulation)
    worst = max(omega_of(q, formulation, zi) for q, zi in zip(probs, parts))
    print(info, "worst instance omega", worst)
    assert worst <= tol


def test_batched_equals_single_solves():
    """Each instance of a batch reaches the solution of its own single solve
    (both certified).  The instance is ordered exactly as in its single
    analysis (same nnz(L), checked on the CPU), but the two runs are not
    bitwise equal, for two reasons: (1) the launch class of a front depends
    on how many fronts share its level (in a level with few compact fronts
    one launch of the large-front kernel factors all of them, in a
    512-instance level the compact kernel does; their diagonal blocks use
    different elimination orders), and the sweep schedule does too
    (dependency-driven above the single-wave levels for one instance, level
    by level for a large batch); (2) a batch refines until every instance
    meets the gate, so an instance can take more refinement steps than its
    single solve.  The results agree to the level the conditioning allows."""
    probs = [workloads.network_flow(N, seed=70 + i, sigma_range=(-2, 2)) for i, N in enumerate([600, 900, 750])]
    print_case("batched_vs_single", count=len(probs))
    s = Solver(None, "lifted", batch=probs).bind(DEV)
    vals, rhs = _batch_values(probs, "lifted")
    s.factorize(*vals)
    z, _ = s.solve(rhs)
    parts = _split(probs, z.cpu().numpy(), "lifted")
    for q, zi in zip(probs, parts):
        zs, _ = solve_once(q, "lifted", "fp64", 1e-10)
        assert np.abs(zi - zs).max() <= 1e-9 * np.abs(zs).max()


def test_autotune_keeps_gate_and_caches():
    probs = [workloads.network_flow(int(N), seed=90 + i) for i, N in enumerate([700, 1200, 900, 1500])]
    print_case("autotune", count=len(probs))
    vals, rhs = _batch_values(probs, "lifted")
    s = Solver(None, "lifted", "fp32_ir", batch=probs, tol=1e-8).bind(DEV)
    chosen, best = s.autotune(*vals, reps=1)
    assert best > 0 and chosen["compact_front"] in (32, 48, 64)
    z, info = s.solve(rhs)
    parts = _split(probs, z.cpu().numpy(), "lifted")
    assert max(omega_of(q, "lifted", zi) for q, zi in zip(probs, parts)) <= 1e-8
    s2 = Solver(None, "lifted", "fp32_ir", batch=probs, tol=1e-8).bind(DEV)
    chosen2, best2 = s2.autotune(*vals)
    assert best2 == -1.0 and chosen2 == chosen


def test_hykkt_fp32_fallback_gets_its_own_refinement_budget():
    """FP32 + refinement HyKKT with ir_maxit = 1 on diagonals spanning 1e+-8:
    the FP32 attempt exhausts its steps and falls back to the FP64
    refactorization, which then has ir_maxit steps of its own (it needs two
    outer steps here) and meets the FP64 gate."""
    p = workloads.network_flow(10_000, seed=0)
    print_case("hykkt_fp32_fallback_budget", n=p.n)
    z, info = solve_once(p, "hykkt", "fp32_ir", 1e-10, ir_maxit=1)
    om = omega_of(p, "hykkt", z)
    print(info, "oracle omega", om)
    assert info["status"] == 0 and info["fallback"] == 2 and om <= 1e-10


def test_fp32_failure_makes_next_systems_fp64_with_backoff():
    """An FP32_IR handle on diagonals spanning 1e+-8: the first system gives
    the FP32 factor up without PCG steps (floored pivots or a first backward
    error above 0.1) and refactorizes in FP64; the next four systems are
    factorized in FP64 from the start (fallback 8); the sixth tries FP32
    again, fails again, and the next eight are FP64.  Every system meets the
    gate by the oracle's certificate."""
    p = workloads.network_flow(3000, seed=4)
    print_case("fp32_history", n=p.n)
    s = Solver(p, "lifted", "fp32_ir", tol=1e-8).bind(DEV)
    w, g, h, _, _ = device_values(p, DEV, "lifted")
    rng = np.random.default_rng(12)
    b = torch.as_tensor(p.b, device=DEV)
    seen = []
    for k in range(14):
        sx, ss = workloads.log_uniform(rng, p.n), workloads.log_uniform(rng, p.m)
        s.factorize(w, g, h, torch.as_tensor(sx, device=DEV), torch.as_tensor(ss, device=DEV))
        z, info = s.solve(b)
        torch.cuda.synchronize()
        seen.append(info["fallback"])
        q = dataclasses.replace(p, sigma_x=sx, sigma_s=ss)
        assert info["status"] == 0 and omega_of(q, "lifted", z.cpu().numpy()) <= 1e-8
        if k == 0:
            assert info["pcg_iters"] == 0
    print(seen)
    assert seen == [2] + [8] * 4 + [2] + [8] * 8
