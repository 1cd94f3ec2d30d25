"""CPU tests of the library boundary and of its host symbolic analysis.

* the shared library loads and exports every entry point of include/ckkt.h;
* malformed patterns are rejected with CKKT_ERR_PATTERN / CKKT_ERR_ARG;
* the analysis (ordering, etree, supernodes, multifrontal maps, level
  schedule) is checked by running the numeric phase on the host over the
  same plan and certifying the result with the oracle;
* analysis invariants: nnz(L) against a naive symbolic elimination, and
  the factor flop count.
No GPU is needed.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2405_14236_amd import _lib, workloads
from paper_2405_14236_amd.solver import Solver
from tests._common import omega_kgamma, sigma_rows

from oracle import sparse as osp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ckkt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ckkt_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert {n for n, _, _ in _lib.SIGNATURES} == set(names)


def test_status_strings():
    lib = _lib.load()
    for s in range(0, -10, -1):
        assert lib.ckkt_status_string(s)


def _bad(p, **changes):
    q = workloads.KKTProblem(**{**p.__dict__, **changes})
    with pytest.raises(_lib.CkktError) as e:
        Solver(q)
    return e.value.status


def test_pattern_errors():
    p = workloads.tiny_grid(0, nx=3, ny=3)
    w_idx = p.w_idx.copy()
    # upper-triangle entry in W
    i = 5
    a = p.w_ptr[i]
    w_up = w_idx.copy(); w_up[a] = p.n - 1
    assert _bad(p, w_idx=w_up) == -2
    # unsorted / duplicate columns in H
    h = p.h_idx.copy()
    r = int(np.argmax(np.diff(p.h_ptr) >= 2))
    h[p.h_ptr[r] + 1] = h[p.h_ptr[r]]
    assert _bad(p, h_idx=h) == -2
    # out of range column in G
    g = p.g_idx.copy(); g[0] = p.n + 3
    assert _bad(p, g_idx=g) == -2
    # inconsistent row pointer
    gp = p.g_ptr.copy(); gp[1] = gp[2] + 1
    assert _bad(p, g_ptr=gp) == -2


def test_bad_enum_is_arg_error():
    lib = _lib.load()
    p = workloads.tiny_grid(0, nx=2, ny=2)
    from paper_2405_14236_amd.solver import _pattern, options
    pat, keep = _pattern(p, 7)
    h = ctypes.c_void_p()
    ws = ctypes.c_size_t()
    assert lib.ckkt_analyze(ctypes.byref(pat), ctypes.byref(options()), ctypes.byref(h), ctypes.byref(ws)) == -1


def test_solve_before_bind_is_state_error():
    lib = _lib.load()
    s = Solver(workloads.tiny_grid(0, nx=2, ny=2))
    si = _lib.SolveInfo()
    assert lib.ckkt_solve(s.h, None, None, ctypes.byref(si), None) == -6
    assert lib.ckkt_factorize(s.h, None, None, None, None, None, 0.0, None) == -6


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("formulation", ["lifted", "hykkt"])
def test_host_run_of_plan_matches_oracle_tiny(seed, formulation):
    p = workloads.tiny_grid(seed)
    s = Solver(p, formulation)
    gamma = 1e7
    ss = p.sigma_s if formulation == "lifted" else p.sigma_s_ineq
    x, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, gamma, p.b)
    assert st == 0 and fc == -1
    assert omega_kgamma(p, x, p.b, gamma) < 1e-12 if formulation == "hykkt" else True
    if formulation == "lifted":
        P = osp.Problem(p)
        assert osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, x, p.b) < 1e-12


@pytest.mark.parametrize("ordering", ["amd", "natural"])
@pytest.mark.parametrize("relax", [0, 1])
def test_host_run_orderings_and_relaxation(ordering, relax):
    p = workloads.tiny_grid(3, nx=6, ny=5, sigma_range=(-3, 3))
    s = Solver(p, "lifted", ordering=ordering, relax=relax)
    x, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s, 0.0, p.b)
    P = osp.Problem(p)
    assert st == 0
    assert osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, x, p.b) < 1e-13


def test_host_run_network_flow_with_big_fronts():
    """A network-flow problem large enough to use the tiled front layout."""
    p = workloads.network_flow(4000, seed=4)
    s = Solver(p, "lifted", lds_front_max=64)
    inf = s.info()
    assert inf["n_big_fronts"] > 0 and inf["n_levels"] > 3
    x, st, fc = s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, p.sigma_s, 0.0, p.b)
    P = osp.Problem(p)
    assert st == 0
    assert osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, x, p.b) < 1e-10


def test_not_spd_reported_with_column():
    p = workloads.tiny_grid(0, nx=3, ny=3, sigma_range=(-1, 1))
    w = p.w_val.copy()
    # make one diagonal entry of W hugely negative
    i = 7
    diag_pos = p.w_ptr[i + 1] - 1
    assert p.w_idx[diag_pos] == i
    w[diag_pos] = -1e6
    s = Solver(p, "lifted")
    x, st, fc = s.host_factor_solve(w, p.g_val, p.h_val, p.sigma_x, p.sigma_s, 0.0, p.b)
    assert st == -3 and fc >= 0


def naive_symbolic_nnz(n, rows_cols, perm):
    """nnz(L) by explicit symbolic elimination on the permuted graph (tiny n)."""
    ip = np.empty(n, int); ip[perm] = np.arange(n)
    adj = [set() for _ in range(n)]
    for i, j in rows_cols:
        a, b = ip[i], ip[j]
        if a != b:
            adj[a].add(b); adj[b].add(a)
    nnz = 0
    for k in range(n):
        higher = {v for v in adj[k] if v > k}
        nnz += 1 + len(higher)
        for u in higher:
            adj[u] |= higher - {u}
    return nnz


def test_nnz_l_matches_naive_elimination():
    p = workloads.tiny_grid(5, nx=5, ny=4)
    s = Solver(p, "lifted", ordering="natural", relax=0)
    inf = s.info()
    pairs = []
    for i in range(p.n):
        for k in range(p.w_ptr[i], p.w_ptr[i + 1]):
            pairs.append((i, p.w_idx[k]))
    for ptr, idx in ((p.g_ptr, p.g_idx), (p.h_ptr, p.h_idx)):
        for r in range(len(ptr) - 1):
            cols = idx[ptr[r]:ptr[r + 1]]
            pairs += [(a, b) for a in cols for b in cols]
    # natural ordering + postorder relabelling keeps fill; compare with natural
    assert inf["nnz_l"] == naive_symbolic_nnz(p.n, pairs, np.arange(p.n))
    # flop formula: sum_j (eta_j^2 + 2 eta_j + 1) >= nnz_l
    assert inf["factor_flops"] >= inf["nnz_l"]


def test_amd_reduces_fill():
    p = workloads.network_flow(800, seed=2)
    nat = Solver(p, "lifted", ordering="natural").info()["nnz_l"]
    amd = Solver(p, "lifted", ordering="amd").info()["nnz_l"]
    assert amd < 0.5 * nat


def test_batch_analysis_is_block_diagonal():
    probs = [workloads.network_flow(int(N), seed=10 + i) for i, N in enumerate([300, 450, 380])]
    s = Solver(None, "lifted", batch=probs)
    inf = s.info()
    singles = [Solver(q, "lifted").info() for q in probs]
    assert inf["n"] == sum(q.n for q in probs)
    assert inf["nnz_k"] == sum(x["nnz_k"] for x in singles)
    # every block is ordered on its own (the same AMD ordering as the single analysis)
    assert inf["nnz_l"] == sum(x["nnz_l"] for x in singles)
    # host run of the union equals the union of host runs (certificate per block)
    w = np.concatenate([q.w_val for q in probs])
    g = np.concatenate([q.g_val for q in probs])
    h = np.concatenate([q.h_val for q in probs])
    sx = np.concatenate([q.sigma_x for q in probs])
    ss = np.concatenate([q.sigma_s[:q.m_eq] for q in probs] + [q.sigma_s[q.m_eq:] for q in probs])
    b = np.concatenate([q.b for q in probs])
    x, st, fc = s.host_factor_solve(w, g, h, sx, ss, 0.0, b)
    assert st == 0
    off = 0
    for q in probs:
        P = osp.Problem(q)
        xi = x[off:off + q.n]
        assert osp.omega_condensed(P.W, q.sigma_x, P.J, q.sigma_s, xi, q.b) < 1e-10
        off += q.n


def _bad_batch(probs):
    with pytest.raises(_lib.CkktError) as e:
        Solver(None, "lifted", batch=probs)
    return e.value.status


def test_batch_instance_pattern_errors():
    """Every instance of a batch is validated on its own before it is
    ordered: an index at or beyond the instance's own n is a pattern error
    even when it lies inside the union (it would name another instance's
    variable), and so are a bad row pointer and an unsorted row."""
    import dataclasses
    a, b = workloads.tiny_grid(0, nx=3, ny=3), workloads.tiny_grid(1, nx=4, ny=3)
    assert b.n > a.n
    g = a.g_idx.copy(); g[0] = a.n          # in range of the union, not of instance 0
    assert _bad_batch([dataclasses.replace(a, g_idx=g), b]) == -2
    h = b.h_idx.copy(); h[-1] = b.n + 7      # beyond the last instance
    assert _bad_batch([a, dataclasses.replace(b, h_idx=h)]) == -2
    w = a.w_idx.copy(); w[a.w_ptr[4]] = 6    # above the diagonal of row 4
    assert _bad_batch([dataclasses.replace(a, w_idx=w), b]) == -2
    gp = b.g_ptr.copy(); gp[1] = -5          # pointer decreases (and is negative)
    assert _bad_batch([a, dataclasses.replace(b, g_ptr=gp)]) == -2
    # the valid batch still analyses
    assert Solver(None, "lifted", batch=[a, b]).info()["n"] == a.n + b.n


def test_dual_reg_arguments_rejected_without_gpu():
    """ckkt_factorize_dual_reg: HyKKT handles and 0 < delta_c with finite 1/delta_c only."""
    p = workloads.tiny_grid(0, nx=3, ny=3)
    lib = _lib.load()
    lifted = Solver(p, "lifted")
    assert lib.ckkt_factorize_dual_reg(lifted.h, None, None, None, None, None, 1e-4, None) == -1
    hy = Solver(p, "hykkt")
    for dc in (0.0, -1.0, float("nan"), float("inf"), 1e-320):
        assert lib.ckkt_factorize_dual_reg(hy.h, None, None, None, None, None, dc, None) == -1, dc
    assert lib.ckkt_factorize_dual_reg(hy.h, None, None, None, None, None, 1e-4, None) == -6  # no workspace
    assert lib.ckkt_factorize_dual_reg(None, None, None, None, None, None, 1e-4, None) == -1


def test_augmented_step_arguments_rejected_without_gpu():
    p = workloads.tiny_grid(0, nx=3, ny=3)
    lib = _lib.load()
    si = _lib.SolveInfo()
    s = Solver(p, "hykkt")  # no workspace bound
    args = [None] * 8
    assert lib.ckkt_solve_augmented(s.h, *args, ctypes.byref(si), None) == -6
    sb = Solver(None, "lifted", batch=[p, workloads.tiny_grid(1, nx=3, ny=3)])
    assert lib.ckkt_solve_augmented(sb.h, *args, ctypes.byref(si), None) == -1
    assert lib.ckkt_solve_augmented(None, *args, None, None) == -1
    assert lib.ckkt_recover_bound_dual(-1, None, None, 0.0, None, None, None) == -1
    assert lib.ckkt_recover_bound_dual(4, None, None, 0.0, None, None, None) == -1
    assert lib.ckkt_recover_bound_dual(0, None, None, float("nan"), None, None, None) == -1
    assert lib.ckkt_recover_bound_dual(0, None, None, 0.1, None, None, None) == 0
