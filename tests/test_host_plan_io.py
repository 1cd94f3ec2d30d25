"""Checkpoint and resume of the symbolic phase (ckkt_plan_save / load): a
handle built from a saved plan has the same analysis (sizes, levels) and
gives bitwise the same host factor-solve as the handle that was analysed;
batch plans and split dense rows round-trip too; truncated, corrupted or
foreign buffers are refused.  CPU only."""
import ctypes

import numpy as np
import pytest

from paper_2405_14236_amd import _lib, workloads
from paper_2405_14236_amd.solver import Solver

KEYS = ("n", "m_eq", "m_ineq", "nnz_k", "nnz_l", "nnz_l_stored", "factor_flops", "n_supernodes", "n_levels",
        "max_front", "n_big_fronts", "workspace_bytes", "n_dense_rows")


def _host(s, p, form):
    ss = p.sigma_s if form == "lifted" else p.sigma_s_ineq
    return s.host_factor_solve(p.w_val, p.g_val, p.h_val, p.sigma_x, ss, 1e7, p.b)


@pytest.mark.parametrize("form,opts", [("lifted", {}), ("hykkt", {}), ("lifted", {"lds_front_max": 64}),
                                       ("lifted", {"ordering": "natural"})])
def test_plan_round_trip(form, opts):
    p = workloads.network_flow(400, seed=5)
    s = Solver(p, form, **opts)
    blob = s.save_plan()
    t = Solver.from_plan(blob)
    a, b = s.info(), t.info()
    assert {k: a[k] for k in KEYS} == {k: b[k] for k in KEYS}
    assert t.formulation == s.formulation
    x0, st0, _ = _host(s, p, form)
    x1, st1, _ = _host(t, p, form)
    assert st0 == st1 == 0 and np.array_equal(x0, x1)
    assert t.save_plan() == blob


def test_plan_round_trip_batch_and_dense_rows():
    probs = [workloads.network_flow(int(N), seed=20 + i) for i, N in enumerate([300, 420])]
    s = Solver(None, "lifted", batch=probs)
    t = Solver.from_plan(s.save_plan())
    assert {k: s.info()[k] for k in KEYS} == {k: t.info()[k] for k in KEYS}
    p = workloads.with_dense_rows(workloads.tiny_grid(60), count=2, frac=0.5, seed=60)
    s = Solver(p, "lifted", dense_row_min=50)
    t = Solver.from_plan(s.save_plan())
    assert t.info()["n_dense_rows"] == 2
    x0, _, _ = _host(s, p, "lifted")
    x1, _, _ = _host(t, p, "lifted")
    assert np.array_equal(x0, x1)
    with pytest.raises(_lib.CkktError):  # the plan's split rows need FP64
        Solver.from_plan(s.save_plan(), precision="fp32_ir")


def test_bad_plan_buffers_refused():
    p = workloads.tiny_grid(61)
    blob = Solver(p, "lifted").save_plan()
    lib = _lib.load()
    bad = [blob[:-1], blob[:40], b"X" + blob[1:], blob[:100] + bytes([blob[100] ^ 1]) + blob[101:], b""]
    for b in bad:
        h, ws = ctypes.c_void_p(), ctypes.c_size_t()
        buf = ctypes.create_string_buffer(b, max(len(b), 1))
        assert lib.ckkt_plan_load(buf, len(b), None, ctypes.byref(h), ctypes.byref(ws)) == -1
        assert not h.value
    size = ctypes.c_size_t()
    s = Solver(p, "lifted")
    assert lib.ckkt_plan_size(s.h, ctypes.byref(size)) == 0 and size.value == len(blob)
    small = ctypes.create_string_buffer(10)
    assert lib.ckkt_plan_save(s.h, small, 10) == -1
