"""The symbolic factorization on the GPU (ckkt_analyze_device,
ckkt_batch_analyze_device) against the host analysis.

Both take the same host ordering; the device computes the elimination tree,
postorder, K lower CSC, column counts, front row lists, relative positions
and the assembly's product slots.  Every array of the plan is integer work,
so the bar is bitwise: the serialized plans are equal except for the
analysis time (the payload's last field) and the checksum over it.  Cases:
the small grid, both network flows (66,000 and 528,000 variables), the
3-D PDE-control pattern (10^3 and 48^3 grids), HyKKT, split dense rows,
natural ordering, no amalgamation, a diagonal-only pattern, a single
variable, and batches of 12 and 512 instances.  One device-analysed handle
is also factorized and solved, bitwise like the host-analysed one.
"""
import types

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import rhs_of

pytestmark = pytest.mark.gpu
DEV = "cuda"

# payload's last field (analysis seconds, float64) + FNV-1a checksum (uint64)
TAIL = 16


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def assert_same_plan(host, dev):
    a, b = host.save_plan(), dev.save_plan()
    assert len(a) == len(b)
    if a[:-TAIL] != b[:-TAIL]:
        raw_a = np.frombuffer(a[:len(a) - TAIL], dtype=np.uint8)
        raw_b = np.frombuffer(b[:len(b) - TAIL], dtype=np.uint8)
        first = int(np.argmax(raw_a != raw_b))
        raise AssertionError(f"plans differ from byte {first} of {len(a)}")
    hi, di = host.info(), dev.info()
    for key in ("nnz_k", "nnz_l", "n_supernodes", "n_levels", "max_front", "workspace_bytes"):
        assert hi[key] == di[key], key


def both(prob, form="lifted", **opts):
    torch.cuda.synchronize()
    host = Solver(prob, form, **opts)
    dev = Solver(prob, form, analysis="device", **opts)
    return host, dev


@pytest.mark.parametrize("name,form,opts", [
    ("tiny", "lifted", {}),
    ("tiny", "hykkt", {}),
    ("tiny", "lifted", {"ordering": "natural"}),
    ("tiny", "lifted", {"relax": 0}),
    ("netflow10k", "lifted", {}),
    ("netflow10k", "hykkt", {}),
    ("pde10", "lifted", {}),
])
def test_device_plan_equals_host_plan(name, form, opts):
    prob = {"tiny": lambda: workloads.tiny_grid(0),
            "netflow10k": lambda: workloads.network_flow(10_000, seed=0),
            "pde10": lambda: workloads.pde_control(10)}[name]()
    print_case("plan", workload=name, form=form, n=prob.n, **opts)
    host, dev = both(prob, form, **opts)
    assert_same_plan(host, dev)


def test_device_plan_split_dense_rows():
    p = workloads.with_dense_rows(workloads.tiny_grid(46, sigma_range=(-8, 8)), count=3, frac=0.6, seed=46)
    print_case("plan_dense_rows", n=p.n)
    host, dev = both(p, "lifted", dense_row_min=60)
    assert dev.info()["n_dense_rows"] == 3
    assert_same_plan(host, dev)


def _diagonal_problem(n, m_eq=0):
    """W diagonal, optional equality rows with one entry each: K is diagonal."""
    ar = np.arange(n, dtype=np.int32)
    g_idx = np.arange(m_eq, dtype=np.int32) % max(n, 1)
    return types.SimpleNamespace(
        n=n, m_eq=m_eq, m_ineq=0,
        w_ptr=np.arange(n + 1, dtype=np.int32), w_idx=ar, w_val=np.ones(n),
        g_ptr=np.arange(m_eq + 1, dtype=np.int32), g_idx=g_idx, g_val=np.ones(m_eq),
        h_ptr=np.zeros(1, dtype=np.int32), h_idx=np.zeros(0, dtype=np.int32), h_val=np.zeros(0))


@pytest.mark.parametrize("n,m_eq", [(1, 0), (7, 0), (7, 3)])
def test_device_plan_degenerate_patterns(n, m_eq):
    p = _diagonal_problem(n, m_eq)
    print_case("plan_degenerate", n=n, m_eq=m_eq)
    host, dev = both(p, "lifted")
    assert_same_plan(host, dev)


def test_device_plan_network_flow_528k():
    p = workloads.network_flow(80_000, seed=0)
    print_case("plan_netflow80k", n=p.n)
    host, dev = both(p, "lifted")
    assert_same_plan(host, dev)
    print("host analysis s", host.info()["analyze_seconds"], "device", dev.info()["analyze_seconds"])


def test_device_plan_pde48():
    p = workloads.pde_control(48)
    print_case("plan_pde48", n=p.n)
    host, dev = both(p, "lifted")
    assert_same_plan(host, dev)
    print("host analysis s", host.info()["analyze_seconds"], "device", dev.info()["analyze_seconds"])


@pytest.mark.parametrize("count", [12, 512])
def test_device_plan_batch(count):
    probs = workloads.batch_network_flow(count, seed=0)
    print_case("plan_batch", count=count, n=sum(q.n for q in probs))
    torch.cuda.synchronize()
    host = Solver(None, "lifted", batch=probs)
    dev = Solver(None, "lifted", batch=probs, analysis="device")
    assert_same_plan(host, dev)
    print("host analysis s", host.info()["analyze_seconds"], "device", dev.info()["analyze_seconds"])


def test_device_analysed_handle_solves_like_host():
    p = workloads.network_flow(10_000, seed=0)
    print_case("solve_after_device_analysis", n=p.n)
    host, dev = both(p, "lifted")
    xs = []
    for s in (host, dev):
        s.bind(DEV)
        s.factorize(*device_values(p, DEV, "lifted"))
        x, info = s.solve(torch.as_tensor(rhs_of(p, "lifted"), device=DEV))
        torch.cuda.synchronize()
        assert info["status"] == 0
        xs.append(x.cpu().numpy())
    assert np.array_equal(xs[0], xs[1])
