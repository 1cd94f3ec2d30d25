"""Parity at the full sizes of the target configurations, in the launch
configuration bench.py times, certified by the oracle's componentwise
backward error (a property that holds at any size; the oracle's own solves
are too slow here):

* 512 independent network-flow instances (4.3 M variables) as one batch,
  FP64: every instance meets the gate;
* the 3-D Poisson control problem on a 48^3 grid (n = 124,416, a dense
  11,007-row root front), LiftedKKT FP64;
* HyKKT on the 80,000-node network flow (n = 528,000)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import omega_of, rhs_of

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def test_batch_512_instances_fp64():
    probs = workloads.batch_network_flow(512, seed=0)
    print_case("batch512", count=len(probs), n=sum(q.n for q in probs))
    s = Solver(None, "lifted", batch=probs).bind(DEV)
    t = lambda arrs: torch.as_tensor(np.concatenate(arrs), device=DEV)
    w = t([q.w_val for q in probs])
    g = t([q.g_val for q in probs])
    h = t([q.h_val for q in probs])
    sx = t([q.sigma_x for q in probs])
    ss = t([q.sigma_s[:q.m_eq] for q in probs] + [q.sigma_s[q.m_eq:] for q in probs])
    b = t([q.b for q in probs])
    s.factorize(w, g, h, sx, ss)
    x, info = s.solve(b)
    torch.cuda.synchronize()
    x = x.cpu().numpy()
    worst, off = 0.0, 0
    for q in probs:
        worst = max(worst, omega_of(q, "lifted", x[off:off + q.n]))
        off += q.n
    print(info, "worst instance omega", worst)
    assert info["status"] == 0 and worst <= 1e-10


def test_pde48_lifted_fp64():
    p = workloads.pde_control(48)
    print_case("pde48", n=p.n)
    s = Solver(p, "lifted").bind(DEV)
    assert s.info()["max_front"] > 10_000
    s.factorize(*device_values(p, DEV, "lifted"))
    x, info = s.solve(torch.as_tensor(p.b, device=DEV))
    torch.cuda.synchronize()
    om = omega_of(p, "lifted", x.cpu().numpy())
    print(info, "oracle omega", om)
    assert info["status"] == 0 and om <= 1e-10


def test_netflow80k_hykkt_fp64():
    p = workloads.network_flow(80_000, seed=0)
    print_case("netflow80k_hykkt", n=p.n)
    s = Solver(p, "hykkt").bind(DEV)
    s.factorize(*device_values(p, DEV, "hykkt"), gamma=1e7)
    z, info = s.solve(torch.as_tensor(rhs_of(p, "hykkt"), device=DEV))
    torch.cuda.synchronize()
    om = omega_of(p, "hykkt", z.cpu().numpy())
    print(info, "oracle omega", om)
    assert info["status"] == 0 and om <= 1e-10
