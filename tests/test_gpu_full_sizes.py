"""Parity at the full sizes of the target configurations, in the launch
configuration bench.py times, certified by the oracle's componentwise
backward error (a property that holds at any size; the oracle's own solves
are too slow here):

* 512 independent network-flow instances (4.3 M variables) as one batch,
  FP64: every instance meets the gate;
* the 3-D Poisson control problem on a 48^3 grid (n = 124,416, a dense
  11,007-row root front), LiftedKKT FP64;
* HyKKT on the 80,000-node network flow (n = 528,000);
* the FP32 factor with FP64 refinement on systems 0, 30 and 59 of the
  60-system IPM-like sequence of that network flow, and on all 512 batch
  instances;
* PCG around a stale factor (D = I and the trained learned diagonal) on
  held-out systems of the 48^3 PDE-control sequence.
Gate of the FP32 + refinement and PCG forms: oracle omega <= 1e-8."""
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


def test_seq80k_fp32_ir_spot_systems():
    from oracle import sparse as osp
    p = workloads.network_flow(80_000, seed=0)
    seq = workloads.ipm_sigma_sequence(p, 60, seed=0)
    print_case("seq80k_fp32_ir", n=p.n, systems=(0, 30, 59))
    s = Solver(p, "lifted", "fp32_ir", tol=1e-8).bind(DEV)
    w, g, h, _, _ = device_values(p, DEV, "lifted")
    b = torch.as_tensor(p.b, device=DEV)
    P = osp.Problem(p)
    for k in (0, 30, 59):
        sx, ss = seq[k]
        s.factorize(w, g, h, torch.as_tensor(sx, device=DEV), torch.as_tensor(ss, device=DEV))
        x, info = s.solve(b, raise_on_error=False)
        torch.cuda.synchronize()
        om = osp.omega_condensed(P.W, sx, P.J, ss, x.cpu().numpy(), p.b)
        print(k, info, "oracle omega", om, flush=True)
        assert info["status"] == 0 and om <= 1e-8


def test_batch_512_instances_fp32_ir():
    probs = workloads.batch_network_flow(512, seed=0)
    print_case("batch512_fp32_ir", count=len(probs), n=sum(q.n for q in probs))
    s = Solver(None, "lifted", "fp32_ir", batch=probs, tol=1e-8).bind(DEV)
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
    assert info["status"] == 0 and worst <= 1e-8


def test_pde48_stale_pcg_identity_and_learned():
    from oracle import sparse as osp
    from paper_2405_14236_amd.solver import init_mlp_params
    p = workloads.pde_control(48)
    num = 80
    seq = workloads.ipm_sigma_sequence(p, num, seed=0)
    print_case("pde48_pcg", n=p.n)
    w, g, h, _, _ = device_values(p, DEV, "lifted")
    T = lambda a: torch.as_tensor(a, device=DEV)
    rng = np.random.default_rng(11)
    rhs = [rng.standard_normal(p.n) for _ in range(num)]
    # training pairs from the FP64 path (systems 0..19)
    s64 = Solver(p, "lifted", "fp64").bind(DEV)
    targets = []
    for k in range(20):
        s64.factorize(w, g, h, T(seq[k][0]), T(seq[k][1]))
        x, _ = s64.solve(T(rhs[k]))
        targets.append(x)
    torch.cuda.synchronize()
    del s64
    s = Solver(p, "lifted", "fp32_ir", learned=1).bind(DEV)
    s.factorize(w, g, h, T(seq[10][0]), T(seq[10][1]))
    prm = init_mlp_params(0, device=DEV)
    m, v = torch.zeros_like(prm), torch.zeros_like(prm)
    step = 0
    for _ in range(3):
        for k in range(20):
            if k != 10:
                step += 1
                s.mlp_train_step((w, g, h, T(seq[k][0]), T(seq[k][1])), 0.0, T(rhs[k]), targets[k], prm, m, v,
                                 step, 3e-3)
    P = osp.Problem(p)
    for params in (None, prm):
        s.factorize(w, g, h, T(seq[19][0]), T(seq[19][1]))
        for k in (20, 50, 79):
            x, si = s.pcg_solve((w, g, h, T(seq[k][0]), T(seq[k][1])), 0.0, params, T(rhs[k]), maxit=50,
                                tol=1e-8, allow_refactor=True, raise_on_error=False)
            torch.cuda.synchronize()
            om = osp.omega_condensed(P.W, seq[k][0], P.J, seq[k][1], x.cpu().numpy(), rhs[k])
            print("learned" if params is not None else "identity", k, si, "oracle omega", om, flush=True)
            assert si["status"] == 0 and om <= 1e-8
