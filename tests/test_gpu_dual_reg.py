"""GPU parity of HyKKT with dual regularization delta_c > 0 (Remark 1,
eqn:primal; ckkt_factorize_dual_reg): the direct solve through K_gamma with
gamma = 1/delta_c against the oracle's sparse solve of K1 with -delta_c I
(SuperLU on the saddle matrix, refined), the backward error on
K1(delta_c) computed by the oracle, no CG, and the return to the CG path
after a plain factorization."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def run(p, delta_c, s=None):
    s = s or Solver(p, "hykkt").bind(DEV)
    vals = device_values(p, DEV, "hykkt")
    s.factorize_dual_reg(*vals, delta_c)
    rhs = torch.as_tensor(np.concatenate([p.r1bar, p.r2bar]), device=DEV)
    sol, info = s.solve(rhs, raise_on_error=False)
    torch.cuda.synchronize()
    return s, vals, sol.cpu().numpy(), info


def omega(p, z, delta_c):
    P = osp.Problem(p)
    return osp.omega_k1(P.W, p.sigma_x, P.H, p.sigma_s_ineq, P.G, z[:p.n], z[p.n:], p.r1bar, p.r2bar, delta_c)


@pytest.mark.parametrize("delta_c", [1e-8, 1e-6, 1e-3, 1.0])
@pytest.mark.parametrize("size", ["n300_wellcond", "n300", "n1200"])
def test_dual_reg_matches_oracle(size, delta_c):
    p = {"n300_wellcond": lambda: workloads.tiny_grid(14, sigma_range=(-1, 1)),
         "n300": lambda: workloads.tiny_grid(15),
         "n1200": lambda: workloads.tiny_grid(16, nx=20, ny=20)}[size]()
    print_case("dual_reg", size=size, n=p.n, delta_c=delta_c)
    _, _, z, info = run(p, delta_c)
    assert info["status"] == 0 and info["cg_iters"] == 0, info
    om = omega(p, z, delta_c)
    print("omega", om, info)
    assert om <= 1e-10
    assert abs(info["omega"] - om) <= 1e-14 + 0.1 * om
    P = osp.Problem(p)
    dx, dy, hist = osp.solve_k1(P, p.sigma_x, p.sigma_s_ineq, p.r1bar, p.r2bar, delta_c=delta_c)
    fe = max(np.abs(z[:p.n] - dx).max() / np.abs(dx).max(), np.abs(z[p.n:] - dy).max() / np.abs(dy).max())
    print("forward error vs oracle", fe, hist[-1])
    if size == "n300_wellcond":
        assert fe <= 1e-8


def test_dual_reg_full_size():
    p = workloads.network_flow(10_000, seed=0)
    print_case("dual_reg_full", n=p.n, delta_c=1e-7)
    _, _, z, info = run(p, 1e-7)
    assert info["status"] == 0 and info["cg_iters"] == 0, info
    om = omega(p, z, 1e-7)
    print("omega", om, info)
    assert om <= 1e-10


def test_plain_factorize_returns_to_cg():
    p = workloads.tiny_grid(17)
    print_case("dual_reg_then_plain", n=p.n)
    s, vals, _, info = run(p, 1e-4)
    assert info["cg_iters"] == 0
    rhs = torch.as_tensor(np.concatenate([p.r1bar, p.r2bar]), device=DEV)
    s.factorize(*vals, gamma=1e7)
    z1, i1 = s.solve(rhs)
    s0 = Solver(p, "hykkt").bind(DEV)
    s0.factorize(*vals, gamma=1e7)
    z0, i0 = s0.solve(rhs)
    torch.cuda.synchronize()
    assert i1["cg_iters"] > 0 and i1 == i0
    assert torch.equal(z1, z0)
