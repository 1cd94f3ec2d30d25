"""GPU parity with dense Jacobian rows split off the condensed matrix
(opt.dense_row_min): the device factor of K_s plus the Woodbury step inside
every factor application (refinement, HyKKT's CG, the K2 Newton step) solves
the FULL system to the gates, certified by the oracle on the full data;
the split and unsplit handles agree on well-conditioned inputs; at the
66,000-variable size, four rows over half of the variables (whose J^T J
block alone would hold ~5e8 entries) are solved through the split."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import newton as on
from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import omega_of, rhs_of

pytestmark = pytest.mark.gpu
DEV = "cuda"
GAMMA = 1e7


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def solve(p, form, **opts):
    s = Solver(p, form, **opts).bind(DEV)
    s.factorize(*device_values(p, DEV, form), gamma=GAMMA)
    rhs = torch.as_tensor(rhs_of(p, form), device=DEV)
    sol, info = s.solve(rhs, raise_on_error=False)
    torch.cuda.synchronize()
    return s, sol.cpu().numpy(), info


@pytest.mark.parametrize("case", [(45, (-1, 1), 2, 0.8), (46, (-8, 8), 3, 0.6), (47, (-8, 8), 8, 0.3)])
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_split_dense_rows_match_oracle(form, case):
    seed, sig, count, frac = case
    p = workloads.with_dense_rows(workloads.tiny_grid(seed, sigma_range=sig), count=count, frac=frac, seed=seed)
    print_case("dense_rows", form=form, seed=seed, n=p.n, count=count, frac=frac)
    s, x, info = solve(p, form, dense_row_min=60)
    assert s.info()["n_dense_rows"] == count
    assert info["status"] == 0, info
    om = omega_of(p, form, x, GAMMA)
    print("omega", om, info)
    assert om <= 1e-10
    _, x0, info0 = solve(p, form)
    assert info0["status"] == 0
    fe = np.abs(x - x0).max() / np.abs(x0).max()
    print("split vs unsplit", fe)
    if sig == (-1, 1):
        assert fe <= 1e-8


def test_split_dense_rows_k2_step():
    p = workloads.with_dense_rows(workloads.tiny_grid(48, sigma_range=(-1, 1)), count=3, frac=0.7, seed=48)
    print_case("dense_rows_k2", n=p.n)
    s = Solver(p, "lifted", dense_row_min=60).bind(DEV)
    s.factorize(*device_values(p, DEV, "lifted"), gamma=GAMMA)
    rng = np.random.default_rng(48)
    r = [rng.standard_normal(k) for k in (p.n, p.m, 0, p.m)]
    t = [torch.as_tensor(a, device=DEV) for a in r]
    dx, ds, _, dz, info = s.solve_augmented(t[0], t[1], None, t[3])
    torch.cuda.synchronize()
    assert info["status"] == 0, info
    P = osp.Problem(p)
    import scipy.sparse as sp
    om = on.omega_k2(P.W, p.sigma_x, sp.csr_matrix((0, p.n)), P.J, p.sigma_s, r[0], r[1], r[2], r[3],
                     dx.cpu().numpy(), ds.cpu().numpy(), np.zeros(0), dz.cpu().numpy())
    print("omega", om, info)
    assert om <= 1e-10


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_split_dense_rows_full_size(form):
    p = workloads.with_dense_rows(workloads.network_flow(10_000, seed=0), count=4, frac=0.5, seed=1)
    print_case("dense_rows_full", form=form, n=p.n, m_ineq=p.m_ineq)
    s, x, info = solve(p, form, dense_row_min=1000)
    assert s.info()["n_dense_rows"] == 4
    assert info["status"] == 0, info
    om = omega_of(p, form, x, GAMMA)
    print("omega", om, info)
    assert om <= 1e-10
