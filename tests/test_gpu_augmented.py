"""GPU parity of the Newton step on the augmented system K2
(ckkt_solve_augmented) and of the bound-multiplier step of K3
(ckkt_recover_bound_dual) against the oracle (oracle/newton.py):

* small and mid-size inputs, both formulations: the four blocks against the
  oracle's dense condensed route (itself pinned to dense K2 and K3 solves),
  K2's backward error <= 1e-10 by the oracle, the library's own omega equal
  to it to rounding;
* the 66,000-variable workload: K2's backward error by the oracle (sparse);
* d_v elementwise against the oracle;
* HyKKT solves of K1 and of K2 interleaved on one handle give the results
  of fresh handles bitwise (the CG iteration graph is shared);
* a handle factorized with dual regularization is refused.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dense as od
from oracle import newton as on
from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values, recover_bound_dual

pytestmark = pytest.mark.gpu
DEV = "cuda"
GAMMA = 1e7


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def t(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def k2_blocks(p, form, dense=True):
    if dense:
        W, G, H = od.problem_dense(p)
    else:
        P = osp.Problem(p)
        W, G, H = P.W, P.G, P.H
    if form == "lifted":
        if dense:
            return W, np.zeros((0, p.n)), np.vstack([G, H]), p.sigma_s
        import scipy.sparse as sp
        return W, sp.csr_matrix((0, p.n)), sp.vstack([G, H]).tocsr(), p.sigma_s
    return W, G, H, p.sigma_s_ineq


def rhs(p, form, seed):
    rng = np.random.default_rng(seed)
    ms = p.m if form == "lifted" else p.m_ineq
    me = 0 if form == "lifted" else p.m_eq
    return [rng.standard_normal(k) for k in (p.n, ms, me, ms)]


def gpu_step(p, form, r, s=None):
    if s is None:
        s = Solver(p, form).bind(DEV)
        s.factorize(*device_values(p, DEV, form), gamma=GAMMA)
    r1, r2, r3, r4 = (t(a) for a in r)
    dx, ds, dy, dz, info = s.solve_augmented(r1, r2, r3 if form == "hykkt" else None, r4)
    torch.cuda.synchronize()
    out = [dx.cpu().numpy(), ds.cpu().numpy(), dy.cpu().numpy() if dy is not None else np.zeros(0),
           dz.cpu().numpy()]
    return s, out, info


CASES = [(lambda: workloads.tiny_grid(31, nx=4, ny=3, sigma_range=(-1, 1)), True),
         (lambda: workloads.tiny_grid(32, sigma_range=(-1, 1)), True),
         (lambda: workloads.tiny_grid(33), False),
         (lambda: workloads.tiny_grid(34, nx=20, ny=20), False)]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_augmented_step_matches_oracle(form, case):
    make, wellcond = CASES[case]
    p = make()
    print_case("augmented", form=form, case=case, n=p.n)
    r = rhs(p, form, 100 + case)
    _, d, info = gpu_step(p, form, r)
    assert info["status"] == 0, info
    W, G, H, E = k2_blocks(p, form)
    om = on.omega_k2(W, p.sigma_x, G, H, E, *r, *d)
    print("omega", om, info)
    assert om <= 1e-10
    assert abs(info["omega"] - om) <= 1e-14 + 0.1 * om
    ref = on.solve_augmented(W, p.sigma_x, G, H, E, *r)
    fe = max(np.abs(a - b).max() / np.abs(b).max() for a, b in zip(d, ref) if b.size)
    print("forward error vs oracle", fe)
    if wellcond:
        assert fe <= 1e-8


@pytest.mark.parametrize("form", ["lifted", "hykkt"])
def test_augmented_step_full_size(form):
    p = workloads.network_flow(10_000, seed=0)
    print_case("augmented_full", form=form, n=p.n)
    r = rhs(p, form, 7)
    _, d, info = gpu_step(p, form, r)
    assert info["status"] == 0, info
    W, G, H, E = k2_blocks(p, form, dense=False)
    om = on.omega_k2(W, p.sigma_x, G, H, E, *r, *d)
    print("omega", om, info)
    assert om <= 1e-10


def test_bound_dual_step_matches_oracle():
    rng = np.random.default_rng(8)
    k = 100_003
    s, v = 10.0 ** rng.uniform(-6, 2, k), 10.0 ** rng.uniform(-6, 2, k)
    ds = rng.standard_normal(k)
    mu = 1e-3
    print_case("bound_dual", count=k)
    dv = recover_bound_dual(t(s), t(v), mu, t(ds)).cpu().numpy()
    ref = on.bound_dual_step(s, v, mu, ds)
    assert np.all(np.abs(dv - ref) <= 8e-16 * (np.abs(v * ds / s) + mu / s + np.abs(v)))


def test_hykkt_k1_and_k2_interleaved_bitwise():
    p = workloads.tiny_grid(35)
    print_case("interleaved", n=p.n)
    vals = device_values(p, DEV, "hykkt")
    rk1 = t(np.concatenate([p.r1bar, p.r2bar]))
    r = rhs(p, "hykkt", 9)
    s = Solver(p, "hykkt").bind(DEV)
    s.factorize(*vals, gamma=GAMMA)
    z_a, i_a = s.solve(rk1)
    _, d_a, j_a = gpu_step(p, "hykkt", r, s)
    z_b, i_b = s.solve(rk1)
    _, d_b, j_b = gpu_step(p, "hykkt", r, s)
    torch.cuda.synchronize()
    f1 = Solver(p, "hykkt").bind(DEV)
    f1.factorize(*vals, gamma=GAMMA)
    z_f, i_f = f1.solve(rk1)
    f2 = Solver(p, "hykkt").bind(DEV)
    f2.factorize(*vals, gamma=GAMMA)
    _, d_f, j_f = gpu_step(p, "hykkt", r, f2)
    torch.cuda.synchronize()
    assert torch.equal(z_a, z_f) and torch.equal(z_b, z_f) and i_a == i_f == i_b
    for a, b, c in zip(d_a, d_b, d_f):
        assert np.array_equal(a, c) and np.array_equal(b, c)
    assert j_a == j_f == j_b


def test_dual_reg_handle_refused():
    p = workloads.tiny_grid(36)
    print_case("dual_reg_refused", n=p.n)
    s = Solver(p, "hykkt").bind(DEV)
    s.factorize_dual_reg(*device_values(p, DEV, "hykkt"), 1e-6)
    r = [t(a) for a in rhs(p, "hykkt", 10)]
    *_, info = s.solve_augmented(*r, raise_on_error=False)
    assert info["status"] == -6
