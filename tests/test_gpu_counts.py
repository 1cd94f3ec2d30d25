"""Iteration counts of the GPU path against the oracle's step-by-step
algorithms on the same right-hand sides:

* HyKKT (Sec. 3.1, eq:kkt:schurcomplhykkt): the CG iterations of the first
  outer step (whose right-hand side is rbar itself) against
  oracle.sparse.hykkt_steps (plain CG from y0 = 0, stop at
  ||r_k||_2 <= 1e-10 ||r_0||_2), within 2, on the 66,000-variable network
  flow at two values of gamma;
* PCG around a stale factor: the iterations to omega <= 1e-8 against
  oracle.mlp.pcg with M^{-1} = D K_s^{-1} D (D = I and D from the oracle's
  MLP forward on the oracle's features with the same parameters), within 2,
  on systems where that PCG converges steadily.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from oracle import mlp as om
from oracle import sparse as osp
from paper_2405_14236_amd import workloads
from paper_2405_14236_amd.solver import Solver, device_values
from tests._common import rhs_of

pytestmark = pytest.mark.gpu
DEV = "cuda"


def print_case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


@pytest.mark.parametrize("gamma", [1e5, 1e7])
def test_hykkt_first_step_cg_count_matches_oracle(gamma):
    p = workloads.network_flow(10_000, seed=0)
    print_case("hykkt_cg_count", n=p.n, gamma=gamma)
    # tol = 1: the solve stops after its first outer step, so cg_iters is
    # the CG count of HyKKT on rbar itself
    s = Solver(p, "hykkt", tol=1.0).bind(DEV)
    s.factorize(*device_values(p, DEV, "hykkt"), gamma=gamma)
    _, info = s.solve(torch.as_tensor(rhs_of(p, "hykkt"), device=DEV))
    torch.cuda.synchronize()
    P = osp.Problem(p)
    _, _, it, ok = osp.hykkt_steps(P, p.sigma_x, p.sigma_s_ineq, p.r1bar, p.r2bar, gamma, cg_tol=1e-10)
    print(info, "oracle CG iterations", it)
    assert ok and info["refine_steps"] == 0
    assert abs(info["cg_iters"] - it) <= 2


def _stale_pcg_oracle(p, seq, k_stale, k, b, theta):
    """Oracle PCG on system k around the exact factor of system k_stale."""
    P = osp.Problem(p)
    sxs, sss = seq[k_stale]
    sx, ss = seq[k]
    Ks = osp.assemble_condensed(P.W, sxs, P.J, sss).tocsc()
    lu = spla.splu(Ks)
    if theta is None:
        D = np.ones(p.n)
    else:
        f = om.features(p.n, p.w_ptr, p.w_idx, p.w_val, P.J, sx, ss, sxs, sss)
        D = om.diag_of(om.forward(theta, f)[0])
    apply_K = lambda v: osp.apply_condensed(P.W, sx, P.J, ss, v)
    tol_fn = lambda x: osp.omega_condensed(P.W, sx, P.J, ss, x, b) <= 1e-8
    x, it, ok = om.pcg(apply_K, b, lambda r: D * lu.solve(D * r), np.zeros(p.n), tol_fn, 50)
    return it, ok


@pytest.mark.parametrize("learned", [False, True])
def test_stale_pcg_count_matches_oracle(learned):
    p = workloads.pde_control(8)
    seq = workloads.ipm_sigma_sequence(p, 20, seed=0)
    print_case("stale_pcg_count", n=p.n, learned=learned)
    s = Solver(p, "lifted", "fp64", learned=1).bind(DEV)
    w, g, h, _, _ = device_values(p, DEV, "lifted")
    T = lambda a: torch.as_tensor(a, device=DEV)
    s.factorize(w, g, h, T(seq[10][0]), T(seq[10][1]))
    theta = None
    prm = None
    if learned:
        theta = om.init_params(3)
        # output weights halved: D stays within a few percent of a constant
        # (1.022..1.026 on system 12), which already moves the count from the
        # 2 iterations of D = I to 18..30, while every system still converges
        # within 50 (larger weights leave the oracle's PCG unconverged too)
        theta[-65:-1] *= 0.5
        theta = theta.astype(np.float32).astype(np.float64)
        prm = T(theta.astype(np.float32))
    b = np.random.default_rng(4).standard_normal(p.n)
    # systems 12..16: on the later systems (17..19) PCG with this D converges
    # slowly and irregularly (the oracle needs 32, 36, 29 iterations) and the
    # count follows the rounding of D (GPU FP32 features and MLP against the
    # oracle's FP64 ones: 37 against 29 on system 19), so they are not compared
    for k in (12, 14, 16):
        _, si = s.pcg_solve((w, g, h, T(seq[k][0]), T(seq[k][1])), 0.0, prm, T(b), maxit=50, tol=1e-8,
                            allow_refactor=False, raise_on_error=False)
        it, ok = _stale_pcg_oracle(p, seq, 10, k, b, theta)
        print(k, si, "oracle PCG iterations", it, ok)
        assert si["status"] == 0 and ok
        assert abs(si["pcg_iters"] - it) <= 2
