"""Why the learned diagonal does not beat D = I on the IPM-like sequences
(CPU evidence for the learned preconditioner's negative result).

PCG around a stale factor with M^{-1} = D K_s^{-1} D converges at the rate
set by the spread of the generalized eigenvalues of (K_k, D^{-1} K_s
D^{-1}).  On the 8^3 PDE-control sequence (stale system 10, new system 16)
the diagonal weights of the rows drift geometrically by two group factors
(active rows up, the rest down), so the spectrum of K_s^{-1} K_k has two
clusters whose extreme eigenvectors spread over many variables.  Starting
from D = I, L-BFGS on log kappa over every positive diagonal (exact
gradient, checked by finite differences here) and the Jacobi choice
D = (diag K_s / diag K_k)^{1/2} both change kappa by less than 0.1 %: no
diagonal correction, learned or not, can make PCG converge faster here.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as so

from oracle import sparse as osp
from paper_2405_14236_amd import workloads


def _pencil():
    p = workloads.pde_control(8)
    seq = workloads.ipm_sigma_sequence(p, 20, seed=0)
    P = osp.Problem(p)
    Ks = osp.assemble_condensed(P.W, seq[10][0], P.J, seq[10][1]).toarray()
    Kk = osp.assemble_condensed(P.W, seq[16][0], P.J, seq[16][1]).toarray()
    return Ks, Kk


def _log_kappa(Ks, Kk, u):
    """log of lambda_max / lambda_min of (Kk, D^-1 Ks D^-1), D = diag(e^u),
    and its gradient: with Kk v = lambda B v, v^T B v = 1 and
    dB/du_j = -(e_j e_j^T B + B e_j e_j^T), d lambda / d u_j = 2 lambda v_j (B v)_j."""
    d = np.exp(u)
    B = Ks / np.outer(d, d)
    lam, V = sla.eigh(Kk, B)
    vmin, vmax = V[:, 0], V[:, -1]
    return np.log(lam[-1] / lam[0]), 2.0 * vmax * (B @ vmax) - 2.0 * vmin * (B @ vmin)


def test_gradient_matches_finite_differences():
    Ks, Kk = _pencil()
    rng = np.random.default_rng(0)
    u = 0.05 * rng.standard_normal(Ks.shape[0])
    f0, g = _log_kappa(Ks, Kk, u)
    # the five largest components (the eigensolver's rounding swamps
    # central differences of the tiny ones)
    for j in np.argsort(-np.abs(g))[:5]:
        e = np.zeros_like(u)
        e[j] = 1e-4
        fd = (_log_kappa(Ks, Kk, u + e)[0] - _log_kappa(Ks, Kk, u - e)[0]) / 2e-4
        assert abs(fd - g[j]) <= 1e-2 * abs(g[j]), (j, fd, g[j])


def test_no_diagonal_tightens_the_two_cluster_spectrum():
    Ks, Kk = _pencil()
    n = Ks.shape[0]
    k_id = np.exp(_log_kappa(Ks, Kk, np.zeros(n))[0])
    assert k_id > 100.0  # the stale factor alone leaves a wide spectrum
    k_jac = np.exp(_log_kappa(Ks, Kk, 0.5 * np.log(np.diag(Ks) / np.diag(Kk)))[0])
    r = so.minimize(lambda u: _log_kappa(Ks, Kk, u), np.zeros(n), jac=True, method="L-BFGS-B",
                    options=dict(maxiter=200))
    k_best = np.exp(r.fun)
    print(f"kappa: D = I {k_id:.4f}, Jacobi {k_jac:.4f}, best diagonal found {k_best:.4f}")
    assert k_best >= 0.999 * k_id and k_jac >= 0.999 * k_id
