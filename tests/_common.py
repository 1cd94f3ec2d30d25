"""Helpers shared by the test modules (not a test module itself)."""
import numpy as np
import scipy.sparse as sp

from oracle import sparse as osp


def sigma_rows(p, formulation, gamma):
    """Row weights of the condensed matrix: LiftedKKT sigma_s on J = [G; H];
    HyKKT gamma on G rows and sigma_s on H rows (K_gamma)."""
    if formulation == "lifted":
        return p.sigma_s
    return np.concatenate([np.full(p.m_eq, gamma), p.sigma_s_ineq])


def omega_of(p, formulation, sol, gamma=1e7):
    """Oracle certificate of a solution (componentwise backward error)."""
    P = osp.Problem(p)
    if formulation == "lifted":
        return osp.omega_condensed(P.W, p.sigma_x, P.J, p.sigma_s, sol, p.b)
    dx, dy = sol[:p.n], sol[p.n:]
    return osp.omega_k1(P.W, p.sigma_x, P.H, p.sigma_s_ineq, P.G, dx, dy, p.r1bar, p.r2bar)


def omega_kgamma(p, x, b, gamma):
    """Certificate of x = K_gamma^{-1} b (one application of the factor)."""
    P = osp.Problem(p)
    J = sp.vstack([P.G, P.H]).tocsr()
    return osp.omega_condensed(P.W, p.sigma_x, J, sigma_rows(p, "hykkt", gamma), x, b)


def rhs_of(p, formulation):
    return p.b if formulation == "lifted" else np.concatenate([p.r1bar, p.r2bar])


def plant_negative_curvature(p, formulation, theta, gamma=1e7):
    """Copy of ``p`` whose W diagonal is lowered uniformly so that the smallest
    eigenvalue of the condensed matrix (K for LiftedKKT, K_gamma for HyKKT)
    is exactly -theta.  Dense eigenvalues: small problems only."""
    import dataclasses
    from oracle import dense as od
    W, G, H = od.problem_dense(p)
    if formulation == "lifted":
        K = od.condensed_matrix(W, p.sigma_x, np.vstack([G, H]), p.sigma_s)
    else:
        K = od.k_gamma(W, p.sigma_x, H, p.sigma_s_ineq, G, gamma)
    shift = np.linalg.eigvalsh(K)[0] + theta
    w = p.w_val.copy()
    for i in range(p.n):
        for k in range(p.w_ptr[i], p.w_ptr[i + 1]):
            if p.w_idx[k] == i:
                w[k] -= shift
    return dataclasses.replace(p, w_val=w, name=f"{p.name}+curv{theta:g}")
