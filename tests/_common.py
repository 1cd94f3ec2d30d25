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
