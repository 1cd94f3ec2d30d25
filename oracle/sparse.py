"""Sparse FP64 oracle for the large workloads (test infrastructure only).

Same definitions as ``oracle.dense`` but with scipy.sparse matrices so the
n ~ 1e5 workloads fit.  The direct solves use SuperLU
(``scipy.sparse.linalg.splu``) as a library primitive; FP64 Richardson
refinement with the *unassembled* operator (Sec. 2.2, "Iterative
refinement") brings the solution to the residual gate.

Residual definitions used throughout (the paper never defines its
"relative residual"; this is the reading used by the whole project):

    omega(x)   = max_i |b - K x|_i / (|W||x| + sigma_x|x| + |J|^T (sigma_s (|J||x|)) + |b|)_i
                 the componentwise relative backward error with respect to
                 the problem data (Oettli-Prager): the smallest eps such that
                 x solves exactly a system whose W, J, sigma and b entries are
                 each perturbed by a relative amount <= eps.  This is the
                 gated "relative residual".
    rho_K(x)   = ||b - K x||_inf / ||b||_inf   (unscaled; reported only)
    rho_K1, omega_K1: the same on K1 = [[K, G^T], [G, 0]] for HyKKT,
                 measured on K1 and not on the gamma-reformulated system.

Why the unscaled rho_K is not gated: with diagonals spanning 1e-8..1e8 the
rounding of x itself (not the solver) leaves rho_K ~ 1e-10..1e-8; the
error analysis of Sec. 4 (Prop. prop:cond:boundcondensedmatrix) measures
rounding as relative perturbations of W, A and D, which is what omega is.

K is always applied unassembled, W x + sigma_x * x + J^T (sigma_s * (J x)),
so the certificate does not inherit the O(u sigma) rounding of the
assembled matrix (Prop. prop:cond:boundcondensedmatrix).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------- inputs ----

def csr(nrows, ncols, ptr, idx, val):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(idx), np.asarray(ptr)),
                         shape=(nrows, ncols))


def sym_from_lower(n, ptr, idx, val):
    L = csr(n, n, ptr, idx, val)
    D = sp.diags(L.diagonal())
    return (L + L.T - D).tocsr()


class Problem:
    """Sparse matrices of a workloads.KKTProblem-like object."""

    def __init__(self, p):
        self.n, self.m_eq, self.m_ineq = p.n, p.m_eq, p.m_ineq
        self.W = sym_from_lower(p.n, p.w_ptr, p.w_idx, p.w_val)
        self.G = csr(p.m_eq, p.n, p.g_ptr, p.g_idx, p.g_val)
        self.H = csr(p.m_ineq, p.n, p.h_ptr, p.h_idx, p.h_val)
        self.J = sp.vstack([self.G, self.H]).tocsr()


# ------------------------------------------------------------- operators ----

def apply_condensed(W, sigma_x, J, sigma_s, x):
    """K x = W x + sigma_x * x + J^T (sigma_s * (J x)), unassembled
    (Sec. 2.2, K1; Sec. 3.2, eq:liftedkkt)."""
    return W @ x + sigma_x * x + J.T @ (sigma_s * (J @ x))


def abs_row_bound(W, sigma_x, J, sigma_s):
    """Upper bound of the row sums of |K| (for ||K||_inf)."""
    aJ = abs(J)
    return abs(W) @ np.ones(W.shape[0]) + sigma_x + aJ.T @ (sigma_s * (aJ @ np.ones(J.shape[1])))


def assemble_condensed(W, sigma_x, J, sigma_s):
    """Assembled K (scipy CSC); used only to build the direct factor."""
    return (W + sp.diags(sigma_x) + J.T @ sp.diags(sigma_s) @ J).tocsc()


def assemble_k_gamma(W, sigma_x, H, sigma_h, G, gamma):
    """K_gamma = W + diag(sigma_x) + H^T diag(sigma_h) H + gamma G^T G (eq:kkt:hykkt)."""
    return (W + sp.diags(sigma_x) + H.T @ sp.diags(sigma_h) @ H + gamma * (G.T @ G)).tocsc()


def k1_matrix(K, G, delta_c=0.0):
    """[[K, G^T], [G, -delta_c I]] (Sec. 2.2, K1; delta_c = 0 on the hot path,
    delta_c > 0 is the dual regularization of Remark 1)."""
    if delta_c == 0.0:
        return sp.bmat([[K, G.T], [G, None]]).tocsc()
    return sp.bmat([[K, G.T], [G, -delta_c * sp.identity(G.shape[0])]]).tocsc()


# ------------------------------------------------------------- residuals ----

def rho_condensed(W, sigma_x, J, sigma_s, x, b):
    r = b - apply_condensed(W, sigma_x, J, sigma_s, x)
    return np.abs(r).max() / max(np.abs(b).max(), 1e-300)


def omega_condensed(W, sigma_x, J, sigma_s, x, b):
    """Componentwise relative backward error w.r.t. (W, sigma_x, J, sigma_s, b)."""
    r = b - apply_condensed(W, sigma_x, J, sigma_s, x)
    ax = np.abs(x)
    aJ = abs(J)
    den = abs(W) @ ax + np.abs(sigma_x) * ax + aJ.T @ (np.abs(sigma_s) * (aJ @ ax)) + np.abs(b)
    return _cw_ratio(r, den)


def _cw_ratio(r, den):
    r = np.abs(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, r / np.where(den > 0, den, 1.0), np.where(r > 0, np.inf, 0.0))
    return float(q.max()) if q.size else 0.0


def eta_condensed(W, sigma_x, J, sigma_s, x, b):
    r = b - apply_condensed(W, sigma_x, J, sigma_s, x)
    knorm = abs_row_bound(W, sigma_x, J, sigma_s).max()
    return np.abs(r).max() / (knorm * np.abs(x).max() + np.abs(b).max())


def k1_residual(W, sigma_x, H, sigma_h, G, dx, dy, r1bar, r2bar, delta_c=0.0):
    """Residual blocks of K1 = [[K, G^T], [G, -delta_c I]] with K unassembled."""
    row1 = r1bar - (apply_condensed(W, sigma_x, H, sigma_h, dx) + G.T @ dy)
    row2 = r2bar - (G @ dx - delta_c * dy)
    return row1, row2


def omega_k1(W, sigma_x, H, sigma_h, G, dx, dy, r1bar, r2bar, delta_c=0.0):
    """Componentwise relative backward error of (dx, dy) on K1 w.r.t. its data
    (delta_c is one more datum of the second block row)."""
    row1, row2 = k1_residual(W, sigma_x, H, sigma_h, G, dx, dy, r1bar, r2bar, delta_c)
    ax, ay = np.abs(dx), np.abs(dy)
    aH, aG = abs(H), abs(G)
    den1 = (abs(W) @ ax + np.abs(sigma_x) * ax + aH.T @ (np.abs(sigma_h) * (aH @ ax))
            + aG.T @ ay + np.abs(r1bar))
    den2 = aG @ ax + abs(delta_c) * ay + np.abs(r2bar)
    return max(_cw_ratio(row1, den1), _cw_ratio(row2, den2))


def rho_k1(W, sigma_x, H, sigma_h, G, dx, dy, r1bar, r2bar, delta_c=0.0):
    row1, row2 = k1_residual(W, sigma_x, H, sigma_h, G, dx, dy, r1bar, r2bar, delta_c)
    num = max(np.abs(row1).max(), np.abs(row2).max() if row2.size else 0.0)
    den = max(np.abs(r1bar).max(), np.abs(r2bar).max() if r2bar.size else 0.0)
    return num / max(den, 1e-300)


# ---------------------------------------------------------------- solves ----

def _lu_spd(A):
    """SuperLU with symmetric fill-reducing ordering and no pivoting: on an
    SPD matrix this is an LL^T-equivalent factorization."""
    return spla.splu(A, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                     options=dict(SymmetricMode=True))


def solve_lifted(P: Problem, sigma_x, sigma_s, b, tol=1e-15, maxit=5):
    """LiftedKKT (Sec. 3.2): factor K_tau once, then Richardson refinement
    x <- x + K_tau^{-1} (b - K_tau x) with the unassembled FP64 operator
    (Sec. 2.2, "Iterative refinement").  Returns (x, omega history)."""
    K = assemble_condensed(P.W, sigma_x, P.J, sigma_s)
    lu = _lu_spd(K)
    x = lu.solve(b)
    hist = [omega_condensed(P.W, sigma_x, P.J, sigma_s, x, b)]
    for _ in range(maxit):
        if hist[-1] <= tol:
            break
        r = b - apply_condensed(P.W, sigma_x, P.J, sigma_s, x)
        x = x + lu.solve(r)
        hist.append(omega_condensed(P.W, sigma_x, P.J, sigma_s, x, b))
    return x, hist


def solve_k1(P: Problem, sigma_x, sigma_h, r1bar, r2bar, tol=1e-15, maxit=5, delta_c=0.0):
    """(d_x, d_y) of K1 directly (Sec. 2.2; with -delta_c I in its (2,2)
    block when delta_c > 0, Remark 1): SuperLU with pivoting on the
    indefinite saddle matrix, refined with the unassembled K1.  Returns
    (d_x, d_y, omega history)."""
    n = P.n
    K = assemble_condensed(P.W, sigma_x, P.H, sigma_h)
    lu = spla.splu(k1_matrix(K, P.G, delta_c))
    rhs = np.concatenate([r1bar, r2bar])
    sol = lu.solve(rhs)
    hist = []
    for _ in range(maxit + 1):
        dx, dy = sol[:n], sol[n:]
        row1, row2 = k1_residual(P.W, sigma_x, P.H, sigma_h, P.G, dx, dy, r1bar, r2bar, delta_c)
        res = np.concatenate([row1, row2])
        hist.append(omega_k1(P.W, sigma_x, P.H, sigma_h, P.G, dx, dy, r1bar, r2bar, delta_c))
        if hist[-1] <= tol:
            break
        sol = sol + lu.solve(res)
    return sol[:n], sol[n:], hist


def hykkt_steps(P: Problem, sigma_x, sigma_h, r1bar, r2bar, gamma, cg_tol=1e-10,
                cg_maxit=None):
    """HyKKT's three steps (Sec. 3.1) with a sparse factor of K_gamma:
    factor, CG on S_gamma (x0 = 0, stop at ||r_k|| <= tol ||c||), recovery.
    Returns (d_x, d_y, cg iterations, converged)."""
    Kg = assemble_k_gamma(P.W, sigma_x, P.H, sigma_h, P.G, gamma)
    lu = _lu_spd(Kg)
    G = P.G
    s = r1bar + gamma * (G.T @ r2bar)
    c = G @ lu.solve(s) - r2bar
    if cg_maxit is None:
        cg_maxit = max(1, min(G.shape[0], 1000))
    y = np.zeros_like(c)
    r = c.copy()
    p = r.copy()
    rr = float(r @ r)
    stop = cg_tol * np.sqrt(float(c @ c))
    it, ok = 0, np.sqrt(rr) <= stop
    while not ok and it < cg_maxit:
        it += 1
        q = G @ lu.solve(G.T @ p)
        alpha = rr / float(p @ q)
        y += alpha * p
        r -= alpha * q
        rr_new = float(r @ r)
        ok = np.sqrt(rr_new) <= stop
        p = r + (rr_new / rr) * p
        rr = rr_new
    dx = lu.solve(s - G.T @ y)
    return dx, y, it, ok
