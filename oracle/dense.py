"""Dense FP64 oracle for the paper's KKT forms (test infrastructure only).

Everything here is the plain definition, written with numpy dense matrices
so a reader can check it against the paper by eye.  It is meant for tiny
inputs (n up to a few hundred).

Notation (Sec. 2.2): W Hessian (symmetric), G equality Jacobian (m_e x n),
H inequality Jacobian (m_i x n), D_H per-row diagonal, delta_w folded into
the primal diagonal ``sigma_x``, delta_c = 0 unless stated (Remark 1).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


# ---------------------------------------------------------------- inputs ----

def sym_from_lower_csr(n, ptr, idx, val):
    """Dense symmetric W from its lower triangle given in CSR."""
    W = np.zeros((n, n))
    for i in range(n):
        for k in range(ptr[i], ptr[i + 1]):
            j = idx[k]
            W[i, j] = val[k]
            W[j, i] = val[k]
    return W


def csr_to_dense(nrows, ncols, ptr, idx, val):
    A = np.zeros((nrows, ncols))
    for i in range(nrows):
        for k in range(ptr[i], ptr[i + 1]):
            A[i, idx[k]] += val[k]
    return A


def problem_dense(p):
    """(W, G, H) dense from a workloads.KKTProblem-like object."""
    W = sym_from_lower_csr(p.n, p.w_ptr, p.w_idx, p.w_val)
    G = csr_to_dense(p.m_eq, p.n, p.g_ptr, p.g_idx, p.g_val)
    H = csr_to_dense(p.m_ineq, p.n, p.h_ptr, p.h_idx, p.h_val)
    return W, G, H


# ------------------------------------------------------- condensed forms ----

def condensed_matrix(W, sigma_x, J, sigma_s):
    """K = W + diag(sigma_x) + J^T diag(sigma_s) J.

    Sec. 2.2 (K1): K := W + delta_w I + H^T D_H H.  With J = H_tau = [G; H]
    this is LiftedKKT's K_tau (Sec. 3.2, eq:liftedkkt).
    """
    return W + np.diag(sigma_x) + J.T @ np.diag(sigma_s) @ J


def k_gamma(W, sigma_x, H, sigma_h, G, gamma):
    """K_gamma = K + gamma G^T G with K = W + diag(sigma_x) + H^T diag(sigma_h) H
    (Sec. 3.1, eq:kkt:hykkt)."""
    return condensed_matrix(W, sigma_x, H, sigma_h) + gamma * (G.T @ G)


def assemble_bruteforce(W, sigma_x, J, sigma_s):
    """Entry-by-entry sum over constraint rows: K_ij = W_ij + [i=j] sigma_x_i
    + sum_r sigma_s_r J_ri J_rj.  Pure-Python loops; tiny inputs only."""
    n = W.shape[0]
    K = W.copy()
    for i in range(n):
        K[i, i] += sigma_x[i]
    for r in range(J.shape[0]):
        nz = [c for c in range(n) if J[r, c] != 0.0]
        for i in nz:
            for j in nz:
                K[i, j] += sigma_s[r] * J[r, i] * J[r, j]
    return K


# -------------------------------------------------------- augmented (K2) ----

def augmented_k2(W, sigma_x, G, H, Ds, delta_w=0.0, delta_c=0.0):
    """The augmented system K2 (Sec. 2.2):

        [ W + dw I    0          G^T      H^T   ]
        [ 0           Ds + dw I  0        I     ]
        [ G           0          -dc I    0     ]
        [ H           I          0        -dc I ]

    Here ``sigma_x`` adds to the (1,1) block the way delta_w I does, so the
    primal diagonal may be any nonnegative vector.
    """
    n, me, mi = W.shape[0], G.shape[0], H.shape[0]
    N = n + mi + me + mi
    M = np.zeros((N, N))
    ix, isl, iy, iz = slice(0, n), slice(n, n + mi), slice(n + mi, n + mi + me), slice(n + mi + me, N)
    M[ix, ix] = W + np.diag(sigma_x) + delta_w * np.eye(n)
    M[isl, isl] = np.diag(Ds) + delta_w * np.eye(mi)
    M[ix, iy] = G.T
    M[iy, ix] = G
    M[ix, iz] = H.T
    M[iz, ix] = H
    M[isl, iz] = np.eye(mi)
    M[iz, isl] = np.eye(mi)
    M[iy, iy] = -delta_c * np.eye(me)
    M[iz, iz] = -delta_c * np.eye(mi)
    return M


def condensed_diagonals(Ds, delta_w=0.0, delta_c=0.0):
    """C = (I + dc (Ds + dw I))^-1 and D_H = (Ds + dw I) C  (Sec. 2.2, K1)."""
    C = 1.0 / (1.0 + delta_c * (Ds + delta_w))
    return C, (Ds + delta_w) * C


def condensed_rhs(r1, r2, r3, r4, H, Ds, delta_w=0.0, delta_c=0.0):
    """(rbar1, rbar2) = -(r1 + H^T (D_H r4 - C r2), r3)  (Sec. 2.2, K1).

    The sign follows the definition in K1; it is re-derived from rows 1, 2
    and 4 of K2 in the pin tests.
    """
    C, DH = condensed_diagonals(Ds, delta_w, delta_c)
    return -(r1 + H.T @ (DH * r4 - C * r2)), -r3


def recover_slacks(dx, r2, r4, H, Ds, delta_w=0.0, delta_c=0.0):
    """d_z = -C r2 + D_H (H dx + r4),  d_s = -(Ds + dw I)^-1 (r2 + d_z)  (Sec. 2.2)."""
    C, DH = condensed_diagonals(Ds, delta_w, delta_c)
    dz = -C * r2 + DH * (H @ dx + r4)
    ds = -(r2 + dz) / (Ds + delta_w)
    return ds, dz


def condensed_k1(K, G, delta_c=0.0):
    """K1 = [[K, G^T], [G, -dc I]]  (Sec. 2.2)."""
    n, me = K.shape[0], G.shape[0]
    M = np.zeros((n + me, n + me))
    M[:n, :n] = K
    M[:n, n:] = G.T
    M[n:, :n] = G
    M[n:, n:] = -delta_c * np.eye(me)
    return M


# ---------------------------------------------------------------- solves ----

def solve_lifted(W, sigma_x, J, sigma_s, b):
    """d_x = K_tau^{-1} b  (Sec. 3.2, eq:liftedkkt), dense LU."""
    return np.linalg.solve(condensed_matrix(W, sigma_x, J, sigma_s), b)


def solve_k1(K, G, r1bar, r2bar, delta_c=0.0):
    """(d_x, d_y) from K1 directly (Sec. 2.2), dense LU."""
    sol = np.linalg.solve(condensed_k1(K, G, delta_c), np.concatenate([r1bar, r2bar]))
    return sol[:K.shape[0]], sol[K.shape[0]:]


def solve_hykkt_system(K, G, r1bar, r2bar, gamma):
    """(d_x, d_y) from the gamma-reformulated saddle system eq:kkt:hykkt
    [[K_gamma, G^T], [G, 0]] (d_x, d_y) = (r1bar + gamma G^T r2bar, r2bar)."""
    n = K.shape[0]
    M = condensed_k1(K + gamma * (G.T @ G), G)
    rhs = np.concatenate([r1bar + gamma * (G.T @ r2bar), r2bar])
    sol = np.linalg.solve(M, rhs)
    return sol[:n], sol[n:]


def primal_schur_delta_c(K, G, r1bar, r2bar, delta_c):
    """Remark 1 (eqn:primal) for delta_c > 0.

    Eliminating d_y = (G d_x - r2bar)/delta_c from K1 gives
    (K + G^T G / delta_c) d_x = r1bar + G^T r2bar / delta_c.  The printed
    right-hand side drops the G^T in front of r2bar (its sizes do not
    match); this is the reading used here.
    """
    dx = np.linalg.solve(K + (G.T @ G) / delta_c, r1bar + G.T @ r2bar / delta_c)
    dy = (G @ dx - r2bar) / delta_c
    return dx, dy


def cg(apply_A, c, tol, maxit):
    """Plain conjugate gradient (Hestenes-Stiefel) from x0 = 0.

    Stops when ||r_k||_2 <= tol * ||c||_2.  Returns (x, iterations,
    converged, residual norms)."""
    x = np.zeros_like(c)
    r = c.copy()
    p = r.copy()
    rr = float(r @ r)
    stop = tol * np.sqrt(float(c @ c))
    hist = [np.sqrt(rr)]
    if np.sqrt(rr) <= stop:
        return x, 0, True, hist
    for k in range(1, maxit + 1):
        q = apply_A(p)
        alpha = rr / float(p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rr_new = float(r @ r)
        hist.append(np.sqrt(rr_new))
        if np.sqrt(rr_new) <= stop:
            return x, k, True, hist
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, maxit, False, hist


def hykkt_steps(K, G, r1bar, r2bar, gamma, cg_tol=1e-10, cg_maxit=None):
    """HyKKT as its three steps (Sec. 3.1):

    1. assemble K_gamma = K + gamma G^T G and take its Cholesky factor;
    2. CG on S_gamma d_y = G K_gamma^{-1} (r1bar + gamma G^T r2bar) - r2bar
       (eq:kkt:schurcomplhykkt) with S_gamma = G K_gamma^{-1} G^T;
    3. d_x = K_gamma^{-1} (r1bar + gamma G^T r2bar - G^T d_y).
    """
    Kg = K + gamma * (G.T @ G)
    Lc = np.linalg.cholesky(Kg)

    def kinv(v):
        return scipy.linalg.cho_solve((Lc, True), v)

    s = r1bar + gamma * (G.T @ r2bar)
    c = G @ kinv(s) - r2bar
    if cg_maxit is None:
        cg_maxit = max(1, min(G.shape[0], 1000))
    dy, iters, ok, hist = cg(lambda p: G @ kinv(G.T @ p), c, cg_tol, cg_maxit)
    dx = kinv(s - G.T @ dy)
    return dx, dy, iters, ok


# -------------------------------------------------------------- spectral ----

def inertia(M, rtol=1e-10):
    """(n_+, n_-, n_0) from the eigenvalues of a symmetric matrix."""
    ev = np.linalg.eigvalsh(M)
    tol = rtol * max(1.0, np.abs(ev).max())
    return int((ev > tol).sum()), int((ev < -tol).sum()), int((np.abs(ev) <= tol).sum())


def null_range_bases(G):
    """Orthonormal [Y Z]: Z spans Ker(G), Y its complement (via SVD)."""
    U, s, Vt = np.linalg.svd(G)
    rank = int((s > s.max() * 1e-12).sum()) if s.size else 0
    V = Vt.T
    return V[:, :rank], V[:, rank:], s[:rank]


def gamma_threshold(K, G):
    """Sufficient gamma for K_gamma > 0 (Remark in Sec. 3.1, eq:kkt:boundgamma):

        gamma_ = (||K||^2 / lam_min(Z^T K Z) - lam_min(Y^T K Y)) / sigma_min(G)^2
    """
    Y, Z, s = null_range_bases(G)
    lz = np.linalg.eigvalsh(Z.T @ K @ Z).min()
    ly = np.linalg.eigvalsh(Y.T @ K @ Y).min()
    normK = np.linalg.norm(K, 2)
    return (normK ** 2 / lz - ly) / s.min() ** 2


def schur_gamma(K, G, gamma):
    """S_gamma = G K_gamma^{-1} G^T (Sec. 3.1)."""
    Kg = K + gamma * (G.T @ G)
    return G @ np.linalg.solve(Kg, G.T)


# ------------------------------------------------------------- residuals ----

def rel_residual(M, x, b):
    """||b - M x||_inf / ||b||_inf."""
    return np.abs(b - M @ x).max() / max(np.abs(b).max(), 1e-300)


def omega_bruteforce(W, sigma_x, J, sigma_s, x, b):
    """Componentwise relative backward error with respect to the data
    (Oettli-Prager), one row at a time: row i's residual divided by the sum
    of the magnitudes of every product that forms (K x)_i, plus |b_i|.
    Pure-Python loops; tiny inputs only."""
    n, m = W.shape[0], J.shape[0]
    worst = 0.0
    for i in range(n):
        acc, mag = 0.0, abs(b[i])
        for j in range(n):
            acc += W[i, j] * x[j]
            mag += abs(W[i, j] * x[j])
        acc += sigma_x[i] * x[i]
        mag += abs(sigma_x[i] * x[i])
        for r in range(m):
            if J[r, i] == 0.0:
                continue
            for j in range(n):
                t = J[r, i] * sigma_s[r] * J[r, j] * x[j]
                acc += t
                mag += abs(t)
        res = abs(b[i] - acc)
        worst = max(worst, res / mag if mag > 0 else (np.inf if res > 0 else 0.0))
    return worst
