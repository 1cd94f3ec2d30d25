"""Newton-step recovery around the condensed solve (test infrastructure only).

The augmented system K2 (Sec. 2.2, eq:kkt:augmented) with delta_c = 0 is

    [ W + Sx   0    G^T   H^T ] [d_x]     [r1]
    [ 0        E    0     I   ] [d_s]     [r2]
    [ G        0    0     0   ] [d_y] = - [r3]
    [ H        I    0     0   ] [d_z]     [r4]

where Sx is the primal diagonal (delta_w I, generalised to any nonnegative
diagonal) and E = D_s + delta_w I the slack diagonal (D_s = S^-1 V).  For
LiftedKKT every constraint row carries a slack (the equalities are relaxed,
Sec. 3.2), so G is empty and H = J; for HyKKT G is the equality Jacobian.
Condensing the slack rows gives the condensed system with D_H = E
(Sec. 2.2, K1), and the slack block is recovered afterwards
(oracle.dense.recover_slacks).  The bound multipliers follow from the last
block row of the unreduced system K3 (eq:kkt:unreduced):
d_v = -S^-1 (V d_s - mu e) - v (Sec. 2.2).

The accuracy measure of a step is the componentwise relative backward error
of K2 with respect to its data (W, Sx, G, H, E and the right-hand side),
the same Oettli-Prager measure used for the condensed systems.

This module shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

from oracle import dense as od


def unreduced_k3(W, sigma_x, G, H, s, v):
    """K3 of eq:kkt:unreduced, with W + diag(sigma_x) as its Hessian block.

    Unknown order (d_x, d_s, d_y, d_z, d_v); the right-hand side is
    -(grad L, z - v, g, h + s, S v - mu e)."""
    n, me, mi = W.shape[0], G.shape[0], H.shape[0]
    N = n + mi + me + mi + mi
    M = np.zeros((N, N))
    ix = slice(0, n)
    isl = slice(n, n + mi)
    iy = slice(n + mi, n + mi + me)
    iz = slice(n + mi + me, n + 2 * mi + me)
    iv = slice(n + 2 * mi + me, N)
    M[ix, ix] = W + np.diag(sigma_x)
    M[ix, iy] = G.T
    M[ix, iz] = H.T
    M[isl, iz] = np.eye(mi)
    M[isl, iv] = -np.eye(mi)
    M[iy, ix] = G
    M[iz, ix] = H
    M[iz, isl] = np.eye(mi)
    M[iv, isl] = np.diag(v)
    M[iv, iv] = np.diag(s)
    return M


def solve_augmented(W, sigma_x, G, H, E, r1, r2, r3, r4):
    """(d_x, d_s, d_y, d_z) of K2 (delta_c = 0) through the condensed system:
    rbar from eq K1's definition, a dense K1 solve, then the slack recovery."""
    rb1, rb2 = od.condensed_rhs(r1, r2, r3, r4, H, E)
    K = od.condensed_matrix(W, sigma_x, H, E)
    dx, dy = od.solve_k1(K, G, rb1, rb2)
    ds, dz = od.recover_slacks(dx, r2, r4, H, E)
    return dx, ds, dy, dz


def bound_dual_step(s, v, mu, ds):
    """d_v from the last block row of K3: V d_s + S d_v = -(S v - mu e)."""
    return -(v * ds - mu) / s - v


def k2_residual(W, sigma_x, G, H, E, r1, r2, r3, r4, dx, ds, dy, dz):
    """Blocks of -r - K2 d (delta_c = 0), with the matrix applied blockwise."""
    R1 = -r1 - ((W @ dx + sigma_x * dx) + G.T @ dy + H.T @ dz)
    R2 = -r2 - (E * ds + dz)
    R3 = -r3 - G @ dx
    R4 = -r4 - (H @ dx + ds)
    return R1, R2, R3, R4


def _ratio(num, den):
    num, den = np.abs(num), np.asarray(den)
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))
    return float(out.max()) if out.size else 0.0


def omega_k2(W, sigma_x, G, H, E, r1, r2, r3, r4, dx, ds, dy, dz):
    """Componentwise relative backward error of (d_x, d_s, d_y, d_z) on K2:
    max_i |res_i| / (|K2| |d| + |r|)_i with |K2| taken block by block."""
    R1, R2, R3, R4 = k2_residual(W, sigma_x, G, H, E, r1, r2, r3, r4, dx, ds, dy, dz)
    ax, asl, ay, az = np.abs(dx), np.abs(ds), np.abs(dy), np.abs(dz)
    aG, aH = abs(G), abs(H)  # abs(): dense arrays or scipy.sparse matrices
    d1 = abs(W) @ ax + np.abs(sigma_x) * ax + aG.T @ ay + aH.T @ az + np.abs(r1)
    d2 = np.abs(E) * asl + az + np.abs(r2)
    d3 = aG @ ax + np.abs(r3)
    d4 = aH @ ax + asl + np.abs(r4)
    return max(_ratio(R1, d1), _ratio(R2, d2), _ratio(R3, d3), _ratio(R4, d4))
