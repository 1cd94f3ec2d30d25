"""Inertia correction of the condensed matrix (test infrastructure only).

The augmented system K2 (Sec. 2.2, eq:kkt:augmented) carries a primal
regularization delta_w >= 0 on both its primal block and its slack block.
Its inertia must be (n + m_i, m_i + m_e, 0), and when it is not, the paper
raises delta_w by the inertia-controlling rule of Waechter & Biegler (2006,
Sec. 3.1), to which it defers for the details (Sec. 2.2; Remark 1).  Through
Sylvester's law (eq:ipm:inertia) a correct inertia is the same thing as a
positive definite condensed matrix: LiftedKKT's K_tau (Sec. 3.2,
eq:liftedkkt), and HyKKT's K_gamma once gamma exceeds its threshold
(Sec. 3.1).  A failed Cholesky factorization is therefore the signal to try
the next delta_w, and no inertia count is needed.

Condensing K2 with delta_w (delta_c = 0, so C = I) gives
    K(delta_w) = W + diag(sigma_x) + delta_w I + J^T diag(sigma_s + delta_w) J,
i.e. delta_w is added to the primal diagonal and to every slack weight.  For
HyKKT only the inequality rows have slacks; G keeps its weight gamma.

The rule (Waechter & Biegler, Sec. 3.1, Algorithm IC; the zero-eigenvalue
branch that sets delta_c is absent because a Cholesky factorization cannot
tell a zero eigenvalue from a negative one and delta_c = 0 on this path):
  1. try delta_w = 0;
  2. first nonzero trial: delta_w_0 if no earlier call needed one
     (delta_w_last = 0), else max(delta_w_min, kappa_minus * delta_w_last);
  3. on failure multiply by kappa_plus_bar (delta_w_last = 0) or kappa_plus
     (delta_w_last > 0) and try again, giving up above delta_w_max;
  4. a successful nonzero delta_w becomes the new delta_w_last; a success at
     delta_w = 0 leaves delta_w_last as it was.
The default constants are the ones Waechter & Biegler publish with the rule.

This module shares nothing with the HIP path.
"""
from __future__ import annotations

import numpy as np

from oracle import dense as od

DEFAULTS = dict(delta_w_min=1e-20, delta_w_0=1e-4, delta_w_max=1e40,
                kappa_minus=1.0 / 3.0, kappa_plus=8.0, kappa_plus_bar=100.0)


def regularized_diagonals(sigma_x, sigma_s, delta_w):
    """Diagonals of the condensed matrix of K2 with delta_w on its primal and
    slack blocks (delta_c = 0): sigma_x + delta_w and sigma_s + delta_w."""
    return np.asarray(sigma_x) + delta_w, np.asarray(sigma_s) + delta_w


def cholesky_ok(M):
    """True when the dense Cholesky factorization of M exists (LAPACK)."""
    try:
        np.linalg.cholesky(M)
        return True
    except np.linalg.LinAlgError:
        return False


def correct(factor_ok, delta_w_last=0.0, params=None):
    """Runs the rule on a predicate ``factor_ok(delta_w) -> bool``.

    Returns (delta_w, tried, delta_w_last_new): the accepted delta_w (None
    when every trial up to delta_w_max failed), the list of trials in order,
    and the delta_w_last to carry into the next call.
    """
    p = dict(DEFAULTS, **(params or {}))
    tried = [0.0]
    if factor_ok(0.0):
        return 0.0, tried, delta_w_last
    if delta_w_last == 0.0:
        delta, grow = p["delta_w_0"], p["kappa_plus_bar"]
    else:
        delta, grow = max(p["delta_w_min"], p["kappa_minus"] * delta_w_last), p["kappa_plus"]
    while delta <= p["delta_w_max"]:
        tried.append(delta)
        if factor_ok(delta):
            return delta, tried, delta
        delta *= grow
    return None, tried, delta_w_last


def lifted_matrix(W, sigma_x, J, sigma_s, delta_w):
    """K_tau of eq:liftedkkt built from K2 with regularization delta_w."""
    sx, ss = regularized_diagonals(sigma_x, sigma_s, delta_w)
    return od.condensed_matrix(W, sx, J, ss)


def hykkt_matrix(W, sigma_x, H, sigma_h, G, gamma, delta_w):
    """K_gamma of eq:kkt:hykkt built from K2 with regularization delta_w."""
    sx, sh = regularized_diagonals(sigma_x, sigma_h, delta_w)
    return od.k_gamma(W, sx, H, sh, G, gamma)


def lifted_correction(W, sigma_x, J, sigma_s, delta_w_last=0.0, params=None):
    return correct(lambda d: cholesky_ok(lifted_matrix(W, sigma_x, J, sigma_s, d)), delta_w_last, params)


def hykkt_correction(W, sigma_x, H, sigma_h, G, gamma, delta_w_last=0.0, params=None):
    return correct(lambda d: cholesky_ok(hykkt_matrix(W, sigma_x, H, sigma_h, G, gamma, d)),
                   delta_w_last, params)
