"""Exact rational arithmetic for tiny KKT systems (test infrastructure only).

Used to write the golden fixtures: the augmented system K2 (Sec. 2.2) is
solved exactly with ``fractions.Fraction`` Gauss-Jordan elimination, which
shares nothing with the floating-point code paths.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Sequence


def solve_exact(A: Sequence[Sequence[Fraction]], b: Sequence[Fraction]) -> List[Fraction]:
    """x with A x = b, exactly (Gauss-Jordan with first-nonzero pivoting)."""
    n = len(A)
    M = [[Fraction(v) for v in row] + [Fraction(bi)] for row, bi in zip(A, b)]
    for col in range(n):
        piv = next((r for r in range(col, n) if M[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular matrix")
        M[col], M[piv] = M[piv], M[col]
        pv = M[col][col]
        M[col] = [v / pv for v in M[col]]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col]
                M[r] = [a - f * c for a, c in zip(M[r], M[col])]
    return [M[r][n] for r in range(n)]


def augmented_k2_exact(W, sigma_x, G, H, Ds):
    """K2 (Sec. 2.2, delta_w = delta_c = 0 with the primal diagonal sigma_x)
    as a list of Fraction rows; W is a full symmetric list of lists."""
    n, me, mi = len(W), len(G), len(H)
    N = n + mi + me + mi
    Z = Fraction(0)
    M = [[Z] * N for _ in range(N)]
    for i in range(n):
        for j in range(n):
            M[i][j] = Fraction(W[i][j])
        M[i][i] += Fraction(sigma_x[i])
    for k in range(mi):
        M[n + k][n + k] = Fraction(Ds[k])
        M[n + k][n + mi + me + k] = Fraction(1)
        M[n + mi + me + k][n + k] = Fraction(1)
    for r in range(me):
        for j in range(n):
            M[n + mi + r][j] = Fraction(G[r][j])
            M[j][n + mi + r] = Fraction(G[r][j])
    for r in range(mi):
        for j in range(n):
            M[n + mi + me + r][j] = Fraction(H[r][j])
            M[j][n + mi + me + r] = Fraction(H[r][j])
    return M
