"""Writes the exact-arithmetic golden fixtures in this folder.

Each fixture is a tiny KKT system with rational data whose augmented form
K2 (Sec. 2.2, eq. K2) is solved exactly by ``oracle.exact``.  The stored
solutions are therefore independent of every floating-point code path; the
tests check the condensed FP64 oracle (K1 / eq:liftedkkt / eq:kkt:hykkt)
and, through it, the HIP path against them.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact import augmented_k2_exact, solve_exact  # noqa: E402


def frac_list(v):
    return [str(x) for x in v]


def case_hykkt():
    # n = 3, m_e = 1, m_i = 2
    W = [[F(4), F(1), F(0)], [F(1), F(3), F(-1, 2)], [F(0), F(-1, 2), F(2)]]
    sigma_x = [F(1, 10), F(0), F(3)]
    G = [[F(1), F(-2), F(1, 3)]]
    H = [[F(0), F(1), F(1)], [F(2), F(0), F(-1)]]
    Ds = [F(1000), F(1, 1000)]
    r1 = [F(1), F(-2), F(1, 2)]
    r2 = [F(3), F(-1)]
    r3 = [F(1, 4)]
    r4 = [F(-1), F(2)]
    M = augmented_k2_exact(W, sigma_x, G, H, Ds)
    sol = solve_exact(M, [-v for v in r1 + r2 + r3 + r4])
    n, mi, me = 3, 2, 1
    return dict(
        citation="Sec. 2.2, eq. K2 (augmented system, delta_w = delta_c = 0) solved exactly; "
                 "condensed forms K1 and eq:kkt:hykkt must reproduce d_x, d_y",
        n=n, m_eq=me, m_ineq=mi,
        W=[frac_list(r) for r in W], sigma_x=frac_list(sigma_x), G=[frac_list(r) for r in G],
        H=[frac_list(r) for r in H], Ds=frac_list(Ds), r1=frac_list(r1), r2=frac_list(r2),
        r3=frac_list(r3), r4=frac_list(r4),
        dx=frac_list(sol[:n]), ds=frac_list(sol[n:n + mi]), dy=frac_list(sol[n + mi:n + mi + me]),
        dz=frac_list(sol[n + mi + me:]))


def case_lifted():
    # n = 4, all three rows are (relaxed) inequality rows: J = [G; H]
    W = [[F(2), F(-1), F(0), F(0)], [F(-1), F(2), F(-1), F(0)],
         [F(0), F(-1), F(2), F(-1)], [F(0), F(0), F(-1), F(2)]]
    sigma_x = [F(1, 100), F(0), F(5), F(1, 2)]
    J = [[F(1), F(1), F(0), F(0)], [F(0), F(3), F(0), F(-1)], [F(1, 2), F(0), F(-1), F(1)]]
    Ds = [F(10 ** 8), F(1, 10 ** 8), F(7, 3)]
    r1 = [F(1), F(0), F(-1), F(2)]
    r2 = [F(1, 2), F(-3), F(1)]
    r4 = [F(2), F(1, 5), F(-1)]
    M = augmented_k2_exact(W, sigma_x, [], J, Ds)
    sol = solve_exact(M, [-v for v in r1 + r2 + r4])
    n, mi = 4, 3
    return dict(
        citation="Sec. 2.2, eq. K2 without equality block (LiftedKKT, Sec. 3.2 eq:liftedkkt: "
                 "equalities relaxed into inequality rows H_tau) solved exactly",
        n=n, m_eq=0, m_ineq=mi,
        W=[frac_list(r) for r in W], sigma_x=frac_list(sigma_x), J=[frac_list(r) for r in J],
        Ds=frac_list(Ds), r1=frac_list(r1), r2=frac_list(r2), r4=frac_list(r4),
        dx=frac_list(sol[:n]), ds=frac_list(sol[n:n + mi]), dz=frac_list(sol[n + mi:]))


if __name__ == "__main__":
    for name, fn in [("tiny_hykkt_k2.json", case_hykkt), ("tiny_lifted_k2.json", case_lifted)]:
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(fn(), f, indent=1)
        print("wrote", name)
