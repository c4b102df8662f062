"""Exact rational brute force over all vertex triples (tests only).

P_bal is the four-term sum of the paper's Section 3 evaluated in exact rational
arithmetic on the FP64 inputs (every FP64 number is a rational), and the
decisions are the definitions "Uncertain Balanced Triangle" (P_bal >= t) and
"Uncertain Unbalanced Triangle" (P_unbal > t) taken literally. Nothing here uses
the product form s = d1 d2 d3, so it checks the oracle's FP64 rule independently.
"""
from fractions import Fraction as F
from itertools import combinations


def p_bal(pa, pb, pc):
    qa, qb, qc = 1 - pa, 1 - pb, 1 - pc
    return pa * pb * pc + pa * qb * qc + qa * pb * qc + qa * qb * pc


def edge_map(lo, hi, p):
    return {(int(a), int(b)): F(float(x)) for a, b, x in zip(lo, hi, p)}


def triangles(n, E):
    for i, j, k in combinations(range(n), 3):
        if (i, j) in E and (i, k) in E and (j, k) in E:
            yield i, j, k


def classify_all(n, lo, hi, p, t):
    E = edge_map(lo, hi, p)
    tt = F(float(t))
    bal, unbal = [], []
    for i, j, k in triangles(n, E):
        pb = p_bal(E[(i, j)], E[(i, k)], E[(j, k)])
        if pb >= tt:
            bal.append((i, j, k))
        if 1 - pb > tt:
            unbal.append((i, j, k))
    return bal, unbal


def expected(n, lo, hi, p):
    E = edge_map(lo, hi, p)
    return sum((p_bal(E[(i, j)], E[(i, k)], E[(j, k)]) for i, j, k in triangles(n, E)), F(0))


def grad_two_point(n, lo, hi, p, e):
    """E(p_e = 1) - E(p_e = 0): equals dE/dp_e because E is affine in each p_e."""
    E = edge_map(lo, hi, p)
    key = (int(lo[e]), int(hi[e]))
    tot = F(0)
    for i, j, k in triangles(n, E):
        tri = [(i, j), (i, k), (j, k)]
        if key not in tri:
            continue
        vals1 = [F(1) if x == key else E[x] for x in tri]
        vals0 = [F(0) if x == key else E[x] for x in tri]
        tot += p_bal(*vals1) - p_bal(*vals0)
    return tot
