"""Brute-force alpha complex for tiny inputs, straight from the definitions.

Used only to pin the oracle. Independent of oracle/ and of the HIP path: it
forms every ortho-centre by solving its linear system in exact rationals
(fractions.Fraction), tests every other ball against it, and breaks exact ties
by simulation of simplicity computed as finite differences of the (affine in
the weights) power difference, so it needs no derivative formulas.

Definitions (Masood, Ray, Natarajan, Sec. 2.2-2.4):
  pi(p, b) = |p - p_b|^2 - W_b,  W_b = r_b^2.
  sigma is in D iff some point is equidistant in power from sigma's balls and
  no closer to any other ball. For a tetrahedron that point is unique (its
  ortho-centre). For a lower simplex, its dual power face is non-empty iff the
  ortho-centre is such a point (Gabriel) or one of its immediate cofaces is in
  D. Size = OrthoSize when Gabriel, else the least Size of a coface in D.
  K_alpha = {sigma in D : Size(sigma) <= alpha}.
Ties: W_i -> W_i + eps_i, eps ranked by input index (lower index dominates).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations


def quantise(xyz, radii, alpha):
    P = [tuple(int(round(float(c) * 1000.0)) for c in p) for p in xyz]
    R = [int(round(float(r) * 1000.0)) for r in radii]
    W = [r * r for r in R]
    aq = int(round(float(alpha) * 1e6))
    return P, W, aq


def _sub(a, b):
    return (a[0] - b[0], a[1] - b[1], a[2] - b[2])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _solve(M, rhs):
    """Gaussian elimination over Fractions; returns None if singular."""
    n = len(M)
    A = [[Fraction(x) for x in row] + [Fraction(r)] for row, r in zip(M, rhs)]
    for col in range(n):
        piv = next((r for r in range(col, n) if A[r][col] != 0), None)
        if piv is None:
            return None
        A[col], A[piv] = A[piv], A[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [A[i][n] / A[i][i] for i in range(n)]


def orthocentre(P, W, sigma):
    """Point of aff(sigma) with equal power distance to sigma's balls (absolute coords)."""
    p0 = P[sigma[0]]
    if len(sigma) == 1:
        return tuple(Fraction(c) for c in p0)
    a = [_sub(P[v], p0) for v in sigma[1:]]
    G = [[_dot(ai, aj) for aj in a] for ai in a]
    beta = [Fraction(_dot(ai, ai) - W[v] + W[sigma[0]], 2) for ai, v in zip(a, sigma[1:])]
    lam = _solve(G, beta)
    if lam is None:
        return None
    return tuple(p0[k] + sum(l * ai[k] for l, ai in zip(lam, a)) for k in range(3))


def power(c, P, W, i):
    d = (c[0] - P[i][0], c[1] - P[i][1], c[2] - P[i][2])
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - W[i]


def violation_sign(P, W, sigma, q, c=None):
    """Sign of pi(c,q) - pi(c,sigma_0) at sigma's ortho-centre c, ties broken by SoS."""
    def g(Wx, cx=None):
        cx = orthocentre(P, Wx, sigma) if cx is None else cx
        return power(cx, P, Wx, q) - power(cx, P, Wx, sigma[0])

    base = g(W, c)
    if base != 0:
        return 1 if base > 0 else -1
    for j in sorted(list(sigma) + [q]):
        Wj = list(W)
        Wj[j] += 1
        d = g(Wj) - base
        if d != 0:
            return 1 if d > 0 else -1
    raise AssertionError("simulation of simplicity did not resolve a tie")


def _independent(P, sigma):
    if len(sigma) <= 1:
        return True
    p0 = P[sigma[0]]
    a = [_sub(P[v], p0) for v in sigma[1:]]
    G = [[_dot(ai, aj) for aj in a] for ai in a]
    if len(a) == 1:
        return G[0][0] != 0
    if len(a) == 2:
        return G[0][0] * G[1][1] - G[0][1] * G[1][0] != 0
    det = (a[0][0] * (a[1][1] * a[2][2] - a[1][2] * a[2][1]) - a[0][1] * (a[1][0] * a[2][2] - a[1][2] * a[2][0])
           + a[0][2] * (a[1][0] * a[2][1] - a[1][1] * a[2][0]))
    return det != 0


def alpha_complex(xyz, radii, alpha):
    """Returns (K, D): K[d] = sorted list of (simplex tuple, Size as Fraction in mA^2)
    for simplices with Size <= alpha_q, D[d] = number of simplices of D."""
    P, W, aq = quantise(xyz, radii, alpha)
    n = len(P)
    size = [dict() for _ in range(4)]  # simplices of D with their Size
    for d in (3, 2, 1, 0):
        for sigma in combinations(range(n), d + 1):
            if not _independent(P, sigma):
                continue
            c0 = orthocentre(P, W, sigma)
            gab = all(violation_sign(P, W, sigma, q, c0) >= 0 for q in range(n) if q not in sigma)
            if d == 3:
                if gab:
                    c = orthocentre(P, W, sigma)
                    size[3][sigma] = power(c, P, W, sigma[0])
                continue
            cof = [s for t, s in size[d + 1].items() if set(sigma) <= set(t)]
            if not gab and not cof:
                continue
            if gab:
                c = orthocentre(P, W, sigma)
                size[d][sigma] = power(c, P, W, sigma[0])
            else:
                size[d][sigma] = min(cof)
    K = [sorted((s, v) for s, v in size[d].items() if v <= aq) for d in range(4)]
    D = [len(size[d]) for d in range(4)]
    return K, D
