"""Euler characteristic of a union of balls from its Cech nerve (tiny inputs).

Independent of oracle/ and of the HIP path. The grown balls B(p_i, sqrt(W_i +
alpha)) meet in a common point iff min_p max_i (|p - p_i|^2 - W_i) <= alpha.
The minimiser of that strictly convex function is the ortho-centre of its
active set A, and lies in conv(A) (first-order optimality), so it is found by
trying every affinely independent subset. Helly's theorem in R^3: a family of
convex sets has a common point iff every four of them do, so nerve simplices
are grown from pairs, triples and quadruples. The nerve theorem then gives
chi(union) = sum over nerve simplices S of (-1)^(|S|-1); the alpha complex is
homotopy equivalent to the same union (it is the nerve of the balls clipped
to their power cells).
"""
from __future__ import annotations

from fractions import Fraction
from itertools import combinations

import bruteforce as bf


def minmax_power(P, W, S):
    """min_p max_{i in S} pi(p, b_i), exact (inputs assumed free of ties)."""
    best = None
    for k in range(1, len(S) + 1):
        for T in combinations(S, k):
            if not bf._independent(P, T):
                continue
            c = bf.orthocentre(P, W, T)
            # barycentric coordinates of c in T
            p0 = P[T[0]]
            if k > 1:
                a = [bf._sub(P[v], p0) for v in T[1:]]
                G = [[bf._dot(ai, aj) for aj in a] for ai in a]
                rhs = [sum((c[m] - p0[m]) * ai[m] for m in range(3)) for ai in a]
                lam = bf._solve(G, rhs)
                bary = [1 - sum(lam)] + lam
                if any(x < 0 for x in bary):
                    continue
            val = bf.power(c, P, W, T[0])
            if all(bf.power(c, P, W, j) <= val for j in S if j not in T):
                if best is None or val < best:
                    best = val
    return best


def union_euler(xyz, radii, alpha):
    P, W, aq = bf.quantise(xyz, radii, alpha)
    n = len(P)
    memo = {}

    def meets(S):
        if S not in memo:
            memo[S] = minmax_power(P, W, S) <= aq
        return memo[S]

    chi = 0

    def grow(S):
        nonlocal chi
        chi += 1 if len(S) % 2 == 1 else -1
        for j in range(S[-1] + 1, n):
            T = S + (j,)
            ok = True
            for m in range(1, min(3, len(S)) + 1):
                for sub in combinations(S, m):
                    if not meets(tuple(sorted(sub + (j,)))):
                        ok = False
                        break
                if not ok:
                    break
            if ok:
                grow(T)

    for i in range(n):
        if -W[i] <= aq:
            grow((i,))
    return chi
