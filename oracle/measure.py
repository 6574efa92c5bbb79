"""Volume and surface area of a union of balls from its alpha complex at
alpha = 0, and their gradients. Test infrastructure only, like the rest of
this package.

The paper motivates the alpha complex by the volume and area of molecules
(Sec. 1). The method here is the short inclusion-exclusion over the dual
complex K (Edelsbrunner 1995, "The union of balls and its dual shape"):

    V = sum over sigma in K of (-1)^dim(sigma) vol(intersection of the balls of sigma)
    A = sum over sigma in K, over i in sigma, of (-1)^dim(sigma) area(S_i inside the other balls of sigma)

Every term is a closed form in float64, written out below for 1 to 4 balls.
The pieces of one intersection I = B_0 & ... & B_{k-1}:

* Farthest-power split. Where ball i has the largest power, I coincides with
  B_i; so I splits into pieces R_i bounded by the sphere patch P_i = S_i & I
  and by flat faces F_ij on the radical planes H_ij. Coning each piece from
  its own centre gives vol(I) = (1/3) [sum_i r_i |P_i| - sum_{i<j} d_ij |F_ij|].
* Faces. F_ij is the radical disk of i and j cut by the half-planes where i
  keeps the largest power: the whole disk (2 balls), a circular segment cut
  by the power line of the triangle (3 balls), the fan from the orthocentre
  over the arc between two triple points (4 balls).
* Patches. P_i is bounded by arcs of the circles S_i & S_j; its area follows
  from Gauss-Bonnet: |P_i| = r_i^2 (2 pi - sum of exterior corner angles)
  - r_i sum_arcs t_ij phi_ij, with t_ij the signed distance from the centre
  of i to H_ij and phi_ij the central angle of the arc.
* Gradients (the complex held fixed). dV/dr_i is the patch area, dV/dp_i
  its vector area sum_j |F_ij| u_ij. The first variation of the boundary area
  of I when sphere i moves with normal speed v is int_{P_i} (2/r_i) v dA plus,
  along each boundary arc of P_i, int v cot(psi/2) ds, psi being the interior
  dihedral angle of I along that arc.

Simplices of K_0 have OrthoSize <= 0 (a face's OrthoSize never exceeds its
cofaces'), so their balls share a point of equal power: the triple points and
the orthocentre exist. Inputs are the float64 coordinates themselves (not the
quantised ones the complex was built from), so square roots and arc cosines
are clamped at the boundary of their domain.
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def _unit(v):
    n = np.linalg.norm(v, axis=-1, keepdims=True)
    return v / np.where(n > 0, n, 1.0)


def _radical_point(P, R):
    """Point of equal power of k = 3 balls (in the plane of the centres) or
    k = 4 balls, and minus that power (rho^2). P: (m,k,3), R: (m,k)."""
    E = P[:, 1:, :] - P[:, :1, :]                       # (m,k-1,3) edges from ball 0
    rhs = 0.5 * (np.einsum("mkc,mkc->mk", E, E) - R[:, 1:] ** 2 + R[:, :1] ** 2)
    if P.shape[1] == 3:
        G = np.einsum("mkc,mlc->mkl", E, E)             # Gram matrix of the two edges
        lam = np.linalg.solve(G, rhs[..., None])[..., 0]
        z = np.einsum("mk,mkc->mc", lam, E)
    else:
        z = np.linalg.solve(E, rhs[..., None])[..., 0]
    rho2 = R[:, 0] ** 2 - np.einsum("mc,mc->m", z, z)
    return P[:, 0, :] + z, rho2


def _pairs(k):
    return [(a, b) for a in range(k) for b in range(a + 1, k)]


def _ccw_angle(x, y, axis):
    """Angle in [0, 2 pi) that turns x into y counter-clockwise about axis."""
    ang = np.arctan2(np.einsum("mc,mc->m", np.cross(x, y), axis), np.einsum("mc,mc->m", x, y))
    return np.where(ang < 0, ang + 2 * math.pi, ang)


def _corner_angle(v, p, r, ua, ub):
    """Exterior angle of the patch on sphere (p, r) at corner v, between the
    arcs cut by planes with normals ua and ub: the angle between the two
    normals projected on the tangent plane at v."""
    n = (v - p) / r[:, None]
    ga = _unit(ua - np.einsum("mc,mc->m", ua, n)[:, None] * n)
    gb = _unit(ub - np.einsum("mc,mc->m", ub, n)[:, None] * n)
    return np.arccos(np.clip(np.einsum("mc,mc->m", ga, gb), -1.0, 1.0))


def intersection_terms(P, R):
    """Closed-form pieces of the intersection of the k balls of each of m
    simplices. P: (m,k,3) centres, R: (m,k) radii, 1 <= k <= 4.

    Returns vol (m,), area (m,k) = |P_i|, vec (m,k,3) = vector area of P_i,
    arc_len (m,k) = sum over boundary arcs of P_i of cot(psi/2) * length, and
    arc_vec (m,k,3) = sum over those arcs of cot(psi/2) * int n_i ds.
    """
    P = np.asarray(P, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    m, k = R.shape
    area = np.zeros((m, k))
    vec = np.zeros((m, k, 3))
    arc_len = np.zeros((m, k))
    arc_vec = np.zeros((m, k, 3))
    if k == 1:
        return FOUR_PI / 3 * R[:, 0] ** 3, FOUR_PI * R ** 2, vec, arc_len, arc_vec

    if k >= 3:
        centre, rho2 = _radical_point(P, R)
        rho = np.sqrt(np.maximum(rho2, 0.0))
    corner = np.zeros((m, k))      # sum of exterior corner angles of each patch
    turn = np.zeros((m, k))        # sum of t_ij * phi_ij over the arcs of each patch
    flat = np.zeros(m)             # sum of d_ij * |F_ij|

    if k == 3:
        nrm = _unit(np.cross(P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]))
        corners = [centre + rho[:, None] * nrm, centre - rho[:, None] * nrm]
    if k == 4:
        # one vertex of I per triple: the triple point inside the fourth ball
        tri_vertex = {}
        for opp in range(4):
            t = [x for x in range(4) if x != opp]
            nt = _unit(np.cross(P[:, t[1]] - P[:, t[0]], P[:, t[2]] - P[:, t[0]]))
            side = np.sign(np.einsum("mc,mc->m", nt, P[:, opp] - P[:, t[0]]))
            nt = nt * np.where(side == 0, 1.0, side)[:, None]      # towards the fourth centre
            beta = np.einsum("mc,mc->m", nt, centre - P[:, t[0]])
            tau = -beta + np.sqrt(np.maximum(beta * beta + rho2, 0.0))
            tri_vertex[tuple(t)] = centre + tau[:, None] * nt

    for a, b in _pairs(k):
        dv = P[:, b] - P[:, a]
        d = np.linalg.norm(dv, axis=1)
        u = dv / d[:, None]
        ta = (d * d + R[:, a] ** 2 - R[:, b] ** 2) / (2 * d)    # p_a to H_ab, towards b
        tb = d - ta
        o = P[:, a] + ta[:, None] * u                             # centre of the circle S_a & S_b
        a2 = np.maximum(R[:, a] ** 2 - ta * ta, 0.0)
        rad = np.sqrt(a2)
        others = [x for x in range(k) if x not in (a, b)]
        if k == 2:
            phi = np.full(m, 2 * math.pi)
            face = math.pi * a2
            mid = np.zeros((m, 3))
        elif k == 3:
            c = others[0]
            w = _unit((P[:, c] - P[:, a]) - np.einsum("mc,mc->m", P[:, c] - P[:, a], u)[:, None] * u)
            s = np.einsum("mc,mc->m", centre - o, w)              # power line's offset from o
            half = np.arccos(np.clip(s / np.where(rad > 0, rad, 1.0), -1.0, 1.0))
            half = np.where(rad > 0, half, 0.0)
            face = a2 * half - s * np.sqrt(np.maximum(a2 - s * s, 0.0))
            phi = 2 * half
            mid = w
        else:
            e, f = others
            q1 = tri_vertex[tuple(sorted((a, b, e)))]
            q2 = tri_vertex[tuple(sorted((a, b, f)))]
            # orient the plane so that the wedge c->q1, c->q2 turns counter-clockwise
            sgn = np.sign(np.einsum("mc,mc->m", np.cross(q1 - centre, q2 - centre), u))
            axis = u * np.where(sgn == 0, 1.0, sgn)[:, None]
            phi = np.where(rad > 0, _ccw_angle(q1 - o, q2 - o, axis), 0.0)
            face = 0.5 * (a2 * phi + np.einsum("mc,mc->m", np.cross(o - centre, q2 - q1), axis))
            e1 = _unit(q1 - o)
            mid = np.cos(phi / 2)[:, None] * e1 + np.sin(phi / 2)[:, None] * np.cross(axis, e1)
        flat += d * face
        turn[:, a] += ta * phi
        turn[:, b] += tb * phi
        vec[:, a] += face[:, None] * u
        vec[:, b] -= face[:, None] * u
        # interior dihedral angle psi of I along the arc: cos psi = -n_a . n_b
        cos_psi = -(R[:, a] ** 2 + R[:, b] ** 2 - d * d) / (2 * R[:, a] * R[:, b])
        cot_half = np.sqrt(np.maximum(1 + cos_psi, 0.0) / np.maximum(1 - cos_psi, 1e-300))
        arc_len[:, a] += cot_half * rad * phi
        arc_len[:, b] += cot_half * rad * phi
        radial = (a2 * 2 * np.sin(phi / 2))[:, None] * mid       # int (x - o) ds over the arc
        axial = (rad * phi)[:, None] * u
        arc_vec[:, a] += cot_half[:, None] * (ta[:, None] * axial + radial) / R[:, a][:, None]
        arc_vec[:, b] += cot_half[:, None] * (-tb[:, None] * axial + radial) / R[:, b][:, None]

    if k == 3:
        for i in range(3):
            j, l = [x for x in range(3) if x != i]
            uj, ul = _unit(P[:, j] - P[:, i]), _unit(P[:, l] - P[:, i])
            for v in corners:
                corner[:, i] += _corner_angle(v, P[:, i], R[:, i], uj, ul)
    if k == 4:
        for t, v in tri_vertex.items():
            for i in t:
                j, l = [x for x in t if x != i]
                uj, ul = _unit(P[:, j] - P[:, i]), _unit(P[:, l] - P[:, i])
                corner[:, i] += _corner_angle(v, P[:, i], R[:, i], uj, ul)

    area = R ** 2 * (2 * math.pi - corner) - R * turn
    vol = (np.einsum("mk,mk->m", R, area) - flat) / 3.0
    return vol, area, vec, arc_len, arc_vec


def union_measure(simplices, xyz, radii, with_grad: bool = False):
    """V and A of the union of the balls from K_0 given as four simplex arrays
    of input ids (counts x (dim+1)). With with_grad, also returns dV/dx (n,3),
    dV/dr (n,), dA/dx (n,3), dA/dr (n,), with the complex held fixed."""
    xyz = np.asarray(xyz, dtype=np.float64)
    radii = np.asarray(radii, dtype=np.float64)
    n = len(radii)
    V = 0.0
    A = 0.0
    gVx = np.zeros((n, 3))
    gVr = np.zeros(n)
    gAx = np.zeros((n, 3))
    gAr = np.zeros(n)
    for dim in range(4):
        s = np.asarray(simplices[dim], dtype=np.int64).reshape(-1, dim + 1)
        if len(s) == 0:
            continue
        sign = -1.0 if dim % 2 else 1.0
        vol, area, vec, arc_len, arc_vec = intersection_terms(xyz[s], radii[s])
        V += sign * vol.sum()
        A += sign * area.sum()
        if with_grad:
            r = radii[s]
            for c in range(dim + 1):
                idx = s[:, c]
                np.add.at(gVr, idx, sign * area[:, c])
                np.add.at(gVx, idx, sign * vec[:, c])
                np.add.at(gAr, idx, sign * (2 * area[:, c] / r[:, c] + arc_len[:, c]))
                np.add.at(gAx, idx, sign * (2 * vec[:, c] / r[:, c][:, None] + arc_vec[:, c]))
    if with_grad:
        return V, A, gVx, gVr, gAx, gAr
    return V, A
