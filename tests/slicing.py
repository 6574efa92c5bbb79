"""Volume and boundary area of a union of balls by slicing: an independent
check of the inclusion-exclusion formulas, for a few dozen balls at most.

Each plane z = const cuts the balls in disks. The union's cross-section area
follows from Green's theorem over the arcs of the disk boundaries that no
other disk covers; Archimedes' hat-box theorem gives the boundary area, since
on a sphere of radius r the area between two planes is r times the azimuth
swept times their distance. Both are integrated over z with Gauss-Legendre
panels whose ends sit at every z where the arc structure changes (poles,
extremes of the circles where two spheres meet, triple points), after a
cosine change of variable that smooths the square-root behaviour there.
No alpha complex is involved.
"""
import math

import numpy as np

GL_X, GL_W = np.polynomial.legendre.leggauss(48)


def _slice(z, P, R):
    """Cross-section area of the union at height z and, per ball, the azimuth
    of its circle at that height that lies outside every other disk."""
    dz = z - P[:, 2]
    rho2 = R * R - dz * dz
    act = np.nonzero(rho2 > 0)[0]
    exposed = np.zeros(len(R))
    area = 0.0
    c = P[act, :2]
    rho = np.sqrt(rho2[act])
    for ii, i in enumerate(act):
        cov = []
        full = False
        for jj in range(len(act)):
            if jj == ii:
                continue
            D = math.hypot(c[jj, 0] - c[ii, 0], c[jj, 1] - c[ii, 1])
            if D >= rho[ii] + rho[jj] or D + rho[jj] <= rho[ii]:
                continue
            if D + rho[ii] <= rho[jj]:
                full = True
                break
            half = math.acos(max(-1.0, min(1.0, (rho[ii] ** 2 + D * D - rho[jj] ** 2) / (2 * rho[ii] * D))))
            mid = math.atan2(c[jj, 1] - c[ii, 1], c[jj, 0] - c[ii, 0])
            lo = (mid - half) % (2 * math.pi)
            hi = lo + 2 * half
            if hi > 2 * math.pi:
                cov += [(lo, 2 * math.pi), (0.0, hi - 2 * math.pi)]
            else:
                cov.append((lo, hi))
        if full:
            continue
        cov.sort()
        gaps = []
        pos = 0.0
        for lo, hi in cov:
            if lo > pos:
                gaps.append((pos, lo))
            pos = max(pos, hi)
        if pos < 2 * math.pi:
            gaps.append((pos, 2 * math.pi))
        cx, cy, r = c[ii, 0], c[ii, 1], rho[ii]
        for t1, t2 in gaps:
            exposed[i] += t2 - t1
            area += 0.5 * (r * r * (t2 - t1) + r * (cx * (math.sin(t2) - math.sin(t1)) - cy * (math.cos(t2) - math.cos(t1))))
    return area, exposed


def _breakpoints(P, R):
    zs = list(P[:, 2] - R) + list(P[:, 2] + R)
    n = len(R)
    for i in range(n):
        for j in range(i + 1, n):
            dv = P[j] - P[i]
            d = np.linalg.norm(dv)
            if d >= R[i] + R[j] or d <= abs(R[i] - R[j]):
                continue
            u = dv / d
            t = (d * d + R[i] ** 2 - R[j] ** 2) / (2 * d)
            a = math.sqrt(max(R[i] ** 2 - t * t, 0.0))
            oz = P[i, 2] + t * u[2]
            e = a * math.sqrt(max(1 - u[2] ** 2, 0.0))
            zs += [oz - e, oz + e]
            for k in range(j + 1, n):
                E = np.array([P[j] - P[i], P[k] - P[i]])
                rhs = 0.5 * (np.sum(E * E, axis=1) - np.array([R[j], R[k]]) ** 2 + R[i] ** 2)
                G = E @ E.T
                if abs(np.linalg.det(G)) < 1e-12:
                    continue
                z = np.linalg.solve(G, rhs) @ E
                rho2 = R[i] ** 2 - z @ z
                if rho2 <= 0:
                    continue
                nrm = np.cross(E[0], E[1])
                nrm /= np.linalg.norm(nrm)
                y = P[i] + z
                zs += [y[2] + math.sqrt(rho2) * nrm[2], y[2] - math.sqrt(rho2) * nrm[2]]
    return np.unique(np.array(zs))


def union_volume_area(xyz, radii, nodes=48):
    """(V, A) of the union of the balls, by quadrature over z with `nodes`
    Gauss-Legendre nodes per panel."""
    gx, gw = (GL_X, GL_W) if nodes == 48 else np.polynomial.legendre.leggauss(nodes)
    P = np.asarray(xyz, dtype=np.float64)
    R = np.asarray(radii, dtype=np.float64)
    zb = _breakpoints(P, R)
    V = 0.0
    expo = np.zeros(len(R))
    for z0, z1 in zip(zb[:-1], zb[1:]):
        if z1 - z0 <= 0:
            continue
        # z = z0 + (z1 - z0) (1 - cos(pi s)) / 2, s in [0, 1]
        s = 0.5 * (gx + 1.0)
        w = 0.5 * gw
        for sk, wk in zip(s, w):
            z = z0 + (z1 - z0) * 0.5 * (1 - math.cos(math.pi * sk))
            jac = (z1 - z0) * 0.5 * math.pi * math.sin(math.pi * sk)
            a, e = _slice(z, P, R)
            V += wk * jac * a
            expo += wk * jac * e
    return V, float(np.sum(R * expo))
