// Volume and boundary area of the union of the balls, from the alpha complex
// at alpha = 0, and their gradients (the complex held fixed).
//
// The union's measure is the alternating sum, over the simplices of the dual
// complex, of the measure of the intersection of their balls (the short
// inclusion-exclusion of Edelsbrunner, 1995); the paper names volume and area
// as what the alpha complex of a molecule is for (Sec. 1). Per simplex of k
// balls, with I the intersection:
//   vol(I)  = (1/3) [ sum_i r_i |P_i| - sum_{i<j} d_ij |F_ij| ]
// where P_i is the patch of sphere i on the boundary of I and F_ij the flat
// face of I on the radical plane of i and j once I is split by the farthest-
// power diagram of its balls (each piece coned from its own centre).
//   |P_i|  = r_i^2 (2 pi - sum of exterior corner angles) - r_i sum_j t_ij phi_ij
// by Gauss-Bonnet, t_ij being the signed distance from centre i to the plane
// and phi_ij the central angle of the boundary arc on the circle S_i & S_j.
// Gradients: d vol / d r_i = |P_i|; d vol / d p_i = sum_j |F_ij| u_ij; the
// boundary area moves by (2 / r_i) times the patch's (vector) area plus
// cot(psi/2) times the length (or int n ds) of each boundary arc of P_i, psi
// the interior dihedral angle of I there.
//
// One thread per simplex; float64 throughout. The coordinates are the
// caller's float64 ones (not the quantised values the complex was built
// from), so square roots and arc cosines are clamped to their domain.
#pragma once
#include "common.hpp"

namespace acx {

struct D3 {
    double x, y, z;
};
__device__ __forceinline__ D3 d3(double x, double y, double z) { return D3{x, y, z}; }
__device__ __forceinline__ D3 operator+(D3 a, D3 b) { return d3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ D3 operator-(D3 a, D3 b) { return d3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ D3 operator*(double s, D3 a) { return d3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ D3 cross(D3 a, D3 b) {
    return d3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ D3 unit(D3 a) {
    const double n = sqrt(dot(a, a));
    return n > 0 ? (1.0 / n) * a : a;
}
__device__ __forceinline__ double clamp1(double x) { return fmin(1.0, fmax(-1.0, x)); }

constexpr double PI = 3.14159265358979323846;

// Terms of corner c (ball c) of one simplex of K balls: what the patch P_c
// and the faces and arcs around it contribute. Summed over the corners:
// vol is the intersection's volume (each flat face's d |F| is split evenly
// between its two balls) and area the boundary area. The arc terms are
// computed only if GRAD.
struct CornerTerms {
    double vol;      // (1/3) [r_c |P_c| - 1/2 sum_b d_cb |F_cb|]
    double area;     // |P_c|
    D3 vec;          // vector area of P_c: sum_b |F_cb| u_cb
    double arc_len;  // sum over the arcs of P_c of cot(psi/2) * length
    D3 arc_vec;      // sum over the arcs of P_c of cot(psi/2) * int n_c ds
};

// Exterior angle at corner v of the patch on sphere (p, r) between the arcs
// cut by the planes with normals ua and ub.
__device__ __forceinline__ double corner_angle(D3 v, D3 p, double r, D3 ua, D3 ub) {
    const D3 n = (1.0 / r) * (v - p);
    const D3 ga = unit(ua - dot(ua, n) * n);
    const D3 gb = unit(ub - dot(ub, n) * n);
    return acos(clamp1(dot(ga, gb)));
}

// Vertex of the intersection of 4 balls on the power line of the triple
// opposite ball f: the triple point inside ball f. c is the ortho-centre.
__device__ __forceinline__ D3 triple_vertex(const D3 *P, int f, D3 c, double rho2) {
    const int t0 = f == 0 ? 1 : 0, t1 = f <= 1 ? 2 : 1, t2 = f == 3 ? 2 : 3;  // the balls other than f, ascending
    D3 nt = unit(cross(P[t1] - P[t0], P[t2] - P[t0]));
    if (dot(nt, P[f] - P[t0]) < 0) nt = -1.0 * nt;
    const double beta = dot(nt, c - P[t0]);
    const double tau = -beta + sqrt(fmax(beta * beta + rho2, 0.0));
    return c + tau * nt;
}

// The corner is ball 0: callers rotate the simplex's balls so that every
// index below is a compile-time constant (no scratch arrays).
template <int K, bool GRAD>
__device__ void corner_terms(const D3 *P, const double *R, CornerTerms &o) {
    constexpr int cc = 0;
    o.vec = d3(0, 0, 0);
    o.arc_len = 0;
    o.arc_vec = d3(0, 0, 0);
    if (K == 1) {
        o.vol = 4.0 / 3.0 * PI * R[0] * R[0] * R[0];
        o.area = 4.0 * PI * R[0] * R[0];
        return;
    }
    // point of equal power (in the plane of the centres when K = 3) and rho^2
    D3 c = P[0];
    double rho2 = 0;
    if (K >= 3) {
        const D3 e1 = P[1] - P[0], e2 = P[2] - P[0];
        const double h1 = 0.5 * (dot(e1, e1) - R[1] * R[1] + R[0] * R[0]);
        const double h2 = 0.5 * (dot(e2, e2) - R[2] * R[2] + R[0] * R[0]);
        D3 z;
        if (K == 3) {
            const double g11 = dot(e1, e1), g12 = dot(e1, e2), g22 = dot(e2, e2);
            const double det = g11 * g22 - g12 * g12;
            const double l1 = (h1 * g22 - h2 * g12) / det, l2 = (h2 * g11 - h1 * g12) / det;
            z = l1 * e1 + l2 * e2;
        } else {
            const D3 e3 = P[3] - P[0];
            const double h3 = 0.5 * (dot(e3, e3) - R[3] * R[3] + R[0] * R[0]);
            const D3 c23 = cross(e2, e3), c31 = cross(e3, e1), c12 = cross(e1, e2);
            z = (1.0 / dot(e1, c23)) * (h1 * c23 + h2 * c31 + h3 * c12);
        }
        c = P[0] + z;
        rho2 = R[0] * R[0] - dot(z, z);
    }
    const double rho = sqrt(fmax(rho2, 0.0));
    // K = 4: the triple points the corner's patch and arcs need (triples
    // containing ball 0), indexed by the ball opposite the triple
    D3 tv[4];
    if (K == 4) {
#pragma unroll
        for (int f = 1; f < 4; f++) tv[f] = triple_vertex(P, f, c, rho2);
    }
    const double rc = R[cc];
    double turn = 0, flat = 0, corner = 0;
#pragma unroll
    for (int b = 1; b < K; b++) {
        const D3 dv = P[b] - P[cc];
        const double d = sqrt(dot(dv, dv));
        const D3 u = (1.0 / d) * dv;
        const double tc = (d * d + rc * rc - R[b] * R[b]) / (2 * d);  // centre c to the plane, towards b
        const D3 oc = P[cc] + tc * u;                                  // centre of the circle S_c & S_b
        const double a2 = fmax(rc * rc - tc * tc, 0.0);
        const double rad = sqrt(a2);
        double phi, face;
        D3 mid = d3(0, 0, 0);
        if (K == 2) {
            phi = 2 * PI;
            face = PI * a2;
        } else if (K == 3) {
            const int e = 3 - cc - b;
            const D3 w = unit((P[e] - P[cc]) - dot(P[e] - P[cc], u) * u);
            const double sw = dot(c - oc, w);
            const double half = rad > 0 ? acos(clamp1(sw / rad)) : 0.0;
            face = a2 * half - sw * sqrt(fmax(a2 - sw * sw, 0.0));
            phi = 2 * half;
            mid = w;
        } else {
            // the other two balls e < f
            const int e = b == 1 ? 2 : 1, f = b == 3 ? 2 : 3;
            // the arc runs between the triple points of (c, b, e) and (c, b, f)
            const D3 q1 = tv[f], q2 = tv[e];
            D3 axis = u;
            if (dot(cross(q1 - c, q2 - c), u) < 0) axis = -1.0 * u;
            const D3 r1 = q1 - oc, r2 = q2 - oc;
            double ang = atan2(dot(cross(r1, r2), axis), dot(r1, r2));
            if (ang < 0) ang += 2 * PI;
            phi = rad > 0 ? ang : 0.0;
            face = 0.5 * (a2 * phi + dot(cross(oc - c, q2 - q1), axis));
            const D3 e1 = unit(r1);
            mid = cos(0.5 * phi) * e1 + sin(0.5 * phi) * cross(axis, e1);
        }
        flat += d * face;
        turn += tc * phi;
        o.vec = o.vec + face * u;
        if (GRAD) {
            const double cos_psi = -(rc * rc + R[b] * R[b] - d * d) / (2 * rc * R[b]);
            const double cot_half = sqrt(fmax(1 + cos_psi, 0.0) / fmax(1 - cos_psi, 1e-300));
            const double len = rad * phi;
            o.arc_len += cot_half * len;
            const D3 radial = (a2 * 2 * sin(0.5 * phi)) * mid;  // int (x - o) ds over the arc
            o.arc_vec = o.arc_vec + (cot_half / rc) * ((tc * len) * u + radial);
        }
    }
    // exterior angles at the corners of P_c
    if (K == 3) {
        const D3 nrm = unit(cross(P[1] - P[0], P[2] - P[0]));
        constexpr int j = 1, l = 2;
        const D3 uj = unit(P[j] - P[cc]), ul = unit(P[l] - P[cc]);
        corner = corner_angle(c + rho * nrm, P[cc], rc, uj, ul) + corner_angle(c - rho * nrm, P[cc], rc, uj, ul);
    }
    if (K == 4) {
#pragma unroll
        for (int f = 1; f < 4; f++) {
            const int j = f == 1 ? 2 : 1, l = f == 3 ? 2 : 3;  // the balls other than 0 and f
            corner += corner_angle(tv[f], P[cc], rc, unit(P[j] - P[cc]), unit(P[l] - P[cc]));
        }
    }
    o.area = rc * rc * (2 * PI - corner) - rc * turn;
    o.vol = (rc * o.area - 0.5 * flat) / 3.0;
}

// Balls of simplex s, rotated so that corner c comes first.
template <int K>
__device__ __forceinline__ void load_balls(const int *__restrict__ simp, long long s, int c0,
                                           const double *__restrict__ xyz, const double *__restrict__ rad, D3 *P,
                                           double *R) {
#pragma unroll
    for (int c = 0; c < K; c++) {
        const int id = simp[s * K + (c0 + c) % K];
        const double *p = xyz + 3LL * id;
        P[c] = d3(p[0], p[1], p[2]);
        R[c] = rad[id];
    }
}

constexpr int MEASURE_BLOCK = 256;

// One thread per (simplex, corner) of dimension K - 1 (thread t: simplex
// t / K, corner t % K). Per block: the signed sums of the corners' volume
// and patch-area parts, written to part[2 * block] and part[2 * block + 1].
template <int K>
__global__ void __launch_bounds__(MEASURE_BLOCK) k_measure_fwd(const int *__restrict__ simp, long long m,
                                                                const double *__restrict__ xyz,
                                                                const double *__restrict__ rad, double *__restrict__ part) {
    __shared__ double sv[MEASURE_BLOCK / WAVE], sa[MEASURE_BLOCK / WAVE];
    const long long t = (long long)blockIdx.x * MEASURE_BLOCK + threadIdx.x;
    double v = 0, a = 0;
    if (t < m * K) {
        D3 P[K];
        double R[K];
        load_balls<K>(simp, t / K, (int)(t % K), xyz, rad, P, R);
        CornerTerms ct;
        corner_terms<K, false>(P, R, ct);
        v = ct.vol;
        a = ct.area;
        if ((K - 1) & 1) {
            v = -v;
            a = -a;
        }
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        v += __shfl_down(v, off, WAVE);
        a += __shfl_down(a, off, WAVE);
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        sv[w] = v;
        sa[w] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tv = 0, ta = 0;
        for (int k = 0; k < MEASURE_BLOCK / WAVE; k++) {
            tv += sv[k];
            ta += sa[k];
        }
        part[2 * blockIdx.x] = tv;
        part[2 * blockIdx.x + 1] = ta;
    }
}

__global__ void __launch_bounds__(MEASURE_BLOCK) k_measure_total(const double *__restrict__ part, int nb,
                                                                  double *__restrict__ out) {
    __shared__ double sv[MEASURE_BLOCK], sa[MEASURE_BLOCK];
    double v = 0, a = 0;
    for (int b = threadIdx.x; b < nb; b += MEASURE_BLOCK) {
        v += part[2 * b];
        a += part[2 * b + 1];
    }
    sv[threadIdx.x] = v;
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int h = MEASURE_BLOCK / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            sv[threadIdx.x] += sv[threadIdx.x + h];
            sa[threadIdx.x] += sa[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sv[0];
        out[1] = sa[0];
    }
}

// Per incidence slot (simplex s, corner c at slot base + s*K + c; one thread
// each): the corner's contribution gV * d(V)/d(p, r) + gA * d(A)/d(p, r),
// as (x, y, z, r), with (gV, gA) = (g[0], g[1]) read from device memory.
// VA: the block's signed volume and area parts too, as k_measure_fwd writes
// them (forward and backward in one pass).
template <int K, bool VA>
__global__ void __launch_bounds__(MEASURE_BLOCK) k_measure_bwd(const int *__restrict__ simp, long long m,
                                                                const double *__restrict__ xyz,
                                                                const double *__restrict__ rad,
                                                                const double *__restrict__ g,
                                                                double4 *__restrict__ contrib,
                                                                double *__restrict__ part) {
    const long long t = (long long)blockIdx.x * MEASURE_BLOCK + threadIdx.x;
    const double sg = ((K - 1) & 1) ? -1.0 : 1.0;
    double v = 0, a = 0;
    if (t < m * K) {
        const double gV = g[0], gA = g[1];
        D3 P[K];
        double R[K];
        load_balls<K>(simp, t / K, (int)(t % K), xyz, rad, P, R);
        CornerTerms ct;
        corner_terms<K, true>(P, R, ct);
        const double ir = 2.0 / R[0];
        const D3 gx = (sg * gV) * ct.vec + (sg * gA) * (ir * ct.vec + ct.arc_vec);
        const double gr = sg * (gV * ct.area + gA * (ir * ct.area + ct.arc_len));
        contrib[t] = make_double4(gx.x, gx.y, gx.z, gr);
        v = sg * ct.vol;
        a = sg * ct.area;
    }
    if (!VA) return;
    __shared__ double sv[MEASURE_BLOCK / WAVE], sa[MEASURE_BLOCK / WAVE];
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        v += __shfl_down(v, off, WAVE);
        a += __shfl_down(a, off, WAVE);
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        sv[w] = v;
        sa[w] = a;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tv = 0, ta = 0;
        for (int k = 0; k < MEASURE_BLOCK / WAVE; k++) {
            tv += sv[k];
            ta += sa[k];
        }
        part[2 * blockIdx.x] = tv;
        part[2 * blockIdx.x + 1] = ta;
    }
}

// vstart[i] = first position of vertex i in the sorted incidence keys (i in [0, n]).
__global__ void __launch_bounds__(MEASURE_BLOCK) k_incidence_start(const unsigned *__restrict__ key, long long M, int n,
                                                                    int *__restrict__ vstart) {
    const long long i = (long long)blockIdx.x * MEASURE_BLOCK + threadIdx.x;
    if (i > n) return;
    long long lo = 0, hi = M;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)key[mid] < i) lo = mid + 1; else hi = mid;
    }
    vstart[i] = (int)lo;
}

// Gradient of ball i: the sum of its incidence slots' contributions, in slot
// order (deterministic).
__global__ void __launch_bounds__(MEASURE_BLOCK) k_measure_gather(const int *__restrict__ vstart,
                                                                   const int *__restrict__ slot,
                                                                   const double4 *__restrict__ contrib, int n,
                                                                   double *__restrict__ dxyz, double *__restrict__ dr) {
    const int i = blockIdx.x * MEASURE_BLOCK + threadIdx.x;
    if (i >= n) return;
    double gx = 0, gy = 0, gz = 0, gr = 0;
    for (int q = vstart[i]; q < vstart[i + 1]; q++) {
        const double4 c = contrib[slot[q]];
        gx += c.x;
        gy += c.y;
        gz += c.z;
        gr += c.w;
    }
    dxyz[3LL * i] = gx;
    dxyz[3LL * i + 1] = gy;
    dxyz[3LL * i + 2] = gz;
    dr[i] = gr;
}

__global__ void __launch_bounds__(MEASURE_BLOCK) k_iota(int *__restrict__ p, long long m) {
    const long long i = (long long)blockIdx.x * MEASURE_BLOCK + threadIdx.x;
    if (i < m) p[i] = (int)i;
}

}  // namespace acx
