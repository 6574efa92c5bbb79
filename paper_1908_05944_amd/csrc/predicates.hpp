// Exact geometric predicates for the alpha-complex kernels (gfx950 device code).
//
// Notation (Masood, Ray, Natarajan, Sec. 2.2-2.4): ball b_i has integer centre
// X_i (milli-angstrom) and weight W_i = R_i^2; pi(p, b_i) = |p - X_i|^2 - W_i.
// For a simplex sigma = (v0..vd) put the origin at v0: a_k = X_vk - X_v0 and
// beta_k = |a_k|^2 - W_vk + W_v0. Its ortho-centre c (relative to v0) lies in
// the affine hull of sigma with 2 a_k . c = beta_k (condition AC1), and
// OrthoSize(sigma) = |c|^2 - W_v0 (Sec. 2.3).
//
//   d = 1: c = beta a / (2 |a|^2)
//   d = 2: n = a1 x a2, c = (beta1 (a2 x n) + beta2 (n x a1)) / (2 |n|^2)
//   d = 3: D = det[a1; a2; a3], c = (beta1 a2xa3 + beta2 a3xa1 + beta3 a1xa2) / (2 D)
//
// AC3 (Step 1 of Sec. 3.1) is the unperturbed closed test OrthoSize <= alpha.
// AC2 at c (Steps 2-5): a query ball q with b = X_q - X_v0 and
// gamma = |b|^2 - W_q + W_v0 violates iff pi(c, q) < pi(c, v0), i.e. iff
// gamma - 2 c.b < 0; each test below evaluates a positive multiple P of that
// difference. Exact ties are broken by simulation of simplicity: W_i -> W_i + eps_i
// with eps ranked by input index, lower index dominating; P is affine in the
// weights, so a zero P takes the sign of its first non-zero weight partial in
// input-index order (the W_q partial is never zero).
//
// Arithmetic: every relative coordinate of a candidate is below 2^14 in
// magnitude (edge length <= 2 sqrt(W_max + alpha) < 2^14), so d <= 1 runs in
// exact int64 and d = 2, 3 use a floating-point filter with a static error
// bound and an exact __int128 fallback. The bounds allow for fused
// multiply-add contraction (a contracted a*b+c rounds once instead of twice).
// The exact integers the filters start from are formed in the cheapest exact
// way: products of two coordinate differences (below 2^28) as 24-bit
// multiplies (full rate; a 32-bit multiply issues at a quarter of that), and
// products of a difference with a cross-product component (below 2^43) as
// float64 products, which are exact below 2^53; the values, and so every
// filter decision, are those of the plain integer formulas.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acx {

typedef __int128 i128;
typedef long long i64;

// 2^-53, the unit roundoff of float64.
#define ACX_U 1.1102230246251565e-16

struct PredParams {
    i64 aq;        // alpha in mA^2
    i64 sg2;       // W_max + aq: squared grown radius bound
    double bmax;   // bound on |b_i| for AC2 queries: 2 sqrt(sg2)
    double gmax;   // bound on |gamma|: 4 sg2 + W_max
    i64 sgc;       // ceil(sqrt(sg2))
    int force_exact;
};

// a * b for |a|, |b| < 2^23 and |a b| < 2^31 (exact)
__device__ __forceinline__ int m24(int a, int b) { return __mul24(a, b); }

struct Counters {
    unsigned long long exact_fallbacks;
    int dup;       // duplicate centres seen
    int lookup;    // a facet lookup failed (must not happen)
    int Nn, E, T, Q;  // neighbour entries and candidate counts, copied from scan totals
    int m0, m1, m2, m3;
    int overflow;  // a single-pass stage ran out of its per-block room (then the two-pass path runs)
    // recorded builds only (sizes fixed in advance): the live candidate
    // counts the later launches read, and why the build stopped (0: it did not)
    int El, Tl, Ql;
    int stop;
};

__device__ __forceinline__ int sgn128(i128 v) { return (v > 0) - (v < 0); }
__device__ __forceinline__ int sgn64(i64 v) { return (v > 0) - (v < 0); }

// First non-zero partial in input-index order.
template <int K>
__device__ __forceinline__ int sos_first(const int (&ids)[K], const i128 (&coef)[K]) {
    unsigned used = 0;
    for (int s = 0; s < K; s++) {
        int best = -1;
        for (int t = 0; t < K; t++)
            if (!((used >> t) & 1u) && (best < 0 || ids[t] < ids[best])) best = t;
        used |= 1u << best;
        if (coef[best] != 0) return coef[best] > 0 ? 1 : -1;
    }
    return 0;
}

__device__ __forceinline__ void note_fallback(Counters *cnt) { atomicAdd(&cnt->exact_fallbacks, 1ull); }

// ---------------------------------------------------------------------------
// Vertex (d = 0): AC2 at the ball's own centre. P = |b|^2 - W_q + W_v.
// Sorted-order indices are passed with the input-order map `perm`; input ids
// are read only when simulation of simplicity has to decide. Queries come
// from neighbour lists, so |b| <= 2 sqrt(sg2) < 2^14 and P fits in int32.
__device__ __forceinline__ int vertex_violation_sign(int4 v, int sv, int4 q, int sq, const int *perm) {
    const int bx = q.x - v.x, by = q.y - v.y, bz = q.z - v.z;
    const int P = m24(bx, bx) + m24(by, by) + m24(bz, bz) - q.w + v.w;
    if (P) return P > 0 ? 1 : -1;
    // partials: W_q -> -1, W_v -> +1
    return perm[sq] < perm[sv] ? -1 : 1;
}

// ---------------------------------------------------------------------------
// Edge (d = 1). |a| < 2^14, so |a|^2 and beta fit in int32; products are
// filtered in float64 and decided exactly in int64 when the filter cannot.
struct Edge {
    int4 v0;
    int ax, ay, az, den, beta;
};

__device__ __forceinline__ Edge edge_setup(int4 v0, int4 v1) {
    Edge e;
    e.v0 = v0;
    e.ax = v1.x - v0.x; e.ay = v1.y - v0.y; e.az = v1.z - v0.z;
    e.den = m24(e.ax, e.ax) + m24(e.ay, e.ay) + m24(e.az, e.az);
    e.beta = e.den - v1.w + v0.w;
    return e;
}

// AC3 for an edge: beta^2 <= 4 |a|^2 (W0 + alpha). Equivalent to the grown
// spheres (radius^2 W + alpha) crossing. Needs |a|^2 <= 4 sg2 (checked by caller).
__device__ __forceinline__ bool edge_ac3(const Edge &e, i64 aq) {
    const i64 rhs = 4 * (i64)e.den * ((i64)e.v0.w + aq);
    return (i64)e.beta * e.beta <= rhs;
}

__device__ __forceinline__ double edge_orthosize(const Edge &e) {
    const double b = (double)e.beta;
    return b * b / (4.0 * (double)e.den) - (double)e.v0.w;
}

// Floating-point filter of edge_violation_sign: the sign of P when the
// rounding bound certifies it, 0 when the exact path has to decide.
__device__ __forceinline__ int edge_violation_filter(const Edge &e, int4 q) {
    const int bx = q.x - e.v0.x, by = q.y - e.v0.y, bz = q.z - e.v0.z;
    const int gam = m24(bx, bx) + m24(by, by) + m24(bz, bz) - q.w + e.v0.w;
    const int t = m24(e.ax, bx) + m24(e.ay, by) + m24(e.az, bz);
    const double p1 = (double)e.den * (double)gam, p2 = (double)e.beta * (double)t;
    const double P = p1 - p2;
    const double eb = 4.0 * ACX_U * (fabs(p1) + fabs(p2));
    return (P > eb) - (P < -eb);
}

// P = |a|^2 gamma - beta (a.b)
__device__ __forceinline__ int edge_violation_sign(const Edge &e, int s0, int s1, int4 q, int sq, const int *perm,
                                                   int force_exact) {
    const int bx = q.x - e.v0.x, by = q.y - e.v0.y, bz = q.z - e.v0.z;
    const int gam = m24(bx, bx) + m24(by, by) + m24(bz, bz) - q.w + e.v0.w;
    const int t = m24(e.ax, bx) + m24(e.ay, by) + m24(e.az, bz);
    if (!force_exact) {
        const double p1 = (double)e.den * (double)gam, p2 = (double)e.beta * (double)t;
        const double P = p1 - p2;
        const double eb = 4.0 * ACX_U * (fabs(p1) + fabs(p2));
        if (P > eb) return 1;
        if (P < -eb) return -1;
    }
    const i64 P = (i64)e.den * gam - (i64)e.beta * t;
    if (P) return P > 0 ? 1 : -1;
    int ids[3] = {perm[sq], perm[s1], perm[s0]};
    i128 coef[3] = {-(i128)e.den, (i128)t, (i128)e.den - t};
    return sos_first<3>(ids, coef);
}

// ---------------------------------------------------------------------------
// Triangle (d = 2).
struct Tri {
    int4 v0;
    int nx, ny, nz;          // n = a1 x a2 (components below 2^29)
    double ux, uy, uz;       // a2 x n (exact integers below 2^44)
    double wx, wy, wz;       // n x a1
    int b1, b2;              // beta1, beta2
    i64 den;                 // |n|^2
    double Mx, My, Mz;       // b1 u + b2 w (rounded)
    double eP;               // filter bound for AC2
};

// a * c - b * d for exact integer products below 2^53 (the result too): exact
__device__ __forceinline__ double cross_d(int a, int c, int b, int d) {
    return (double)a * (double)c - (double)b * (double)d;
}

__device__ __forceinline__ Tri tri_setup(int4 v0, int4 v1, int4 v2, const PredParams &pp) {
    Tri t;
    t.v0 = v0;
    const int a1x = v1.x - v0.x, a1y = v1.y - v0.y, a1z = v1.z - v0.z;
    const int a2x = v2.x - v0.x, a2y = v2.y - v0.y, a2z = v2.z - v0.z;
    t.nx = m24(a1y, a2z) - m24(a1z, a2y);
    t.ny = m24(a1z, a2x) - m24(a1x, a2z);
    t.nz = m24(a1x, a2y) - m24(a1y, a2x);
    t.ux = cross_d(a2y, t.nz, a2z, t.ny);
    t.uy = cross_d(a2z, t.nx, a2x, t.nz);
    t.uz = cross_d(a2x, t.ny, a2y, t.nx);
    t.wx = cross_d(t.ny, a1z, t.nz, a1y);
    t.wy = cross_d(t.nz, a1x, t.nx, a1z);
    t.wz = cross_d(t.nx, a1y, t.ny, a1x);
    t.b1 = m24(a1x, a1x) + m24(a1y, a1y) + m24(a1z, a1z) - v1.w + v0.w;
    t.b2 = m24(a2x, a2x) + m24(a2y, a2y) + m24(a2z, a2z) - v2.w + v0.w;
    t.den = (i64)t.nx * t.nx + (i64)t.ny * t.ny + (i64)t.nz * t.nz;
    const double b1 = (double)t.b1, b2 = (double)t.b2;
    t.Mx = b1 * t.ux + b2 * t.wx;
    t.My = b1 * t.uy + b2 * t.wy;
    t.Mz = b1 * t.uz + b2 * t.wz;
    const double ab1 = fabs(b1), ab2 = fabs(b2);
    const double Mabs = ab1 * (fabs(t.ux) + fabs(t.uy) + fabs(t.uz)) + ab2 * (fabs(t.wx) + fabs(t.wy) + fabs(t.wz));
    t.eP = 16.0 * ACX_U * ((double)t.den * pp.gmax + pp.bmax * Mabs);
    return t;
}

__device__ __forceinline__ bool tri_degenerate(const Tri &t) { return t.nx == 0 && t.ny == 0 && t.nz == 0; }

// Candidate test of a triangle (Step 1): not collinear, and AC3 in Gram form,
// beta^T adj(G) beta <= 4 det(G) (W0 + alpha) with G the Gram matrix of
// (a1, a2) and det(G) = |n|^2, from the edge vectors only (the AC2 data of
// tri_setup is not needed to decide candidacy).
__device__ __forceinline__ bool tri_candidate(int4 v0, int4 v1, int4 v2, const PredParams &pp, Counters *cnt) {
    const int a1x = v1.x - v0.x, a1y = v1.y - v0.y, a1z = v1.z - v0.z;
    const int a2x = v2.x - v0.x, a2y = v2.y - v0.y, a2z = v2.z - v0.z;
    const int nx = m24(a1y, a2z) - m24(a1z, a2y), ny = m24(a1z, a2x) - m24(a1x, a2z),
              nz = m24(a1x, a2y) - m24(a1y, a2x);
    if (nx == 0 && ny == 0 && nz == 0) return false;
    const i64 den = (i64)nx * nx + (i64)ny * ny + (i64)nz * nz;
    const int g11 = m24(a1x, a1x) + m24(a1y, a1y) + m24(a1z, a1z);
    const int g12 = m24(a1x, a2x) + m24(a1y, a2y) + m24(a1z, a2z);
    const int g22 = m24(a2x, a2x) + m24(a2y, a2y) + m24(a2z, a2z);
    const int b1 = g11 - v1.w + v0.w, b2 = g22 - v2.w + v0.w;
    const i64 wa = v0.w + pp.aq;
    if (!pp.force_exact) {
        const double db1 = (double)b1, db2 = (double)b2;
        const double q1 = (double)g22 * (db1 * db1), q2 = 2.0 * (double)g12 * (db1 * db2), q3 = (double)g11 * (db2 * db2);
        const double Q = q1 - q2 + q3;
        const double R = 4.0 * (double)den * (double)wa;
        const double e = 16.0 * ACX_U * (fabs(q1) + fabs(q2) + fabs(q3) + fabs(R));
        const double diff = Q - R;
        if (diff < -e) return true;
        if (diff > e) return false;
        note_fallback(cnt);
    }
    const i128 Q = (i128)g22 * b1 * b1 - (i128)2 * g12 * b1 * b2 + (i128)g11 * b2 * b2;
    const i128 R = (i128)4 * den * wa;
    return Q <= R;
}

__device__ __forceinline__ double tri_orthosize(const Tri &t) {
    // |c|^2 = |M|^2 / (4 den^2)
    const double M2 = t.Mx * t.Mx + t.My * t.My + t.Mz * t.Mz;
    const double d = (double)t.den;
    return M2 / (4.0 * d * d) - (double)t.v0.w;
}

// Floating-point filter of tri_violation_sign: the sign of P when the
// rounding bound certifies it, 0 when the exact path has to decide.
__device__ __forceinline__ int tri_violation_filter(const Tri &t, int4 q) {
    const int bx = q.x - t.v0.x, by = q.y - t.v0.y, bz = q.z - t.v0.z;
    const int gam = m24(bx, bx) + m24(by, by) + m24(bz, bz) - q.w + t.v0.w;
    const double P = (double)t.den * (double)gam - (t.Mx * (double)bx + t.My * (double)by + t.Mz * (double)bz);
    return (P > t.eP) - (P < -t.eP);
}

// Exact sign of P (int128), with simulation of simplicity on a tie.
__device__ __forceinline__ int tri_violation_exact(const Tri &t, int s0, int s1, int s2, int4 q, int sq,
                                                   const int *perm);

// P = |n|^2 gamma - M.b
__device__ __forceinline__ int tri_violation_sign(const Tri &t, int s0, int s1, int s2, int4 q, int sq, const int *perm,
                                                  const PredParams &pp, Counters *cnt) {
    if (!pp.force_exact) {
        const int f = tri_violation_filter(t, q);
        if (f) return f;
        note_fallback(cnt);
    }
    return tri_violation_exact(t, s0, s1, s2, q, sq, perm);
}

__device__ __forceinline__ int tri_violation_exact(const Tri &t, int s0, int s1, int s2, int4 q, int sq,
                                                   const int *perm) {
    const i64 bx = q.x - t.v0.x, by = q.y - t.v0.y, bz = q.z - t.v0.z;
    const i64 gam = bx * bx + by * by + bz * bz - q.w + t.v0.w;
    // u, w are exact integers below 2^44 held in float64
    const i64 ux = (i64)t.ux, uy = (i64)t.uy, uz = (i64)t.uz, wx = (i64)t.wx, wy = (i64)t.wy, wz = (i64)t.wz;
    const i128 Mx = (i128)t.b1 * ux + (i128)t.b2 * wx;
    const i128 My = (i128)t.b1 * uy + (i128)t.b2 * wy;
    const i128 Mz = (i128)t.b1 * uz + (i128)t.b2 * wz;
    const i128 P = (i128)t.den * gam - (Mx * bx + My * by + Mz * bz);
    if (P != 0) return sgn128(P);
    const i64 ub = ux * bx + uy * by + uz * bz;
    const i64 wb = wx * bx + wy * by + wz * bz;
    int ids[4] = {perm[sq], perm[s1], perm[s2], perm[s0]};
    i128 coef[4] = {-(i128)t.den, (i128)ub, (i128)wb, (i128)t.den - ub - wb};
    return sos_first<4>(ids, coef);
}

// ---------------------------------------------------------------------------
// Tetrahedron (d = 3).
struct Tet {
    int4 v0;
    int c1x, c1y, c1z, c2x, c2y, c2z, c3x, c3y, c3z;  // a2xa3, a3xa1, a1xa2 (components below 2^29)
    int b1, b2, b3;
    i64 D;
    double Mx, My, Mz, Mabs2, eP;
};

__device__ __forceinline__ Tet tet_setup(int4 v0, int4 v1, int4 v2, int4 v3, const PredParams &pp) {
    Tet t;
    t.v0 = v0;
    const int a1x = v1.x - v0.x, a1y = v1.y - v0.y, a1z = v1.z - v0.z;
    const int a2x = v2.x - v0.x, a2y = v2.y - v0.y, a2z = v2.z - v0.z;
    const int a3x = v3.x - v0.x, a3y = v3.y - v0.y, a3z = v3.z - v0.z;
    t.c1x = m24(a2y, a3z) - m24(a2z, a3y); t.c1y = m24(a2z, a3x) - m24(a2x, a3z); t.c1z = m24(a2x, a3y) - m24(a2y, a3x);
    t.c2x = m24(a3y, a1z) - m24(a3z, a1y); t.c2y = m24(a3z, a1x) - m24(a3x, a1z); t.c2z = m24(a3x, a1y) - m24(a3y, a1x);
    t.c3x = m24(a1y, a2z) - m24(a1z, a2y); t.c3y = m24(a1z, a2x) - m24(a1x, a2z); t.c3z = m24(a1x, a2y) - m24(a1y, a2x);
    // D = a1 . c1: products below 2^43, sum below 2^45, exact in float64
    t.D = (i64)((double)a1x * (double)t.c1x + (double)a1y * (double)t.c1y + (double)a1z * (double)t.c1z);
    t.b1 = m24(a1x, a1x) + m24(a1y, a1y) + m24(a1z, a1z) - v1.w + v0.w;
    t.b2 = m24(a2x, a2x) + m24(a2y, a2y) + m24(a2z, a2z) - v2.w + v0.w;
    t.b3 = m24(a3x, a3x) + m24(a3y, a3y) + m24(a3z, a3z) - v3.w + v0.w;
    const double b1 = (double)t.b1, b2 = (double)t.b2, b3 = (double)t.b3;
    t.Mx = b1 * (double)t.c1x + b2 * (double)t.c2x + b3 * (double)t.c3x;
    t.My = b1 * (double)t.c1y + b2 * (double)t.c2y + b3 * (double)t.c3y;
    t.Mz = b1 * (double)t.c1z + b2 * (double)t.c2z + b3 * (double)t.c3z;
    const double ab1 = fabs(b1), ab2 = fabs(b2), ab3 = fabs(b3);
    const double mx = ab1 * fabs((double)t.c1x) + ab2 * fabs((double)t.c2x) + ab3 * fabs((double)t.c3x);
    const double my = ab1 * fabs((double)t.c1y) + ab2 * fabs((double)t.c2y) + ab3 * fabs((double)t.c3y);
    const double mz = ab1 * fabs((double)t.c1z) + ab2 * fabs((double)t.c2z) + ab3 * fabs((double)t.c3z);
    t.Mabs2 = mx * mx + my * my + mz * mz;
    t.eP = 16.0 * ACX_U * (fabs((double)t.D) * pp.gmax + pp.bmax * (mx + my + mz));
    return t;
}

__device__ __forceinline__ void tet_exact_M(const Tet &t, i128 &Mx, i128 &My, i128 &Mz) {
    Mx = (i128)t.b1 * t.c1x + (i128)t.b2 * t.c2x + (i128)t.b3 * t.c3x;
    My = (i128)t.b1 * t.c1y + (i128)t.b2 * t.c2y + (i128)t.b3 * t.c3y;
    Mz = (i128)t.b1 * t.c1z + (i128)t.b2 * t.c2z + (i128)t.b3 * t.c3z;
}

// AC3 for a tetrahedron: |M|^2 <= 4 D^2 (W0 + alpha).
__device__ __forceinline__ bool tet_ac3(const Tet &t, const PredParams &pp, Counters *cnt) {
    const i64 wa = t.v0.w + pp.aq;
    if (!pp.force_exact) {
        const double L = t.Mx * t.Mx + t.My * t.My + t.Mz * t.Mz;
        const double Dd = (double)t.D;
        const double R = 4.0 * (Dd * Dd) * (double)wa;
        const double e = 16.0 * ACX_U * (t.Mabs2 + fabs(R));
        const double diff = L - R;
        if (diff < -e) return true;
        if (diff > e) return false;
        note_fallback(cnt);
    }
    i128 Mx, My, Mz;
    tet_exact_M(t, Mx, My, Mz);
    const i128 L = Mx * Mx + My * My + Mz * Mz;
    const i128 R = (i128)4 * ((i128)t.D * t.D) * wa;
    return L <= R;
}

__device__ __forceinline__ double tet_orthosize(const Tet &t) {
    const double M2 = t.Mx * t.Mx + t.My * t.My + t.Mz * t.Mz;
    const double d = (double)t.D;
    return M2 / (4.0 * d * d) - (double)t.v0.w;
}

// P = sign(D) (D gamma - M.b)
__device__ __forceinline__ int tet_violation_sign(const Tet &t, int s0, int s1, int s2, int s3, int4 q, int sq,
                                                  const int *perm, const PredParams &pp, Counters *cnt) {
    const int bx = q.x - t.v0.x, by = q.y - t.v0.y, bz = q.z - t.v0.z;
    const int gam = m24(bx, bx) + m24(by, by) + m24(bz, bz) - q.w + t.v0.w;
    const int sD = t.D > 0 ? 1 : -1;
    if (!pp.force_exact) {
        const double P = (double)t.D * (double)gam - (t.Mx * (double)bx + t.My * (double)by + t.Mz * (double)bz);
        if (P > t.eP) return sD;
        if (P < -t.eP) return -sD;
        note_fallback(cnt);
    }
    i128 Mx, My, Mz;
    tet_exact_M(t, Mx, My, Mz);
    const i128 P = (i128)t.D * gam - (Mx * bx + My * by + Mz * bz);
    if (P != 0) return sD * sgn128(P);
    const i64 k1 = (i64)t.c1x * bx + (i64)t.c1y * by + (i64)t.c1z * bz;
    const i64 k2 = (i64)t.c2x * bx + (i64)t.c2y * by + (i64)t.c2z * bz;
    const i64 k3 = (i64)t.c3x * bx + (i64)t.c3y * by + (i64)t.c3z * bz;
    int ids[5] = {perm[sq], perm[s1], perm[s2], perm[s3], perm[s0]};
    i128 coef[5] = {-(i128)(t.D > 0 ? t.D : -t.D), (i128)sD * k1, (i128)sD * k2, (i128)sD * k3,
                    (i128)sD * (t.D - k1 - k2 - k3)};
    return sos_first<5>(ids, coef);
}

}  // namespace acx
