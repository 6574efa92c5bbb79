// Alpha sweep (gfx950 device code): the complexes of one ball set for many
// alpha values from the candidates of the largest.
//
// For a candidate simplex the AC3 test "OrthoSize <= alpha" (Sec. 3.1,
// Step 1) is monotone in alpha, so it holds exactly from an integer
// threshold on (alpha in mA^2): the least integer a with OrthoSize <= a. AC2
// (Steps 2-5) does not depend on alpha. The preparation kernels below find
// each candidate's threshold once with the exact predicates and lay every
// per-candidate quantity out in the output order (rows sorted by input ids),
// with face references given as places in that order. The kernels of one
// alpha are then integer comparisons, the attachment of Steps 3-5 and a
// compaction, all streaming over the output order.
#pragma once
#include "kernels.hpp"

namespace acx {

// Least integer a in (lo, hi] with ac3(a) true, for an exact test that is
// false at lo and at every a below the threshold, and true at hi and above.
// A float64 estimate of the OrthoSize is corrected by exact tests; bisection
// backs the correction up.
template <class F>
__device__ int entry_threshold(double est, i64 lo, i64 hi, F &&ac3) {
    i64 a = (i64)ceil(est);
    a = a <= lo ? lo + 1 : (a > hi ? hi : a);
    for (int it = 0; it < 4 && a < hi && !ac3(a); it++) a++;
    for (int it = 0; it < 4 && a - 1 > lo && ac3(a - 1); it++) a--;
    if (ac3(a) && (a - 1 <= lo || !ac3(a - 1))) return (int)a;
    i64 l = lo, h = hi;
    while (h - l > 1) {
        const i64 m = l + (h - l) / 2;
        if (ac3(m)) h = m; else l = m;
    }
    return (int)h;
}

constexpr int NO_ENTRY = INT_MAX;  // threshold of a candidate that fails AC2

// Edges: candidate e goes to place p = spos[e] of the output order.
__global__ void __launch_bounds__(BLOCK) k_sweep_prep_edge(const int4 *__restrict__ atom, const int *__restrict__ up,
                                                            const int *__restrict__ edge_i, int E,
                                                            const unsigned char *__restrict__ egab,
                                                            const int *__restrict__ spos, i64 aq_max,
                                                            int *__restrict__ thr, double *__restrict__ sz,
                                                            int2 *__restrict__ ends) {
    const int e = xcd_block() * BLOCK + threadIdx.x;
    if (e >= E) return;
    const int i = edge_i[e], j = up[e];
    const int p = spos[e];
    ends[p] = make_int2(i, j);
    if (!egab[e]) {
        thr[p] = NO_ENTRY;
        return;
    }
    const int4 vi = atom[i], vj = atom[j];
    const Edge ed = edge_setup(vi, vj);
    thr[p] = entry_threshold(edge_orthosize(ed), -(i64)vi.w - 1, aq_max, [&](i64 a) { return edge_ac3(ed, a); });
    sz[p] = edge_size_canon(vi, vj);
}

// Triangles: threshold, Size (the canonical OrthoSize), and the places of
// the three edges in the edge output order.
__global__ void __launch_bounds__(BLOCK) k_sweep_prep_tri(const int4 *__restrict__ atom, const int *__restrict__ up,
                                                           const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                           const int *__restrict__ tri_e, int T,
                                                           const unsigned char *__restrict__ tgab,
                                                           const double *__restrict__ tsize,
                                                           const int2 *__restrict__ tedge, const int *__restrict__ spos_t,
                                                           const int *__restrict__ spos_e, PredParams pp,
                                                           int *__restrict__ thr, double *__restrict__ sz,
                                                           int4 *__restrict__ face, Counters *cnt) {
    const int t = xcd_block() * BLOCK + threadIdx.x;
    if (t >= T) return;
    const int e = tri_e[t];
    const int p = spos_t[t];
    const int2 f = tedge[t];
    face[p] = make_int4(spos_e[e], f.x < 0 ? -1 : spos_e[f.x], f.y < 0 ? -1 : spos_e[f.y], 0);
    if (!tgab[t]) {
        thr[p] = NO_ENTRY;
        return;
    }
    const int4 vi = atom[edge_i[e]], vj = atom[up[e]], vk = atom[tri_k[t]];
    PredParams q = pp;
    thr[p] = entry_threshold(tri_orthosize(tri_setup(vi, vj, vk, pp)), -(i64)vi.w - 1, pp.aq, [&](i64 a) {
        q.aq = a;
        return tri_candidate(vi, vj, vk, q, cnt);
    });
    sz[p] = tsize[t];
}

// Tetrahedra: threshold (AC2 from k_tet_ac2<true> in qgab), Size, and the
// places of the four facets in the triangle output order.
__global__ void __launch_bounds__(BLOCK) k_sweep_prep_tet(const int4 *__restrict__ atom, const int *__restrict__ up,
                                                           const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                           const int *__restrict__ tri_e, const int *__restrict__ tet_t,
                                                           const int *__restrict__ tet_l, int Q,
                                                           const unsigned char *__restrict__ qgab,
                                                           const double *__restrict__ qsize,
                                                           const int4 *__restrict__ tface, const int *__restrict__ spos_q,
                                                           const int *__restrict__ spos_t, PredParams pp,
                                                           int *__restrict__ thr, double *__restrict__ sz,
                                                           int4 *__restrict__ face, Counters *cnt) {
    const int c = xcd_block() * BLOCK + threadIdx.x;
    if (c >= Q) return;
    const int p = spos_q[c];
    if (!qgab[c]) {
        thr[p] = NO_ENTRY;
        return;
    }
    const int t = tet_t[c];
    const int e = tri_e[t];
    const int4 v0 = atom[edge_i[e]];
    const Tet te = tet_setup(v0, atom[up[e]], atom[tri_k[t]], atom[tet_l[c]], pp);
    PredParams q = pp;
    thr[p] = entry_threshold(tet_orthosize(te), -(i64)v0.w - 1, pp.aq, [&](i64 a) {
        q.aq = a;
        return tet_ac3(te, q, cnt);
    });
    sz[p] = qsize[c];
    const int4 f = tface[c];
    auto at = [&](int x) { return x < 0 ? -1 : spos_t[x]; };
    face[p] = make_int4(at(f.x), at(f.y), at(f.z), at(f.w));
}

// A kept coface records itself on face f unless f passes AC2 (threshold not
// NO_ENTRY: such a face is in K with its own Size whenever a coface is).
__device__ __forceinline__ void sweep_mark(const int *__restrict__ thr, int *att, long long *mins, int f,
                                           long long key, Counters *cnt) {
    if (f < 0) { atomicOr(&cnt->lookup, 1); return; }
    if (thr[f] != NO_ENTRY) return;
    atomicOr(&att[f], 1);
    atomicMin(&mins[f], key);
}

// The kernels of one alpha run one thread per row of the output order, in
// blocks of BLOCK rows; each writes its rows' kept flags and its block's
// kept total (tsum), whose scan places the kept rows in k_sweep_write.

// One alpha (aq in mA^2), tetrahedra in output order (Step 2).
__global__ void __launch_bounds__(BLOCK) k_sweep_tets(int Q, i64 aq, const int *__restrict__ thr3,
                                                       const double *__restrict__ sz3, const int4 *__restrict__ face3,
                                                       const int *__restrict__ thr2, int *__restrict__ tri_att,
                                                       long long *__restrict__ tri_min, unsigned char *__restrict__ in_s,
                                                       double *__restrict__ sz_s, int *__restrict__ tsum,
                                                       Counters *cnt) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    const bool in = p < Q && thr3[p] <= aq;
    if (p < Q) in_s[p] = in;
    if (in) {
        const double sz = sz3[p];
        sz_s[p] = sz;
        const long long key = ordered_from_double(sz);
        const int4 f = face3[p];
        sweep_mark(thr2, tri_att, tri_min, f.x, key, cnt);
        sweep_mark(thr2, tri_att, tri_min, f.y, key, cnt);
        sweep_mark(thr2, tri_att, tri_min, f.z, key, cnt);
        sweep_mark(thr2, tri_att, tri_min, f.w, key, cnt);
    }
    int tot;
    (void)block_exclusive_scan<BLOCK>(in, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One alpha, triangles in output order (Step 3).
__global__ void __launch_bounds__(BLOCK) k_sweep_tris(int T, i64 aq, const int *__restrict__ thr2,
                                                       const double *__restrict__ sz2, const int4 *__restrict__ face2,
                                                       const int *__restrict__ tri_att,
                                                       const long long *__restrict__ tri_min,
                                                       const int *__restrict__ thr1, int *__restrict__ edge_att,
                                                       long long *__restrict__ edge_min,
                                                       unsigned char *__restrict__ in_s, double *__restrict__ sz_s,
                                                       int *__restrict__ tsum, Counters *cnt) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    bool in = false;
    if (p < T) {
        const bool gab = thr2[p] <= aq;
        in = gab || tri_att[p];
        in_s[p] = in;
        if (in) {
            const double sz = gab ? sz2[p] : double_from_ordered(tri_min[p]);
            sz_s[p] = sz;
            const long long key = ordered_from_double(sz);
            const int4 f = face2[p];
            sweep_mark(thr1, edge_att, edge_min, f.x, key, cnt);
            sweep_mark(thr1, edge_att, edge_min, f.y, key, cnt);
            sweep_mark(thr1, edge_att, edge_min, f.z, key, cnt);
        }
    }
    int tot;
    (void)block_exclusive_scan<BLOCK>(in, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One alpha, edges in output order (Step 4); kept edges record themselves on
// their ends that fail AC2 (Step 5).
__global__ void __launch_bounds__(BLOCK) k_sweep_edges(int E, i64 aq, const int *__restrict__ thr1,
                                                        const double *__restrict__ sz1, const int2 *__restrict__ ends,
                                                        const int *__restrict__ edge_att,
                                                        const long long *__restrict__ edge_min,
                                                        const unsigned char *__restrict__ vgab,
                                                        int *__restrict__ vert_att, long long *__restrict__ vert_min,
                                                        unsigned char *__restrict__ in_s, double *__restrict__ sz_s,
                                                        int *__restrict__ tsum) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    bool in = false;
    if (p < E) {
        const bool gab = thr1[p] <= aq;
        in = gab || edge_att[p];
        in_s[p] = in;
        if (in) {
            const double sz = gab ? sz1[p] : double_from_ordered(edge_min[p]);
            sz_s[p] = sz;
            const long long key = ordered_from_double(sz);
            const int2 v = ends[p];
            if (!vgab[v.x]) { atomicOr(&vert_att[v.x], 1); atomicMin(&vert_min[v.x], key); }
            if (!vgab[v.y]) { atomicOr(&vert_att[v.y], 1); atomicMin(&vert_min[v.y], key); }
        }
    }
    int tot;
    (void)block_exclusive_scan<BLOCK>(in, &tot);
    if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// One alpha, output of dimension K - 1: the kept rows in output order, each
// at its block's offset (toff: exclusive scan of the block totals) plus its
// place among the block's kept rows.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_sweep_write(const unsigned char *__restrict__ in_s,
                                                        const int *__restrict__ toff, const int *__restrict__ rows_s,
                                                        const double *__restrict__ sz_s, int m, int *__restrict__ out,
                                                        double *__restrict__ out_size) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    const bool in = p < m && in_s[p];
    int tot;
    const int local = block_exclusive_scan<BLOCK>(in, &tot);
    if (!in) return;
    const int o = toff[blockIdx.x] + local;
#pragma unroll
    for (int u = 0; u < K; u++) out[(long long)o * K + u] = rows_s[(long long)p * K + u];
    out_size[o] = sz_s[p] / 1.0e6;  // mA^2 -> A^2
}

}  // namespace acx
