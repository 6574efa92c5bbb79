// HIP kernels of the alpha-complex pipeline for gfx950.
//
// Stages (Masood, Ray, Natarajan, Sec. 3.1 Steps 1-5 and Sec. 4.2-4.5):
//   quantise  -> integer milli-angstrom balls, bounding box, validation
//   binning   -> counting sort of the balls by uniform-grid cell (Sec. 4.2)
//   neighbours-> per ball: every ball whose grown ball (radius^2 W + alpha)
//                meets its own (the only possible AC2 violators of any
//                candidate it belongs to), and the upper candidate edges,
//                Sigma_ortho^1 (Sec. 4.3)
//   triangles -> Sigma_ortho^2 from pairs of candidate edges (Sec. 4.3)
//   tetrahedra-> Sigma_ortho^3 from candidate triangles, each tested at once
//                with AC2 at its ortho-centre (Step 2); survivors mark their
//                facets attached (Step 3, first half)
//   finalise  -> triangles, edges, vertices: a candidate is in K_alpha iff it
//                passes AC2 at its own ortho-centre or is a face of a kept
//                coface (Steps 3-5, Lemmas 1-2); Size is its OrthoSize when it
//                passes AC2, else the least Size of a kept coface (Sec. 2.3)
//   emit      -> input ids, sorted within a row, rows sorted (bucket by the
//                first id, then each bucket sorted in place)
#pragma once
#include "common.hpp"
#include "predicates.hpp"

namespace acx {

struct Stats {
    int minx, miny, minz, maxx, maxy, maxz;
    int wmax, flags;  // flags: 1 invalid value, 2 out of range
};

struct Grid {
    int ox, oy, oz;   // low corner (mA)
    int s;            // cell side (mA)
    int nx, ny, nz;
    int reach;        // cells to scan on each side for neighbours
};

constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// Quantise: x -> rint(1000 x) (round half to even), W = R^2.
__global__ void __launch_bounds__(BLOCK) k_quantise(const double *__restrict__ xyz, const double *__restrict__ r,
                                                     int n, int4 *__restrict__ q, Stats *st) {
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN}, wmax = 0, flags = 0;
    for (int i = blockIdx.x * BLOCK + threadIdx.x; i < n; i += gridDim.x * BLOCK) {
        int c[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double v = xyz[3 * (long long)i + a];
            c[a] = 0;
            if (!isfinite(v)) { flags |= 1; continue; }
            const double s = v * 1000.0;
            if (!(fabs(s) < 524288.0)) { flags |= 2; continue; }
            c[a] = (int)rint(s);
            if (c[a] >= 524288 || c[a] <= -524288) flags |= 2;
            mn[a] = min(mn[a], c[a]);
            mx[a] = max(mx[a], c[a]);
        }
        const double rv = r[i];
        int W = 0;
        if (!isfinite(rv) || !(rv > 0.0)) {
            flags |= 1;
        } else {
            const double rs = rv * 1000.0;
            if (!(rs < 8192.0)) {
                flags |= 2;
            } else {
                const int R = (int)rint(rs);
                if (R < 1) flags |= 1;
                W = R * R;
            }
        }
        wmax = max(wmax, W);
        q[i] = make_int4(c[0], c[1], c[2], W);
    }
    // wave reduction, then one atomic per wave
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            mn[a] = min(mn[a], __shfl_xor(mn[a], off, WAVE));
            mx[a] = max(mx[a], __shfl_xor(mx[a], off, WAVE));
        }
        wmax = max(wmax, __shfl_xor(wmax, off, WAVE));
        flags |= __shfl_xor(flags, off, WAVE);
    }
    if (lane_id() == 0) {
        atomicMin(&st->minx, mn[0]); atomicMin(&st->miny, mn[1]); atomicMin(&st->minz, mn[2]);
        atomicMax(&st->maxx, mx[0]); atomicMax(&st->maxy, mx[1]); atomicMax(&st->maxz, mx[2]);
        atomicMax(&st->wmax, wmax);
        atomicOr(&st->flags, flags);
    }
}

__global__ void k_stats_init(Stats *st) {
    st->minx = st->miny = st->minz = INT_MAX;
    st->maxx = st->maxy = st->maxz = INT_MIN;
    st->wmax = 0;
    st->flags = 0;
}

template <class T>
__global__ void __launch_bounds__(BLOCK) k_fill(T *__restrict__ p, T v, long long n) {
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) p[i] = v;
}

// ---------------------------------------------------------------------------
// Binning (Sec. 4.2): cell key, histogram, scatter, then a deterministic order
// inside each cell (by input index).
__device__ __forceinline__ long long cell_of(const Grid &g, int x, int y, int z) {
    const int cx = (x - g.ox) / g.s, cy = (y - g.oy) / g.s, cz = (z - g.oz) / g.s;
    return ((long long)cz * g.ny + cy) * g.nx + cx;
}

__global__ void __launch_bounds__(BLOCK) k_cell_hist(const int4 *__restrict__ q, int n, Grid g,
                                                      long long *__restrict__ key, int *__restrict__ cell_count) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int4 a = q[i];
    const long long c = cell_of(g, a.x, a.y, a.z);
    key[i] = c;
    atomicAdd(&cell_count[c], 1);
}

__global__ void __launch_bounds__(BLOCK) k_scatter(const int4 *__restrict__ q, const long long *__restrict__ key, int n,
                                                    int *__restrict__ cursor, int4 *__restrict__ tmp_atom,
                                                    int *__restrict__ tmp_perm) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int pos = atomicAdd(&cursor[key[i]], 1);
    tmp_atom[pos] = q[i];
    tmp_perm[pos] = i;
}

// Also flags duplicate centres (equal centres share a cell).
__global__ void __launch_bounds__(BLOCK) k_cell_order(const int4 *__restrict__ tmp_atom, const int *__restrict__ tmp_perm,
                                                       int n, Grid g, const int *__restrict__ cell_start,
                                                       int4 *__restrict__ atom, int *__restrict__ perm, Counters *cnt) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n) return;
    const int4 a = tmp_atom[p];
    const int me = tmp_perm[p];
    const long long c = cell_of(g, a.x, a.y, a.z);
    const int s = cell_start[c], e = cell_start[c + 1];
    int rank = 0;
    bool dup = false;
    for (int k = s; k < e; k++) {
        rank += tmp_perm[k] < me;
        if (k != p) {
            const int4 b = tmp_atom[k];
            dup |= b.x == a.x && b.y == a.y && b.z == a.z;
        }
    }
    if (dup) atomicOr(&cnt->dup, 1);
    atom[s + rank] = a;
    perm[s + rank] = me;
}

// ---------------------------------------------------------------------------
// Neighbour lists and candidate edges (Sec. 4.3, first step). A thread per
// ball scans the cells within `reach`; cells of one grid row are contiguous
// in the sorted order, so each (dz, dy) row is one contiguous range.
template <bool FILL>
__global__ void __launch_bounds__(BLOCK) k_neighbours(const int4 *__restrict__ atom, int n, Grid g,
                                                       const int *__restrict__ cell_start, PredParams pp,
                                                       int *__restrict__ deg_n, int *__restrict__ deg_up,
                                                       const int *__restrict__ nbr_start, const int *__restrict__ up_start,
                                                       int *__restrict__ nbr, int *__restrict__ up,
                                                       int *__restrict__ edge_i, Counters *cnt) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int4 a = atom[i];
    const i64 ra = (i64)a.w + pp.aq;
    int cn = 0, cu = 0;
    if (ra >= 0) {
        const int pn = FILL ? nbr_start[i] : 0, pu = FILL ? up_start[i] : 0;
        const int cx = (a.x - g.ox) / g.s, cy = (a.y - g.oy) / g.s, cz = (a.z - g.oz) / g.s;
        const int x0 = max(cx - g.reach, 0), x1 = min(cx + g.reach, g.nx - 1);
        const int y0 = max(cy - g.reach, 0), y1 = min(cy + g.reach, g.ny - 1);
        const int z0 = max(cz - g.reach, 0), z1 = min(cz + g.reach, g.nz - 1);
        const i64 lim = 4 * pp.sg2;
        for (int z = z0; z <= z1; z++)
            for (int y = y0; y <= y1; y++) {
                const long long rb = ((long long)z * g.ny + y) * g.nx;
                const int s = cell_start[rb + x0], e = cell_start[rb + x1 + 1];
                for (int j = s; j < e; j++) {
                    if (j == i) continue;
                    const int4 b = atom[j];
                    const i64 dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                    const i64 d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 > lim) continue;
                    if (d2 == 0) continue; /* duplicates are reported by k_cell_order */
                    const i64 rb2 = (i64)b.w + pp.aq;
                    if (rb2 < 0) continue;
                    // grown balls meet: d <= rho_a + rho_b
                    const i64 L = d2 - ra - rb2;
                    if (L > 0 && L * L > 4 * ra * rb2) continue;
                    if (FILL) nbr[pn + cn] = j;
                    cn++;
                    if (j > i) {
                        const Edge ed = edge_setup(a, b);
                        if (edge_ac3(ed, pp.aq)) {
                            if (FILL) { up[pu + cu] = j; edge_i[pu + cu] = i; }
                            cu++;
                        }
                    }
                }
            }
    }
    if (!FILL) { deg_n[i] = cn; deg_up[i] = cu; }
}

// Position of b in the (sorted) upper-edge list of a, i.e. the edge id; -1 if absent.
__device__ __forceinline__ int find_edge(const int *__restrict__ up_start, const int *__restrict__ up, int a, int b) {
    int lo = up_start[a], hi = up_start[a + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = up[mid];
        if (v == b) return mid;
        if (v < b) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// Triangle id of (a < b < c); -1 if absent.
__device__ __forceinline__ int find_tri(const int *__restrict__ up_start, const int *__restrict__ up,
                                        const int *__restrict__ tri_start, const int *__restrict__ tri_k, int a, int b,
                                        int c) {
    const int e = find_edge(up_start, up, a, b);
    if (e < 0) return -1;
    int lo = tri_start[e], hi = tri_start[e + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = tri_k[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Candidate triangles (Sec. 4.3): for an edge (i, j), every k > j adjacent to
// both by a candidate edge, not collinear, with OrthoSize <= alpha.
template <bool FILL>
__global__ void __launch_bounds__(BLOCK) k_triangles(const int4 *__restrict__ atom, const int *__restrict__ up_start,
                                                      const int *__restrict__ up, const int *__restrict__ edge_i, int E,
                                                      PredParams pp, int *__restrict__ tri_cnt,
                                                      const int *__restrict__ tri_start, int *__restrict__ tri_k,
                                                      int *__restrict__ tri_e, Counters *cnt) {
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= E) return;
    const int i = edge_i[e], j = up[e];
    int pa = e + 1;
    const int ea = up_start[i + 1];
    int pb = up_start[j];
    const int eb = up_start[j + 1];
    const int4 vi = atom[i], vj = atom[j];
    int c = 0;
    const int out = FILL ? tri_start[e] : 0;
    while (pa < ea && pb < eb) {
        const int ka = up[pa], kb = up[pb];
        if (ka < kb) { pa++; continue; }
        if (kb < ka) { pb++; continue; }
        pa++; pb++;
        const Tri t = tri_setup(vi, vj, atom[ka], pp);
        if (tri_degenerate(t) || !tri_ac3(t, pp, cnt)) continue;
        if (FILL) { tri_k[out + c] = ka; tri_e[out + c] = e; }
        c++;
    }
    if (!FILL) tri_cnt[e] = c;
}

// ---------------------------------------------------------------------------
// Candidate tetrahedra with AC2 (Steps 1-2): for a triangle (i, j, k), every
// l > k adjacent to all three by candidate edges (all six edges in
// Sigma_ortho^1 suffice since OrthoSize grows from face to coface), not flat,
// with OrthoSize <= alpha; kept iff no ball is strictly closer in power to its
// ortho-centre. Kept tetrahedra mark their four facets.
__device__ __forceinline__ void mark_face(int *att, long long *mins, int f, long long key, Counters *cnt) {
    if (f < 0) { atomicOr(&cnt->lookup, 1); return; }
    atomicOr(&att[f], 1);
    atomicMin(&mins[f], key);
}

__global__ void __launch_bounds__(BLOCK) k_tetrahedra(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                       const int *__restrict__ nbr_start, const int *__restrict__ nbr,
                                                       const int *__restrict__ up_start, const int *__restrict__ up,
                                                       const int *__restrict__ edge_i, const int *__restrict__ tri_start,
                                                       const int *__restrict__ tri_k, const int *__restrict__ tri_e,
                                                       int T, PredParams pp, int *__restrict__ tri_att,
                                                       long long *__restrict__ tri_min, int4 *__restrict__ k3,
                                                       double *__restrict__ k3_size, int cap3, Counters *cnt) {
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    if (t >= T) return;
    const int e = tri_e[t];
    const int i = edge_i[e], j = up[e], k = tri_k[t];
    int pa = e + 1;
    const int ea = up_start[i + 1];
    int pb = up_start[j];
    const int eb = up_start[j + 1];
    int pc = up_start[k];
    const int ec = up_start[k + 1];
    const int4 vi = atom[i], vj = atom[j], vk = atom[k];
    const int ns = nbr_start[i], ne = nbr_start[i + 1];
    while (pa < ea && pb < eb && pc < ec) {
        const int la = up[pa], lb = up[pb], lc = up[pc];
        const int m = max(la, max(lb, lc));
        if (la < m) { pa++; continue; }
        if (lb < m) { pb++; continue; }
        if (lc < m) { pc++; continue; }
        pa++; pb++; pc++;
        const int l = m;
        const Tet te = tet_setup(vi, vj, vk, atom[l], pp);
        if (te.D == 0 || !tet_ac3(te, pp, cnt)) continue;
        bool keep = true;
        for (int p = ns; p < ne; p++) {
            const int q = nbr[p];
            if (q == j || q == k || q == l) continue;
            if (tet_violation_sign(te, i, j, k, l, atom[q], q, perm, pp, cnt) < 0) { keep = false; break; }
        }
        if (!keep) continue;
        const double sz = tet_orthosize(te);
        const int slot = atomicAdd(&cnt->k3, 1);
        if (slot < cap3) { k3[slot] = make_int4(i, j, k, l); k3_size[slot] = sz; }
        const long long key = ordered_from_double(sz);
        mark_face(tri_att, tri_min, t, key, cnt);
        mark_face(tri_att, tri_min, find_tri(up_start, up, tri_start, tri_k, i, j, l), key, cnt);
        mark_face(tri_att, tri_min, find_tri(up_start, up, tri_start, tri_k, i, k, l), key, cnt);
        mark_face(tri_att, tri_min, find_tri(up_start, up, tri_start, tri_k, j, k, l), key, cnt);
    }
}

// Triangles (Step 3): kept iff AC2 holds at the ortho-centre or a kept
// tetrahedron has it as a facet.
__global__ void __launch_bounds__(BLOCK) k_tri_final(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                      const int *__restrict__ nbr_start, const int *__restrict__ nbr,
                                                      const int *__restrict__ up_start, const int *__restrict__ up,
                                                      const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                      const int *__restrict__ tri_e, int T, PredParams pp,
                                                      const int *__restrict__ tri_att,
                                                      const long long *__restrict__ tri_min, int *__restrict__ edge_att,
                                                      long long *__restrict__ edge_min, int4 *__restrict__ k2,
                                                      double *__restrict__ k2_size, Counters *cnt) {
    const int t = blockIdx.x * BLOCK + threadIdx.x;
    const bool valid = t < T;
    bool in = false;
    int i = 0, j = 0, k = 0, e = 0;
    double sz = 0.0;
    if (valid) {
        e = tri_e[t];
        i = edge_i[e]; j = up[e]; k = tri_k[t];
        const Tri tr = tri_setup(atom[i], atom[j], atom[k], pp);
        bool gab = true;
        const int ns = nbr_start[i], ne = nbr_start[i + 1];
        for (int p = ns; p < ne; p++) {
            const int q = nbr[p];
            if (q == j || q == k) continue;
            if (tri_violation_sign(tr, i, j, k, atom[q], q, perm, pp, cnt) < 0) { gab = false; break; }
        }
        in = gab || tri_att[t];
        sz = gab ? tri_orthosize(tr) : double_from_ordered(tri_min[t]);
    }
    const int slot = wave_append(&cnt->k2, in);
    if (in) {
        k2[slot] = make_int4(i, j, k, 0);
        k2_size[slot] = sz;
        const long long key = ordered_from_double(sz);
        mark_face(edge_att, edge_min, e, key, cnt);
        mark_face(edge_att, edge_min, find_edge(up_start, up, i, k), key, cnt);
        mark_face(edge_att, edge_min, find_edge(up_start, up, j, k), key, cnt);
    }
}

// Edges (Step 4).
__global__ void __launch_bounds__(BLOCK) k_edge_final(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                       const int *__restrict__ nbr_start, const int *__restrict__ nbr,
                                                       const int *__restrict__ up, const int *__restrict__ edge_i, int E,
                                                       const int *__restrict__ edge_att,
                                                       const long long *__restrict__ edge_min,
                                                       int *__restrict__ vert_att, long long *__restrict__ vert_min,
                                                       int2 *__restrict__ k1, double *__restrict__ k1_size,
                                                       Counters *cnt) {
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    const bool valid = e < E;
    bool in = false;
    int i = 0, j = 0;
    double sz = 0.0;
    if (valid) {
        i = edge_i[e]; j = up[e];
        const Edge ed = edge_setup(atom[i], atom[j]);
        bool gab = true;
        const int ns = nbr_start[i], ne = nbr_start[i + 1];
        for (int p = ns; p < ne; p++) {
            const int q = nbr[p];
            if (q == j) continue;
            if (edge_violation_sign(ed, i, j, atom[q], q, perm) < 0) { gab = false; break; }
        }
        in = gab || edge_att[e];
        sz = gab ? edge_orthosize(ed) : double_from_ordered(edge_min[e]);
    }
    const int slot = wave_append(&cnt->k1, in);
    if (in) {
        k1[slot] = make_int2(i, j);
        k1_size[slot] = sz;
        const long long key = ordered_from_double(sz);
        atomicOr(&vert_att[i], 1); atomicMin(&vert_min[i], key);
        atomicOr(&vert_att[j], 1); atomicMin(&vert_min[j], key);
    }
}

// Vertices (Step 5): a ball with -W <= alpha is kept iff no ball is strictly
// closer in power to its own centre, or it ends a kept edge.
__global__ void __launch_bounds__(BLOCK) k_vert_final(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                       const int *__restrict__ nbr_start, const int *__restrict__ nbr,
                                                       int n, PredParams pp, int shortcut,
                                                       const int *__restrict__ vert_att,
                                                       const long long *__restrict__ vert_min, int *__restrict__ k0,
                                                       double *__restrict__ k0_size, Counters *cnt) {
    const int v = blockIdx.x * BLOCK + threadIdx.x;
    bool in = false;
    double sz = 0.0;
    if (v < n) {
        const int4 a = atom[v];
        if ((i64)a.w + pp.aq >= 0) {
            bool gab = true;
            if (!shortcut) {
                const int ns = nbr_start[v], ne = nbr_start[v + 1];
                for (int p = ns; p < ne; p++) {
                    const int q = nbr[p];
                    if (vertex_violation_sign(a, v, atom[q], q, perm) < 0) { gab = false; break; }
                }
            }
            in = gab || vert_att[v];
            sz = gab ? -(double)a.w : double_from_ordered(vert_min[v]);
        }
    }
    const int slot = wave_append(&cnt->k0, in);
    if (in) { k0[slot] = v; k0_size[slot] = sz; }
}

// ---------------------------------------------------------------------------
// Emit: rows of sorted-order indices -> rows of input ids sorted ascending,
// rows in lexicographic order. Bucket by the first id (counting sort), then
// insertion-sort each (short) bucket.
template <int K>
__device__ __forceinline__ void load_row(const int *rows, int r, int (&v)[4]) {
    if (K == 1) { v[0] = rows[r]; v[1] = v[2] = v[3] = 0; }
    else if (K == 2) { const int2 t = reinterpret_cast<const int2 *>(rows)[r]; v[0] = t.x; v[1] = t.y; v[2] = v[3] = 0; }
    else { const int4 t = reinterpret_cast<const int4 *>(rows)[r]; v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = K == 4 ? t.w : 0; }
}

template <int K>
__global__ void __launch_bounds__(BLOCK) k_emit_remap(const int *__restrict__ rows, const int *__restrict__ perm, int m,
                                                       int4 *__restrict__ tmp, int *__restrict__ bucket_cnt) {
    const int r = blockIdx.x * BLOCK + threadIdx.x;
    if (r >= m) return;
    int v[4];
    load_row<K>(rows, r, v);
#pragma unroll
    for (int u = 0; u < K; u++) v[u] = perm[v[u]];
#pragma unroll
    for (int a = 1; a < K; a++)
#pragma unroll
        for (int b = a; b > 0; b--)
            if (v[b - 1] > v[b]) { const int s = v[b]; v[b] = v[b - 1]; v[b - 1] = s; }
    tmp[r] = make_int4(v[0], v[1], v[2], v[3]);
    atomicAdd(&bucket_cnt[v[0]], 1);
}

__global__ void __launch_bounds__(BLOCK) k_emit_scatter(const int4 *__restrict__ tmp, const double *__restrict__ size_in,
                                                         int m, int *__restrict__ cursor, int4 *__restrict__ rows2,
                                                         double *__restrict__ size2) {
    const int r = blockIdx.x * BLOCK + threadIdx.x;
    if (r >= m) return;
    const int4 v = tmp[r];
    const int pos = atomicAdd(&cursor[v.x], 1);
    rows2[pos] = v;
    size2[pos] = size_in[r];
}

__device__ __forceinline__ bool row_less(const int4 &a, const int4 &b) {
    if (a.y != b.y) return a.y < b.y;
    if (a.z != b.z) return a.z < b.z;
    return a.w < b.w;
}

template <int K>
__global__ void __launch_bounds__(BLOCK) k_emit_sort(const int4 *__restrict__ rows2, const double *__restrict__ size2,
                                                      const int *__restrict__ bstart, int nb, int *__restrict__ out,
                                                      double *__restrict__ out_size) {
    const int b = blockIdx.x * BLOCK + threadIdx.x;
    if (b >= nb) return;
    const int s = bstart[b], e = bstart[b + 1];
    constexpr int LOCAL = 32;
    if (e - s <= LOCAL) {
        int4 r[LOCAL];
        double z[LOCAL];
        const int m = e - s;
        for (int u = 0; u < m; u++) {
            int4 x = rows2[s + u];
            double y = size2[s + u];
            int w = u;
            while (w > 0 && row_less(x, r[w - 1])) { r[w] = r[w - 1]; z[w] = z[w - 1]; w--; }
            r[w] = x; z[w] = y;
        }
        for (int u = 0; u < m; u++) {
            const int v[4] = {r[u].x, r[u].y, r[u].z, r[u].w};
#pragma unroll
            for (int c = 0; c < K; c++) out[(long long)(s + u) * K + c] = v[c];
            out_size[s + u] = z[u] / 1.0e6;  // mA^2 -> A^2
        }
    } else {
        // long bucket (only on very dense inputs): selection by rank, O(m^2)
        for (int u = s; u < e; u++) {
            const int4 x = rows2[u];
            int rank = 0;
            for (int w = s; w < e; w++) rank += row_less(rows2[w], x);
            const int v[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
            for (int c = 0; c < K; c++) out[(long long)(s + rank) * K + c] = v[c];
            out_size[s + rank] = size2[u] / 1.0e6;
        }
    }
}

}  // namespace acx
