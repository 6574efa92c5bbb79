// Partitioned builds (gfx950 device code): the balls are cut into slabs along
// x, each slab is built with a halo of neighbouring balls, and every simplex
// is kept by exactly one slab, the one holding its owner vertex.
//
// Locality (Sec. 3.1 Steps 1-5, Sec. 4.3): every vertex of a candidate lies
// within 2 s_g of the others (grown balls of radius s_g = sqrt(W_max + alpha)
// meet), a ball violating AC2 for a simplex meets its ortho-centre, which
// lies within s_g of each vertex, and the cofaces that decide a face's Size
// share its vertices. So membership and Size of a simplex depend only on
// balls within 4 s_g of any one of its vertices, and a slab built with every
// ball within 4 s_g (plus a margin) of its core decides the simplices whose
// owner vertex lies in the core exactly as a build of all balls does.
#pragma once
#include "kernels.hpp"

namespace acx {

// Slab of a quantised x coordinate: slabs of width w from x0, the last one
// open to the right; every slab computes it the same way.
__device__ __forceinline__ int slab_of(int x, int x0, int w, int parts) { return min(parts - 1, (x - x0) / w); }

// Balls of slab k's core extended by the halo: flag[i] = 1 if lo - halo <= x_i < hi + halo.
__global__ void __launch_bounds__(BLOCK) k_slab_flags(const int4 *__restrict__ q, int n, int lo, int hi, int halo,
                                                       int *__restrict__ flag) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int x = q[i].x;
    flag[i] = (x >= lo - halo) & (x < hi + halo);
}

// The flagged balls in input order (pos: exclusive scan of flag): their
// float64 coordinates and radii, and their input ids (sel).
__global__ void __launch_bounds__(BLOCK) k_slab_gather(const int *__restrict__ flag, const int *__restrict__ pos, int n,
                                                        const double *__restrict__ xyz, const double *__restrict__ r,
                                                        double *__restrict__ sub_xyz, double *__restrict__ sub_r,
                                                        int *__restrict__ sel) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n || !flag[i]) return;
    const int p = pos[i];
    sub_xyz[3 * (long long)p] = xyz[3 * (long long)i];
    sub_xyz[3 * (long long)p + 1] = xyz[3 * (long long)i + 1];
    sub_xyz[3 * (long long)p + 2] = xyz[3 * (long long)i + 2];
    sub_r[p] = r[i];
    sel[p] = i;
}

// Owner vertex of a row (ids of the slab's build): the vertex with the least
// quantised x, ties to the least input id. flag[s] = 1 if it lies in slab k.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_own_flags(const int *__restrict__ rows, int m, const int *__restrict__ sel,
                                                      const int4 *__restrict__ q, int x0, int w, int parts, int k,
                                                      int *__restrict__ flag) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= m) return;
    int best_x = INT_MAX, best_id = INT_MAX;
#pragma unroll
    for (int u = 0; u < K; u++) {
        const int g = sel[rows[(long long)s * K + u]];
        const int x = q[g].x;
        if (x < best_x || (x == best_x && g < best_id)) {
            best_x = x;
            best_id = g;
        }
    }
    flag[s] = slab_of(best_x, x0, w, parts) == k;
}

// Owned vertices of a slab's build, by input id (a vertex owns itself).
__global__ void __launch_bounds__(BLOCK) k_own_vertices(const int *__restrict__ rows, const double *__restrict__ size,
                                                         int m, const int *__restrict__ sel, const int4 *__restrict__ q,
                                                         int x0, int w, int parts, int k, int *__restrict__ kept,
                                                         double *__restrict__ vsize) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= m) return;
    const int g = sel[rows[s]];
    if (slab_of(q[g].x, x0, w, parts) != k) return;
    kept[g] = 1;
    vsize[g] = size[s];
}

// Kept vertices in input order (pos: exclusive scan of kept).
__global__ void __launch_bounds__(BLOCK) k_vertex_rows(const int *__restrict__ kept, const int *__restrict__ pos,
                                                        const double *__restrict__ vsize, int n, int *__restrict__ out,
                                                        double *__restrict__ out_size) {
    const int u = blockIdx.x * BLOCK + threadIdx.x;
    if (u >= n || !kept[u]) return;
    out[pos[u]] = u;
    out_size[pos[u]] = vsize[u];
}

// The owned rows of a slab in emit form, packed in their order (pos:
// exclusive scan of flag): key = least input id (a row's ids ascend in the
// slab's ids, and sel keeps their order), payload = the other input ids and
// the Size bits (K = 2, 3), or the row's place idx_base + pos among the rows
// of all slabs, whose Size goes to out_size[pos] (K = 4). Sizes stay in A^2.
// The emit (radix sort by bucket, k_emit_block) then merges the rows of all
// slabs into output order.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_own_emit(const int *__restrict__ rows, const double *__restrict__ size, int m,
                                                     const int *__restrict__ flag, const int *__restrict__ pos,
                                                     const int *__restrict__ sel, int idx_base,
                                                     unsigned *__restrict__ key,
                                                     typename EmitPay<K>::type *__restrict__ pay,
                                                     double *__restrict__ out_size) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= m || !flag[s]) return;
    const int p = pos[s];
    int v[4] = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < K; u++) v[u] = sel[rows[(long long)s * K + u]];
    emit_pack<K>(true, v, size[s], idx_base + p, 0, key[p], pay[p]);
    if (K == 4) out_size[p] = size[s];
}

// Host-streamed slabs: the device holds only the slab (core and halo), so the
// owner test reads the slab's own quantised x (qx, slab ids) and input ids
// (sel, slab ids) instead of arrays over all balls.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_own_flags_local(const int *__restrict__ rows, int m,
                                                            const int *__restrict__ sel, const int *__restrict__ qx,
                                                            int x0, int w, int parts, int k, int *__restrict__ flag) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= m) return;
    int best_x = INT_MAX, best_id = INT_MAX;
#pragma unroll
    for (int u = 0; u < K; u++) {
        const int l = rows[(long long)s * K + u];
        const int x = qx[l], g = sel[l];
        if (x < best_x || (x == best_x && g < best_id)) {
            best_x = x;
            best_id = g;
        }
    }
    flag[s] = slab_of(best_x, x0, w, parts) == k;
}

// Owned vertices of a host-streamed slab, packed (pos: exclusive scan of
// flag, set by k_own_flags_local<1>): input id and Size.
__global__ void __launch_bounds__(BLOCK) k_own_vertices_local(const int *__restrict__ rows,
                                                               const double *__restrict__ size, int m,
                                                               const int *__restrict__ flag, const int *__restrict__ pos,
                                                               const int *__restrict__ sel, int *__restrict__ out_id,
                                                               double *__restrict__ out_size) {
    const int s = blockIdx.x * BLOCK + threadIdx.x;
    if (s >= m || !flag[s]) return;
    out_id[pos[s]] = sel[rows[s]];
    out_size[pos[s]] = size[s];
}

}  // namespace acx
