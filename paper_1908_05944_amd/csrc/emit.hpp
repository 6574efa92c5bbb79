// Emit: the kept simplices as rows of input ids, ascending inside a row, rows
// in lexicographic order, each with its Size (Sec. 2.3; the paper outputs
// membership only).
//
// The pruning kernels key every candidate by the least input id of its row
// with the remaining ids and its Size (for a tetrahedron: its candidate
// index) as payload; a candidate that is not kept gets the drop key, the
// first key of the bucket after every input id's. A bucket is 2^shift
// consecutive ids (at most EK_KEYS; smaller for small inputs, so that there
// are some hundred buckets). A stable LSD radix sort over the key bits above
// the bucket (8-bit passes) makes every bucket's rows contiguous, the dropped
// rows last; k_key_starts finds where each
// bucket starts, and k_emit_block finishes one bucket per block in LDS: it
// loads the bucket's rows, counts the rows of each id with LDS atomics, scans
// the counts, orders the rows by id, ranks each row in its id's group by the
// remaining ids and writes it to its final place. Every global access is a
// contiguous range; no global atomics, no scattered writes (a bucket with more
// rows than LDS holds is finished through global scratch instead).
#pragma once
#include "common.hpp"
#include "radix.hpp"

namespace acx {

// Sort payload of a row: the ids after the least, then the Size bits (edges,
// triangles) or the candidate index (tetrahedra, whose Size is read at the
// end: they are few).
template <int K> struct EmitPay;
template <> struct EmitPay<2> { typedef uint3 type; };  // v1, Size bits
template <> struct EmitPay<3> { typedef uint4 type; };  // v1, v2, Size bits
template <> struct EmitPay<4> { typedef uint4 type; };  // v1, v2, v3, candidate

__device__ __forceinline__ uint2 bits_of(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return make_uint2((unsigned)b, (unsigned)(b >> 32));
}
__device__ __forceinline__ double double_of(unsigned lo, unsigned hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Key and payload of a candidate with input ids v[0..K) (any order): key =
// least id, payload = the others ascending and `size` (K = 2, 3) or the
// candidate index c (K = 4). Not kept: the drop key, empty payload.
template <int K>
__device__ __forceinline__ void emit_pack(bool kept, int (&v)[4], double size, int c, unsigned drop, unsigned &key,
                                          typename EmitPay<K>::type &pay) {
    pay = typename EmitPay<K>::type{};
    if (!kept) {
        key = drop;
        return;
    }
#pragma unroll
    for (int a = 1; a < K; a++)
#pragma unroll
        for (int b = a; b > 0; b--)
            if (v[b - 1] > v[b]) { const int t = v[b]; v[b] = v[b - 1]; v[b - 1] = t; }
    key = (unsigned)v[0];
    if constexpr (K == 2) {
        const uint2 z = bits_of(size);
        pay = make_uint3((unsigned)v[1], z.x, z.y);
    } else if constexpr (K == 3) {
        const uint2 z = bits_of(size);
        pay = make_uint4((unsigned)v[1], (unsigned)v[2], z.x, z.y);
    } else {
        pay = make_uint4((unsigned)v[1], (unsigned)v[2], (unsigned)v[3], (unsigned)c);
    }
}

// Payloads held in registers as uint4 (a 12-byte uint3 in an array of a
// batch ends up in scratch memory; uint4 stays in registers).
__device__ __forceinline__ uint4 widen(const uint3 &q) { return make_uint4(q.x, q.y, q.z, 0u); }
__device__ __forceinline__ uint4 widen(const uint4 &q) { return q; }
template <class P> __device__ __forceinline__ P narrow(const uint4 &q);
template <> __device__ __forceinline__ uint3 narrow<uint3>(const uint4 &q) { return make_uint3(q.x, q.y, q.z); }
template <> __device__ __forceinline__ uint4 narrow<uint4>(const uint4 &q) { return q; }

template <int K>
__device__ __forceinline__ void pay_ids(const uint4 &q, unsigned (&r)[3]) {
    if constexpr (K == 2) { r[0] = q.x; r[1] = 0; r[2] = 0; }
    else if constexpr (K == 3) { r[0] = q.x; r[1] = q.y; r[2] = 0; }
    else { r[0] = q.x; r[1] = q.y; r[2] = q.z; }
}

template <int K>
__device__ __forceinline__ double pay_size(const uint4 &q, const double *__restrict__ size) {
    if constexpr (K == 2) return double_of(q.y, q.z);
    else if constexpr (K == 3) return double_of(q.z, q.w);
    else return size[q.w];
}

constexpr int EK_SHIFT = 9;              // largest bucket: 2^EK_SHIFT ids
constexpr int EK_KEYS = 1 << EK_SHIFT;
constexpr int EK_BLOCK = 256;
// Rows a block orders in LDS, per dimension. The host picks each dimension's
// bucket size so that its expected largest bucket fits (a row is keyed by its
// least id, so the lowest ids of a randomly numbered input key about K times
// the mean number of rows per id).
template <int K> constexpr int ek_rows() { return K == 4 ? 512 : 2048; }
// What a row holds in LDS besides its 16-bit id in the bucket and its place
// in the order. Edges: only the other id (8 bytes a row, about 18 KB a block,
// eight blocks per CU); the Size bits are read again from the bucket's
// payload when the row is written, from cache, as the block has just read
// them. Triangles and tetrahedra: the whole payload (20 bytes a row; a
// triangle block, about 42 KB, leaves room for three per CU). The edge emit
// ends the build, so it gains from the occupancy; the triangle emit runs on
// the second stream beside the edge path, and slim triangle rows (six blocks
// per CU) did not shorten the build (2.185 against 2.190 ms), so they keep
// the payload and do not read it twice.
template <int K> constexpr bool ek_slim() { return K == 2; }

template <int K>
__device__ __forceinline__ void write_row(int *__restrict__ out, long long pos, unsigned k, const unsigned (&r)[3]) {
    if constexpr (K == 2) {
        *reinterpret_cast<int2 *>(out + pos * 2) = make_int2((int)k, (int)r[0]);
    } else if constexpr (K == 4) {
        *reinterpret_cast<int4 *>(out + pos * 4) = make_int4((int)k, (int)r[0], (int)r[1], (int)r[2]);
    } else {
        out[pos * K] = (int)k;
#pragma unroll
        for (int c = 1; c < K; c++) out[pos * K + c] = (int)r[c - 1];
    }
}

__device__ __forceinline__ bool ids_less(const unsigned (&v)[3], const unsigned (&r)[3]) {
    return v[0] != r[0] ? v[0] < r[0] : (v[1] != r[1] ? v[1] < r[1] : v[2] < r[2]);
}

// Block b finishes bucket b (b < nb, the drop key's bucket): its rows
// [start[b], start[b + 1]) of key / pay are written, in order, to out /
// out_size at the same places (every row before the bucket belongs to smaller
// ids). Block 0 writes the kept count start[nb] to *m_out. gkey / gpay (m
// entries) are scratch for a bucket with more than ek_rows<K>() rows. Sizes are
// converted from mA^2 to A^2 when to_A2 is set (emit of a build), else copied
// (merge of rows that are already output).
// single > 0: one block takes every row unsorted (at most ek_rows<K>(), ids
// below single <= EK_KEYS, shift EK_SHIFT): the rows whose key is single or
// more are dropped ones and skipped, and the block writes the kept count.
// `start` is then unused and the row count is rows_cap, or *live if given.
// A build of a few hundred balls then needs no radix sort.
template <int K>
__global__ void __launch_bounds__(EK_BLOCK) k_emit_block(const unsigned *__restrict__ key,
                                                          const typename EmitPay<K>::type *__restrict__ pay,
                                                          const int *__restrict__ start, int shift, int nb,
                                                          unsigned *__restrict__ gkey,
                                                          typename EmitPay<K>::type *__restrict__ gpay,
                                                          const double *__restrict__ size_in, int to_A2,
                                                          int *__restrict__ out, double *__restrict__ out_size,
                                                          int *__restrict__ m_out, int single = 0, int rows_cap = 0,
                                                          const int *__restrict__ live = nullptr) {
    constexpr int NI = K - 1;  // ids after the least
    constexpr bool SLIM = ek_slim<K>();
    constexpr int NW = SLIM ? NI : (K == 2 ? 3 : 4);  // payload words held in LDS
    constexpr int ROWS = ek_rows<K>();
    __shared__ unsigned sid[NW][ROWS];      // the bucket's rows' other ids (payloads), in load order
    __shared__ unsigned short skey[ROWS];   // their ids less the bucket's first
    __shared__ unsigned short sord[ROWS];   // load positions in id order
    // rows per id; then each id's first place; after the ordering, where each
    // id's group ends (= the next id's first place)
    __shared__ int cnt[EK_KEYS + 1];
    __shared__ int wsum[EK_BLOCK / WAVE];
    constexpr unsigned short DROPPED = 0xFFFF;  // skey of a skipped row (single block)
    const int b = blockIdx.x, t = threadIdx.x;
    const bool one = single > 0;
    if (!one && b == 0 && t == 0) *m_out = start[nb];
    const int bs = one ? 0 : start[b], rows = one ? live_count(rows_cap, live) : start[b + 1] - bs;
    const unsigned k0 = (unsigned)b << shift;  // the bucket's ids: [k0, k0 + 2^shift), 2^shift <= EK_KEYS
    for (int k = t; k <= EK_KEYS; k += EK_BLOCK) cnt[k] = 0;
    __syncthreads();
    const bool lds = rows <= ROWS;
    // counts per id (and, in LDS, the rows' ids); four rows per thread loaded
    // together
    for (int p0 = t; p0 < rows; p0 += 4 * EK_BLOCK) {
        unsigned kk[4];
        uint4 q[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int p = p0 + u * EK_BLOCK;
            kk[u] = p < rows ? key[bs + p] - k0 : 0u;
            q[u] = p < rows && lds ? widen(pay[bs + p]) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int p = p0 + u * EK_BLOCK;
            if (p >= rows) continue;
            const bool drop = one && kk[u] >= (unsigned)single;  // k0 = 0 in a single block
            if (!drop) atomicAdd(&cnt[kk[u]], 1);
            if (lds) {
                skey[p] = drop ? DROPPED : (unsigned short)kk[u];
                sid[0][p] = q[u].x;
                if constexpr (NW >= 2) sid[1][p] = q[u].y;
                if constexpr (NW >= 3) sid[2][p] = q[u].z;
                if constexpr (NW >= 4) sid[3][p] = q[u].w;
            }
        }
    }
    __syncthreads();
    // exclusive scan of the counts (EK_KEYS / EK_BLOCK per thread)
    {
        constexpr int PT = EK_KEYS / EK_BLOCK;
        int c[PT], s = 0;
#pragma unroll
        for (int u = 0; u < PT; u++) {
            c[u] = cnt[t * PT + u];
            s += c[u];
        }
        const int incl = wave_inclusive_scan(s);
        if (lane_id() == WAVE - 1) wsum[t / WAVE] = incl;
        __syncthreads();
        int run = incl - s;
        for (int w = 0; w < t / WAVE; w++) run += wsum[w];
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PT; u++) {
            cnt[t * PT + u] = run;
            run += c[u];
        }
        if (t == EK_BLOCK - 1) {
            cnt[EK_KEYS] = run;
            if (one) *m_out = run;  // the kept rows
        }
    }
    __syncthreads();
    if (lds) {
        // order the rows by id (within an id in atomics' order), then rank
        // each row in its id's group by the remaining ids
        for (int p = t; p < rows; p += EK_BLOCK)
            if (skey[p] != DROPPED) sord[atomicAdd(&cnt[skey[p]], 1)] = (unsigned short)p;
        __syncthreads();
        const int kept = one ? cnt[EK_KEYS] : rows;
        for (int s = t; s < kept; s += EK_BLOCK) {
            const int p = sord[s];
            uint4 me;  // Size bits or candidate index
            if constexpr (SLIM) {
                me = widen(pay[bs + p]);
            } else {
                me.x = sid[0][p];
                me.y = sid[NW >= 2 ? 1 : 0][p];
                me.z = sid[NW >= 3 ? 2 : 0][p];
                me.w = NW >= 4 ? sid[NW >= 4 ? 3 : 0][p] : 0u;
            }
            const int k = skey[p];
            const int g0 = k > 0 ? cnt[k - 1] : 0, g1 = cnt[k];
            unsigned r[3];
            r[0] = sid[0][p];
            r[1] = NI >= 2 ? sid[NI >= 2 ? 1 : 0][p] : 0u;
            r[2] = NI >= 3 ? sid[NI >= 3 ? 2 : 0][p] : 0u;
            int rank = 0;
            for (int q = g0; q < g1; q++) {
                const int o = sord[q];
                const unsigned v[3] = {sid[0][o], NI >= 2 ? sid[NI >= 2 ? 1 : 0][o] : 0u,
                                       NI >= 3 ? sid[NI >= 3 ? 2 : 0][o] : 0u};
                rank += (q != s) && ids_less(v, r);
            }
            const long long pos = (long long)bs + g0 + rank;
            write_row<K>(out, pos, k0 + k, r);
            const double z = pay_size<K>(me, size_in);
            out_size[pos] = to_A2 ? z / 1.0e6 : z;
        }
        return;
    }
    // a bucket beyond LDS: rows placed in their id's group in global scratch
    // (the bucket's own range of gkey / gpay), ranked from there
    for (int p = t; p < rows; p += EK_BLOCK) {
        const unsigned kk = key[bs + p] - k0;
        const int slot = atomicAdd(&cnt[kk], 1);
        gkey[bs + slot] = kk;
        gpay[bs + slot] = pay[bs + p];
    }
    __threadfence_block();
    __syncthreads();
    for (int s = t; s < rows; s += EK_BLOCK) {
        const int k = (int)gkey[bs + s];
        const int g0 = k > 0 ? cnt[k - 1] : 0, g1 = cnt[k];
        const uint4 me = widen(gpay[bs + s]);
        unsigned r[3];
        pay_ids<K>(me, r);
        int rank = 0;
        for (int q = g0; q < g1; q++) {
            unsigned v[3];
            pay_ids<K>(widen(gpay[bs + q]), v);
            rank += (q != s) && ids_less(v, r);
        }
        const long long pos = (long long)bs + g0 + rank;
        write_row<K>(out, pos, k0 + k, r);
        const double z = pay_size<K>(me, size_in);
        out_size[pos] = to_A2 ? z / 1.0e6 : z;
    }
}

// ---------------------------------------------------------------------------
// Vertices in input order. k_vert_final writes one float64 per ball to its
// input position: its Size in mA^2, or NaN when the ball is not in K_alpha;
// the kept flags for the scan are taken from those words in order.
__global__ void __launch_bounds__(256) k_vert_flags(const double *__restrict__ vsize_in, int n, int *__restrict__ flag) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u < n) flag[u] = vsize_in[u] == vsize_in[u];  // not NaN
}

__global__ void __launch_bounds__(256) k_vert_emit(const double *__restrict__ vsize_in, const int *__restrict__ vpos,
                                                    int n, int *__restrict__ out, double *__restrict__ out_size) {
    const int u = blockIdx.x * 256 + threadIdx.x;
    if (u >= n) return;
    const double z = vsize_in[u];
    if (z != z) return;
    const int p = vpos[u];
    out[p] = u;
    out_size[p] = z / 1.0e6;  // mA^2 -> A^2
}

}  // namespace acx
