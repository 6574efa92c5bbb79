// Emit: the kept simplices as rows of input ids, ascending inside a row, rows
// in lexicographic order, each with its Size (Sec. 2.3; the paper outputs
// membership only).
//
// The pruning kernels key every candidate by the least input id of its row
// (not kept: n, after every id) with the remaining ids and its Size (for a
// tetrahedron: its candidate index) as payload. A stable LSD radix pass over
// the high bits of the key (one 8-bit pass below 2^22 balls, two above)
// groups the rows into coarse buckets; k_emit_bucket then finishes EB_KEYS
// consecutive keys per block: the per-key counts by LDS atomics and their
// scan give every key's place, each row is put in its key's group, and its
// rank in the group by the remaining ids gives its final place. The rows of
// one key are few (a ball's upper edges, triangles or tetrahedra), so the
// rank is a short walk; no global atomics and no device-wide sort passes over
// the low bits.
#pragma once
#include "common.hpp"

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
// candidate index c (K = 4). Not kept: key n, empty payload.
template <int K>
__device__ __forceinline__ void emit_pack(bool kept, int (&v)[4], double size, int c, int n, unsigned &key,
                                          typename EmitPay<K>::type &pay) {
    pay = typename EmitPay<K>::type{};
    if (!kept) {
        key = (unsigned)n;
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

template <int K>
__device__ __forceinline__ void pay_ids(const typename EmitPay<K>::type &q, unsigned (&r)[3]) {
    if constexpr (K == 2) { r[0] = q.x; r[1] = 0; r[2] = 0; }
    else if constexpr (K == 3) { r[0] = q.x; r[1] = q.y; r[2] = 0; }
    else { r[0] = q.x; r[1] = q.y; r[2] = q.z; }
}

template <int K>
__device__ __forceinline__ double pay_size(const typename EmitPay<K>::type &q, const double *__restrict__ size) {
    if constexpr (K == 2) return double_of(q.y, q.z);
    else if constexpr (K == 3) return double_of(q.z, q.w);
    else return size[q.w];
}

// First position p in [0, m) with (key[p] >> shift) >= b (key sorted by key >> shift).
__device__ __forceinline__ int coarse_lower_bound(const unsigned *__restrict__ key, int m, int shift, long long b) {
    int lo = 0, hi = m;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)(key[mid] >> shift) < b) lo = mid + 1; else hi = mid;
    }
    return lo;
}

constexpr int EB_KEYS = 4096;   // keys finished by one block
constexpr int EB_BLOCK = 512;
constexpr int EB_PER_THREAD = EB_KEYS / EB_BLOCK;

// Block b finishes the keys [b EB_KEYS, (b + 1) EB_KEYS) of key / pay (m rows
// sorted by key >> shift), using gkey / gpay (m entries) as scratch, and
// writes the kept rows (key < n) to out / out_size at their final places;
// the block holding key n writes the kept count to *m_out (the host sets it
// to m beforehand, for when every row is kept). Sizes are converted from
// mA^2 to A^2 when to_A2 is set (emit of a build), else copied (merge of
// rows that are already output).
template <int K>
__global__ void __launch_bounds__(EB_BLOCK) k_emit_bucket(const unsigned *__restrict__ key,
                                                           const typename EmitPay<K>::type *__restrict__ pay, int m,
                                                           int n, int shift, unsigned *__restrict__ gkey,
                                                           typename EmitPay<K>::type *__restrict__ gpay,
                                                           const double *__restrict__ size_in, int to_A2,
                                                           int *__restrict__ out, double *__restrict__ out_size,
                                                           int *__restrict__ m_out, const int *__restrict__ live = nullptr) {
    typedef typename EmitPay<K>::type P;
    m = live_count(m, live);
    __shared__ int cnt[EB_KEYS];  // per-key counts, then each key's first place in the block's range
    __shared__ int cur[EB_KEYS];  // placement cursors
    __shared__ int wsum[EB_BLOCK / WAVE];
    __shared__ int below_s;
    const long long k0 = (long long)blockIdx.x * EB_KEYS;
    const int t = threadIdx.x;
    // the rows of the coarse buckets that hold this block's keys
    const int bs = coarse_lower_bound(key, m, shift, k0 >> shift);
    const int be = coarse_lower_bound(key, m, shift, ((k0 + EB_KEYS - 1) >> shift) + 1);
#pragma unroll
    for (int u = 0; u < EB_PER_THREAD; u++) cnt[u * EB_BLOCK + t] = 0;
    if (t == 0) below_s = 0;
    __syncthreads();
    // sweep 1: counts per key; rows of the buckets with keys below this block's
    int below = 0;
    for (int e = bs + t; e < be; e += EB_BLOCK) {
        const long long kk = key[e];
        if (kk < k0) below++;
        else if (kk < k0 + EB_KEYS) atomicAdd(&cnt[kk - k0], 1);
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) below += __shfl_down(below, off, WAVE);
    if (lane_id() == 0 && below) atomicAdd(&below_s, below);
    __syncthreads();
    // exclusive scan of the counts: EB_PER_THREAD consecutive keys per thread
    int c[EB_PER_THREAD], s = 0;
#pragma unroll
    for (int u = 0; u < EB_PER_THREAD; u++) {
        c[u] = cnt[t * EB_PER_THREAD + u];
        s += c[u];
    }
    const int incl = wave_inclusive_scan(s);
    if (lane_id() == WAVE - 1) wsum[t / WAVE] = incl;
    __syncthreads();
    int run = incl - s, total = 0;
#pragma unroll
    for (int w = 0; w < EB_BLOCK / WAVE; w++) {
        run += w < t / WAVE ? wsum[w] : 0;
        total += wsum[w];
    }
#pragma unroll
    for (int u = 0; u < EB_PER_THREAD; u++) {
        cnt[t * EB_PER_THREAD + u] = run;
        cur[t * EB_PER_THREAD + u] = run;
        run += c[u];
    }
    __syncthreads();
    const int gs = bs + below_s;  // global place of the block's first row
    // the kept rows of the range end where key n starts (if n is in it)
    const bool has_n = (long long)n >= k0 && (long long)n < k0 + EB_KEYS;
    const int kept_end = has_n ? cnt[n - k0] : total;
    if (has_n && t == 0) *m_out = gs + kept_end;
    // sweep 2: every kept row into its key's group (order inside a group is
    // the atomics' order; the rank below fixes it)
    for (int e = bs + t; e < be; e += EB_BLOCK) {
        const long long kk = key[e];
        if (kk < k0 || kk >= k0 + EB_KEYS || kk >= n) continue;
        const int p = atomicAdd(&cur[kk - k0], 1);
        gkey[gs + p] = (unsigned)kk;
        gpay[gs + p] = pay[e];
    }
    __syncthreads();
    // sweep 3: rank inside the group by the remaining ids, then the final write
    for (int p = t; p < kept_end; p += EB_BLOCK) {
        const unsigned kk = gkey[gs + p];
        const int loc = (int)(kk - k0);
        const int g0 = cnt[loc], g1 = loc + 1 < EB_KEYS ? cnt[loc + 1] : total;
        const P me = gpay[gs + p];
        unsigned r[3];
        pay_ids<K>(me, r);
        int rank = 0;
        for (int q = g0; q < g1; q++) {
            if (q == p) continue;
            unsigned o[3];
            pay_ids<K>(gpay[gs + q], o);
            rank += o[0] != r[0] ? o[0] < r[0] : (o[1] != r[1] ? o[1] < r[1] : o[2] < r[2]);
        }
        const long long pos = (long long)gs + g0 + rank;
        out[pos * K] = (int)kk;
#pragma unroll
        for (int u = 1; u < K; u++) out[pos * K + u] = (int)r[u - 1];
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
