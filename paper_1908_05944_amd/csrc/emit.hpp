// Emit: the kept simplices as rows of input ids, ascending inside a row, rows
// in lexicographic order, each with its Size (Sec. 2.3; the paper outputs
// membership only).
//
// The pruning kernels key every candidate by the least input id of its row
// with the remaining ids and its Size (for a tetrahedron: its candidate
// index) as payload; a candidate that is not kept gets the drop key, the
// first key of the coarse bucket after every input id's. A stable LSD radix
// pass over the high bits of the key (one 8-bit pass below 2^22 balls, two
// above) groups the rows into coarse buckets, the dropped rows in one bucket
// of their own at the end; k_emit_bucket then finishes EB_KEYS consecutive
// keys per block: the per-key counts by LDS atomics and their scan give every
// key's place, each row is put in its key's group, and its rank in the group
// by the remaining ids gives its final place. The rows of one key are few (a
// ball's upper edges, triangles or tetrahedra), so the rank is a short walk;
// no global atomics, no device-wide sort passes over the low bits, and (above
// 2^19 balls, where coarse buckets are whole multiples of a block's keys) no
// block reads the dropped rows.
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
constexpr int EB_BATCH1 = 32;  // keys per thread loaded together in the counting sweep
constexpr int EB_BATCH2 = 8;   // rows per thread loaded together in the placing sweep
constexpr int EB_WIN = 2048;   // rows ranked together in LDS

// Block b finishes the keys [b EB_KEYS, (b + 1) EB_KEYS) of key / pay (m rows
// sorted by key >> shift), using gkey / gpay (m entries) as scratch, and
// writes the kept rows (key < drop) to out / out_size at their final places;
// the last block writes the kept count to *m_out. The grid covers the input
// ids, so every block's first key lies below the drop key, whose coarse
// bucket follows all others. Sizes are converted from mA^2 to A^2 when to_A2
// is set (emit of a build), else copied (merge of rows that are already
// output).
template <int K>
__global__ void __launch_bounds__(EB_BLOCK) k_emit_bucket(const unsigned *__restrict__ key,
                                                           const typename EmitPay<K>::type *__restrict__ pay, int m,
                                                           unsigned drop, int shift, unsigned *__restrict__ gkey,
                                                           typename EmitPay<K>::type *__restrict__ gpay,
                                                           const double *__restrict__ size_in, int to_A2,
                                                           int *__restrict__ out, double *__restrict__ out_size,
                                                           int *__restrict__ m_out, const int *__restrict__ digit_tot,
                                                           const int *__restrict__ live = nullptr) {
    typedef typename EmitPay<K>::type P;
    m = live_count(m, live);
    __shared__ int cnt[EB_KEYS];  // per-key counts, then each key's first place in the block's range
    // placement cursors (int[EB_KEYS]) in sweeps 1-2, then the window of rows
    // ranked in LDS in sweep 3
    __shared__ uint4 sh[EB_WIN];
    static_assert(sizeof(uint4) * EB_WIN >= sizeof(int) * EB_KEYS, "the cursors fit in the row window");
    int *const cur = reinterpret_cast<int *>(sh);
    __shared__ int wsum[EB_BLOCK / WAVE];
    __shared__ int below_s;
    const long long k0 = (long long)blockIdx.x * EB_KEYS;
    const int t = threadIdx.x;
    // the rows of the coarse buckets that hold this block's keys: from the
    // digit totals of a single radix pass (the coarse bucket is the digit),
    // else by binary search
    const int c_lo = (int)(k0 >> shift), c_hi = (int)((k0 + EB_KEYS - 1) >> shift) + 1;
    int bs, be;
    if (digit_tot) {
        __shared__ int part[2][EB_BLOCK / WAVE];
        int a = 0, b = 0;
        if (t < RS_BINS) {
            const int v = digit_tot[t];
            a = t < c_lo ? v : 0;
            b = t < c_hi ? v : 0;
        }
        for (int off = WAVE / 2; off > 0; off >>= 1) {
            a += __shfl_down(a, off, WAVE);
            b += __shfl_down(b, off, WAVE);
        }
        if (lane_id() == 0) {
            part[0][t / WAVE] = a;
            part[1][t / WAVE] = b;
        }
        __syncthreads();
        bs = 0;
        be = 0;
#pragma unroll
        for (int w = 0; w < EB_BLOCK / WAVE; w++) {
            bs += part[0][w];
            be += part[1][w];
        }
    } else {
        bs = coarse_lower_bound(key, m, shift, c_lo);
        be = coarse_lower_bound(key, m, shift, c_hi);
    }
#pragma unroll
    for (int u = 0; u < EB_PER_THREAD; u++) cnt[u * EB_BLOCK + t] = 0;
    if (t == 0) below_s = 0;
    __syncthreads();
    // sweep 1: counts per key; rows of the buckets with keys below this block's.
    // The sweeps load a batch of entries per thread before using any (one
    // latency per batch, not per entry); keys are below 2^31, and a slot past
    // the range holds 0xffffffff, which no test takes.
    const unsigned ku0 = (unsigned)k0, ku1 = (unsigned)min(k0 + EB_KEYS, (long long)drop);
    int below = 0;
    for (int e0 = bs + t; e0 < be; e0 += EB_BLOCK * EB_BATCH1) {
        unsigned kb[EB_BATCH1];
#pragma unroll
        for (int u = 0; u < EB_BATCH1; u++) {
            const int e = e0 + u * EB_BLOCK;
            kb[u] = e < be ? key[e] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < EB_BATCH1; u++) {
            const unsigned kk = kb[u];
            if (kk < ku0) below++;  // kept: k0 < drop
            else if (kk < ku1) atomicAdd(&cnt[kk - ku0], 1);
        }
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
    const int kept_end = total;
    if (blockIdx.x == gridDim.x - 1 && t == 0) *m_out = coarse_lower_bound(key, m, shift, (long long)(drop >> shift));
    // sweep 2: every kept row into its key's group (order inside a group is
    // the atomics' order; the rank below fixes it)
    for (int e0 = bs + t; e0 < be; e0 += EB_BLOCK * EB_BATCH2) {
        unsigned kb[EB_BATCH2];
        uint4 pb[EB_BATCH2];
#pragma unroll
        for (int u = 0; u < EB_BATCH2; u++) {
            const int e = e0 + u * EB_BLOCK;
            kb[u] = e < be ? key[e] : 0xffffffffu;
        }
#pragma unroll
        for (int u = 0; u < EB_BATCH2; u++) {
            const bool mine = kb[u] >= ku0 && kb[u] < ku1;
            pb[u] = mine ? widen(pay[e0 + u * EB_BLOCK]) : make_uint4(0u, 0u, 0u, 0u);
        }
#pragma unroll
        for (int u = 0; u < EB_BATCH2; u++) {
            const unsigned kk = kb[u];
            if (kk < ku0 || kk >= ku1) continue;
            const int p = atomicAdd(&cur[kk - ku0], 1);
            gkey[gs + p] = kk;
            gpay[gs + p] = narrow<P>(pb[u]);
        }
    }
    __syncthreads();
    // sweep 3: rank inside the group by the remaining ids, then the final
    // write. The placed rows go through LDS in windows of at most EB_WIN rows
    // that end at a group boundary, so each rank walk reads its group from
    // LDS (a group longer than a window, which the keys here never have, is
    // cut and its rows beyond the window read from global memory).
    for (int w0 = 0; w0 < kept_end;) {
        int w1 = min(w0 + EB_WIN, kept_end);
        if (w1 < kept_end) {
            const int gb = cnt[gkey[gs + w1] - k0];  // start of the group holding row w1
            if (gb > w0) w1 = gb;
        }
        __syncthreads();  // the previous window is done with sh (and sweep 2 with the cursors)
        for (int p = w0 + t; p < w1; p += EB_BLOCK) sh[p - w0] = widen(gpay[gs + p]);
        __syncthreads();
        for (int p = w0 + t; p < w1; p += EB_BLOCK) {
            const unsigned kk = gkey[gs + p];
            const int loc = (int)(kk - k0);
            const int g0 = cnt[loc], g1 = loc + 1 < EB_KEYS ? cnt[loc + 1] : total;
            const uint4 me = sh[p - w0];
            unsigned r[3];
            pay_ids<K>(me, r);
            int rank = 0;
            for (int q = g0; q < g1; q++) {
                if (q == p) continue;
                const uint4 o = q >= w0 && q < w1 ? sh[q - w0] : widen(gpay[gs + q]);
                unsigned v[3];
                pay_ids<K>(o, v);
                rank += v[0] != r[0] ? v[0] < r[0] : (v[1] != r[1] ? v[1] < r[1] : v[2] < r[2]);
            }
            const long long pos = (long long)gs + g0 + rank;
            out[pos * K] = (int)kk;
#pragma unroll
            for (int c = 1; c < K; c++) out[pos * K + c] = (int)r[c - 1];
            const double z = pay_size<K>(me, size_in);
            out_size[pos] = to_A2 ? z / 1.0e6 : z;
        }
        w0 = w1;
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
