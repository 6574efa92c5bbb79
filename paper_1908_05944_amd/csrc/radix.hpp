// Stable least-significant-digit radix sort of (uint32 key, payload) pairs.
//
// One pass per 8-bit digit: a tile histogram kernel (LDS counters) into the
// digit-major table [256][tiles], a prefix kernel over each digit's row, and
// a scatter kernel. In the scatter each wave owns a contiguous chunk of the
// tile and ranks its elements among equal digits with ballots and per-wave
// LDS counters (no block barrier inside the sweep); one block scan over
// (digit, wave) counts then gives every element its stable place, the tile
// is laid out in LDS in digit order and written so that each digit's run
// (about tile / 256 elements) goes to consecutive addresses: writing each
// element straight from its lane would scatter partial-line stores over the
// whole output. No global atomics are used: on MI355X
// device-scope atomics go through the memory-side fabric and run far below
// the memory bandwidth.
#pragma once
#include "common.hpp"

namespace acx {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_BLOCK = 256;
constexpr int RS_IPT = 8;
constexpr int RS_TILE = RS_BLOCK * RS_IPT;
static_assert(RS_BINS == RS_BLOCK, "one histogram bin per thread");

__global__ void __launch_bounds__(RS_BLOCK) k_rs_hist(const unsigned *__restrict__ keys, int n, int shift,
                                                       int *__restrict__ hist, int tiles,
                                                       const int *__restrict__ live = nullptr) {
    n = live_count(n, live);
    __shared__ int h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * RS_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (RS_BINS - 1)], 1);
    }
    __syncthreads();
    hist[(long long)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Per digit d (one block each): exclusive prefix over the tiles of the
// digit's row hist[d][0..tiles), in place, and the digit's total. The digit
// bases (a scan of the 256 totals) are taken by each scatter block itself.
constexpr int RS_PREFIX_BLOCK = 1024;
constexpr int RS_PREFIX_IPT = 8;

__global__ void __launch_bounds__(RS_PREFIX_BLOCK) k_rs_digit_prefix(int *__restrict__ hist, int tiles,
                                                                      int *__restrict__ totals) {
    __shared__ int wsum[RS_PREFIX_BLOCK / WAVE];
    __shared__ int carry_s;
    int *row = hist + (long long)blockIdx.x * tiles;
    int carry = 0;
    for (int c0 = 0; c0 < tiles; c0 += RS_PREFIX_BLOCK * RS_PREFIX_IPT) {
        const int base = c0 + threadIdx.x * RS_PREFIX_IPT;
        int v[RS_PREFIX_IPT];
        int s = 0;
#pragma unroll
        for (int k = 0; k < RS_PREFIX_IPT; k++) {
            v[k] = base + k < tiles ? row[base + k] : 0;
            s += v[k];
        }
        const int incl = wave_inclusive_scan(s);
        const int w = threadIdx.x / WAVE;
        if (lane_id() == WAVE - 1) wsum[w] = incl;
        __syncthreads();
        int run = carry + incl - s;
        for (int k = 0; k < w; k++) run += wsum[k];
#pragma unroll
        for (int k = 0; k < RS_PREFIX_IPT; k++) {
            if (base + k < tiles) row[base + k] = run;
            run += v[k];
        }
        if (threadIdx.x == RS_PREFIX_BLOCK - 1) carry_s = run;
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

// Payload as held in registers: a 12-byte uint3 in an array ends up in
// scratch memory, so it is widened to a uint4.
template <class P> struct RsReg { typedef P type; };
template <> struct RsReg<uint3> { typedef uint4 type; };
template <class P> __device__ __forceinline__ P rs_to_reg(const P &p) { return p; }
__device__ __forceinline__ uint4 rs_to_reg(const uint3 &p) { return make_uint4(p.x, p.y, p.z, 0u); }
template <class P, class R> __device__ __forceinline__ P rs_from_reg(const R &r) { return r; }
template <> __device__ __forceinline__ uint3 rs_from_reg<uint3, uint4>(const uint4 &r) { return make_uint3(r.x, r.y, r.z); }

template <class P>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_scatter(const unsigned *__restrict__ kin, const P *__restrict__ pin,
                                                          unsigned *__restrict__ kout, P *__restrict__ pout, int n,
                                                          int shift, const int *__restrict__ prefix,
                                                          const int *__restrict__ totals, int tiles,
                                                          const int *__restrict__ live = nullptr) {
    n = live_count(n, live);
    // consecutive tiles on one XCD: their pieces of each digit run are
    // adjacent, so the partial lines they write meet in that XCD's L2
    const int tb = xcd_block(n / RS_TILE + (n % RS_TILE != 0));
    constexpr int NW = RS_BLOCK / WAVE;
    constexpr int CHUNK = WAVE * RS_IPT;  // each wave owns a contiguous chunk of the tile
    __shared__ int gbase[RS_BINS];        // output start of each digit for this tile
    __shared__ int wcnt[NW][RS_BINS];     // per-wave digit counts, then per-wave digit starts
    __shared__ int wsum[NW];
    __shared__ unsigned skey[RS_TILE];
    __shared__ P spay[RS_TILE];
    const int lane = lane_id(), wave = threadIdx.x / WAVE;
    {
        // output start of digit d for this tile: the totals of the digits
        // below d, plus digit d's count in the tiles before this one
        const int t = totals[threadIdx.x];
        const int incl = wave_inclusive_scan(t);
        if (lane == WAVE - 1) wsum[wave] = incl;
        __syncthreads();
        int below = incl - t;
        for (int w = 0; w < wave; w++) below += wsum[w];
        gbase[threadIdx.x] = below + prefix[(long long)threadIdx.x * tiles + tb];
    }
#pragma unroll
    for (int w = 0; w < NW; w++) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    // sweep: rank each element among the equal digits of its wave so far
    const unsigned long long lt = (1ull << lane) - 1ull;
    const long long base = (long long)tb * RS_TILE + (long long)wave * CHUNK;
    // keys, payloads and ranks stay in registers; every load of the tile is
    // issued before the first ballot
    typedef typename RsReg<P>::type R;
    unsigned key[RS_IPT];
    R pv[RS_IPT];
    int rank[RS_IPT];
#pragma unroll
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * WAVE + lane;
        key[r] = idx < n ? kin[idx] : 0u;
        pv[r] = idx < n ? rs_to_reg(pin[idx]) : R{};
    }
#pragma unroll
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * WAVE + lane;
        const bool valid = idx < n;
        const unsigned d = (key[r] >> shift) & (RS_BINS - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < RS_BITS; bit++) {
            const unsigned long long m = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? m : ~m;
        }
        const int leader = valid ? __ffsll((long long)peers) - 1 : 0;
        int old = 0;
        if (valid && lane == leader) {
            old = wcnt[wave][d];
            wcnt[wave][d] = old + __popcll(peers);
        }
        old = __shfl(old, leader, WAVE);
        rank[r] = valid ? old + __popcll(peers & lt) : -1;
    }
    __syncthreads();
    // tile-local start of (digit, wave): digits in order, waves in order
    {
        const int d = threadIdx.x;
        int c[NW], tot = 0;
#pragma unroll
        for (int w = 0; w < NW; w++) { c[w] = wcnt[w][d]; tot += c[w]; }
        const int incl = wave_inclusive_scan(tot);
        if (lane == WAVE - 1) wsum[wave] = incl;
        __syncthreads();
        int start = incl - tot;
        for (int w = 0; w < wave; w++) start += wsum[w];
#pragma unroll
        for (int w = 0; w < NW; w++) { wcnt[w][d] = start; start += c[w]; }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RS_IPT; r++) {
        if (rank[r] < 0) continue;
        const unsigned d = (key[r] >> shift) & (RS_BINS - 1);
        const int lpos = wcnt[wave][d] + rank[r];
        skey[lpos] = key[r];
        spay[lpos] = rs_from_reg<P>(pv[r]);
    }
    __syncthreads();
    // the tile in digit order: each digit's run goes to consecutive addresses;
    // a digit's tile-local start is the start of its first wave
    const long long tbase = (long long)tb * RS_TILE;
    const int cnt = (int)min((long long)RS_TILE, (long long)n - tbase);
    for (int p = threadIdx.x; p < cnt; p += RS_BLOCK) {
        const unsigned k = skey[p];
        const unsigned d = (k >> shift) & (RS_BINS - 1);
        const int g = gbase[d] + (p - wcnt[0][d]);
        kout[g] = k;
        pout[g] = spay[p];
    }
}

// Starts of key ranges in sorted keys: start[c] = the first row whose
// key >> shift is at least c, for c = 0..nb (rows sorted by key >> shift; row
// p, 0 <= p <= m, writes the starts of the ranges in (range of row p - 1,
// range of row p], with row m in range nb). The bucket starts of the emit
// (every bucket holds rows, so each thread fills only a few starts). A thread
// takes KS_PT consecutive rows (one 16-byte load); `key` is 16-byte aligned.
// One pass over the keys: no count array, no scan.
constexpr int KS_BLOCK = 256;
constexpr int KS_PT = 4;
__global__ void __launch_bounds__(KS_BLOCK) k_key_starts(const unsigned *__restrict__ key, int m, int shift, int nb,
                                                        int *__restrict__ start, const int *__restrict__ live = nullptr) {
    m = live_count(m, live);
    const long long p0 = ((long long)blockIdx.x * KS_BLOCK + threadIdx.x) * KS_PT;
    if (p0 > m) return;
    unsigned k[KS_PT];
    if (p0 + KS_PT <= m) {
        const uint4 v = *reinterpret_cast<const uint4 *>(key + p0);
        k[0] = v.x; k[1] = v.y; k[2] = v.z; k[3] = v.w;
    } else {
#pragma unroll
        for (int u = 0; u < KS_PT; u++) k[u] = p0 + u < m ? key[p0 + u] : 0u;
    }
    int prev = p0 == 0 ? -1 : min((int)(key[p0 - 1] >> shift), nb);
#pragma unroll
    for (int u = 0; u < KS_PT; u++) {
        const long long p = p0 + u;
        if (p > m) break;
        const int cur = p == m ? nb : min((int)(k[u] >> shift), nb);
        for (int c = prev + 1; c <= cur; c++) start[c] = (int)p;
        prev = cur;
    }
}

}  // namespace acx
