// Stable least-significant-digit radix sort of (uint32 key, payload) pairs.
//
// One pass per 8-bit digit: a tile histogram kernel (LDS counters), a
// device-wide exclusive scan of the digit-major table [256][tiles], and a
// scatter kernel. The scatter ranks each tile's elements stably by digit
// (wave-level match by ballots, waves taking their offsets in order), places
// them in LDS in digit order, and then writes the tile out so that each
// digit's run (about tile / 256 elements) goes to consecutive addresses:
// writing each element straight from its lane would scatter partial-line
// stores over the whole output. No global atomics are used: on MI355X
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
                                                       int *__restrict__ hist, int tiles) {
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

template <class P>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_scatter(const unsigned *__restrict__ kin, const P *__restrict__ pin,
                                                          unsigned *__restrict__ kout, P *__restrict__ pout, int n,
                                                          int shift, const int *__restrict__ offs,
                                                          const int *__restrict__ hist, int tiles) {
    __shared__ int gbase[RS_BINS];  // output start of each digit for this tile
    __shared__ int lbase[RS_BINS];  // start of each digit inside the tile
    __shared__ int run[RS_BINS];
    __shared__ int grp[RS_BLOCK / WAVE][WAVE];
    __shared__ int wsum[RS_BLOCK / WAVE];
    __shared__ unsigned skey[RS_TILE];
    __shared__ P spay[RS_TILE];
    const int lane = lane_id(), wave = threadIdx.x / WAVE;
    gbase[threadIdx.x] = offs[(long long)threadIdx.x * tiles + blockIdx.x];
    {
        // tile-local exclusive scan of this tile's digit counts
        const int h = hist[(long long)threadIdx.x * tiles + blockIdx.x];
        const int incl = wave_inclusive_scan(h);
        if (lane == WAVE - 1) wsum[wave] = incl;
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wave; w++) off += wsum[w];
        lbase[threadIdx.x] = off + incl - h;
    }
    run[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long lt = (1ull << lane) - 1ull;
    const long long base = (long long)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * RS_BLOCK + threadIdx.x;
        const bool valid = idx < n;
        unsigned key = 0;
        P pay{};
        if (valid) { key = kin[idx]; pay = pin[idx]; }
        const unsigned d = (key >> shift) & (RS_BINS - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RS_BITS; b++) {
            const unsigned long long m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const int leader = valid ? __ffsll((long long)peers) - 1 : 0;
        const int rank = __popcll(peers & lt);
        // waves take their offsets in order, so equal digits keep input order
        for (int w = 0; w < RS_BLOCK / WAVE; w++) {
            if (wave == w && valid && lane == leader) {
                const int old = run[d];
                run[d] = old + __popcll(peers);
                grp[w][lane] = old;
            }
            __syncthreads();
        }
        if (valid) {
            const int lpos = lbase[d] + grp[wave][leader] + rank;
            skey[lpos] = key;
            spay[lpos] = pay;
        }
        __syncthreads();
    }
    // the tile in digit order: each digit's run goes to consecutive addresses
    const int cnt = (int)min((long long)RS_TILE, (long long)n - base);
    for (int p = threadIdx.x; p < cnt; p += RS_BLOCK) {
        const unsigned key = skey[p];
        const unsigned d = (key >> shift) & (RS_BINS - 1);
        const int g = gbase[d] + (p - lbase[d]);
        kout[g] = key;
        pout[g] = spay[p];
    }
}

}  // namespace acx
