// Stable least-significant-digit radix sort of (uint32 key, payload) pairs.
//
// One pass per digit of BITS bits (8 or 11): a tile histogram kernel (LDS
// counters), a device-wide exclusive scan of the digit-major table
// [2^BITS][tiles], and a scatter kernel that ranks each tile's elements
// stably by digit (wave-level match by ballots, waves taking their offsets in
// order) and writes them to their final place for that pass. Wider digits
// mean fewer passes over the data (22-bit keys: 2 passes instead of 3) for a
// larger offset table. No global atomics are used: on MI355X
// device-scope atomics go through the memory-side fabric and are far slower
// than LDS traffic.
#pragma once
#include "common.hpp"

namespace acx {

constexpr int RS_BLOCK = 256;
constexpr int RS_IPT = 16;
constexpr int RS_TILE = RS_BLOCK * RS_IPT;

template <int BITS>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_hist(const unsigned *__restrict__ keys, int n, int shift,
                                                       int *__restrict__ hist, int tiles) {
    constexpr int BINS = 1 << BITS;
    __shared__ int h[BINS];
    for (int b = threadIdx.x; b < BINS; b += RS_BLOCK) h[b] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * RS_TILE;
#pragma unroll 4
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * RS_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & (BINS - 1)], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < BINS; b += RS_BLOCK) hist[(long long)b * tiles + blockIdx.x] = h[b];
}

template <class P, int BITS>
__global__ void __launch_bounds__(RS_BLOCK) k_rs_scatter(const unsigned *__restrict__ kin, const P *__restrict__ pin,
                                                          unsigned *__restrict__ kout, P *__restrict__ pout, int n,
                                                          int shift, const int *__restrict__ offs, int tiles) {
    constexpr int BINS = 1 << BITS;
    __shared__ int gbase[BINS];
    __shared__ int run[BINS];
    __shared__ int grp[RS_BLOCK / WAVE][WAVE];
    for (int b = threadIdx.x; b < BINS; b += RS_BLOCK) {
        gbase[b] = offs[(long long)b * tiles + blockIdx.x];
        run[b] = 0;
    }
    __syncthreads();
    const int lane = lane_id(), wave = threadIdx.x / WAVE;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const long long base = (long long)blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_IPT; r++) {
        const long long idx = base + (long long)r * RS_BLOCK + threadIdx.x;
        const bool valid = idx < n;
        unsigned key = 0;
        P pay{};
        if (valid) { key = kin[idx]; pay = pin[idx]; }
        const unsigned d = (key >> shift) & (BINS - 1);
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; b++) {
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
            const int pos = gbase[d] + grp[wave][leader] + rank;
            kout[pos] = key;
            pout[pos] = pay;
        }
        __syncthreads();
    }
}

}  // namespace acx
