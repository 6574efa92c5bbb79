// Stable least-significant-digit radix sort of (uint32 key, payload) pairs.
//
// One pass per 8-bit digit: a tile histogram kernel (LDS counters), a
// device-wide exclusive scan of the digit-major table [256][tiles], and a
// scatter kernel that ranks each tile's elements stably by digit (wave-level
// match by ballots, waves taking their offsets in order) and writes them to
// their final place for that pass. No global atomics are used: on MI355X
// device-scope atomics go through the memory-side fabric and are far slower
// than LDS traffic.
#pragma once
#include "common.hpp"

namespace acx {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_BLOCK = 256;
constexpr int RS_IPT = 16;
constexpr int RS_TILE = RS_BLOCK * RS_IPT;
static_assert(RS_BINS == RS_BLOCK, "one histogram bin per thread");

__global__ void __launch_bounds__(RS_BLOCK) k_rs_hist(const unsigned *__restrict__ keys, int n, int shift,
                                                       int *__restrict__ hist, int tiles) {
    __shared__ int h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * RS_TILE;
#pragma unroll 4
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
                                                          int shift, const int *__restrict__ offs, int tiles) {
    __shared__ int gbase[RS_BINS];
    __shared__ int run[RS_BINS];
    __shared__ int grp[RS_BLOCK / WAVE][WAVE];
    gbase[threadIdx.x] = offs[(long long)threadIdx.x * tiles + blockIdx.x];
    run[threadIdx.x] = 0;
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
            const int pos = gbase[d] + grp[wave][leader] + rank;
            kout[pos] = key;
            pout[pos] = pay;
        }
        __syncthreads();
    }
}

}  // namespace acx
