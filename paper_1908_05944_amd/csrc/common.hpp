// Shared device utilities: wave-level prefix sums and appends, a device-wide
// exclusive scan, and an order-preserving int64 encoding of float64 for
// atomicMin. Wavefronts are 64 lanes wide on gfx950.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace acx {

constexpr int WAVE = 64;

// float64 -> int64 whose signed order matches the float order (no NaNs).
__device__ __forceinline__ long long ordered_from_double(double x) {
    long long b = __double_as_longlong(x);
    return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}
__device__ __forceinline__ double double_from_ordered(long long k) {
    long long b = k >= 0 ? k : (k ^ 0x7fffffffffffffffLL);
    return __longlong_as_double(b);
}
constexpr long long ORDERED_POS_INF = 0x7ff0000000000000LL;  // +inf encoded

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with its own L2. Renumbering the blocks so that every XCD runs one
// contiguous range of the grid keeps spatially neighbouring work (and the
// data it shares) in one L2. A bijection on [0, gridDim.x).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, b = blockIdx.x;
    const int q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int x = b % NUM_XCD, k = b / NUM_XCD;
    return x * q + min(x, r) + k;
}

// The same for a launch sized for a capacity of which only the first `live`
// blocks have work (counts known on the device only): those blocks are
// spread evenly over the XCDs, each XCD taking one contiguous range of them,
// and the idle blocks map onto [live, gridDim.x). Still a bijection on
// [0, gridDim.x); with live = gridDim.x it is xcd_block().
__device__ __forceinline__ int xcd_block(int live) {
    const int nb = gridDim.x, b = blockIdx.x;
    live = min(max(live, 0), nb);
    const int x = b % NUM_XCD, k = b / NUM_XCD;
    const int q = live / NUM_XCD, r = live % NUM_XCD;  // live blocks per XCD
    const int len = q + (x < r);
    if (k < len) return x * q + min(x, r) + k;
    const int Q = nb / NUM_XCD, R = nb % NUM_XCD;  // blocks per XCD
    return live + (x * Q + min(x, R)) - (x * q + min(x, r)) + (k - len);
}

// Item count of a launch: `cap`, the count it was sized for, or, when `live`
// is given, the smaller count an earlier kernel on the stream wrote there
// (launches recorded before their counts are known, as in a captured graph).
__device__ __forceinline__ int live_count(int cap, const int *live) { return live ? min(cap, *live) : cap; }

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        int t = __shfl_up(v, off, WAVE);
        if (lane >= off) v += t;
    }
    return v;
}

// Append one item per lane where pred holds; returns the slot (or -1). Must be
// reached by every active lane of the wave together.
__device__ __forceinline__ int wave_append(int *counter, bool pred) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader, WAVE);
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    return pred ? base + rank : -1;
}

// Exclusive prefix sum over a block of nthreads (a multiple of 64) threads;
// every thread of the block must call it. *total receives the block's sum.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int *total) {
    __shared__ int wsum[NT / WAVE];
    const int incl = wave_inclusive_scan(v);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / WAVE; k++) {
        off += k < w ? wsum[k] : 0;
        tot += wsum[k];
    }
    __syncthreads();  // wsum may be reused by the next call
    *total = tot;
    return off + incl - v;
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan of int32: out[i] = sum(in[0..i)), out[n] = total.
// Tiles of SCAN_TILE items per 256-thread block; tile totals are scanned
// recursively and added back.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_IPT;

// IPT consecutive ints at p[base..base + IPT), zero past n: 16-byte loads
// when the run is whole and p is 16-byte aligned (a lane's run is one
// 16-byte-multiple piece: 4 vector instead of 16 scalar loads per thread).
template <int IPT>
__device__ __forceinline__ void load_run(const int *__restrict__ p, long long base, long long n, int (&v)[IPT]) {
    static_assert(IPT % 4 == 0, "whole int4 pieces");
    if (base + IPT <= n && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
        const int4 *q = reinterpret_cast<const int4 *>(p + base);
#pragma unroll
        for (int k = 0; k < IPT / 4; k++) {
            const int4 x = q[k];
            v[4 * k] = x.x; v[4 * k + 1] = x.y; v[4 * k + 2] = x.z; v[4 * k + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < IPT; k++) v[k] = base + k < n ? p[base + k] : 0;
    }
}
template <int IPT>
__device__ __forceinline__ void store_run(int *__restrict__ p, long long base, long long n, const int (&v)[IPT]) {
    if (base + IPT <= n && ((reinterpret_cast<uintptr_t>(p) & 15) == 0)) {
        int4 *q = reinterpret_cast<int4 *>(p + base);
#pragma unroll
        for (int k = 0; k < IPT / 4; k++) q[k] = make_int4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < IPT; k++)
            if (base + k < n) p[base + k] = v[k];
    }
}

__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_tiles(const int *__restrict__ in, int *__restrict__ out,
                                                            int *__restrict__ tile_sums, long long n) {
    __shared__ int wsum[SCAN_BLOCK / WAVE];
    const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_IPT;
    int v[SCAN_IPT];
    load_run<SCAN_IPT>(in, base, n, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) s += v[k];
    const int incl = wave_inclusive_scan(s);
    const int w = threadIdx.x / WAVE, lane = lane_id();
    if (lane == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < w; k++) woff += wsum[k];
    int run = woff + incl - s;
#pragma unroll
    for (int k = 0; k < SCAN_IPT; k++) {
        const int x = v[k];
        v[k] = run;
        run += x;
    }
    store_run<SCAN_IPT>(out, base, n, v);
    if (threadIdx.x == SCAN_BLOCK - 1) {
        int tot = 0;
        for (int k = 0; k < SCAN_BLOCK / WAVE; k++) tot += wsum[k];
        tile_sums[blockIdx.x] = tot;
    }
}

// Single-block exclusive scan for n <= SCAN_SMALL: out[0..n], out[n] = total.
// 1024 threads with 16 items each: every thread issues its loads together, so
// the scan costs about one memory latency instead of a serial walk.
constexpr int SCAN_SMALL_BLOCK = 1024;
constexpr int SCAN_SMALL_IPT = 16;
constexpr int SCAN_SMALL = SCAN_SMALL_BLOCK * SCAN_SMALL_IPT;

__global__ void __launch_bounds__(SCAN_SMALL_BLOCK) k_scan_small(const int *__restrict__ in, int *__restrict__ out,
                                                                  int n, int *__restrict__ total_to) {
    __shared__ int wsum[SCAN_SMALL_BLOCK / WAVE];
    const int base = threadIdx.x * SCAN_SMALL_IPT;
    int v[SCAN_SMALL_IPT];
    load_run<SCAN_SMALL_IPT>(in, base, n, v);
    int s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_SMALL_IPT; k++) s += v[k];
    const int incl = wave_inclusive_scan(s);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == WAVE - 1) wsum[w] = incl;
    __syncthreads();
    int run = incl - s;
    for (int k = 0; k < w; k++) run += wsum[k];
#pragma unroll
    for (int k = 0; k < SCAN_SMALL_IPT; k++) {
        const int x = v[k];
        v[k] = run;
        run += x;
    }
    store_run<SCAN_SMALL_IPT>(out, base, n, v);
    if (threadIdx.x == SCAN_SMALL_BLOCK - 1) {
        out[n] = run;
        if (total_to) *total_to = run;
    }
}

// Adds tile offsets; block 0 also writes out[n] = total (and *total_to if set).
__global__ void __launch_bounds__(SCAN_BLOCK) k_scan_add_total(int *__restrict__ out, const int *__restrict__ tile_off,
                                                                long long n, int tiles, int *__restrict__ total_to) {
    const long long base = (long long)blockIdx.x * SCAN_TILE;
    const int add = tile_off[blockIdx.x];
    for (int k = threadIdx.x; k < SCAN_TILE; k += SCAN_BLOCK) {
        const long long i = base + k;
        if (i < n) out[i] += add;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[n] = tile_off[tiles];
        if (total_to) *total_to = tile_off[tiles];
    }
}

}  // namespace acx
