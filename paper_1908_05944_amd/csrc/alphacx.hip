// libalphacx: host orchestration and the C ABI declared in include/alphacx.h.
//
// One call runs the whole pipeline of kernels.hpp on one HIP stream. Device
// memory comes from a per-device caching pool, so repeated calls of similar
// size allocate nothing from the runtime after the first.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <limits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <queue>
#include <string>
#include <thread>
#include <vector>

#include "alphacx.h"
#include "kernels.hpp"
#include "measure.hpp"
#include "sweep.hpp"
#include "partition.hpp"
#include "plan.hpp"

using namespace acx;

// ---------------------------------------------------------------------------
// Errors
static thread_local std::string g_last_error;

static ac_status set_error(ac_status st, const std::string &msg) {
    g_last_error = msg;
    return st;
}

struct HipError {
    ac_status st;
    std::string msg;
};

#define HIP_TRY(expr)                                                                                         \
    do {                                                                                                      \
        hipError_t e_ = (expr);                                                                               \
        if (e_ != hipSuccess) {                                                                               \
            throw HipError{e_ == hipErrorOutOfMemory ? AC_E_NOMEM : AC_E_DEVICE,                              \
                           std::string(#expr) + ": " + hipGetErrorString(e_)};                                \
        }                                                                                                     \
    } while (0)

#define LAUNCH_CHECK() HIP_TRY(hipGetLastError())

// ---------------------------------------------------------------------------
// Caching device allocator: blocks are kept per device and size class (next
// power of two) and reused; nothing is returned to the runtime until
// ac_release_workspace().
namespace {
struct Pool {
    std::mutex mu;
    std::map<int, std::multimap<size_t, void *>> free_blocks;  // device -> size -> ptr
    std::map<void *, std::pair<int, size_t>> live;
};
Pool &pool() {
    static Pool *p = new Pool();
    return *p;
}
size_t size_class(size_t n) {
    size_t c = 256;
    while (c < n) c <<= 1;
    return c;
}
}  // namespace

// Bump allocation from a caller-provided region instead of the pool, set for
// the duration of one call on the calling thread (the no-allocation entry
// point): every device buffer of the call, results included, then comes from
// that region, and read-backs go to pageable memory, so the call makes no
// allocation of its own.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
};
static thread_local Arena *t_arena = nullptr;

// Allocations of a recorded build (ac_plan), kept for the plan's lifetime:
// the first fixed run takes pool blocks and records them in order; the run
// that is captured in a graph gets the same blocks back in the same order (its
// requests are the same, since every size is fixed), so the graph's launches
// address memory the plan owns.
struct Recorder {
    std::vector<std::pair<void *, size_t>> blocks;
    size_t next = 0;
    bool replay = false;
};
static thread_local Recorder *t_rec = nullptr;

static void *dev_alloc(size_t n) {
    if (Arena *a = t_arena) {
        const size_t at = (a->used + 255) & ~(size_t)255;
        if (n > a->cap || at > a->cap - n)
            throw HipError{AC_E_CAPACITY, "the call needs more than the " + std::to_string(a->cap >> 20) +
                                              " MiB of fixed scratch (" + std::to_string((at + n) >> 20) +
                                              " MiB requested so far)"};
        a->used = at + n;
        a->peak = std::max(a->peak, a->used);
        return a->base + at;
    }
    if (Recorder *r = t_rec) {
        if (r->replay) {
            if (r->next >= r->blocks.size() || r->blocks[r->next].second < n)
                throw HipError{AC_E_DEVICE, "internal error: a recorded build asked for other buffers than recorded"};
            return r->blocks[r->next++].first;
        }
        t_rec = nullptr;  // a pool block, recorded
        void *p = nullptr;
        try {
            p = dev_alloc(n);
        } catch (...) {
            t_rec = r;
            throw;
        }
        t_rec = r;
        r->blocks.emplace_back(p, n);
        return p;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const size_t c = size_class(n ? n : 1);
    Pool &P = pool();
    {
        std::lock_guard<std::mutex> g(P.mu);
        auto &fb = P.free_blocks[dev];
        auto it = fb.find(c);
        if (it != fb.end()) {
            void *p = it->second;
            fb.erase(it);
            P.live[p] = {dev, c};
            return p;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, c);
    if (e != hipSuccess) {
        // drop cached blocks of this device and retry once
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> g(P.mu);
            for (auto &kv : P.free_blocks[dev]) (void)hipFree(kv.second);
            P.free_blocks[dev].clear();
        }
        HIP_TRY(hipMalloc(&p, c));
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.live[p] = {dev, c};
    return p;
}

static void dev_free(void *p) {
    if (!p) return;
    if (const Arena *a = t_arena)
        if (static_cast<char *>(p) >= a->base && static_cast<char *>(p) < a->base + a->cap) return;
    if (t_rec) return;  // recorded blocks belong to the plan
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    auto it = P.live.find(p);
    if (it == P.live.end()) return;
    P.free_blocks[it->second.first].emplace(it->second.second, p);
    P.live.erase(it);
}

// Allocations of one call, returned to the pool when the call ends.
struct Scope {
    std::vector<void *> held;
    template <class T>
    T *get(size_t count) {
        void *p = dev_alloc(count * sizeof(T));
        held.push_back(p);
        return static_cast<T *>(p);
    }
    ~Scope() {
        for (void *p : held) dev_free(p);
    }
};

// ---------------------------------------------------------------------------
// Result object
struct ac_complex {
    int64_t count[4] = {0, 0, 0, 0};
    int64_t cand[4] = {0, 0, 0, 0};
    int64_t fallbacks = 0;
    int64_t work[2] = {0, 0};
    int64_t n = 0;  // balls in the input
    int64_t n_mol = 1;
    int64_t alpha_q = 0;  // the alpha the complex was built at (mA^2)
    bool batch = false;   // made by ac_alpha_complex_batch
    std::vector<int64_t> mol_rows[4];  // per dimension: first row of each molecule, n_mol + 1 entries
    std::vector<int32_t> h_mol[4];     // per dimension: molecule of each row (built on first ac_molecule)
    int32_t *d_simp[4] = {nullptr, nullptr, nullptr, nullptr};
    double *d_size[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<int32_t> h_simp[4];
    std::vector<double> h_size[4];
    bool host_ready[4] = {false, false, false, false};
    bool device_result = false;
    int device = 0;
    double stage_ms[32];
    // vertex -> incidence slots of the simplices, built on first use by the
    // union-measure backward (slot of corner k of simplex s of dimension d:
    // sum_{e<d} count[e] (e+1) + s (d+1) + k)
    int32_t *inc_slot = nullptr;
    int32_t *inc_start = nullptr;
    // work buffers of the union-measure calls, kept with the complex so that
    // those calls need no allocation or host synchronisation after the first
    double *meas_part = nullptr;    // block partial sums of V and A, then V, A
    double4 *meas_contrib = nullptr;  // per incidence slot gradient terms
};

static void free_complex(ac_complex *c) {
    if (!c) return;
    for (int d = 0; d < 4; d++) {
        dev_free(c->d_simp[d]);
        dev_free(c->d_size[d]);
    }
    dev_free(c->inc_slot);
    dev_free(c->inc_start);
    dev_free(c->meas_part);
    dev_free(c->meas_contrib);
    delete c;
}

// ---------------------------------------------------------------------------
static inline unsigned grid_for(long long n) {
    long long b = (n + BLOCK - 1) / BLOCK;
    return (unsigned)(b < 1 ? 1 : b);
}

template <class T>
static void fill(T *p, T v, long long n, hipStream_t s) {
    if (n <= 0) return;
    long long b = (n + BLOCK - 1) / BLOCK;
    if (b > 65536) b = 65536;
    k_fill<T><<<(unsigned)b, BLOCK, 0, s>>>(p, v, n);
    LAUNCH_CHECK();
}

// out[0..n] = exclusive scan of in[0..n), out[n] = total (also stored to
// *total_to when given). One launch up to SCAN_SMALL items, three above
// (tile scan, scan of tile sums, add).
static void scan_i32(const int *in, int *out, long long n, hipStream_t s, Scope &sc, int *total_to = nullptr) {
    if (n <= 0) {
        fill<int>(out, 0, 1, s);
        if (total_to) fill<int>(total_to, 0, 1, s);
        return;
    }
    if (n <= SCAN_SMALL) {
        k_scan_small<<<1, SCAN_SMALL_BLOCK, 0, s>>>(in, out, (int)n, total_to);
        LAUNCH_CHECK();
        return;
    }
    const long long tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int *sums = sc.get<int>(tiles);
    int *offs = sc.get<int>(tiles + 1);
    k_scan_tiles<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, out, sums, n);
    LAUNCH_CHECK();
    scan_i32(sums, offs, tiles, s, sc);
    k_scan_add_total<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(out, offs, n, (int)tiles, total_to);
    LAUNCH_CHECK();
}

// Pinned host block of this thread for device-to-host read-backs (a copy to
// pageable memory takes a slower staged path). Every use synchronises the
// stream before the block is read or reused, so one block per thread serves
// all calls; it is kept until the process ends.
static void *pinned_block(size_t bytes) {
    thread_local void *p = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (p) HIP_TRY(hipHostFree(p));
        p = nullptr;
        cap = 0;
        const size_t c = std::max<size_t>(bytes, 4096);
        HIP_TRY(hipHostMalloc(&p, c, hipHostMallocPortable));
        cap = c;
    }
    return p;
}

// Copies n items from the device into h through the pinned block (synchronises s).
template <class T>
static void read_back(T *h, const T *d, size_t n, hipStream_t s) {
    if (n == 0) return;
    if (t_arena) {
        // no pinned block (that would be an allocation): pageable copy
        HIP_TRY(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return;
    }
    void *b = pinned_block(n * sizeof(T));
    HIP_TRY(hipMemcpyAsync(b, d, n * sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(h, b, n * sizeof(T));
}

template <class T>
static T read_one(const T *d, hipStream_t s) {
    T h;
    read_back(&h, d, 1, s);
    return h;
}

// Exact 64-bit sum of n int32 counts (synchronises the stream). The
// counted-fill fallbacks check their totals with it before 32-bit scans.
static long long total_i64(const int *x, long long n, hipStream_t s, Scope &sc) {
    if (n <= 0) return 0;
    long long b = (n + BLOCK - 1) / BLOCK;
    if (b > 1024) b = 1024;
    long long *part = sc.get<long long>(b + 1);
    k_sum_i64<<<(unsigned)b, BLOCK, 0, s>>>(x, n, part);
    k_fold_i64<<<1, 1, 0, s>>>(part, (int)b, part + b);
    LAUNCH_CHECK();
    return read_one(part + b, s);
}

static void check_total(long long t, const char *what) {
    if (t >= (long long)INT_MAX)
        throw HipError{AC_E_CAPACITY, std::string("more than 2^31 - 1 ") + what + " (32-bit indices)"};
}

static long long isqrt_ceil(long long v) {
    if (v <= 0) return 0;
    long long r = (long long)std::sqrt((double)v);
    while (r * r > v) r--;
    while (r * r < v) r++;
    return r;
}

// Candidate arrays of one call, used by the emit stage.
struct Cands {
    const int *up, *edge_i, *tri_k, *tri_e, *tet_t, *tet_l, *perm;
};

// Stable LSD radix sort of (key, payload) on bits [lo, hi) of key, 8 bits per
// pass. key / pay are set to the buffers that hold the result (the inputs' or
// scratch of the scope); *spare_key / *spare_pay (if given) to two other
// buffers of n entries.
template <class P>
static void radix_sort(unsigned *&key, P *&pay, int n, int lo, int hi, hipStream_t s, Scope &sc,
                       unsigned **spare_key = nullptr, P **spare_pay = nullptr, const int *live = nullptr) {
    unsigned *k2 = sc.get<unsigned>(n > 0 ? n : 1);
    P *p2 = sc.get<P>(n > 0 ? n : 1);
    unsigned *kin = key, *kout = k2;
    P *pin = pay, *pout = p2;
    if (n > 1 && hi > lo) {
        const int tiles = (n + RS_TILE - 1) / RS_TILE;
        int *hist = sc.get<int>((size_t)RS_BINS * tiles);
        int *totals = sc.get<int>(RS_BINS);
        for (int shift = lo; shift < hi; shift += RS_BITS) {
            k_rs_hist<<<tiles, RS_BLOCK, 0, s>>>(kin, n, shift, hist, tiles, live);
            k_rs_digit_prefix<<<RS_BINS, RS_PREFIX_BLOCK, 0, s>>>(hist, tiles, totals);
            k_rs_scatter<P><<<tiles, RS_BLOCK, 0, s>>>(kin, pin, kout, pout, n, shift, hist, totals, tiles, live);
            LAUNCH_CHECK();
            std::swap(kin, kout);
            std::swap(pin, pout);
        }
    }
    key = kin;
    pay = pin;
    if (spare_key) *spare_key = kout;
    if (spare_pay) *spare_pay = pout;
}

template <class P>
static void radix_sort(unsigned *&key, P *&pay, int n, int bits, hipStream_t s, Scope &sc) {
    radix_sort<P>(key, pay, n, 0, bits, s, sc);
}

static int bits_for(long long n) {
    int b = 1;
    while ((1LL << b) < n) b++;
    return b;
}

// Emit keys of dimension K - 1 for n balls and M candidates: rows are keyed
// by their least input id (< n); a bucket is 2^shift ids, at most EK_KEYS,
// at least 256 buckets where n allows (so that small inputs still spread over
// many blocks), and small enough that the expected largest bucket, 2^shift K
// M / n rows, stays within 95% of what a block orders in LDS; dropped
// candidates get `drop`, the first key of the bucket after those of every id,
// which fits in `bits` key bits. The radix sort orders bits [shift, bits).
// The pruning kernel that writes the keys and emit_dim take the same M.
struct EmitKeys {
    int bits, shift;
    unsigned drop;
};
template <int K>
static EmitKeys emit_keys(int n, long long M) {
    EmitKeys k;
    k.shift = EK_SHIFT;
    while (k.shift > 0 && ((n >> k.shift) < 256 ||
                           (double)(1LL << k.shift) * K * (double)M > 0.95 * ek_rows<K>() * (double)n))
        k.shift--;
    k.drop = (unsigned)((((long long)n >> k.shift) + 1) << k.shift);
    k.bits = bits_for((long long)k.drop + 1);
    return k;
}

// start[0..nb] of the ranges of key >> shift in m sorted keys (k_key_starts).
static void key_starts(const unsigned *key, long long m, int shift, int nb, int *start, hipStream_t s,
                       const int *live = nullptr) {
    const long long threads = m / KS_PT + 1;  // rows 0..m
    k_key_starts<<<(unsigned)((threads + KS_BLOCK - 1) / KS_BLOCK), KS_BLOCK, 0, s>>>(key, (int)m, shift, nb, start,
                                                                                    live);
    LAUNCH_CHECK();
}

// Emit dimension d = K - 1 from the candidates' keys (least input id; not
// kept: the drop key) and payloads: a radix sort over the key bits above the
// bucket (2^shift ids, emit_keys) makes each bucket contiguous, k_key_starts
// finds the buckets' starts and k_emit_block orders each bucket and writes
// its rows; up to EK_KEYS balls one block takes every row, unsorted. The
// output arrays have room for all M candidates; the kept count goes to
// *m_out on the device. live: the count is read on the device (at most M).
template <int K>
static void emit_dim(unsigned *key, typename EmitPay<K>::type *pay, const double *size_in, int M, int n,
                     hipStream_t s, Scope &sc, ac_complex *res, int d, int *m_out, bool to_A2 = true,
                     const int *live = nullptr) {
    typedef typename EmitPay<K>::type P;
    res->d_simp[d] = static_cast<int32_t *>(dev_alloc((size_t)(M > 0 ? M : 1) * K * sizeof(int32_t)));
    res->d_size[d] = static_cast<double *>(dev_alloc((size_t)(M > 0 ? M : 1) * sizeof(double)));
    if (M == 0) {
        fill<int>(m_out, 0, 1, s);
        return;
    }
    if (n <= EK_KEYS && M <= ek_rows<K>()) {
        // a few hundred balls: one block orders every row, no radix sort
        k_emit_block<K><<<1, EK_BLOCK, 0, s>>>(key, pay, nullptr, EK_SHIFT, 1, nullptr, nullptr, size_in, to_A2 ? 1 : 0,
                                              res->d_simp[d], res->d_size[d], m_out, n, M, live);
        LAUNCH_CHECK();
        return;
    }
    const EmitKeys ek = emit_keys<K>(n, M);
    unsigned *gkey = nullptr;
    P *gpay = nullptr;
    radix_sort<P>(key, pay, M, ek.shift, ek.bits, s, sc, &gkey, &gpay, live);
    const int nb = (int)(ek.drop >> ek.shift);
    int *start = sc.get<int>((size_t)nb + 1);
    key_starts(key, M, ek.shift, nb, start, s, live);
    LAUNCH_CHECK();
    k_emit_block<K><<<(unsigned)nb, EK_BLOCK, 0, s>>>(key, pay, start, ek.shift, nb, gkey, gpay, size_in,
                                                     to_A2 ? 1 : 0, res->d_simp[d], res->d_size[d], m_out);
    LAUNCH_CHECK();
}

// Second stream of the calling thread on the current device, with events for
// its fork from and join into the caller's stream: the emit of triangles,
// tetrahedra and vertices runs there beside the pruning kernels and the edge
// emit. Non-blocking (no implicit order with the null stream), default
// priority; created on first use and kept until the process ends.
struct AuxStream {
    hipStream_t s = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};
static AuxStream &aux_stream() {
    thread_local std::map<int, AuxStream> per_dev;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    AuxStream &a = per_dev[dev];
    if (!a.s) {
        HIP_TRY(hipStreamCreateWithFlags(&a.s, hipStreamNonBlocking));
        // order between two streams of one device: a device-scope release
        // suffices (no system-scope fence, no timing)
        for (hipEvent_t &e : a.ev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
    }
    return a;
}

// `to` waits for the work enqueued on `from` so far (through event e).
static void stream_after(hipStream_t to, hipStream_t from, hipEvent_t e) {
    HIP_TRY(hipEventRecord(e, from));
    HIP_TRY(hipStreamWaitEvent(to, e, 0));
}

// Output order of every candidate of dimension K - 1 (for a sweep): the
// rows sorted as emit_dim sorts them (rows_s) and each candidate's place in
// that order (spos).
template <int K>
static void order_dim(int M, const Cands &cd, int n, hipStream_t s, Scope &sc, int *rows_s, int *spos) {
    typedef typename OrderPay<K>::type P;
    if (M == 0) return;
    unsigned *key = sc.get<unsigned>(M);
    P *pay = sc.get<P>(M);
    k_order_keys<K><<<grid_for(M), BLOCK, 0, s>>>(M, cd.up, cd.edge_i, cd.tri_k, cd.tri_e, cd.tet_t, cd.tet_l, cd.perm,
                                                  key, pay);
    LAUNCH_CHECK();
    radix_sort<P>(key, pay, M, bits_for((long long)n), s, sc);
    k_order_rank<K><<<grid_for(M), BLOCK, 0, s>>>(key, pay, M, rows_s, spos);
    LAUNCH_CHECK();
}

struct Options {
    int cell_mA = 0;
    int force_exact = 0;
    int vertex_shortcut = 0;
    int profile = 0;
    int cell_order = ORDER_ROW;
};

// Stages timed by HIP events when profiling. A stage lasts from its mark to
// the next mark; "edges_ac2" and "triangles_ac2" are marked only when the AC2
// tests of edges and triangles run as kernels of their own.
enum Stage {
    ST_QUANTISE, ST_BIN, ST_NBR_COUNT, ST_NBR_SCAN, ST_NBR_FILL, ST_TRI_COUNT, ST_TRI_SCAN, ST_TRI_FILL,
    ST_TRI_GABRIEL, ST_TET_COUNT, ST_TET_FILL, ST_TETRA, ST_TRI_FINAL, ST_EDGE_FINAL, ST_VERT_FINAL, ST_EMIT,
    ST_EDGE_AC2, ST_TRI_AC2, ST_COUNT
};
static const char *kStageNames[ST_COUNT] = {
    "quantise", "binning", "neighbours_count", "neighbours_scan", "neighbours_fill", "triangles_count",
    "triangles_scan", "triangles_fill", "triangles_ac2_tetrahedra", "tetrahedra_scan", "tetrahedra_fill", "tetrahedra_ac2",
    "triangles_final", "edges_final", "vertices_final", "emit", "edges_ac2", "triangles_ac2"};
// profile value of the per-step arrangement: every stage timed, edge and
// triangle AC2 in kernels of their own
constexpr int PROFILE_SPLIT = ST_COUNT + 2;

// Events at stage boundaries. Each recorded event costs a few microseconds of
// idle device time between two kernels, so a caller may ask for one stage
// only (its two boundary events). The events come from a per-thread pool
// (creating one in the middle of a build would hold up the host's launches),
// one pool per device (an event belongs to the device it was created on).
static std::vector<hipEvent_t> &event_pool() {
    thread_local std::map<int, std::vector<hipEvent_t>> pools;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    return pools[dev];
}
struct StageTimer {
    bool on = false;
    int only = -1;  // >= 0: record the boundaries of this stage only
    int cur = -1;   // stage running since the last mark
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    int ev_start[ST_COUNT], ev_end[ST_COUNT];
    void start(int profile, hipStream_t st) {
        on = profile != 0;
        only = (profile >= 2 && profile < PROFILE_SPLIT) ? profile - 2 : -1;
        s = st;
        for (int i = 0; i < ST_COUNT; i++) ev_start[i] = ev_end[i] = -1;
    }
    // stage i starts now (i = ST_COUNT: the last stage ends)
    void mark(int i) {
        if (!on) return;
        const bool need = only < 0 || i == only || cur == only;
        if (need) {
            hipEvent_t e;
            std::vector<hipEvent_t> &pool = event_pool();
            if (!pool.empty()) {
                e = pool.back();
                pool.pop_back();
            } else {
                // timing only: no system-scope fence (an L2 writeback and
                // invalidate at every record, which stalls the next kernels)
                HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            }
            ev.push_back(e);
            HIP_TRY(hipEventRecord(e, s));
            const int k = (int)ev.size() - 1;
            if (cur >= 0) ev_end[cur] = k;
            if (i < ST_COUNT) ev_start[i] = k;
        }
        cur = i;
    }
    void collect(double *ms) {
        for (int i = 0; i < ST_COUNT; i++) {
            ms[i] = -1.0;
            if (on && ev_start[i] >= 0 && ev_end[i] >= 0) {
                float f = 0.f;
                if (hipEventElapsedTime(&f, ev[ev_start[i]], ev[ev_end[i]]) == hipSuccess) ms[i] = f;
            }
        }
    }
    ~StageTimer() {
        // back to the pool of this thread and device, for a later build (a
        // re-record of an event still pending only moves it)
        if (ev.empty()) return;
        try {
            std::vector<hipEvent_t> &pool = event_pool();
            for (hipEvent_t e : ev) pool.push_back(e);
        } catch (...) {
            for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        }
    }
};

// Molecules of one call: balls [off[m], off[m+1]) form molecule m, each with
// its own grid (cell side cell_mA[m] if given).
struct Batch {
    std::vector<int64_t> off;
    std::vector<int32_t> cell_mA;
};

// Blocks of the quantise kernel: tiles of at most QTILE balls, each inside one
// molecule; molecule m's tiles are [tile_first[m], tile_first[m+1]).
static void quantise_tiles(const Batch &bt, std::vector<int2> &tiles, std::vector<int> &tile_first) {
    const int n_mol = (int)bt.off.size() - 1;
    tiles.clear();
    tile_first.assign(n_mol + 1, 0);
    for (int m = 0; m < n_mol; m++) {
        tile_first[m] = (int)tiles.size();
        for (int64_t a = bt.off[m]; a < bt.off[m + 1]; a += QTILE)
            tiles.push_back(make_int2((int)a, (int)std::min<int64_t>(a + QTILE, bt.off[m + 1])));
    }
    tile_first[n_mol] = (int)tiles.size();
}

// Sizes of a recorded build (ac_plan). A learning run (learn = true) is an
// ordinary build that notes them; a fixed run takes them, with the plan's
// capacities, instead of reading any count back, so that it is a fixed
// sequence of launches with no host synchronisation (see plan.hpp).
struct Fixed {
    bool learn = true;
    // noted by the learning run
    std::vector<Grid> grids;       // per molecule: cell side, reach, order, balls
    std::vector<long long> cells;  // per molecule: grid cells
    PredParams pp{};
    int wmax = 0, slot = 0;
    long long E = 0, T = 0, Q = 0;
    bool two_pass = false;  // a stage needed the counted fill
    // given to a fixed run (device arrays uploaded before it)
    long long ncell = 0;  // cells of all molecules' capacities
    int E_cap = 1, T_cap = 1, Q_cap = 1;
    const int2 *d_tiles = nullptr;
    const int *d_tile_first = nullptr;
    const Grid *d_tmpl = nullptr;       // recorded grids with each molecule's first cell
    const long long *d_cell_cap = nullptr;
    const long long *d_bound = nullptr;  // first ball of each molecule, n_mol + 1
    // left by a fixed run (device)
    Counters *cnt = nullptr;
    long long *d_rows = nullptr;
};

// The whole pipeline from device arrays, for n_alpha >= 1 alpha values: one
// candidate search at the largest, then pruning and output per value (the
// candidates of a smaller alpha are those of the larger that pass AC3 at the
// smaller, and AC2 does not depend on alpha). Returns AC_OK and outs[k] for
// alphas[k] on success; nothing is left allocated on failure.
static ac_status run_pipeline(const double *d_xyz, const double *d_r, int64_t n64, const Batch &bt,
                              const double *alphas, int n_alpha, const Options &o, hipStream_t s, ac_complex **outs,
                              Fixed *fx = nullptr) {
    for (int k = 0; k < n_alpha; k++) outs[k] = nullptr;
    // fixed: sizes from fx, nothing read back (only with one alpha)
    const bool fixed = fx && !fx->learn;
    if (fx && n_alpha != 1) return set_error(AC_E_INVALID, "a recorded build takes one alpha");
    if (n64 < 1 || n64 >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
    if (n_alpha < 1 || n_alpha > AC_MAX_SWEEP) return set_error(AC_E_INVALID, "number of alpha values out of range");
    std::vector<long long> aqs(n_alpha);
    for (int k = 0; k < n_alpha; k++) {
        if (!std::isfinite(alphas[k])) return set_error(AC_E_INVALID, "alpha is not finite");
        const double as = alphas[k] * 1e6;
        if (!(std::fabs(as) < 67108864.0)) return set_error(AC_E_RANGE, "|alpha| too large for the exact bit budget");
        aqs[k] = (long long)std::nearbyint(as);
    }
    const long long aq = *std::max_element(aqs.begin(), aqs.end());
    const int n = (int)n64;
    Scope sc;
    StageTimer tm;
    std::vector<ac_complex *> rs(n_alpha, nullptr);
    auto new_result = [&]() {
        ac_complex *r = new ac_complex();
        for (double &x : r->stage_ms) x = -1.0;
        HIP_TRY(hipGetDevice(&r->device));
        r->device_result = true;
        return r;
    };
    ac_complex *res = nullptr;
    hipStream_t s_aux = nullptr;  // the second stream, once work was put on it
    try {
        for (int k = 0; k < n_alpha; k++) rs[k] = new_result();
        res = rs[0];
        tm.start(o.profile, s);
        const bool split = o.profile == PROFILE_SPLIT;  // AC2 of edges and triangles as kernels of their own
        // ---- quantise + stats (per molecule) ----
        tm.mark(ST_QUANTISE);
        const int n_mol = (int)bt.off.size() - 1;
        int4 *q = sc.get<int4>(n);
        Counters *cnt = sc.get<Counters>(1);
        static_assert(sizeof(Counters) % sizeof(int) == 0, "Counters cleared as ints");
        fill<int>(reinterpret_cast<int *>(cnt), 0, sizeof(Counters) / sizeof(int), s);  // a kernel: graph-safe
        std::vector<int2> tiles;
        std::vector<int> tile_first;
        quantise_tiles(bt, tiles, tile_first);
        std::vector<Stats> hs(n_mol);
        Stats *st = sc.get<Stats>(n_mol);
        {
            const int2 *d_tiles = fixed ? fx->d_tiles : sc.get<int2>(tiles.size());
            const int *d_tile_first = fixed ? fx->d_tile_first : sc.get<int>(n_mol + 1);
            Stats *part = sc.get<Stats>(tiles.size());
            if (!fixed) {
                HIP_TRY(hipMemcpyAsync(const_cast<int2 *>(d_tiles), tiles.data(), tiles.size() * sizeof(int2),
                                       hipMemcpyHostToDevice, s));
                HIP_TRY(hipMemcpyAsync(const_cast<int *>(d_tile_first), tile_first.data(), (n_mol + 1) * sizeof(int),
                                       hipMemcpyHostToDevice, s));
            }
            k_quantise<<<(unsigned)tiles.size(), BLOCK, 0, s>>>(d_xyz, d_r, d_tiles, q, part);
            LAUNCH_CHECK();
            k_stats_reduce<<<(unsigned)n_mol, BLOCK, 0, s>>>(part, d_tile_first, st);
            LAUNCH_CHECK();
            if (!fixed) read_back(hs.data(), st, (size_t)n_mol, s);
        }
        int flags = 0, wmax = 0;
        for (const Stats &x : hs) {
            flags |= x.flags;
            wmax = std::max(wmax, x.wmax);
        }
        if (fixed) wmax = fx->wmax;  // the device checks that no radius exceeds it
        if (flags & 1) throw HipError{AC_E_INVALID, "non-finite coordinate, or radius not positive"};
        if (flags & 2) throw HipError{AC_E_RANGE, "coordinate or radius outside the exact bit budget"};
        const long long sg2 = (long long)wmax + aq;
        if (sg2 >= (1LL << 26)) throw HipError{AC_E_RANGE, "r_max^2 + alpha too large for the exact bit budget"};
        PredParams pp;
        pp.aq = aq;
        pp.sg2 = sg2 < 0 ? 0 : sg2;
        const long long sgc = isqrt_ceil(pp.sg2);
        pp.sgc = sgc;
        pp.bmax = 2.0 * (double)sgc;
        pp.gmax = 4.0 * (double)pp.sg2 + (double)wmax;
        pp.force_exact = o.force_exact;
        if (fx && fx->learn) {
            fx->pp = pp;
            fx->wmax = wmax;
        }

        // ---- grids: one per molecule, cells numbered consecutively ----
        std::vector<Grid> grids(n_mol);
        long long ncell = 0;
        if (fx && fx->learn) fx->cells.assign(n_mol, 0);
        for (int m = 0; m < n_mol && !fixed; m++) {
            const Stats &h = hs[m];
            const long long nm = bt.off[m + 1] - bt.off[m];
            Grid &g = grids[m];
            g.ox = h.minx; g.oy = h.miny; g.oz = h.minz;
            const long long ex = (long long)h.maxx - h.minx + 1, ey = (long long)h.maxy - h.miny + 1,
                            ez = (long long)h.maxz - h.minz + 1;
            long long side = !bt.cell_mA.empty() ? bt.cell_mA[m] : (o.cell_mA > 0 ? o.cell_mA : (sgc > 0 ? sgc : 1));
            const long long cell_limit = n_mol == 1 ? std::max<long long>(8LL * nm, 1LL << 22)
                                                    : std::max<long long>(8LL * nm, 1LL << 15);
            // cells of the grid: the box, or for a Morton order the cube of
            // 2^L cells a side that holds it (2^(3L) codes)
            auto ncell_of = [&](long long sd) {
                const long long gx = (ex + sd - 1) / sd, gy = (ey + sd - 1) / sd, gz = (ez + sd - 1) / sd;
                if (o.cell_order != ORDER_MORTON) return gx * gy * gz;
                int L = 0;
                while ((1LL << L) < std::max(gx, std::max(gy, gz))) L++;
                return L > MORTON_MAX_BITS ? LLONG_MAX : 1LL << (3 * L);
            };
            while (ncell_of(side) > cell_limit) side = side + side / 4 + 1;
            g.s = (int)side;
            g.nx = (int)((ex + side - 1) / side); g.ny = (int)((ey + side - 1) / side); g.nz = (int)((ez + side - 1) / side);
            g.reach = (int)((2 * sgc + side - 1) / side);
            g.base = ncell;
            g.a0 = (int)bt.off[m];
            g.a1 = (int)bt.off[m + 1];
            g.order = o.cell_order;
            if (fx && fx->learn) fx->cells[m] = ncell_of(side);
            ncell += ncell_of(side);
        }
        if (fx && fx->learn) fx->grids = grids;
        if (fixed) ncell = fx->ncell;
        if (ncell >= (long long)INT_MAX) throw HipError{AC_E_CAPACITY, "too many grid cells"};
        Grid *d_grids = sc.get<Grid>(n_mol);
        if (fixed) {
            // this run's boxes, the recorded sides and capacities
            k_plan_grids<<<grid_for(n_mol), BLOCK, 0, s>>>(st, n_mol, fx->d_tmpl, fx->d_cell_cap, fx->wmax, d_grids,
                                                           cnt);
            LAUNCH_CHECK();
        } else {
            HIP_TRY(hipMemcpyAsync(d_grids, grids.data(), n_mol * sizeof(Grid), hipMemcpyHostToDevice, s));
        }

        // ---- binning ----
        tm.mark(ST_BIN);
        unsigned *ckey = sc.get<unsigned>(n);
        unsigned *cidx = sc.get<unsigned>(n);
        int *cell_count = sc.get<int>(ncell + 1);
        int *cell_start = sc.get<int>(ncell + 1);
        k_cell_key<<<grid_for(n), BLOCK, 0, s>>>(q, n, d_grids, n_mol, ckey, cidx);
        LAUNCH_CHECK();
        radix_sort<unsigned>(ckey, cidx, n, bits_for(ncell), s, sc);
        // the cell table from the populations (most cells are empty, so the
        // starts are not taken from the sorted keys as the emit's buckets are:
        // one thread would fill each run of empty cells)
        fill<int>(cell_count, 0, ncell, s);
        k_cell_runs<<<grid_for(n), BLOCK, 0, s>>>(ckey, n, cell_count);
        LAUNCH_CHECK();
        scan_i32(cell_count, cell_start, ncell, s, sc);
        int4 *atom = sc.get<int4>(n);
        int *perm = sc.get<int>(n);
        k_gather_atoms<<<grid_for(n), BLOCK, 0, s>>>(q, cidx, ckey, n, atom, perm, cnt);
        LAUNCH_CHECK();

        // ---- neighbours and candidate edges: one pass into per-block slabs,
        // then compaction; count, scan and fill if a ball's rows overflow ----
        int *deg_n = sc.get<int>(n), *deg_up = sc.get<int>(n);
        int *nbr_start = sc.get<int>(n + 1), *up_start = sc.get<int>(n + 1);
        unsigned char *vgab = sc.get<unsigned char>(n);
        long long *vert_min = sc.get<long long>(n);
        const unsigned nbN = grid_for(n);
        // slot per ball: wide for grown radii between 1.9 and 2.6 A (alpha > 0
        // with van der Waals radii), where rows outgrow 16 entries; beyond,
        // rows outgrow 32 too and the counted fill runs anyway
        const int slot = (pp.sgc > 1900 && pp.sgc <= 2600) ? NB_SLOT_WIDE : NB_SLOT;
        if (fx && fx->learn) fx->slot = slot;
        const long long nb_slab = (long long)BLOCK * slot;
        int *nslab = sc.get<int>((size_t)nbN * nb_slab + NBR_PAD);
        unsigned *upmask = sc.get<unsigned>(n);
        int *nbtot = sc.get<int>(2 * (size_t)nbN);
        int *nboff = sc.get<int>(nbN + 1), *uboff = sc.get<int>(nbN + 1);
        // the fast exact pair test applies when every scanned offset stays
        // below 26 A per axis, s_g^2 < 2^25 and alpha >= 0 (see k_neighbours)
        bool nb_fast = pp.aq >= 0 && pp.sg2 < (1LL << 25);
        for (const Grid &g : (fixed ? fx->grids : grids))
            nb_fast = nb_fast && (long long)(g.reach + 1) * g.s < 26000;
        tm.mark(ST_NBR_COUNT);
        if (slot == NB_SLOT_WIDE && nb_fast)
            k_neighbours<NB_ONEPASS, NB_SLOT_WIDE, true><<<nbN, BLOCK, 0, s>>>(
                atom, perm, n, d_grids, n_mol, cell_start, pp, deg_n, deg_up, upmask, nslab, nbtot, nullptr, nullptr,
                nullptr, nullptr, nullptr, vgab, vert_min, cnt);
        else if (slot == NB_SLOT_WIDE)
            k_neighbours<NB_ONEPASS, NB_SLOT_WIDE><<<nbN, BLOCK, 0, s>>>(atom, perm, n, d_grids, n_mol, cell_start, pp,
                                                                        deg_n, deg_up, upmask, nslab, nbtot, nullptr,
                                                                        nullptr, nullptr, nullptr, nullptr, vgab, vert_min,
                                                                        cnt);
        else if (nb_fast)
            k_neighbours<NB_ONEPASS, NB_SLOT, true><<<nbN, BLOCK, 0, s>>>(
                atom, perm, n, d_grids, n_mol, cell_start, pp, deg_n, deg_up, upmask, nslab, nbtot, nullptr, nullptr,
                nullptr, nullptr, nullptr, vgab, vert_min, cnt);
        else
            k_neighbours<NB_ONEPASS, NB_SLOT><<<nbN, BLOCK, 0, s>>>(atom, perm, n, d_grids, n_mol, cell_start, pp, deg_n,
                                                                   deg_up, upmask, nslab, nbtot, nullptr, nullptr,
                                                                   nullptr, nullptr, nullptr, vgab, vert_min, cnt);
        LAUNCH_CHECK();
        tm.mark(ST_NBR_SCAN);
        scan_i32(nbtot, nboff, nbN, s, sc, &cnt->Nn);
        scan_i32(nbtot + nbN, uboff, nbN, s, sc, &cnt->E);
        LAUNCH_CHECK();
        Counters c0{};
        if (fixed) {
            k_plan_guard<<<1, WAVE, 0, s>>>(cnt, 0, fx->E_cap);
            LAUNCH_CHECK();
            c0.E = fx->E_cap;
        } else {
            c0 = read_one(cnt, s);
        }
        if (c0.dup) throw HipError{AC_E_DUPLICATE, "two balls have equal quantised centres"};
        const bool nbr_two_pass = c0.overflow != 0;
        if (fx && fx->learn) fx->two_pass |= nbr_two_pass;
        if (!fixed && (nbr_two_pass || (long long)nbN * nb_slab >= (long long)INT_MAX)) {
            // past this size the slab bound no longer keeps the total in 32 bits
            check_total(total_i64(deg_n, n, s, sc), "neighbour entries");
        }
        if (nbr_two_pass) {
            scan_i32(deg_n, nbr_start, n, s, sc, &cnt->Nn);
            scan_i32(deg_up, up_start, n, s, sc, &cnt->E);
            LAUNCH_CHECK();
            c0 = read_one(cnt, s);
        }
        const int E = c0.E, Nn = c0.Nn;
        if (fx && fx->learn) fx->E = E;
        const int *E_live = fixed ? &cnt->El : nullptr;  // fixed: the launches below read the count
        // neighbour rows: in the slabs after the one-pass search, else in CSR
        int *nbr = nbr_two_pass ? sc.get<int>((size_t)(Nn > 0 ? Nn : 1) + NBR_PAD) : nslab;
        int *up = sc.get<int>(E > 0 ? E : 1);
        int *edge_i = sc.get<int>(E > 0 ? E : 1);
        tm.mark(ST_NBR_FILL);
        if (!nbr_two_pass) {
            if (slot == NB_SLOT_WIDE)
                k_nbr_compact<NB_SLOT_WIDE><<<nbN, BLOCK, 0, s>>>(deg_n, deg_up, upmask, n, nslab, uboff, nbr_start,
                                                                 up_start, up, edge_i, fixed ? &cnt->stop : nullptr);
            else
                k_nbr_compact<NB_SLOT><<<nbN, BLOCK, 0, s>>>(deg_n, deg_up, upmask, n, nslab, uboff, nbr_start, up_start,
                                                            up, edge_i, fixed ? &cnt->stop : nullptr);
        } else if (nb_fast) {
            k_neighbours<NB_FILL, NB_SLOT, true><<<nbN, BLOCK, 0, s>>>(atom, perm, n, d_grids, n_mol, cell_start, pp,
                                                                      nullptr, nullptr, nullptr, nullptr, nullptr,
                                                                      nbr_start, up_start, nbr, up, edge_i, vgab,
                                                                      vert_min, cnt);
        } else {
            k_neighbours<NB_FILL, NB_SLOT><<<nbN, BLOCK, 0, s>>>(atom, perm, n, d_grids, n_mol, cell_start, pp, nullptr,
                                                                nullptr, nullptr, nullptr, nullptr, nbr_start, up_start,
                                                                nbr, up, edge_i, vgab, vert_min, cnt);
        }
        LAUNCH_CHECK();
        const int *nbr_cnt = deg_n;
        unsigned char *egab = sc.get<unsigned char>(E > 0 ? E : 1);
        long long *edge_min = sc.get<long long>(E > 0 ? E : 1);
        if (split && E > 0) {
            tm.mark(ST_EDGE_AC2);
            k_edge_ac2<<<grid_for(E), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up, edge_i, E, pp, egab,
                                                    edge_min);
            LAUNCH_CHECK();
        }

        // ---- candidate triangles (with AC2 of the edges): one pass into
        // per-block slabs, then compaction; two passes if a slab overflows ----
        int *tri_cnt = sc.get<int>(E > 0 ? E : 1);
        int *tri_start = sc.get<int>(E + 1);
        const unsigned nbE = grid_for(E);
        int *tslab = sc.get<int>((size_t)nbE * TRI_SLAB);
        int *tbtot = sc.get<int>(nbE);
        int *tboff = sc.get<int>(nbE + 1);
        tm.mark(ST_TRI_COUNT);
        fill<int>(&cnt->overflow, 0, 1, s);
        if (E > 0) {
            if (split)
                k_triangles<TRI_ONEPASS, false><<<nbE, BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up,
                                                                     edge_i, E, pp, tri_cnt, egab, edge_min, tslab,
                                                                     tbtot, nullptr, nullptr, nullptr, cnt);
            else
                k_triangles<TRI_ONEPASS><<<nbE, BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i,
                                                              E, pp, tri_cnt, egab, edge_min, tslab, tbtot, nullptr,
                                                              nullptr, nullptr, cnt, E_live);
            LAUNCH_CHECK();
            tm.mark(ST_TRI_SCAN);
            scan_i32(tbtot, tboff, nbE, s, sc, &cnt->T);
            LAUNCH_CHECK();
        } else {
            tm.mark(ST_TRI_SCAN);
            fill<int>(&cnt->T, 0, 1, s);
        }
        Counters ct{};
        if (fixed) {
            k_plan_guard<<<1, WAVE, 0, s>>>(cnt, 1, fx->T_cap);
            LAUNCH_CHECK();
            ct.T = fx->T_cap;
        } else {
            ct = read_one(cnt, s);
        }
        const bool tri_two_pass = ct.overflow != 0;
        if (fx && fx->learn) fx->two_pass |= tri_two_pass;
        if (!fixed && (tri_two_pass || (long long)nbE * TRI_SLAB >= (long long)INT_MAX)) {
            // past this size the slab bound no longer keeps the total in 32 bits
            check_total(total_i64(tri_cnt, E, s, sc), "candidate triangles");
        }
        if (tri_two_pass) {
            scan_i32(tri_cnt, tri_start, E, s, sc, &cnt->T);
            LAUNCH_CHECK();
            ct = read_one(cnt, s);
        }
        const int T = ct.T;
        if (fx && fx->learn) fx->T = T;
        const int *T_live = fixed ? &cnt->Tl : nullptr;
        int *tri_k = sc.get<int>(T > 0 ? T : 1);
        int *tri_e = sc.get<int>(T > 0 ? T : 1);
        unsigned char *tgab = sc.get<unsigned char>(T > 0 ? T : 1);
        double *tsize = sc.get<double>(T > 0 ? T : 1);
        long long *tri_min = sc.get<long long>(T > 0 ? T : 1);
        int *tet_cnt = sc.get<int>(T > 0 ? T : 1);
        int *tet_start = sc.get<int>(T + 1);
        tm.mark(ST_TRI_FILL);
        if (fixed) fill<int>(tri_start, 0, 1, s);  // no edge at run time leaves tri_start[0] unwritten
        if (E > 0 && !tri_two_pass) {
            k_tri_compact<<<(nbE + TRI_CB - 1) / TRI_CB, BLOCK, 0, s>>>(tri_cnt, E, tslab, tboff, tri_start, tri_k,
                                                                       tri_e, E_live);
            LAUNCH_CHECK();
        } else if (T > 0) {
            k_triangles<TRI_FILL><<<nbE, BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i, E, pp,
                                                       nullptr, nullptr, nullptr, nullptr, nullptr, tri_start, tri_k,
                                                       tri_e, cnt);
            LAUNCH_CHECK();
        }
        if (E == 0) fill<int>(tri_start, 0, 1, s);
        // ---- AC2 of triangles and candidate tetrahedra: one pass into
        // per-block slabs, then compaction; two passes if a slab overflows ----
        const unsigned nbT = grid_for(T);
        int *qslab = sc.get<int>((size_t)nbT * TET_SLAB);
        int *qbtot = sc.get<int>(nbT);
        int *qboff = sc.get<int>(nbT + 1);
        if (split && T > 0) {
            tm.mark(ST_TRI_AC2);
            k_tri_ac2<<<grid_for(T), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up, edge_i, tri_k, tri_e, T, pp,
                                                   tgab, tsize, tri_min, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TRI_GABRIEL);
        fill<int>(&cnt->overflow, 0, 1, s);
        if (T > 0) {
            if (split)
                k_tet_candidates<TET_ONEPASS, false><<<nbT, BLOCK, 0, s>>>(
                    atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i, tri_k, tri_e, T, pp, tgab, tsize, tri_min,
                    tet_cnt, qslab, qbtot, nullptr, nullptr, nullptr, cnt);
            else
                k_tet_candidates<TET_ONEPASS><<<nbT, BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up,
                                                                   edge_i, tri_k, tri_e, T, pp, tgab, tsize, tri_min,
                                                                   tet_cnt, qslab, qbtot, nullptr, nullptr, nullptr, cnt,
                                                                   T_live);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TET_COUNT);
        if (T > 0) {
            scan_i32(qbtot, qboff, nbT, s, sc, &cnt->Q);
            LAUNCH_CHECK();
        } else {
            fill<int>(&cnt->Q, 0, 1, s);
        }
        Counters cq{};
        if (fixed) {
            k_plan_guard<<<1, WAVE, 0, s>>>(cnt, 2, fx->Q_cap);
            LAUNCH_CHECK();
            cq.Q = fx->Q_cap;
        } else {
            cq = read_one(cnt, s);
        }
        const bool tet_two_pass = cq.overflow != 0;
        if (fx && fx->learn) fx->two_pass |= tet_two_pass;
        if (tet_two_pass) {
            check_total(total_i64(tet_cnt, T, s, sc), "candidate tetrahedra");
            scan_i32(tet_cnt, tet_start, T, s, sc, &cnt->Q);
            LAUNCH_CHECK();
            cq = read_one(cnt, s);
        }
        const int Q = cq.Q;
        if (fx && fx->learn) fx->Q = Q;
        const int *Q_live = fixed ? &cnt->Ql : nullptr;
        int *tet_t = sc.get<int>(Q > 0 ? Q : 1);
        int *tet_l = sc.get<int>(Q > 0 ? Q : 1);
        double *qsize = sc.get<double>(Q > 0 ? Q : 1);
        tm.mark(ST_TET_FILL);
        if (T > 0 && !tet_two_pass) {
            k_tet_compact<<<nbT, BLOCK, 0, s>>>(tet_cnt, T, qslab, qboff, tet_t, tet_l, T_live);
            LAUNCH_CHECK();
        } else if (Q > 0) {
            k_tet_candidates<TET_FILL><<<nbT, BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i,
                                                            tri_k, tri_e, T, pp, nullptr, nullptr, nullptr, nullptr,
                                                            nullptr, nullptr, tet_start, tet_t, tet_l, cnt);
            LAUNCH_CHECK();
        }

        // ---- pruning: tetrahedra, then triangles, edges, vertices ----
        int *tri_att = nullptr, *edge_att = nullptr, *vert_att = nullptr;  // sweep only
        double *vsize_in = sc.get<double>(n);
        int *vflag = sc.get<int>(n);
        int *vpos = sc.get<int>(n + 1);
        auto prune_init = [&]() {
            const long long mx = std::max<long long>(std::max<long long>(T, E), n);
            const long long nb = std::min<long long>((mx + BLOCK - 1) / BLOCK, 65536);
            k_prune_init<<<(unsigned)nb, BLOCK, 0, s>>>(T, E, n, tri_att, tri_min, edge_att, edge_min, vert_att, vert_min);
            LAUNCH_CHECK();
        };
        // vertices of one alpha (Step 5), then their output in input order
        auto vert_final = [&](const PredParams &pa) {
            k_vert_final<<<grid_for(n), BLOCK, 0, s>>>(atom, perm, n, pa, o.vertex_shortcut, vgab, vert_min, vsize_in);
            LAUNCH_CHECK();
        };
        auto vert_emit = [&](ac_complex *r, int *m_out, hipStream_t se) {
            k_vert_flags<<<grid_for(n), BLOCK, 0, se>>>(vsize_in, n, vflag);
            LAUNCH_CHECK();
            scan_i32(vflag, vpos, n, se, sc, m_out);
            r->d_simp[0] = static_cast<int32_t *>(dev_alloc((size_t)n * sizeof(int32_t)));
            r->d_size[0] = static_cast<double *>(dev_alloc((size_t)n * sizeof(double)));
            k_vert_emit<<<grid_for(n), BLOCK, 0, se>>>(vsize_in, vpos, n, r->d_simp[0], r->d_size[0]);
            LAUNCH_CHECK();
        };
        // rows of each molecule of a batch in the sorted outputs of r (device)
        auto mol_rows = [&](ac_complex *r, Counters *cm, long long *d_rows, const long long *d_bound) {
            const unsigned nb = (unsigned)((n_mol + 1 + BLOCK - 1) / BLOCK);
            k_row_lower_bound<1><<<nb, BLOCK, 0, s>>>(r->d_simp[0], &cm->m0, d_bound, n_mol + 1, d_rows);
            k_row_lower_bound<2><<<nb, BLOCK, 0, s>>>(r->d_simp[1], &cm->m1, d_bound, n_mol + 1, d_rows + (n_mol + 1));
            k_row_lower_bound<3><<<nb, BLOCK, 0, s>>>(r->d_simp[2], &cm->m2, d_bound, n_mol + 1, d_rows + 2 * (n_mol + 1));
            k_row_lower_bound<4><<<nb, BLOCK, 0, s>>>(r->d_simp[3], &cm->m3, d_bound, n_mol + 1, d_rows + 3 * (n_mol + 1));
            LAUNCH_CHECK();
        };
        long long *d_bound = nullptr;
        if (n_mol > 1 && fixed) {
            d_bound = const_cast<long long *>(fx->d_bound);
        } else if (n_mol > 1) {
            d_bound = sc.get<long long>(n_mol + 1);
            HIP_TRY(hipMemcpyAsync(d_bound, bt.off.data(), (n_mol + 1) * sizeof(long long), hipMemcpyHostToDevice, s));
        }
        // per-alpha kept counts (m0..m3 of cs[k]); the main counters keep the
        // fallback count and the lookup flag
        Counters *cs = cnt;
        if (n_alpha > 1) {
            cs = sc.get<Counters>(n_alpha);
            HIP_TRY(hipMemsetAsync(cs, 0, n_alpha * sizeof(Counters), s));
        }
        long long *d_rows = n_mol > 1 ? sc.get<long long>((size_t)n_alpha * 4 * (n_mol + 1)) : nullptr;

        if (n_alpha == 1) {
            // every candidate leaves its pruning kernel with its emit key
            // (least input id, n if not kept) and payload
            unsigned *qkey = sc.get<unsigned>(Q > 0 ? Q : 1), *tkey = sc.get<unsigned>(T > 0 ? T : 1);
            unsigned *ekey = sc.get<unsigned>(E > 0 ? E : 1);
            EmitPay<4>::type *qpay = sc.get<EmitPay<4>::type>(Q > 0 ? Q : 1);
            EmitPay<3>::type *tpay = sc.get<EmitPay<3>::type>(T > 0 ? T : 1);
            EmitPay<2>::type *epay = sc.get<EmitPay<2>::type>(E > 0 ? E : 1);
            // Each dimension's emit needs only its own pruning kernel: the
            // emit of the tetrahedra, the triangles and the vertices runs on a
            // second stream beside the later pruning kernels and the edge emit
            // (the longest); the streams join before the counts are read.
            // Measured on the 3M-atom shell: 2.470 ms per build against 2.508
            // on one stream (a kernel on either stream mostly fills the GPU,
            // so the other stream's kernels run in its gaps). Small builds
            // keep one stream (the waits between streams cost more than the
            // overlap gains: 260 atoms, 0.36 ms against 0.31), and so do a
            // profile that times these stages and a build on fixed scratch
            // (which creates no stream or event).
            const bool one_stream =
                n < (1 << 20) || (tm.on && (tm.only < 0 || tm.only >= ST_TETRA)) || t_arena;
            AuxStream *ax = one_stream ? nullptr : &aux_stream();
            hipStream_t s2 = ax ? ax->s : s;
            s_aux = ax ? ax->s : nullptr;
            tm.mark(ST_TETRA);
            if (Q > 0) {
                k_tet_ac2<false><<<grid_for(Q), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i,
                                                              tri_start, tri_k, tri_e, tet_t, tet_l, Q, pp, tgab, tri_min,
                                                              nullptr, qsize, nullptr, emit_keys<4>(n, Q).drop, qkey, qpay, cnt,
                                                              Q_live);
                LAUNCH_CHECK();
            }
            auto emit_tets = [&]() { emit_dim<4>(qkey, qpay, qsize, Q, n, s2, sc, res, 3, &cnt->m3, true, Q_live); };
            auto emit_tris = [&]() { emit_dim<3>(tkey, tpay, nullptr, T, n, s2, sc, res, 2, &cnt->m2, true, T_live); };
            if (ax) {
                stream_after(s2, s, ax->ev[0]);
                emit_tets();
            }
            tm.mark(ST_TRI_FINAL);
            if (T > 0) {
                k_tri_final<<<grid_for(T), BLOCK, 0, s>>>(up_start, up, edge_i, tri_k, tri_e, T, tgab, tsize, tri_min, egab,
                                                         edge_min, perm, emit_keys<3>(n, T).drop, tkey, tpay, cnt, T_live);
                LAUNCH_CHECK();
            }
            if (ax) {
                stream_after(s2, s, ax->ev[1]);
                emit_tris();
            }
            tm.mark(ST_EDGE_FINAL);
            if (E > 0) {
                k_edge_final<<<grid_for(E), BLOCK, 0, s>>>(atom, up, edge_i, E, egab, edge_min, vgab, vert_min, perm,
                                                          emit_keys<2>(n, E).drop, ekey, epay, E_live);
                LAUNCH_CHECK();
            }
            tm.mark(ST_VERT_FINAL);
            vert_final(pp);
            if (ax) {
                stream_after(s2, s, ax->ev[2]);
                vert_emit(res, &cnt->m0, s2);
            }
            // ---- emit ----
            tm.mark(ST_EMIT);
            if (!ax) vert_emit(res, &cnt->m0, s);
            emit_dim<2>(ekey, epay, nullptr, E, n, s, sc, res, 1, &cnt->m1, true, E_live);
            if (ax) {
                stream_after(s, s2, ax->ev[3]);
            } else {
                emit_tris();
                emit_tets();
            }
            if (n_mol > 1) mol_rows(res, cnt, d_rows, d_bound);
        } else {
            // ---- sweep: AC2 of the tetrahedra, the output order of every
            // candidate and each candidate's AC3 threshold once; then per
            // alpha, comparisons, pruning and compaction in output order ----
            tm.mark(ST_TETRA);
            tri_att = sc.get<int>(T > 0 ? T : 1);
            edge_att = sc.get<int>(E > 0 ? E : 1);
            vert_att = sc.get<int>(n);
            unsigned char *qin = sc.get<unsigned char>(Q > 0 ? Q : 1);
            int4 *tface = sc.get<int4>(Q > 0 ? Q : 1);
            if (Q > 0) {
                k_tet_ac2<true><<<grid_for(Q), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i,
                                                             tri_start, tri_k, tri_e, tet_t, tet_l, Q, pp, tgab, nullptr,
                                                             qin, qsize, tface, emit_keys<4>(n, Q).drop, nullptr, nullptr, cnt);
                LAUNCH_CHECK();
            }
            int2 *tedge = sc.get<int2>(T > 0 ? T : 1);
            if (T > 0) {
                k_tri_edges<<<grid_for(T), BLOCK, 0, s>>>(up_start, up, edge_i, tri_k, tri_e, T, tedge);
                LAUNCH_CHECK();
            }
            const Cands cd{up, edge_i, tri_k, tri_e, tet_t, tet_l, perm};
            const int M[4] = {n, E, T, Q};
            int *rows_s[4] = {}, *spos[4] = {}, *thr[4] = {}, *tsum[4] = {}, *toff[4] = {};
            unsigned char *in_s[4] = {};
            double *sz_s[4] = {}, *szp[4] = {};
            for (int d = 1; d <= 3; d++) {
                const int m = M[d] > 0 ? M[d] : 1;
                const unsigned nb = grid_for(m);
                rows_s[d] = sc.get<int>((size_t)m * (d + 1));
                spos[d] = sc.get<int>(m);
                in_s[d] = sc.get<unsigned char>(m);
                tsum[d] = sc.get<int>(nb);
                toff[d] = sc.get<int>((size_t)nb + 1);
                sz_s[d] = sc.get<double>(m);
                thr[d] = sc.get<int>(m);
                szp[d] = sc.get<double>(m);
            }
            int2 *ends = sc.get<int2>(E > 0 ? E : 1);
            int4 *face2 = sc.get<int4>(T > 0 ? T : 1);
            int4 *face3 = sc.get<int4>(Q > 0 ? Q : 1);
            order_dim<2>(E, cd, n, s, sc, rows_s[1], spos[1]);
            order_dim<3>(T, cd, n, s, sc, rows_s[2], spos[2]);
            order_dim<4>(Q, cd, n, s, sc, rows_s[3], spos[3]);
            if (E > 0) {
                k_sweep_prep_edge<<<grid_for(E), BLOCK, 0, s>>>(atom, up, edge_i, E, egab, spos[1], aq, thr[1], szp[1],
                                                               ends);
                LAUNCH_CHECK();
            }
            if (T > 0) {
                k_sweep_prep_tri<<<grid_for(T), BLOCK, 0, s>>>(atom, up, edge_i, tri_k, tri_e, T, tgab, tsize, tedge,
                                                              spos[2], spos[1], pp, thr[2], szp[2], face2, cnt);
                LAUNCH_CHECK();
            }
            if (Q > 0) {
                k_sweep_prep_tet<<<grid_for(Q), BLOCK, 0, s>>>(atom, up, edge_i, tri_k, tri_e, tet_t, tet_l, Q, qin, qsize,
                                                              tface, spos[3], spos[2], pp, thr[3], szp[3], face3, cnt);
                LAUNCH_CHECK();
            }
            tm.mark(ST_EMIT);
            for (int k = 0; k < n_alpha; k++) {
                PredParams pa = pp;
                pa.aq = aqs[k];
                ac_complex *r = rs[k];
                prune_init();
                if (Q > 0) {
                    k_sweep_tets<<<grid_for(Q), BLOCK, 0, s>>>(Q, pa.aq, thr[3], szp[3], face3, thr[2], tri_att, tri_min,
                                                              in_s[3], sz_s[3], tsum[3], cnt);
                    LAUNCH_CHECK();
                }
                if (T > 0) {
                    k_sweep_tris<<<grid_for(T), BLOCK, 0, s>>>(T, pa.aq, thr[2], szp[2], face2, tri_att, tri_min, thr[1],
                                                              edge_att, edge_min, in_s[2], sz_s[2], tsum[2], cnt);
                    LAUNCH_CHECK();
                }
                if (E > 0) {
                    k_sweep_edges<<<grid_for(E), BLOCK, 0, s>>>(E, pa.aq, thr[1], szp[1], ends, edge_att, edge_min, vgab,
                                                               vert_att, vert_min, in_s[1], sz_s[1], tsum[1]);
                    LAUNCH_CHECK();
                }
                vert_final(pa);
                vert_emit(r, &cs[k].m0, s);
                int *m_out[4] = {&cs[k].m0, &cs[k].m1, &cs[k].m2, &cs[k].m3};
                for (int d = 1; d <= 3; d++) {
                    const int K = d + 1;
                    r->d_simp[d] = static_cast<int32_t *>(dev_alloc((size_t)(M[d] > 0 ? M[d] : 1) * K * sizeof(int32_t)));
                    r->d_size[d] = static_cast<double *>(dev_alloc((size_t)(M[d] > 0 ? M[d] : 1) * sizeof(double)));
                    if (M[d] == 0) {
                        fill<int>(m_out[d], 0, 1, s);
                        continue;
                    }
                    const unsigned nb = grid_for(M[d]);
                    scan_i32(tsum[d], toff[d], nb, s, sc, m_out[d]);
                    if (d == 1)
                        k_sweep_write<2><<<nb, BLOCK, 0, s>>>(in_s[d], toff[d], rows_s[d], sz_s[d], M[d], r->d_simp[d],
                                                             r->d_size[d]);
                    else if (d == 2)
                        k_sweep_write<3><<<nb, BLOCK, 0, s>>>(in_s[d], toff[d], rows_s[d], sz_s[d], M[d], r->d_simp[d],
                                                             r->d_size[d]);
                    else
                        k_sweep_write<4><<<nb, BLOCK, 0, s>>>(in_s[d], toff[d], rows_s[d], sz_s[d], M[d], r->d_simp[d],
                                                             r->d_size[d]);
                    LAUNCH_CHECK();
                }
                if (n_mol > 1) mol_rows(r, &cs[k], d_rows + (size_t)k * 4 * (n_mol + 1), d_bound);
            }
        }
        tm.mark(ST_COUNT);
        if (fixed) {
            // nothing is read back: the plan reads the counters after a replay
            fx->cnt = cnt;
            fx->d_rows = d_rows;
            outs[0] = res;
            return AC_OK;
        }

        // ---- results ----
        std::vector<int64_t> rows;
        if (n_mol > 1) {
            rows.resize((size_t)n_alpha * 4 * (n_mol + 1));
            read_back(rows.data(), (const int64_t *)d_rows, rows.size(), s);
        }
        std::vector<Counters> cm(n_alpha);
        if (n_alpha > 1) read_back(cm.data(), cs, (size_t)n_alpha, s);
        const Counters cf = read_one(cnt, s);
        if (n_alpha == 1) cm[0] = cf;
        if (cf.lookup) throw HipError{AC_E_DEVICE, "internal error: a facet of a kept simplex is not a candidate"};
        tm.collect(res->stage_ms);
        for (int k = 0; k < n_alpha; k++) {
            ac_complex *r = rs[k];
            if (k > 0) std::copy(res->stage_ms, res->stage_ms + 32, r->stage_ms);
            r->n_mol = n_mol;
            r->alpha_q = aqs[k];
            r->cand[0] = n;
            r->cand[1] = E;
            r->cand[2] = T;
            r->cand[3] = Q;
            r->fallbacks = (int64_t)cf.exact_fallbacks;
            r->work[0] = ncell;
            r->work[1] = Nn;
            r->n = n;
            r->count[0] = cm[k].m0;
            r->count[1] = cm[k].m1;
            r->count[2] = cm[k].m2;
            r->count[3] = cm[k].m3;
            for (int d = 0; d < 4; d++) {
                if (n_mol > 1) {
                    const int64_t *b0 = rows.data() + ((size_t)k * 4 + d) * (n_mol + 1);
                    r->mol_rows[d].assign(b0, b0 + (n_mol + 1));
                } else {
                    r->mol_rows[d] = {0, r->count[d]};
                }
            }
        }
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);
        if (s_aux) (void)hipStreamSynchronize(s_aux);
        for (ac_complex *r : rs) free_complex(r);
        return set_error(e.st, e.msg);
    }
    for (int k = 0; k < n_alpha; k++) outs[k] = rs[k];
    g_last_error.clear();
    return AC_OK;
}

static ac_status run_pipeline(const double *d_xyz, const double *d_r, int64_t n64, const Batch &bt, double alpha,
                              const Options &o, hipStream_t s, ac_complex **out) {
    return run_pipeline(d_xyz, d_r, n64, bt, &alpha, 1, o, s, out);
}

// ---------------------------------------------------------------------------
// Partitioned build (partition.hpp): slabs along x with a halo of 4 s_g plus
// 2 A, one pipeline run per slab, owned rows kept, then merged in output
// order. Peak scratch memory is that of the largest slab's build.

// Rows of dimension K - 1 that slab k owns, in emit form: flags, their scan
// and count (read back: the slab's memory is freed next), then the packed
// keys, payloads and (tetrahedra) Sizes, appended to the per-slab lists.
struct OwnedRows {
    std::vector<void *> key, pay, size;  // per slab with owned rows
    std::vector<int> count;
    long long total = 0;
    ~OwnedRows() {
        for (auto *v : {&key, &pay, &size})
            for (void *p : *v) dev_free(p);
    }
};

template <int K>
static void own_rows(const ac_complex *ck, const int *sel, const int4 *q, int x0, int w, int parts, int k,
                     hipStream_t s, Scope &sc, OwnedRows &own) {
    typedef typename EmitPay<K>::type P;
    const int d = K - 1;
    const int m = (int)ck->count[d];
    if (m == 0) return;
    int *flag = sc.get<int>(m);
    int *pos = sc.get<int>((size_t)m + 1);
    int *cnt = sc.get<int>(1);
    k_own_flags<K><<<grid_for(m), BLOCK, 0, s>>>(ck->d_simp[d], m, sel, q, x0, w, parts, k, flag);
    LAUNCH_CHECK();
    scan_i32(flag, pos, m, s, sc, cnt);
    const int c = read_one(cnt, s);
    if (c == 0) return;
    check_total(own.total + c, "simplices of one dimension");
    unsigned *key = static_cast<unsigned *>(dev_alloc((size_t)c * sizeof(unsigned)));
    own.key.push_back(key);
    P *pay = static_cast<P *>(dev_alloc((size_t)c * sizeof(P)));
    own.pay.push_back(pay);
    double *size = K == 4 ? static_cast<double *>(dev_alloc((size_t)c * sizeof(double))) : nullptr;
    if (size) own.size.push_back(size);
    k_own_emit<K><<<grid_for(m), BLOCK, 0, s>>>(ck->d_simp[d], ck->d_size[d], m, flag, pos, sel, (int)own.total, key,
                                                pay, size);
    LAUNCH_CHECK();
    own.count.push_back(c);
    own.total += c;
}

// All slabs' owned rows of dimension K - 1 in output order (into r).
template <int K>
static void merge_rows(OwnedRows &own, int n, hipStream_t s, Scope &sc, ac_complex *r, int *m_out) {
    typedef typename EmitPay<K>::type P;
    const int m = (int)own.total;
    unsigned *key = sc.get<unsigned>(m > 0 ? m : 1);
    P *pay = sc.get<P>(m > 0 ? m : 1);
    double *size = K == 4 ? sc.get<double>(m > 0 ? m : 1) : nullptr;
    long long off = 0;
    for (size_t j = 0; j < own.count.size(); j++) {
        const size_t c = (size_t)own.count[j];
        HIP_TRY(hipMemcpyAsync(key + off, own.key[j], c * sizeof(unsigned), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(pay + off, own.pay[j], c * sizeof(P), hipMemcpyDeviceToDevice, s));
        if (size) HIP_TRY(hipMemcpyAsync(size + off, own.size[j], c * sizeof(double), hipMemcpyDeviceToDevice, s));
        off += (long long)c;
    }
    emit_dim<K>(key, pay, size, m, n, s, sc, r, K - 1, m_out, false);
}

static ac_status run_partitioned(const double *d_xyz, const double *d_r, int64_t n64, double alpha, int parts,
                                 const Options &o, hipStream_t s, ac_complex **out) {
    *out = nullptr;
    if (n64 < 1 || n64 >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
    if (parts < 1 || parts > 64) return set_error(AC_E_INVALID, "parts must be in [1, 64]");
    if (!std::isfinite(alpha)) return set_error(AC_E_INVALID, "alpha is not finite");
    const double as = alpha * 1e6;
    if (!(std::fabs(as) < 67108864.0)) return set_error(AC_E_RANGE, "|alpha| too large for the exact bit budget");
    const long long aq = (long long)std::nearbyint(as);
    const int n = (int)n64;
    Scope sc;
    ac_complex *res = nullptr;
    ac_complex *ck = nullptr;
    try {
        // quantised centres, bounding box and the largest weight
        int4 *q = sc.get<int4>(n);
        std::vector<int2> tiles;
        for (int a = 0; a < n; a += QTILE) tiles.push_back(make_int2(a, std::min(a + QTILE, n)));
        int2 *d_tiles = sc.get<int2>(tiles.size());
        int *d_tile_first = sc.get<int>(2);
        const int tf[2] = {0, (int)tiles.size()};
        Stats *part = sc.get<Stats>(tiles.size());
        Stats *st = sc.get<Stats>(1);
        HIP_TRY(hipMemcpyAsync(d_tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(d_tile_first, tf, sizeof(tf), hipMemcpyHostToDevice, s));
        k_quantise<<<(unsigned)tiles.size(), BLOCK, 0, s>>>(d_xyz, d_r, d_tiles, q, part);
        k_stats_reduce<<<1, BLOCK, 0, s>>>(part, d_tile_first, st);
        LAUNCH_CHECK();
        const Stats h = read_one(st, s);
        if (h.flags & 1) throw HipError{AC_E_INVALID, "non-finite coordinate, or radius not positive"};
        if (h.flags & 2) throw HipError{AC_E_RANGE, "coordinate or radius outside the exact bit budget"};
        const long long sg2 = (long long)h.wmax + aq;
        if (sg2 >= (1LL << 26)) throw HipError{AC_E_RANGE, "r_max^2 + alpha too large for the exact bit budget"};
        const int halo = (int)(4 * isqrt_ceil(sg2 < 0 ? 0 : sg2) + 2000);
        const int x0 = h.minx;
        const int w = (int)(((long long)h.maxx - h.minx + parts) / parts);  // ceil((extent + 1) / parts)

        OwnedRows own[4];
        int *kept = sc.get<int>(n);
        double *vsize = sc.get<double>(n);
        fill<int>(kept, 0, n, s);
        int *flag = sc.get<int>(n);
        int *pos = sc.get<int>((size_t)n + 1);
        int *m_sub = sc.get<int>(1);
        long long fallbacks = 0;
        for (int k = 0; k < parts; k++) {
            const int lo = x0 + k * w, hi = k == parts - 1 ? INT_MAX - halo : lo + w;
            k_slab_flags<<<grid_for(n), BLOCK, 0, s>>>(q, n, lo, hi, halo, flag);
            LAUNCH_CHECK();
            scan_i32(flag, pos, n, s, sc, m_sub);
            const int ms = read_one(m_sub, s);
            if (ms == 0) continue;
            double *sub_xyz = sc.get<double>((size_t)ms * 3);
            double *sub_r = sc.get<double>(ms);
            int *sel = sc.get<int>(ms);
            k_slab_gather<<<grid_for(n), BLOCK, 0, s>>>(flag, pos, n, d_xyz, d_r, sub_xyz, sub_r, sel);
            LAUNCH_CHECK();
            Batch bt;
            bt.off = {0, ms};
            Options ok = o;
            ok.profile = 0;
            const ac_status stp = run_pipeline(sub_xyz, sub_r, ms, bt, alpha, ok, s, &ck);
            if (stp != AC_OK) throw HipError{stp, g_last_error};
            fallbacks += ck->fallbacks;
            if (ck->count[0] > 0) {
                k_own_vertices<<<grid_for(ck->count[0]), BLOCK, 0, s>>>(ck->d_simp[0], ck->d_size[0],
                                                                        (int)ck->count[0], sel, q, x0, w, parts, k,
                                                                        kept, vsize);
                LAUNCH_CHECK();
            }
            own_rows<2>(ck, sel, q, x0, w, parts, k, s, sc, own[1]);
            own_rows<3>(ck, sel, q, x0, w, parts, k, s, sc, own[2]);
            own_rows<4>(ck, sel, q, x0, w, parts, k, s, sc, own[3]);
            HIP_TRY(hipStreamSynchronize(s));  // the slab's result is consumed; free it
            free_complex(ck);
            ck = nullptr;
        }
        res = new ac_complex();
        for (double &x : res->stage_ms) x = -1.0;
        HIP_TRY(hipGetDevice(&res->device));
        res->device_result = true;
        // vertices: kept flags by input id
        int *m0 = sc.get<int>(1);
        scan_i32(kept, pos, n, s, sc, m0);
        res->d_simp[0] = static_cast<int32_t *>(dev_alloc((size_t)n * sizeof(int32_t)));
        res->d_size[0] = static_cast<double *>(dev_alloc((size_t)n * sizeof(double)));
        k_vertex_rows<<<grid_for(n), BLOCK, 0, s>>>(kept, pos, vsize, n, res->d_simp[0], res->d_size[0]);
        LAUNCH_CHECK();
        res->count[0] = read_one(m0, s);
        // higher dimensions: every slab's owned rows merged into output order
        int *mcount = sc.get<int>(4);
        merge_rows<2>(own[1], n, s, sc, res, mcount + 1);
        merge_rows<3>(own[2], n, s, sc, res, mcount + 2);
        merge_rows<4>(own[3], n, s, sc, res, mcount + 3);
        for (int d = 1; d <= 3; d++) res->count[d] = own[d].total;
        HIP_TRY(hipStreamSynchronize(s));
        res->n = n;
        res->n_mol = 1;
        for (int d = 0; d < 4; d++) {
            res->cand[d] = -1;
            res->mol_rows[d] = {0, res->count[d]};
        }
        res->fallbacks = fallbacks;
        res->alpha_q = aq;
        res->work[0] = res->work[1] = -1;
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);
        free_complex(ck);
        free_complex(res);
        return set_error(e.st, e.msg);
    }
    *out = res;
    g_last_error.clear();
    return AC_OK;
}

// ---------------------------------------------------------------------------
// Host-streamed partitioned build: inputs and results stay in host memory.
// One slab at a time (its core and halo) is copied to the device, built, and
// the rows it owns are copied back in emit form; the slabs' lists, each
// sorted already, are merged on the host. Device memory is that of one
// slab's build.

template <int K> struct HostPay { static constexpr int words = K == 2 ? 3 : 4; };

// Owned rows of dimension K - 1 of all slabs, in host memory.
struct HostRows {
    std::vector<std::vector<uint32_t>> key, pay;  // per slab
    std::vector<std::vector<double>> size;        // per slab (K = 4)
};

template <int K>
static void own_rows_host(const ac_complex *ck, const int *sel, const int *qx, int x0, int w, int parts, int k,
                          hipStream_t s, Scope &sc, HostRows &hr) {
    typedef typename EmitPay<K>::type P;
    const int d = K - 1;
    const int m = (int)ck->count[d];
    if (m == 0) return;
    int *flag = sc.get<int>(m);
    int *pos = sc.get<int>((size_t)m + 1);
    int *cnt = sc.get<int>(1);
    k_own_flags_local<K><<<grid_for(m), BLOCK, 0, s>>>(ck->d_simp[d], m, sel, qx, x0, w, parts, k, flag);
    LAUNCH_CHECK();
    scan_i32(flag, pos, m, s, sc, cnt);
    const int c = read_one(cnt, s);
    if (c == 0) return;
    unsigned *key = sc.get<unsigned>(c);
    P *pay = sc.get<P>(c);
    double *size = K == 4 ? sc.get<double>(c) : nullptr;
    k_own_emit<K><<<grid_for(m), BLOCK, 0, s>>>(ck->d_simp[d], ck->d_size[d], m, flag, pos, sel, 0, key, pay, size);
    LAUNCH_CHECK();
    static_assert(sizeof(P) == HostPay<K>::words * sizeof(uint32_t), "payload words");
    hr.key.emplace_back((size_t)c);
    hr.pay.emplace_back((size_t)c * HostPay<K>::words);
    HIP_TRY(hipMemcpyAsync(hr.key.back().data(), key, (size_t)c * sizeof(unsigned), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hr.pay.back().data(), pay, (size_t)c * sizeof(P), hipMemcpyDeviceToHost, s));
    if (size) {
        hr.size.emplace_back((size_t)c);
        HIP_TRY(hipMemcpyAsync(hr.size.back().data(), size, (size_t)c * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
}

// K-way merge of the slabs' sorted lists into output order (rows of K input
// ids, Sizes), in parallel over ranges of the least id.
template <int K>
static void merge_host(const HostRows &hr, int n, std::vector<int32_t> &rows, std::vector<double> &sizes) {
    constexpr int W = HostPay<K>::words;
    const size_t L = hr.key.size();
    size_t M = 0;
    for (const auto &k : hr.key) M += k.size();
    rows.assign(M * K + 1, 0);
    sizes.assign(M + 1, 0.0);
    if (M == 0) return;
    auto row_less = [&](size_t a, size_t ra, size_t b, size_t rb) {
        if (hr.key[a][ra] != hr.key[b][rb]) return hr.key[a][ra] < hr.key[b][rb];
        for (int u = 0; u < K - 1; u++) {
            const uint32_t x = hr.pay[a][ra * W + u], y = hr.pay[b][rb * W + u];
            if (x != y) return x < y;
        }
        return false;
    };
    const int T = (int)std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
    std::vector<std::vector<size_t>> lo(T + 1, std::vector<size_t>(L));
    std::vector<size_t> start(T + 1, 0);
    for (int t = 0; t <= T; t++) {
        const uint32_t u = (uint32_t)((long long)n * t / T);
        for (size_t j = 0; j < L; j++) {
            lo[t][j] = t == T ? hr.key[j].size()
                              : (size_t)(std::lower_bound(hr.key[j].begin(), hr.key[j].end(), u) - hr.key[j].begin());
            start[t] += lo[t][j];
        }
    }
    auto work = [&](int t) {
        std::vector<size_t> at = lo[t];
        auto greater = [&](size_t a, size_t b) { return row_less(b, at[b], a, at[a]); };
        std::priority_queue<size_t, std::vector<size_t>, decltype(greater)> heap(greater);
        for (size_t j = 0; j < L; j++)
            if (at[j] < lo[t + 1][j]) heap.push(j);
        size_t out = start[t];
        while (!heap.empty()) {
            const size_t j = heap.top();
            heap.pop();
            const size_t r = at[j];
            rows[out * K] = (int32_t)hr.key[j][r];
            for (int u = 1; u < K; u++) rows[out * K + u] = (int32_t)hr.pay[j][r * W + u - 1];
            if constexpr (K == 4) {
                sizes[out] = hr.size[j][r];
            } else {
                const uint64_t b = (uint64_t)hr.pay[j][r * W + K - 1] | ((uint64_t)hr.pay[j][r * W + K] << 32);
                double z;
                std::memcpy(&z, &b, sizeof z);
                sizes[out] = z;
            }
            out++;
            if (++at[j] < lo[t + 1][j]) heap.push(j);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < T; t++) th.emplace_back(work, t);
    work(0);
    for (auto &x : th) x.join();
}

static ac_status run_streamed(const double *xyz, const double *r, int64_t n64, double alpha, int parts, const Options &o,
                              ac_complex **out) {
    *out = nullptr;
    if (!xyz || !r) return set_error(AC_E_INVALID, "NULL input pointer");
    if (n64 < 1 || n64 >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
    if (parts < 1 || parts > 1024) return set_error(AC_E_INVALID, "parts must be in [1, 1024]");
    if (!std::isfinite(alpha)) return set_error(AC_E_INVALID, "alpha is not finite");
    const double as = alpha * 1e6;
    if (!(std::fabs(as) < 67108864.0)) return set_error(AC_E_RANGE, "|alpha| too large for the exact bit budget");
    const long long aq = (long long)std::nearbyint(as);
    const int n = (int)n64;
    // the slabs' bounds need the quantised x of every ball and the largest
    // weight: the same rounding (half to even) and checks as the device's
    std::vector<int> qx((size_t)n);
    long long wmax = 0;
    for (int i = 0; i < n; i++) {
        const double v = xyz[3 * (size_t)i];
        if (!std::isfinite(v)) return set_error(AC_E_INVALID, "non-finite coordinate, or radius not positive");
        const double sx = v * 1000.0;
        if (!(std::fabs(sx) < 524288.0)) return set_error(AC_E_RANGE, "coordinate or radius outside the exact bit budget");
        qx[i] = (int)std::nearbyint(sx);
        if (qx[i] >= 524288 || qx[i] <= -524288)
            return set_error(AC_E_RANGE, "coordinate or radius outside the exact bit budget");
        const double rv = r[i];
        if (!std::isfinite(rv) || !(rv > 0.0)) return set_error(AC_E_INVALID, "non-finite coordinate, or radius not positive");
        if (!(rv * 1000.0 < 8192.0)) return set_error(AC_E_RANGE, "coordinate or radius outside the exact bit budget");
        const long long R = (long long)std::nearbyint(rv * 1000.0);
        wmax = std::max(wmax, R * R);
    }
    const long long sg2 = wmax + aq;
    if (sg2 >= (1LL << 26)) return set_error(AC_E_RANGE, "r_max^2 + alpha too large for the exact bit budget");
    const int halo = (int)(4 * isqrt_ceil(sg2 < 0 ? 0 : sg2) + 2000);
    const int x0 = *std::min_element(qx.begin(), qx.end()), x1 = *std::max_element(qx.begin(), qx.end());
    const int w = (int)(((long long)x1 - x0 + parts) / parts);  // ceil((extent + 1) / parts)
    hipStream_t s = nullptr;
    ac_complex *res = nullptr, *ck = nullptr;
    void *pin = nullptr;
    try {
        // the slabs' balls (input order) and the largest slab
        std::vector<std::vector<int>> slab((size_t)parts);
        size_t big = 0;
        for (int k = 0; k < parts; k++) {
            const int lo = x0 + k * w, hi = k == parts - 1 ? INT_MAX - halo : lo + w;
            for (int i = 0; i < n; i++)
                if (qx[i] >= lo - halo && qx[i] < hi + halo) slab[k].push_back(i);
            big = std::max(big, slab[k].size());
        }
        const size_t stage = big * (4 * sizeof(double) + 2 * sizeof(int));
        HIP_TRY(hipHostMalloc(&pin, stage > 0 ? stage : 1, hipHostMallocDefault));
        double *hx = static_cast<double *>(pin), *hrad = hx + 3 * big;
        int *hsel = reinterpret_cast<int *>(hrad + big), *hqx = hsel + big;
        std::vector<double> vsize((size_t)n, std::numeric_limits<double>::quiet_NaN());
        HostRows rows[4];
        long long fallbacks = 0;
        for (int k = 0; k < parts; k++) {
            const int ms = (int)slab[k].size();
            if (ms == 0) continue;
            for (int t = 0; t < ms; t++) {
                const int i = slab[k][t];
                hx[3 * t] = xyz[3 * (size_t)i];
                hx[3 * t + 1] = xyz[3 * (size_t)i + 1];
                hx[3 * t + 2] = xyz[3 * (size_t)i + 2];
                hrad[t] = r[i];
                hsel[t] = i;
                hqx[t] = qx[i];
            }
            Scope sc;  // this slab's device memory, back to the pool after the slab
            double *dx = sc.get<double>(3 * (size_t)ms), *dr = sc.get<double>(ms);
            int *dsel = sc.get<int>(ms), *dqx = sc.get<int>(ms);
            HIP_TRY(hipMemcpyAsync(dx, hx, 3 * (size_t)ms * sizeof(double), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(dr, hrad, (size_t)ms * sizeof(double), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(dsel, hsel, (size_t)ms * sizeof(int), hipMemcpyHostToDevice, s));
            HIP_TRY(hipMemcpyAsync(dqx, hqx, (size_t)ms * sizeof(int), hipMemcpyHostToDevice, s));
            Batch bt;
            bt.off = {0, ms};
            Options ok = o;
            ok.profile = 0;
            const ac_status stp = run_pipeline(dx, dr, ms, bt, alpha, ok, s, &ck);
            if (stp != AC_OK) throw HipError{stp, g_last_error};
            fallbacks += ck->fallbacks;
            // vertices the slab owns: input id and Size
            const int m0 = (int)ck->count[0];
            if (m0 > 0) {
                int *flag = sc.get<int>(m0), *pos = sc.get<int>((size_t)m0 + 1), *cnt = sc.get<int>(1);
                k_own_flags_local<1><<<grid_for(m0), BLOCK, 0, s>>>(ck->d_simp[0], m0, dsel, dqx, x0, w, parts, k, flag);
                LAUNCH_CHECK();
                scan_i32(flag, pos, m0, s, sc, cnt);
                const int c = read_one(cnt, s);
                if (c > 0) {
                    int *oid = sc.get<int>(c);
                    double *osz = sc.get<double>(c);
                    k_own_vertices_local<<<grid_for(m0), BLOCK, 0, s>>>(ck->d_simp[0], ck->d_size[0], m0, flag, pos, dsel,
                                                                        oid, osz);
                    LAUNCH_CHECK();
                    std::vector<int> hid((size_t)c);
                    std::vector<double> hsz((size_t)c);
                    HIP_TRY(hipMemcpyAsync(hid.data(), oid, (size_t)c * sizeof(int), hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipMemcpyAsync(hsz.data(), osz, (size_t)c * sizeof(double), hipMemcpyDeviceToHost, s));
                    HIP_TRY(hipStreamSynchronize(s));
                    for (int t = 0; t < c; t++) vsize[hid[t]] = hsz[t];
                }
            }
            own_rows_host<2>(ck, dsel, dqx, x0, w, parts, k, s, sc, rows[1]);
            own_rows_host<3>(ck, dsel, dqx, x0, w, parts, k, s, sc, rows[2]);
            own_rows_host<4>(ck, dsel, dqx, x0, w, parts, k, s, sc, rows[3]);
            HIP_TRY(hipStreamSynchronize(s));
            free_complex(ck);
            ck = nullptr;
        }
        res = new ac_complex();
        for (double &x : res->stage_ms) x = -1.0;
        HIP_TRY(hipGetDevice(&res->device));
        res->device_result = false;
        // vertices in input order
        std::vector<int32_t> &v0 = res->h_simp[0];
        std::vector<double> &z0 = res->h_size[0];
        for (int i = 0; i < n; i++)
            if (vsize[i] == vsize[i]) {
                v0.push_back(i);
                z0.push_back(vsize[i]);
            }
        res->count[0] = (int64_t)v0.size();
        v0.push_back(0);
        z0.push_back(0.0);
        merge_host<2>(rows[1], n, res->h_simp[1], res->h_size[1]);
        merge_host<3>(rows[2], n, res->h_simp[2], res->h_size[2]);
        merge_host<4>(rows[3], n, res->h_simp[3], res->h_size[3]);
        for (int d = 1; d <= 3; d++) res->count[d] = (int64_t)res->h_size[d].size() - 1;
        for (int d = 0; d < 4; d++) {
            res->host_ready[d] = true;
            res->cand[d] = -1;
            res->mol_rows[d] = {0, res->count[d]};
        }
        res->n = n;
        res->n_mol = 1;
        res->alpha_q = aq;
        res->fallbacks = fallbacks;
        res->work[0] = res->work[1] = -1;
        HIP_TRY(hipHostFree(pin));
        pin = nullptr;
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);
        free_complex(ck);
        free_complex(res);
        if (pin) (void)hipHostFree(pin);
        return set_error(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        (void)hipStreamSynchronize(s);
        free_complex(ck);
        free_complex(res);
        if (pin) (void)hipHostFree(pin);
        return set_error(AC_E_NOMEM, "host allocation failed");
    }
    *out = res;
    g_last_error.clear();
    return AC_OK;
}

// ---------------------------------------------------------------------------
// Union volume / area (measure.hpp)

static long long incidence_count(const ac_complex *c) {
    long long M = 0;
    for (int d = 0; d < 4; d++) M += c->count[d] * (d + 1);
    return M;
}

static void check_measure_args(const ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n) {
    if (!c) throw HipError{AC_E_INVALID, "complex is NULL"};
    if (!d_xyz || !d_radii) throw HipError{AC_E_INVALID, "NULL input pointer"};
    if (n != c->n) throw HipError{AC_E_INVALID, "n differs from the number of balls the complex was built on"};
    if (c->alpha_q != 0)
        throw HipError{AC_E_INVALID, "the complex was built at alpha != 0; for the union of grown balls build the "
                                     "complex of radii sqrt(r^2 + alpha) at alpha = 0"};
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) throw HipError{AC_E_INVALID, "the complex lives on another device"};
    if (incidence_count(c) >= INT_MAX) throw HipError{AC_E_CAPACITY, "too many simplex corners"};
}

// Sorts the corners of all simplices by ball id once per complex.
static void ensure_incidence(ac_complex *c, hipStream_t s) {
    if (c->inc_slot) return;
    const long long M = incidence_count(c);
    const int n = (int)c->n;
    int32_t *slot = static_cast<int32_t *>(dev_alloc((size_t)(M > 0 ? M : 1) * sizeof(int32_t)));
    int32_t *start = nullptr;
    try {
        start = static_cast<int32_t *>(dev_alloc((size_t)(n + 1) * sizeof(int32_t)));
        Scope sc;
        unsigned *key = sc.get<unsigned>(M > 0 ? M : 1);
        long long off = 0;
        for (int d = 0; d < 4; d++) {
            const long long m = c->count[d] * (d + 1);
            if (m) HIP_TRY(hipMemcpyAsync(key + off, c->d_simp[d], m * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            off += m;
        }
        if (M > 0) {
            k_iota<<<(unsigned)((M + MEASURE_BLOCK - 1) / MEASURE_BLOCK), MEASURE_BLOCK, 0, s>>>(slot, M);
            LAUNCH_CHECK();
            int32_t *sorted = slot;
            radix_sort<int>(key, sorted, (int)M, bits_for(n), s, sc);
            if (sorted != slot)
                HIP_TRY(hipMemcpyAsync(slot, sorted, (size_t)M * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        }
        k_incidence_start<<<(unsigned)((n + 1 + MEASURE_BLOCK - 1) / MEASURE_BLOCK), MEASURE_BLOCK, 0, s>>>(key, M, n,
                                                                                                          start);
        LAUNCH_CHECK();
        HIP_TRY(hipStreamSynchronize(s));  // before the scope's blocks go back to the pool
    } catch (...) {
        dev_free(slot);
        dev_free(start);
        throw;
    }
    c->inc_slot = slot;
    c->inc_start = start;
}

template <int K>
static void measure_fwd_dim(const ac_complex *c, const double *x, const double *r, double *part, int &nb,
                            hipStream_t s) {
    const long long m = c->count[K - 1];
    if (m == 0) return;
    const unsigned b = (unsigned)((m * K + MEASURE_BLOCK - 1) / MEASURE_BLOCK);
    k_measure_fwd<K><<<b, MEASURE_BLOCK, 0, s>>>(c->d_simp[K - 1], m, x, r, part + 2LL * nb);
    LAUNCH_CHECK();
    nb += (int)b;
}

// Writes V, A to d_out (device), or to the complex's own buffer if d_out is
// NULL; returns where they are.
static double *measure_forward(ac_complex *c, const double *x, const double *r, double *d_out, hipStream_t s) {
    long long nb_total = 0;
    for (int d = 0; d < 4; d++) nb_total += (c->count[d] * (d + 1) + MEASURE_BLOCK - 1) / MEASURE_BLOCK;
    if (!c->meas_part) c->meas_part = static_cast<double *>(dev_alloc((size_t)(2 * nb_total + 2) * sizeof(double)));
    double *part = c->meas_part;
    if (!d_out) d_out = part + 2 * nb_total;
    int nb = 0;
    measure_fwd_dim<1>(c, x, r, part, nb, s);
    measure_fwd_dim<2>(c, x, r, part, nb, s);
    measure_fwd_dim<3>(c, x, r, part, nb, s);
    measure_fwd_dim<4>(c, x, r, part, nb, s);
    k_measure_total<<<1, MEASURE_BLOCK, 0, s>>>(part, nb, d_out);
    LAUNCH_CHECK();
    return d_out;
}

// Backward of dimension K - 1; with part, also the forward's block parts
// (part + 2 nb onwards, nb advanced as in measure_fwd_dim).
template <int K>
static void measure_bwd_dim(const ac_complex *c, const double *x, const double *r, const double *g, double4 *contrib,
                            long long &off, hipStream_t s, double *part = nullptr, int *nb = nullptr) {
    const long long m = c->count[K - 1];
    if (m == 0) return;
    const unsigned b = (unsigned)((m * K + MEASURE_BLOCK - 1) / MEASURE_BLOCK);
    if (part) {
        k_measure_bwd<K, true><<<b, MEASURE_BLOCK, 0, s>>>(c->d_simp[K - 1], m, x, r, g, contrib + off, part + 2LL * *nb);
        *nb += (int)b;
    } else {
        k_measure_bwd<K, false><<<b, MEASURE_BLOCK, 0, s>>>(c->d_simp[K - 1], m, x, r, g, contrib + off, nullptr);
    }
    LAUNCH_CHECK();
    off += m * K;
}

// Validated molecule offsets of a batch call.
static ac_status batch_from(const int64_t *offsets, int64_t n_mol, const int32_t *cell_mA, Batch &bt) {
    if (!offsets) return set_error(AC_E_INVALID, "offsets is NULL");
    if (n_mol < 1 || n_mol > (1 << 20)) return set_error(AC_E_INVALID, "n_mol must be in [1, 2^20]");
    if (offsets[0] != 0) return set_error(AC_E_INVALID, "offsets[0] must be 0");
    bt.off.assign(offsets, offsets + n_mol + 1);
    for (int64_t m = 0; m < n_mol; m++)
        if (bt.off[m + 1] <= bt.off[m]) return set_error(AC_E_INVALID, "offsets must increase strictly (no empty molecule)");
    if (bt.off[n_mol] >= (1 << 26)) return set_error(AC_E_INVALID, "total balls must be below 2^26");
    bt.cell_mA.clear();
    if (cell_mA) {
        bt.cell_mA.assign(cell_mA, cell_mA + n_mol);
        for (int32_t c : bt.cell_mA)
            if (c < 1) return set_error(AC_E_INVALID, "cell sides must be positive");
    }
    return AC_OK;
}

// Time of one pipeline run on its stream (ms): two HIP events around the
// whole run, so that the idle time of its host synchronisations counts and
// no event between stages perturbs it.
static ac_status timed_run(const double *x, const double *r, int64_t n, const Batch &bt, double alpha, Options o,
                           hipStream_t s, double *ms) {
    o.profile = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        throw HipError{AC_E_DEVICE, "hipEventCreate failed"};
    }
    ac_complex *c = nullptr;
    ac_status st = hipEventRecord(e0, s) == hipSuccess ? run_pipeline(x, r, n, bt, alpha, o, s, &c) : AC_E_DEVICE;
    float f = 0.f;
    if (st == AC_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&f, e0, e1) != hipSuccess))
        st = set_error(AC_E_DEVICE, "timing events failed");
    free_complex(c);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = f;
    return st;
}

// Options of a call, validated: every field has a documented range and a
// value outside it is an argument error, not silently replaced.
static Options parse(const ac_options *opt) {
    Options o;
    if (!opt) return o;
    if (opt->reserved != 0) throw HipError{AC_E_INVALID, "ac_options.reserved must be 0"};
    if (opt->cell_mA < 0) throw HipError{AC_E_INVALID, "ac_options.cell_mA must be >= 0"};
    if (opt->wave_tile != 0)
        throw HipError{AC_E_INVALID, "ac_options.wave_tile must be 0 (every kernel maps one item to one lane)"};
    if (opt->capacity_hint != 0)
        throw HipError{AC_E_INVALID, "ac_options.capacity_hint must be 0 (buffers are sized from exact counts)"};
    if (opt->force_exact != 0 && opt->force_exact != 1) throw HipError{AC_E_INVALID, "ac_options.force_exact must be 0 or 1"};
    if (opt->vertex_shortcut != 0 && opt->vertex_shortcut != 1)
        throw HipError{AC_E_INVALID, "ac_options.vertex_shortcut must be 0 or 1"};
    if (opt->profile < 0 || opt->profile > PROFILE_SPLIT)
        throw HipError{AC_E_INVALID, "ac_options.profile must be 0, 1, 2 + a stage index or 2 + the stage count"};
    if (opt->cell_order != ORDER_ROW && opt->cell_order != ORDER_MORTON)
        throw HipError{AC_E_INVALID, "ac_options.cell_order must be 0 (row-major) or 1 (Morton)"};
    o.cell_mA = opt->cell_mA;
    o.force_exact = opt->force_exact;
    o.vertex_shortcut = opt->vertex_shortcut;
    o.profile = opt->profile;
    o.cell_order = opt->cell_order;
    return o;
}

// ---------------------------------------------------------------------------
// Recorded batch builds: one learning build notes the sizes, the fixed
// pipeline is run once to take its buffers and once under stream capture,
// and the captured graph is then replayed on new coordinates.
struct ac_plan {
    int device = 0;
    hipStream_t cap_stream = nullptr;  // the stream the graph was captured on
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Fixed fx;
    Recorder rec;                 // the build's buffers, owned by the plan
    std::vector<void *> consts;   // uploaded tiles, grid templates, capacities, molecule bounds
    // what an ordinary build needs when a replay stops
    const double *d_xyz = nullptr, *d_r = nullptr;
    int64_t n = 0;
    Batch bt;
    double alpha = 0;
    Options o;
    int32_t *out_simp[4] = {};
    double *out_size[4] = {};
    int last_stop = 0;
    int64_t ordinary_builds = 0;
};

static void free_plan(ac_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->cap_stream) {
        (void)hipStreamSynchronize(p->cap_stream);
        (void)hipStreamDestroy(p->cap_stream);
    }
    for (auto &b : p->rec.blocks) dev_free(b.first);
    for (void *c : p->consts) dev_free(c);
    delete p;
}

template <class T>
static T *upload(ac_plan *p, const T *h, size_t n, hipStream_t s) {
    T *d = static_cast<T *>(dev_alloc((n ? n : 1) * sizeof(T)));
    p->consts.push_back(d);
    if (n) HIP_TRY(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, s));
    return d;
}

// Sets t_rec for the duration of a scope.
struct RecordingOn {
    explicit RecordingOn(Recorder *r) { t_rec = r; }
    ~RecordingOn() { t_rec = nullptr; }
};

static ac_status plan_create(const double *d_xyz, const double *d_r, const Batch &bt, double alpha, const Options &o,
                             double headroom, hipStream_t s, ac_plan **out) {
    ac_plan *p = new ac_plan();
    try {
        HIP_TRY(hipGetDevice(&p->device));
        p->d_xyz = d_xyz;
        p->d_r = d_r;
        p->n = bt.off.back();
        p->bt = bt;
        p->alpha = alpha;
        p->o = o;
        const int n_mol = (int)bt.off.size() - 1;
        // 1. an ordinary build notes the sizes
        Fixed &fx = p->fx;
        fx.learn = true;
        ac_complex *r0 = nullptr;
        ac_status st = run_pipeline(d_xyz, d_r, p->n, bt, &alpha, 1, o, s, &r0, &fx);
        if (st != AC_OK) {
            free_plan(p);
            return st;
        }
        free_complex(r0);
        if (fx.two_pass)
            throw HipError{AC_E_CAPACITY, "a stage of this input needs the counted fill (rows longer than the "
                                          "single-pass slots); it has no recorded build"};
        // 2. capacities: the learned sizes with headroom; every molecule's
        // grid gets at least a cell per ball (a stopped molecule uses that)
        auto grow = [&](long long v) {
            const double c = std::ceil((double)v * headroom) + 256.0;
            if (c >= (double)INT_MAX) throw HipError{AC_E_CAPACITY, "planned capacity beyond 2^31"};
            return (int)c;
        };
        fx.E_cap = grow(fx.E);
        fx.T_cap = grow(fx.T);
        fx.Q_cap = grow(fx.Q);
        std::vector<long long> cap(n_mol);
        std::vector<Grid> tmpl = fx.grids;
        long long base = 0;
        for (int m = 0; m < n_mol; m++) {
            cap[m] = std::max<long long>((long long)std::ceil((double)fx.cells[m] * headroom), bt.off[m + 1] - bt.off[m]);
            tmpl[m].base = base;
            base += cap[m];
        }
        if (base >= (long long)INT_MAX) throw HipError{AC_E_CAPACITY, "planned grid cells beyond 2^31"};
        fx.ncell = base;
        std::vector<int2> tiles;
        std::vector<int> tile_first;
        quantise_tiles(bt, tiles, tile_first);
        std::vector<long long> bound(bt.off.begin(), bt.off.end());
        fx.d_tiles = upload(p, tiles.data(), tiles.size(), s);
        fx.d_tile_first = upload(p, tile_first.data(), tile_first.size(), s);
        fx.d_tmpl = upload(p, tmpl.data(), tmpl.size(), s);
        fx.d_cell_cap = upload(p, cap.data(), cap.size(), s);
        fx.d_bound = upload(p, bound.data(), bound.size(), s);
        HIP_TRY(hipStreamSynchronize(s));  // the host arrays above go out of scope
        fx.learn = false;
        // 3. the fixed pipeline once, taking (and recording) its buffers
        HIP_TRY(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
        ac_complex *r1 = nullptr;
        {
            const RecordingOn on(&p->rec);
            st = run_pipeline(d_xyz, d_r, p->n, bt, &alpha, 1, o, p->cap_stream, &r1, &fx);
            if (st != AC_OK) {
                free_plan(p);
                return st;
            }
            for (int d = 0; d < 4; d++) {
                p->out_simp[d] = r1->d_simp[d];
                p->out_size[d] = r1->d_size[d];
            }
            free_complex(r1);  // host object; its arrays are recorded blocks
        }
        Counters c{};
        read_back(&c, fx.cnt, 1, p->cap_stream);
        if (c.stop) throw HipError{AC_E_DEVICE, "internal error: the recorded build stopped on its own input"};
        // 4. the same launches captured in a graph, on the recorded buffers
        p->rec.replay = true;
        p->rec.next = 0;
        {
            const RecordingOn on(&p->rec);
            HIP_TRY(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
            ac_complex *r2 = nullptr;
            try {
                st = run_pipeline(d_xyz, d_r, p->n, bt, &alpha, 1, o, p->cap_stream, &r2, &fx);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(p->cap_stream, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIP_TRY(hipStreamEndCapture(p->cap_stream, &p->graph));
            if (st != AC_OK) {
                free_plan(p);
                return st;
            }
            bool same = p->rec.next == p->rec.blocks.size();
            for (int d = 0; d < 4; d++) same = same && r2->d_simp[d] == p->out_simp[d] && r2->d_size[d] == p->out_size[d];
            free_complex(r2);
            if (!same) throw HipError{AC_E_DEVICE, "internal error: the captured build used other buffers"};
        }
        HIP_TRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        *out = p;
        g_last_error.clear();
        return AC_OK;
    } catch (const HipError &e) {
        t_rec = nullptr;
        free_plan(p);
        return set_error(e.st, e.msg);
    }
}

static ac_status plan_result(ac_plan *p, hipStream_t s, ac_complex **out) {
    const int n_mol = (int)p->bt.off.size() - 1;
    Counters c{};
    read_back(&c, p->fx.cnt, 1, s);
    p->last_stop = c.stop;
    if (c.stop) {
        // the input did not fit the recording: an ordinary build of the same
        // arguments (it also reports invalid input)
        p->ordinary_builds++;
        const ac_status st = run_pipeline(p->d_xyz, p->d_r, p->n, p->bt, &p->alpha, 1, p->o, s, out);
        if (st == AC_OK) (*out)->batch = true;
        return st;
    }
    if (c.lookup) throw HipError{AC_E_DEVICE, "internal error: a facet of a kept simplex is not a candidate"};
    std::vector<int64_t> rows;
    if (n_mol > 1) {
        rows.resize(4 * (size_t)(n_mol + 1));
        read_back(rows.data(), (const int64_t *)p->fx.d_rows, rows.size(), s);
    }
    ac_complex *r = new ac_complex();
    try {
        for (double &x : r->stage_ms) x = -1.0;
        r->device = p->device;
        r->device_result = true;
        r->batch = true;
        r->n_mol = n_mol;
        r->n = p->n;
        r->alpha_q = (int64_t)std::nearbyint(p->alpha * 1e6);
        const int m[4] = {c.m0, c.m1, c.m2, c.m3};
        r->cand[0] = p->n;
        r->cand[1] = c.El;
        r->cand[2] = c.Tl;
        r->cand[3] = c.Ql;
        r->fallbacks = (int64_t)c.exact_fallbacks;
        r->work[0] = p->fx.ncell;
        r->work[1] = c.Nn;
        for (int d = 0; d < 4; d++) {
            r->count[d] = m[d];
            r->d_simp[d] = static_cast<int32_t *>(dev_alloc((size_t)(m[d] > 0 ? m[d] : 1) * (d + 1) * sizeof(int32_t)));
            r->d_size[d] = static_cast<double *>(dev_alloc((size_t)(m[d] > 0 ? m[d] : 1) * sizeof(double)));
            if (m[d] > 0) {
                HIP_TRY(hipMemcpyAsync(r->d_simp[d], p->out_simp[d], (size_t)m[d] * (d + 1) * sizeof(int32_t),
                                       hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipMemcpyAsync(r->d_size[d], p->out_size[d], (size_t)m[d] * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
            }
            if (n_mol > 1) {
                const int64_t *b0 = rows.data() + (size_t)d * (n_mol + 1);
                r->mol_rows[d].assign(b0, b0 + (n_mol + 1));
            } else {
                r->mol_rows[d] = {0, r->count[d]};
            }
        }
    } catch (...) {
        (void)hipStreamSynchronize(s);
        free_complex(r);
        throw;
    }
    *out = r;
    return AC_OK;
}

// ---------------------------------------------------------------------------
// Fixed device scratch of ac_alpha_complex_noalloc. Every device the library
// runs on holds one copy of this array until the process ends. In host code
// its name is only a stand-in: the device address of a device's copy comes
// from hipGetSymbolAddress, taken once per device with that device current,
// and only that address is handed to kernels and copies.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)AC_NOALLOC_SCRATCH_MIB << 20;
// a ball needs more than this much scratch whatever the input (quantised and
// sorted balls, sort keys, neighbour slots)
constexpr size_t NOALLOC_MIN_BYTES_PER_BALL = 128;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu[NOALLOC_MAX_DEVICES];  // held for a whole call: one call per device at a time
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};  // device address of each device's copy, once known
}  // namespace

// Device address of the scratch array on device `dev` (the current device;
// the caller holds g_scratch_mu[dev]).
static char *scratch_on(int dev) {
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw HipError{AC_E_DEVICE, "hipGetSymbolAddress gave no address for the scratch array"};
        g_scratch_ptr[dev] = p;
    }
    return static_cast<char *>(g_scratch_ptr[dev]);
}

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

ac_status ac_alpha_complex_device(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                  const ac_options *opt, void *stream, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    try {
        const Options o = parse(opt);
        if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
        Batch bt;
        bt.off = {0, n};
        return run_pipeline(d_xyz, d_radii, n, bt, alpha, o, static_cast<hipStream_t>(stream), out);
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_complex_noalloc(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                   const ac_options *opt, void *stream, int32_t *const *d_simp,
                                   double *const *d_size, const int64_t *capacity, int64_t *counts) {
    if (!d_simp || !d_size || !capacity || !counts) return set_error(AC_E_INVALID, "NULL output argument");
    for (int d = 0; d < 4; d++) counts[d] = -1;
    ac_complex *c = nullptr;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = -1;
    try {
        const Options o = parse(opt);
        if (o.profile != 0) return set_error(AC_E_INVALID, "ac_options.profile must be 0 (profiling creates HIP events)");
        if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
        if (n < 1 || n >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
        for (int d = 0; d < 4; d++) {
            if (capacity[d] < 0) return set_error(AC_E_INVALID, "capacity must be >= 0");
            if (capacity[d] > 0 && (!d_simp[d] || !d_size[d]))
                return set_error(AC_E_INVALID, "NULL output buffer with a non-zero capacity");
        }
        if ((size_t)n > NOALLOC_SCRATCH_BYTES / NOALLOC_MIN_BYTES_PER_BALL)
            return set_error(AC_E_CAPACITY, "n exceeds what the " + std::to_string(AC_NOALLOC_SCRATCH_MIB) +
                                                " MiB of fixed scratch can hold");
        HIP_TRY(hipGetDevice(&dev));
        if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return set_error(AC_E_DEVICE, "device index out of range");
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    Arena ar;
    struct ArenaOn {
        explicit ArenaOn(Arena *a) { t_arena = a; }
        ~ArenaOn() { t_arena = nullptr; }
    };
    try {
        ar.base = scratch_on(dev);
        ar.cap = NOALLOC_SCRATCH_BYTES;
        const ArenaOn on(&ar);
        Batch bt;
        bt.off = {0, n};
        const Options o = parse(opt);
        const ac_status st = run_pipeline(d_xyz, d_radii, n, bt, alpha, o, s, &c);  // synchronises s on error
        if (st != AC_OK) return st;
        bool fits = true;
        for (int d = 0; d < 4; d++) {
            counts[d] = c->count[d];
            fits = fits && c->count[d] <= capacity[d];
        }
        for (int d = 0; fits && d < 4; d++) {
            const size_t m = (size_t)c->count[d];
            if (m == 0) continue;
            HIP_TRY(hipMemcpyAsync(d_simp[d], c->d_simp[d], m * (d + 1) * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
            HIP_TRY(hipMemcpyAsync(d_size[d], c->d_size[d], m * sizeof(double), hipMemcpyDeviceToDevice, s));
        }
        // the next call may reuse the scratch only once these copies are done
        HIP_TRY(hipStreamSynchronize(s));
        free_complex(c);  // host object only: its arrays lie in the scratch
        c = nullptr;
        if (!fits) return set_error(AC_E_CAPACITY, "an output buffer is smaller than the result (counts holds the sizes)");
        g_last_error.clear();
        return AC_OK;
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);
        if (c) {
            const ArenaOn on(&ar);  // its arrays are scratch, not pool blocks
            free_complex(c);
        }
        return set_error(e.st, e.msg);
    } catch (...) {
        (void)hipStreamSynchronize(s);
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_complex_partitioned(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                       int32_t parts, const ac_options *opt, void *stream, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    try {
        const Options o = parse(opt);
        if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
        return run_partitioned(d_xyz, d_radii, n, alpha, parts, o, static_cast<hipStream_t>(stream), out);
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_complex_partitioned_host(const double *xyz, const double *radii, int64_t n, double alpha,
                                            int32_t parts, const ac_options *opt, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    try {
        const Options o = parse(opt);
        return run_streamed(xyz, radii, n, alpha, parts, o, out);
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_sweep_device(const double *d_xyz, const double *d_radii, int64_t n, const double *alphas,
                                int64_t n_alpha, const ac_options *opt, void *stream, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    if (n_alpha < 1 || n_alpha > AC_MAX_SWEEP) return set_error(AC_E_INVALID, "number of alpha values out of range");
    for (int64_t k = 0; k < n_alpha; k++) out[k] = nullptr;
    try {
        const Options o = parse(opt);
        if (!d_xyz || !d_radii || !alphas) return set_error(AC_E_INVALID, "NULL input pointer");
        Batch bt;
        bt.off = {0, n};
        return run_pipeline(d_xyz, d_radii, n, bt, alphas, (int)n_alpha, o, static_cast<hipStream_t>(stream), out);
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_complex(const double *xyz, const double *radii, int64_t n, double alpha, const ac_options *opt,
                           ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    void *dx = nullptr, *dr = nullptr;
    try {
        const Options o = parse(opt);
        if (!xyz || !radii) return set_error(AC_E_INVALID, "NULL input pointer");
        if (n < 1 || n >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
        dx = dev_alloc((size_t)n * 3 * sizeof(double));
        dr = dev_alloc((size_t)n * sizeof(double));
        HIP_TRY(hipMemcpy(dx, xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(dr, radii, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
        Batch bt;
        bt.off = {0, n};
        ac_status st = run_pipeline(static_cast<double *>(dx), static_cast<double *>(dr), n, bt, alpha, o, nullptr, out);
        dev_free(dx);
        dev_free(dr);
        if (st != AC_OK) return st;
        (*out)->device_result = false;
        for (int d = 0; d < 4; d++)
            if (!ac_simplices(*out, d) || !ac_sizes(*out, d)) {
                ac_free(*out);
                *out = nullptr;
                return set_error(AC_E_DEVICE, "device-to-host copy failed");
            }
        return AC_OK;
    } catch (const HipError &e) {
        dev_free(dx);
        dev_free(dr);
        return set_error(e.st, e.msg);
    } catch (...) {
        dev_free(dx);
        dev_free(dr);
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_alpha_complex_batch(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol,
                                 double alpha, const ac_options *opt, const int32_t *cell_mA, void *stream,
                                 ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    try {
        const Options o = parse(opt);
        if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
        Batch bt;
        const ac_status st = batch_from(offsets, n_mol, cell_mA, bt);
        if (st != AC_OK) return st;
        const ac_status sp = run_pipeline(d_xyz, d_radii, bt.off[n_mol], bt, alpha, o, static_cast<hipStream_t>(stream), out);
        if (sp == AC_OK) (*out)->batch = true;
        return sp;
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_plan_create(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol, double alpha,
                         const ac_options *opt, const int32_t *cell_mA, double headroom, void *stream, ac_plan **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    try {
        const Options o = parse(opt);
        if (o.profile != 0) return set_error(AC_E_INVALID, "ac_options.profile must be 0 for a recorded build");
        if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
        if (!std::isfinite(alpha)) return set_error(AC_E_INVALID, "alpha is not finite");
        if (!(headroom >= 1.0 && headroom <= 16.0)) return set_error(AC_E_INVALID, "headroom must be in [1, 16]");
        Batch bt;
        const ac_status st = batch_from(offsets, n_mol, cell_mA, bt);
        if (st != AC_OK) return st;
        return plan_create(d_xyz, d_radii, bt, alpha, o, headroom, static_cast<hipStream_t>(stream), out);
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

ac_status ac_plan_launch(ac_plan *p, void *stream) {
    if (!p) return set_error(AC_E_INVALID, "plan is NULL");
    try {
        int dev = -1;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != p->device) return set_error(AC_E_INVALID, "the plan was made on another device");
        HIP_TRY(hipGraphLaunch(p->exec, static_cast<hipStream_t>(stream)));
        return AC_OK;
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    }
}

ac_status ac_plan_result(ac_plan *p, void *stream, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!p) return set_error(AC_E_INVALID, "plan is NULL");
    try {
        int dev = -1;
        HIP_TRY(hipGetDevice(&dev));
        if (dev != p->device) return set_error(AC_E_INVALID, "the plan was made on another device");
        const ac_status st = plan_result(p, static_cast<hipStream_t>(stream), out);
        if (st == AC_OK) g_last_error.clear();
        return st;
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
}

int32_t ac_plan_stopped(const ac_plan *p) { return p ? p->last_stop : -1; }

int64_t ac_plan_ordinary_builds(const ac_plan *p) { return p ? p->ordinary_builds : -1; }

void ac_plan_free(ac_plan *p) { free_plan(p); }

int64_t ac_molecule_count(const ac_complex *c) { return c ? c->n_mol : -1; }

const int64_t *ac_molecule_rows(const ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3 || c->mol_rows[dim].empty()) return nullptr;
    return c->mol_rows[dim].data();
}

const int32_t *ac_molecule(ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3 || !c->batch || c->mol_rows[dim].size() != (size_t)c->n_mol + 1) return nullptr;
    std::vector<int32_t> &h = c->h_mol[dim];
    if (h.empty()) {
        const std::vector<int64_t> &r = c->mol_rows[dim];
        h.assign((size_t)c->count[dim] + 1, 0);  // one spare entry: never a zero-length array
        for (int64_t m = 0; m < c->n_mol; m++)
            std::fill(h.begin() + r[m], h.begin() + r[m + 1], (int32_t)m);
    }
    return h.data();
}

ac_status ac_tune_cells(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol, double alpha,
                        const ac_options *opt, void *stream, int32_t *cell_mA_out, int32_t *bucket_out) {
    try {
        const Options o = parse(opt);
        if (!d_xyz || !d_radii || !cell_mA_out) return set_error(AC_E_INVALID, "NULL pointer");
        Batch all;
        ac_status st = batch_from(offsets, n_mol, nullptr, all);
        if (st != AC_OK) return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        // grown radius s_g (mA): the default cell side the candidates scale
        double rmax = 0;
        {
            std::vector<double> hr((size_t)all.off[n_mol]);
            HIP_TRY(hipMemcpyAsync(hr.data(), d_radii, hr.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (double v : hr) rmax = std::max(rmax, v);
        }
        const double sg = std::sqrt(std::max(rmax * rmax + alpha, 1e-6)) * 1000.0;
        static const double kFactor[] = {0.5, 0.7, 1.0, 1.4, 2.0};
        // size buckets: [0, 2k), [2k, 8k), [8k, 32k), [32k, inf)
        auto bucket_of = [](int64_t nm) { return nm < 2000 ? 0 : nm < 8000 ? 1 : nm < 32000 ? 2 : 3; };
        for (int b = 0; b < 4; b++) {
            std::vector<int64_t> mols;
            for (int64_t m = 0; m < n_mol; m++)
                if (bucket_of(all.off[m + 1] - all.off[m]) == b) mols.push_back(m);
            if (mols.empty()) continue;
            // the bucket's molecules, copied into one contiguous sub-batch
            Batch sub;
            sub.off.push_back(0);
            for (int64_t m : mols) sub.off.push_back(sub.off.back() + all.off[m + 1] - all.off[m]);
            const int64_t ns = sub.off.back();
            Scope sc;
            double *x = sc.get<double>(3 * ns), *r = sc.get<double>(ns);
            for (size_t k = 0; k < mols.size(); k++) {
                const int64_t m = mols[k], nm = all.off[m + 1] - all.off[m];
                HIP_TRY(hipMemcpyAsync(x + 3 * sub.off[k], d_xyz + 3 * all.off[m], 3 * nm * sizeof(double),
                                       hipMemcpyDeviceToDevice, s));
                HIP_TRY(hipMemcpyAsync(r + sub.off[k], d_radii + all.off[m], nm * sizeof(double), hipMemcpyDeviceToDevice, s));
            }
            // each side: one warm-up run (fills the pool), then the median of
            // kTuneReps timed runs; another side replaces the default s_g only
            // when it is faster by more than kTuneMargin (run-to-run noise is a
            // few per cent)
            constexpr int kTuneReps = 5;
            constexpr double kTuneMargin = 0.03;
            std::vector<double> med(std::size(kFactor));
            for (size_t fi = 0; fi < std::size(kFactor); fi++) {
                const int32_t side = std::max<int32_t>(1, (int32_t)std::lround(kFactor[fi] * sg));
                sub.cell_mA.assign(mols.size(), side);
                std::vector<double> ts;
                for (int rep = 0; rep <= kTuneReps; rep++) {
                    double tr = 0;
                    st = timed_run(x, r, ns, sub, alpha, o, s, &tr);
                    if (st != AC_OK) return st;
                    if (rep > 0) ts.push_back(tr);
                }
                std::nth_element(ts.begin(), ts.begin() + ts.size() / 2, ts.end());
                med[fi] = ts[ts.size() / 2];
            }
            size_t def = 0;
            while (kFactor[def] != 1.0) def++;
            size_t bi = def;
            for (size_t fi = 0; fi < med.size(); fi++)
                if (med[fi] < med[bi]) bi = fi;
            if (bi != def && med[bi] > (1.0 - kTuneMargin) * med[def]) bi = def;
            const int32_t best = std::max<int32_t>(1, (int32_t)std::lround(kFactor[bi] * sg));
            for (int64_t m : mols) {
                cell_mA_out[m] = best;
                if (bucket_out) bucket_out[m] = b;
            }
            HIP_TRY(hipStreamSynchronize(s));
        }
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    g_last_error.clear();
    return AC_OK;
}

int64_t ac_count(const ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3) return -1;
    return c->count[dim];
}

const int32_t *ac_simplices(ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3) return nullptr;
    if (!c->host_ready[dim]) {
        const size_t m = (size_t)c->count[dim];
        c->h_simp[dim].resize(m * (dim + 1) + 1);
        c->h_size[dim].resize(m + 1);
        if (m) {
            if (hipMemcpy(c->h_simp[dim].data(), c->d_simp[dim], m * (dim + 1) * sizeof(int32_t),
                          hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(c->h_size[dim].data(), c->d_size[dim], m * sizeof(double), hipMemcpyDeviceToHost) !=
                    hipSuccess) {
                set_error(AC_E_DEVICE, "device-to-host copy failed");
                return nullptr;
            }
        }
        c->host_ready[dim] = true;
    }
    return c->h_simp[dim].data();
}

const double *ac_sizes(ac_complex *c, int dim) {
    if (!ac_simplices(c, dim)) return nullptr;
    return c->h_size[dim].data();
}

const int32_t *ac_simplices_device(const ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3 || !c->device_result) return nullptr;
    return c->d_simp[dim];
}

const double *ac_sizes_device(const ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3 || !c->device_result) return nullptr;
    return c->d_size[dim];
}

int64_t ac_candidate_count(const ac_complex *c, int dim) {
    if (!c || dim < 0 || dim > 3) return -1;
    return c->cand[dim];
}

int64_t ac_exact_fallbacks(const ac_complex *c) { return c ? c->fallbacks : -1; }

int64_t ac_work_count(const ac_complex *c, int which) {
    if (!c || which < 0 || which > 1) return -1;
    return c->work[which];
}

ac_status ac_union_measure_device(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                  double *d_out, void *stream) {
    try {
        check_measure_args(c, d_xyz, d_radii, n);
        if (!d_out) throw HipError{AC_E_INVALID, "out is NULL"};
        measure_forward(c, d_xyz, d_radii, d_out, static_cast<hipStream_t>(stream));
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    g_last_error.clear();
    return AC_OK;
}

ac_status ac_union_measure(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n, double *V,
                           double *A, void *stream) {
    if (!V || !A) return set_error(AC_E_INVALID, "V or A is NULL");
    try {
        check_measure_args(c, d_xyz, d_radii, n);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const double *d_out = measure_forward(c, d_xyz, d_radii, nullptr, s);
        double h[2];
        read_back(h, d_out, 2, s);
        *V = h[0];
        *A = h[1];
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    g_last_error.clear();
    return AC_OK;
}

// Backward (and, with d_out, the forward in the same pass) on stream s.
static void measure_backward(ac_complex *c, const double *x, const double *r, int64_t n, const double *g,
                             double *dx, double *dr, double *d_out, hipStream_t s) {
    ensure_incidence(c, s);
    const long long M = incidence_count(c);
    if (!c->meas_contrib) c->meas_contrib = static_cast<double4 *>(dev_alloc((size_t)(M > 0 ? M : 1) * sizeof(double4)));
    double4 *contrib = c->meas_contrib;
    double *part = nullptr;
    if (d_out) {
        long long nb_total = 0;
        for (int d = 0; d < 4; d++) nb_total += (c->count[d] * (d + 1) + MEASURE_BLOCK - 1) / MEASURE_BLOCK;
        if (!c->meas_part) c->meas_part = static_cast<double *>(dev_alloc((size_t)(2 * nb_total + 2) * sizeof(double)));
        part = c->meas_part;
    }
    long long off = 0;
    int nb = 0;
    measure_bwd_dim<1>(c, x, r, g, contrib, off, s, part, &nb);
    measure_bwd_dim<2>(c, x, r, g, contrib, off, s, part, &nb);
    measure_bwd_dim<3>(c, x, r, g, contrib, off, s, part, &nb);
    measure_bwd_dim<4>(c, x, r, g, contrib, off, s, part, &nb);
    if (d_out) {
        k_measure_total<<<1, MEASURE_BLOCK, 0, s>>>(part, nb, d_out);
        LAUNCH_CHECK();
    }
    k_measure_gather<<<(unsigned)((n + MEASURE_BLOCK - 1) / MEASURE_BLOCK), MEASURE_BLOCK, 0, s>>>(
        c->inc_start, c->inc_slot, contrib, (int)n, dx, dr);
    LAUNCH_CHECK();
}

ac_status ac_union_measure_fused(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                 const double *d_grad, double *d_out, double *d_dxyz, double *d_dradii, void *stream) {
    try {
        check_measure_args(c, d_xyz, d_radii, n);
        if (!d_grad || !d_out || !d_dxyz || !d_dradii) throw HipError{AC_E_INVALID, "NULL output or gradient pointer"};
        measure_backward(c, d_xyz, d_radii, n, d_grad, d_dxyz, d_dradii, d_out, static_cast<hipStream_t>(stream));
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    g_last_error.clear();
    return AC_OK;
}

ac_status ac_union_measure_backward(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                    const double *d_grad, double *d_dxyz, double *d_dradii, void *stream) {
    try {
        check_measure_args(c, d_xyz, d_radii, n);
        if (!d_grad || !d_dxyz || !d_dradii) throw HipError{AC_E_INVALID, "NULL gradient pointer"};
        measure_backward(c, d_xyz, d_radii, n, d_grad, d_dxyz, d_dradii, nullptr, static_cast<hipStream_t>(stream));
    } catch (const HipError &e) {
        return set_error(e.st, e.msg);
    } catch (...) {
        return set_error(AC_E_DEVICE, "unexpected host exception");
    }
    g_last_error.clear();
    return AC_OK;
}

void ac_free(ac_complex *c) { free_complex(c); }

int ac_stage_count(void) { return ST_COUNT; }

const char *ac_stage_name(int i) { return (i >= 0 && i < ST_COUNT) ? kStageNames[i] : ""; }

double ac_stage_ms(const ac_complex *c, int i) {
    if (!c || i < 0 || i >= ST_COUNT) return -1.0;
    return c->stage_ms[i];
}

ac_status ac_release_workspace(void) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(AC_E_DEVICE, "hipGetDevice failed");
    Pool &P = pool();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto &kv : P.free_blocks[dev]) (void)hipFree(kv.second);
    P.free_blocks[dev].clear();
    return AC_OK;
}

const char *ac_status_str(ac_status s) {
    switch (s) {
        case AC_OK: return "ok";
        case AC_E_INVALID: return "invalid argument";
        case AC_E_DUPLICATE: return "duplicate centres";
        case AC_E_RANGE: return "input outside the exact-arithmetic range";
        case AC_E_NOMEM: return "out of memory";
        case AC_E_DEVICE: return "HIP device error";
        case AC_E_CAPACITY: return "candidate buffer capacity exceeded";
    }
    return "unknown status";
}

const char *ac_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
