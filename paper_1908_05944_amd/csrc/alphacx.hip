// libalphacx: host orchestration and the C ABI declared in include/alphacx.h.
//
// One call runs the whole pipeline of kernels.hpp on one HIP stream. Device
// memory comes from a per-device caching pool, so repeated calls of similar
// size allocate nothing from the runtime after the first.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "alphacx.h"
#include "kernels.hpp"

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

static void *dev_alloc(size_t n) {
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
    int32_t *d_simp[4] = {nullptr, nullptr, nullptr, nullptr};
    double *d_size[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<int32_t> h_simp[4];
    std::vector<double> h_size[4];
    bool host_ready[4] = {false, false, false, false};
    bool device_result = false;
    int device = 0;
    double stage_ms[32];
};

static void free_complex(ac_complex *c) {
    if (!c) return;
    for (int d = 0; d < 4; d++) {
        dev_free(c->d_simp[d]);
        dev_free(c->d_size[d]);
    }
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

// out[0..n] = exclusive scan of in[0..n), out[n] = total. One launch up to
// SCAN_SMALL items, three above (tile scan, scan of tile sums, add).
static void scan_i32(const int *in, int *out, long long n, hipStream_t s, Scope &sc) {
    if (n <= 0) {
        fill<int>(out, 0, 1, s);
        return;
    }
    if (n <= SCAN_SMALL) {
        k_scan_small<<<1, SCAN_BLOCK, 0, s>>>(in, out, (int)n);
        LAUNCH_CHECK();
        return;
    }
    const long long tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int *sums = sc.get<int>(tiles);
    int *offs = sc.get<int>(tiles + 1);
    k_scan_tiles<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, out, sums, n);
    LAUNCH_CHECK();
    scan_i32(sums, offs, tiles, s, sc);
    k_scan_add_total<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(out, offs, n, (int)tiles);
    LAUNCH_CHECK();
}

template <class T>
static T read_one(const T *d, hipStream_t s) {
    T h;
    HIP_TRY(hipMemcpyAsync(&h, d, sizeof(T), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return h;
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

// Stable LSD radix sort of (key, payload) on the low `bits` bits of key;
// the result ends in key/pay.
template <class P>
static void radix_sort(unsigned *key, P *pay, int n, int bits, hipStream_t s, Scope &sc) {
    if (n <= 1 || bits <= 0) return;
    const int tiles = (n + RS_TILE - 1) / RS_TILE;
    unsigned *k2 = sc.get<unsigned>(n);
    P *p2 = sc.get<P>(n);
    int *hist = sc.get<int>((size_t)RS_BINS * tiles);
    int *offs = sc.get<int>((size_t)RS_BINS * tiles + 1);
    unsigned *kin = key, *kout = k2;
    P *pin = pay, *pout = p2;
    for (int shift = 0; shift < bits; shift += RS_BITS) {
        k_rs_hist<<<tiles, RS_BLOCK, 0, s>>>(kin, n, shift, hist, tiles);
        LAUNCH_CHECK();
        scan_i32(hist, offs, (long long)RS_BINS * tiles, s, sc);
        k_rs_scatter<P><<<tiles, RS_BLOCK, 0, s>>>(kin, pin, kout, pout, n, shift, offs, tiles);
        LAUNCH_CHECK();
        std::swap(kin, kout);
        std::swap(pin, pout);
    }
    if (kin != key) {
        HIP_TRY(hipMemcpyAsync(key, kin, sizeof(unsigned) * n, hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(pay, pin, sizeof(P) * n, hipMemcpyDeviceToDevice, s));
    }
}

static int bits_for(long long n) {
    int b = 1;
    while ((1LL << b) < n) b++;
    return b;
}

// Emit dimension d (K = d + 1 >= 2): kept candidates (flags `in`, compacted
// positions `fpos`), remapped to input ids, radix-sorted by their least id,
// then ranked inside each bucket by the remaining ids.
template <int K>
static void emit_dim(const unsigned char *in, const int *fpos, const double *sizes, int M, const Cands &cd, int n,
                     hipStream_t s, Scope &sc, ac_complex *res, int d, int m_out) {
    typedef typename EmitPay<K>::type P;
    res->count[d] = m_out;
    res->d_simp[d] = static_cast<int32_t *>(dev_alloc((size_t)(m_out > 0 ? m_out : 1) * K * sizeof(int32_t)));
    res->d_size[d] = static_cast<double *>(dev_alloc((size_t)(m_out > 0 ? m_out : 1) * sizeof(double)));
    if (m_out == 0) return;
    unsigned *key = sc.get<unsigned>(m_out);
    P *pay = sc.get<P>(m_out);
    k_emit_keys<K><<<grid_for(M), BLOCK, 0, s>>>(in, fpos, M, cd.up, cd.edge_i, cd.tri_k, cd.tri_e, cd.tet_t,
                                                 cd.tet_l, cd.perm, key, pay);
    LAUNCH_CHECK();
    radix_sort<P>(key, pay, m_out, bits_for(n), s, sc);
    k_emit_rank<K><<<grid_for(m_out), BLOCK, 0, s>>>(key, pay, m_out, sizes, res->d_simp[d], res->d_size[d]);
    LAUNCH_CHECK();
}

struct Options {
    int cell_mA = 0;
    int force_exact = 0;
    int vertex_shortcut = 0;
    int profile = 0;
};

// Stages timed by HIP events when profiling (one event before each).
enum Stage {
    ST_QUANTISE, ST_BIN, ST_NBR_COUNT, ST_NBR_SCAN, ST_NBR_FILL, ST_TRI_COUNT, ST_TRI_SCAN, ST_TRI_FILL,
    ST_TRI_GABRIEL, ST_TET_COUNT, ST_TET_FILL, ST_TETRA, ST_TRI_FINAL, ST_EDGE_FINAL, ST_VERT_FINAL, ST_EMIT,
    ST_COUNT
};
static const char *kStageNames[ST_COUNT] = {
    "quantise", "binning", "neighbours_count", "neighbours_scan", "neighbours_fill", "triangles_count",
    "triangles_scan", "triangles_fill", "triangles_ac2", "tetrahedra_count", "tetrahedra_fill", "tetrahedra_ac2",
    "triangles_final", "edges_final", "vertices_final", "emit"};

struct StageTimer {
    bool on = false;
    hipStream_t s = nullptr;
    hipEvent_t ev[ST_COUNT + 1] = {};
    bool rec[ST_COUNT + 1] = {};
    void start(bool enable, hipStream_t st) {
        on = enable;
        s = st;
        if (!on) return;
        for (int i = 0; i <= ST_COUNT; i++) HIP_TRY(hipEventCreate(&ev[i]));
    }
    void mark(int i) {
        if (!on) return;
        HIP_TRY(hipEventRecord(ev[i], s));
        rec[i] = true;
    }
    void collect(double *ms) {
        for (int i = 0; i < ST_COUNT; i++) {
            ms[i] = -1.0;
            if (on && rec[i] && rec[i + 1]) {
                float f = 0.f;
                if (hipEventElapsedTime(&f, ev[i], ev[i + 1]) == hipSuccess) ms[i] = f;
            }
        }
    }
    ~StageTimer() {
        if (on)
            for (int i = 0; i <= ST_COUNT; i++)
                if (ev[i]) (void)hipEventDestroy(ev[i]);
    }
};

__global__ void __launch_bounds__(BLOCK) k_flags_to_int(const unsigned char *__restrict__ f, long long M,
                                                         int *__restrict__ out) {
    const long long i = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (i < M) out[i] = f[i];
}

// Exclusive scan of 0/1 flags into pos[0..M]; pos[M] is the number set.
static void scan_flags(const unsigned char *flags, long long M, int *pos, hipStream_t s, Scope &sc) {
    if (M <= 0) {
        fill<int>(pos, 0, 1, s);
        return;
    }
    int *work = sc.get<int>(M);
    k_flags_to_int<<<grid_for(M), BLOCK, 0, s>>>(flags, M, work);
    LAUNCH_CHECK();
    scan_i32(work, pos, M, s, sc);
}

// The whole pipeline from device arrays. Returns AC_OK and *out on success.
static ac_status run_pipeline(const double *d_xyz, const double *d_r, int64_t n64, double alpha, const Options &o,
                              hipStream_t s, ac_complex **out) {
    *out = nullptr;
    if (n64 < 1 || n64 >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
    if (!std::isfinite(alpha)) return set_error(AC_E_INVALID, "alpha is not finite");
    const double as = alpha * 1e6;
    if (!(std::fabs(as) < 67108864.0)) return set_error(AC_E_RANGE, "|alpha| too large for the exact bit budget");
    const long long aq = (long long)std::nearbyint(as);
    const int n = (int)n64;
    Scope sc;
    StageTimer tm;
    ac_complex *res = new ac_complex();
    for (double &x : res->stage_ms) x = -1.0;
    HIP_TRY(hipGetDevice(&res->device));
    res->device_result = true;
    try {
        tm.start(o.profile != 0, s);
        // ---- quantise + stats ----
        tm.mark(ST_QUANTISE);
        int4 *q = sc.get<int4>(n);
        Stats *st = sc.get<Stats>(1);
        Counters *cnt = sc.get<Counters>(1);
        HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(Counters), s));
        {
            long long b = grid_for(n);
            if (b > 2048) b = 2048;
            Stats *part = sc.get<Stats>(b);
            k_quantise<<<(unsigned)b, BLOCK, 0, s>>>(d_xyz, d_r, n, q, part);
            LAUNCH_CHECK();
            k_stats_reduce<<<1, BLOCK, 0, s>>>(part, (int)b, st);
            LAUNCH_CHECK();
        }
        const Stats hs = read_one(st, s);
        if (hs.flags & 1) throw HipError{AC_E_INVALID, "non-finite coordinate, or radius not positive"};
        if (hs.flags & 2) throw HipError{AC_E_RANGE, "coordinate or radius outside the exact bit budget"};
        const long long sg2 = (long long)hs.wmax + aq;
        if (sg2 >= (1LL << 26)) throw HipError{AC_E_RANGE, "r_max^2 + alpha too large for the exact bit budget"};
        PredParams pp;
        pp.aq = aq;
        pp.sg2 = sg2 < 0 ? 0 : sg2;
        const long long sgc = isqrt_ceil(pp.sg2);
        pp.sgc = sgc;
        pp.bmax = 2.0 * (double)sgc;
        pp.gmax = 4.0 * (double)pp.sg2 + (double)hs.wmax;
        pp.force_exact = o.force_exact;

        // ---- grid ----
        Grid g;
        g.ox = hs.minx; g.oy = hs.miny; g.oz = hs.minz;
        const long long ex = (long long)hs.maxx - hs.minx + 1, ey = (long long)hs.maxy - hs.miny + 1,
                        ez = (long long)hs.maxz - hs.minz + 1;
        long long side = o.cell_mA > 0 ? o.cell_mA : (sgc > 0 ? sgc : 1);
        const long long cell_limit = std::max<long long>(8LL * n, 1LL << 22);
        auto ncell_of = [&](long long sd) { return ((ex + sd - 1) / sd) * ((ey + sd - 1) / sd) * ((ez + sd - 1) / sd); };
        while (ncell_of(side) > cell_limit) side = side + side / 4 + 1;
        g.s = (int)side;
        g.nx = (int)((ex + side - 1) / side); g.ny = (int)((ey + side - 1) / side); g.nz = (int)((ez + side - 1) / side);
        g.reach = (int)((2 * sgc + side - 1) / side);
        const long long ncell = (long long)g.nx * g.ny * g.nz;

        // ---- binning ----
        tm.mark(ST_BIN);
        unsigned *ckey = sc.get<unsigned>(n);
        unsigned *cidx = sc.get<unsigned>(n);
        int *cell_count = sc.get<int>(ncell + 1);
        int *cell_start = sc.get<int>(ncell + 1);
        k_cell_key<<<grid_for(n), BLOCK, 0, s>>>(q, n, g, ckey, cidx);
        LAUNCH_CHECK();
        radix_sort<unsigned>(ckey, cidx, n, bits_for(ncell), s, sc);
        fill<int>(cell_count, 0, ncell, s);
        k_cell_runs<<<grid_for(n), BLOCK, 0, s>>>(ckey, n, cell_count);
        LAUNCH_CHECK();
        scan_i32(cell_count, cell_start, ncell, s, sc);
        int4 *atom = sc.get<int4>(n);
        int *perm = sc.get<int>(n);
        k_gather_atoms<<<grid_for(n), BLOCK, 0, s>>>(q, ckey, cidx, n, atom, perm, cnt);
        LAUNCH_CHECK();

        // ---- neighbours and candidate edges: count, scan, fill ----
        int *deg_n = sc.get<int>(n), *deg_up = sc.get<int>(n);
        int *nbr_start = sc.get<int>(n + 1), *up_start = sc.get<int>(n + 1);
        unsigned char *vgab = sc.get<unsigned char>(n);
        tm.mark(ST_NBR_COUNT);
        k_neighbours<NB_COUNT><<<grid_for(n), BLOCK, 0, s>>>(atom, perm, n, g, cell_start, pp, deg_n, deg_up, nullptr,
                                                            nullptr, nullptr, nullptr, nullptr, nullptr);
        LAUNCH_CHECK();
        tm.mark(ST_NBR_SCAN);
        scan_i32(deg_n, nbr_start, n, s, sc);
        scan_i32(deg_up, up_start, n, s, sc);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->Nn, nbr_start + n);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->E, up_start + n);
        LAUNCH_CHECK();
        const Counters c0 = read_one(cnt, s);
        if (c0.dup) throw HipError{AC_E_DUPLICATE, "two balls have equal quantised centres"};
        const int E = c0.E, Nn = c0.Nn;
        int *nbr = sc.get<int>(Nn > 0 ? Nn : 1);
        int *up = sc.get<int>(E > 0 ? E : 1);
        int *edge_i = sc.get<int>(E > 0 ? E : 1);
        tm.mark(ST_NBR_FILL);
        k_neighbours<NB_FILL><<<grid_for(n), BLOCK, 0, s>>>(atom, perm, n, g, cell_start, pp, nullptr, nullptr,
                                                           nbr_start, up_start, nbr, up, edge_i, vgab);
        LAUNCH_CHECK();
        const int *nbr_cnt = deg_n;

        // ---- candidate triangles (with AC2 of the edges) ----
        int *tri_cnt = sc.get<int>(E > 0 ? E : 1);
        int *tri_start = sc.get<int>(E + 1);
        unsigned char *egab = sc.get<unsigned char>(E > 0 ? E : 1);
        tm.mark(ST_TRI_COUNT);
        if (E > 0) {
            k_triangles<false><<<grid_for(E), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i, E, pp,
                                                            tri_cnt, egab, nullptr, nullptr, nullptr, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TRI_SCAN);
        scan_i32(tri_cnt, tri_start, E, s, sc);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->T, tri_start + E);
        LAUNCH_CHECK();
        const int T = read_one(cnt, s).T;
        int *tri_k = sc.get<int>(T > 0 ? T : 1);
        int *tri_e = sc.get<int>(T > 0 ? T : 1);
        unsigned char *tgab = sc.get<unsigned char>(T > 0 ? T : 1);
        double *tsize = sc.get<double>(T > 0 ? T : 1);
        int *tet_cnt = sc.get<int>(T > 0 ? T : 1);
        int *tet_start = sc.get<int>(T + 1);
        tm.mark(ST_TRI_FILL);
        if (T > 0) {
            k_triangles<true><<<grid_for(E), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i, E, pp,
                                                           nullptr, nullptr, tri_start, tri_k, tri_e, cnt);
            LAUNCH_CHECK();
        }
        // ---- AC2 of triangles; candidate tetrahedra ----
        tm.mark(ST_TRI_GABRIEL);
        if (T > 0) {
            k_tri_gabriel<<<grid_for(T), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up, edge_i, tri_k, tri_e, T, pp,
                                                       tgab, tsize, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TET_COUNT);
        if (T > 0) {
            k_tet_candidates<false><<<grid_for(T), BLOCK, 0, s>>>(atom, up_start, up, edge_i, tri_k, tri_e, T, pp,
                                                                 tet_cnt, nullptr, nullptr, nullptr, cnt);
            LAUNCH_CHECK();
        }
        scan_i32(tet_cnt, tet_start, T, s, sc);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->Q, tet_start + T);
        LAUNCH_CHECK();
        const int Q = read_one(cnt, s).Q;
        int *tet_t = sc.get<int>(Q > 0 ? Q : 1);
        int *tet_l = sc.get<int>(Q > 0 ? Q : 1);
        unsigned char *qin = sc.get<unsigned char>(Q > 0 ? Q : 1);
        double *qsize = sc.get<double>(Q > 0 ? Q : 1);
        tm.mark(ST_TET_FILL);
        if (Q > 0) {
            k_tet_candidates<true><<<grid_for(T), BLOCK, 0, s>>>(atom, up_start, up, edge_i, tri_k, tri_e, T, pp,
                                                                nullptr, tet_start, tet_t, tet_l, cnt);
            LAUNCH_CHECK();
        }

        // ---- pruning: tetrahedra, then triangles, edges, vertices ----
        int *tri_att = sc.get<int>(T > 0 ? T : 1);
        long long *tri_min = sc.get<long long>(T > 0 ? T : 1);
        int *edge_att = sc.get<int>(E > 0 ? E : 1);
        long long *edge_min = sc.get<long long>(E > 0 ? E : 1);
        int *vert_att = sc.get<int>(n);
        long long *vert_min = sc.get<long long>(n);
        unsigned char *tin = sc.get<unsigned char>(T > 0 ? T : 1);
        unsigned char *ein = sc.get<unsigned char>(E > 0 ? E : 1);
        double *esize = sc.get<double>(E > 0 ? E : 1);
        int *vin_in = sc.get<int>(n);
        double *vsize_in = sc.get<double>(n);
        fill<int>(tri_att, 0, T, s);
        fill<long long>(tri_min, ORDERED_POS_INF, T, s);
        fill<int>(edge_att, 0, E, s);
        fill<long long>(edge_min, ORDERED_POS_INF, E, s);
        fill<int>(vert_att, 0, n, s);
        fill<long long>(vert_min, ORDERED_POS_INF, n, s);
        tm.mark(ST_TETRA);
        if (Q > 0) {
            k_tet_ac2<<<grid_for(Q), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr_cnt, nbr, up_start, up, edge_i, tri_start, tri_k,
                                                   tri_e, tet_t, tet_l, Q, pp, tgab, tri_att, tri_min, qin, qsize, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TRI_FINAL);
        if (T > 0) {
            k_tri_final<<<grid_for(T), BLOCK, 0, s>>>(up_start, up, edge_i, tri_k, tri_e, T, tgab, tsize, tri_att,
                                                     tri_min, tin, egab, edge_att, edge_min, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_EDGE_FINAL);
        if (E > 0) {
            k_edge_final<<<grid_for(E), BLOCK, 0, s>>>(atom, up, edge_i, E, egab, edge_att, edge_min, ein, esize, vgab,
                                                      vert_att, vert_min);
            LAUNCH_CHECK();
        }
        tm.mark(ST_VERT_FINAL);
        k_vert_final<<<grid_for(n), BLOCK, 0, s>>>(atom, perm, n, pp, o.vertex_shortcut, vgab, vert_att, vert_min,
                                                  vin_in, vsize_in);
        LAUNCH_CHECK();

        // ---- emit ----
        tm.mark(ST_EMIT);
        int *vpos = sc.get<int>(n + 1);
        scan_i32(vin_in, vpos, n, s, sc);
        int *epos = sc.get<int>(E + 1), *tpos = sc.get<int>(T + 1), *qpos = sc.get<int>(Q + 1);
        scan_flags(ein, E, epos, s, sc);
        scan_flags(tin, T, tpos, s, sc);
        scan_flags(qin, Q, qpos, s, sc);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->m1, epos + E);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->m2, tpos + T);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->m3, qpos + Q);
        k_copy_int<<<1, 1, 0, s>>>(&cnt->m0, vpos + n);
        LAUNCH_CHECK();
        const Counters cf = read_one(cnt, s);
        const int m0 = cf.m0, m1 = cf.m1, m2 = cf.m2, m3 = cf.m3;
        if (cf.lookup) throw HipError{AC_E_DEVICE, "internal error: a facet of a kept simplex is not a candidate"};
        res->cand[0] = n;
        res->cand[1] = E;
        res->cand[2] = T;
        res->cand[3] = Q;
        res->fallbacks = (int64_t)cf.exact_fallbacks;
        res->count[0] = m0;
        res->d_simp[0] = static_cast<int32_t *>(dev_alloc((size_t)(m0 > 0 ? m0 : 1) * sizeof(int32_t)));
        res->d_size[0] = static_cast<double *>(dev_alloc((size_t)(m0 > 0 ? m0 : 1) * sizeof(double)));
        k_vert_emit<<<grid_for(n), BLOCK, 0, s>>>(vin_in, vpos, vsize_in, n, res->d_simp[0], res->d_size[0]);
        LAUNCH_CHECK();
        const Cands cd{up, edge_i, tri_k, tri_e, tet_t, tet_l, perm};
        emit_dim<2>(ein, epos, esize, E, cd, n, s, sc, res, 1, m1);
        emit_dim<3>(tin, tpos, tsize, T, cd, n, s, sc, res, 2, m2);
        emit_dim<4>(qin, qpos, qsize, Q, cd, n, s, sc, res, 3, m3);
        tm.mark(ST_COUNT);
        HIP_TRY(hipStreamSynchronize(s));
        tm.collect(res->stage_ms);
    } catch (const HipError &e) {
        (void)hipStreamSynchronize(s);
        free_complex(res);
        return set_error(e.st, e.msg);
    }
    *out = res;
    g_last_error.clear();
    return AC_OK;
}

static Options parse(const ac_options *opt) {
    Options o;
    if (opt) {
        o.cell_mA = opt->cell_mA;
        o.force_exact = opt->force_exact != 0;
        o.vertex_shortcut = opt->vertex_shortcut != 0;
        o.profile = opt->profile != 0;
    }
    return o;
}

// ---------------------------------------------------------------------------
// C ABI
extern "C" {

ac_status ac_alpha_complex_device(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                  const ac_options *opt, void *stream, ac_complex **out) {
    if (!out) return set_error(AC_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!d_xyz || !d_radii) return set_error(AC_E_INVALID, "NULL input pointer");
    try {
        return run_pipeline(d_xyz, d_radii, n, alpha, parse(opt), static_cast<hipStream_t>(stream), out);
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
    if (!xyz || !radii) return set_error(AC_E_INVALID, "NULL input pointer");
    if (n < 1 || n >= (1 << 26)) return set_error(AC_E_INVALID, "n must be in [1, 2^26)");
    void *dx = nullptr, *dr = nullptr;
    try {
        dx = dev_alloc((size_t)n * 3 * sizeof(double));
        dr = dev_alloc((size_t)n * sizeof(double));
        HIP_TRY(hipMemcpy(dx, xyz, (size_t)n * 3 * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(dr, radii, (size_t)n * sizeof(double), hipMemcpyHostToDevice));
        ac_status st = run_pipeline(static_cast<double *>(dx), static_cast<double *>(dr), n, alpha, parse(opt), nullptr, out);
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
