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

// out[0..n] = exclusive scan of in[0..n), out[n] = total.
static void scan_i32(const int *in, int *out, long long n, hipStream_t s, Scope &sc) {
    if (n <= 0) {
        fill<int>(out, 0, 1, s);
        return;
    }
    const long long tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    int *sums = sc.get<int>(tiles);
    k_scan_tiles<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(in, out, sums, n);
    LAUNCH_CHECK();
    if (tiles > 1) {
        int *offs = sc.get<int>(tiles + 1);
        scan_i32(sums, offs, tiles, s, sc);
        k_scan_add<<<(unsigned)tiles, SCAN_BLOCK, 0, s>>>(out, offs, n);
        LAUNCH_CHECK();
    }
    k_scan_total<<<1, 1, 0, s>>>(out, in, n);
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

// Emit one dimension: remap to input ids, sort, write result-owned arrays.
template <int K>
static void emit_dim(const int *rows, const double *sizes, int m, const int *perm, int n, hipStream_t s, Scope &sc,
                     ac_complex *res, int d) {
    res->count[d] = m;
    res->d_simp[d] = static_cast<int32_t *>(dev_alloc((size_t)(m > 0 ? m : 1) * K * sizeof(int32_t)));
    res->d_size[d] = static_cast<double *>(dev_alloc((size_t)(m > 0 ? m : 1) * sizeof(double)));
    if (m == 0) return;
    int4 *tmp = sc.get<int4>(m);
    int4 *rows2 = sc.get<int4>(m);
    double *size2 = sc.get<double>(m);
    int *bcnt = sc.get<int>(n);
    int *bstart = sc.get<int>(n + 1);
    fill<int>(bcnt, 0, n, s);
    k_emit_remap<K><<<grid_for(m), BLOCK, 0, s>>>(rows, perm, m, tmp, bcnt);
    LAUNCH_CHECK();
    scan_i32(bcnt, bstart, n, s, sc);
    HIP_TRY(hipMemcpyAsync(bcnt, bstart, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
    k_emit_scatter<<<grid_for(m), BLOCK, 0, s>>>(tmp, sizes, m, bcnt, rows2, size2);
    LAUNCH_CHECK();
    k_emit_sort<K><<<grid_for(n), BLOCK, 0, s>>>(rows2, size2, bstart, n, res->d_simp[d], res->d_size[d]);
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
    ST_TETRA, ST_TRI_FINAL, ST_EDGE_FINAL, ST_VERT_FINAL, ST_EMIT, ST_COUNT
};
static const char *kStageNames[ST_COUNT] = {
    "quantise", "binning", "neighbours_count", "neighbours_scan", "neighbours_fill", "triangles_count",
    "triangles_scan", "triangles_fill", "tetrahedra_ac2", "triangles_final", "edges_final", "vertices_final", "emit"};

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
        k_stats_init<<<1, 1, 0, s>>>(st);
        LAUNCH_CHECK();
        {
            long long b = grid_for(n);
            if (b > 4096) b = 4096;
            k_quantise<<<(unsigned)b, BLOCK, 0, s>>>(d_xyz, d_r, n, q, st);
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
        long long *key = sc.get<long long>(n);
        int *cell_count = sc.get<int>(ncell + 1);
        int *cell_start = sc.get<int>(ncell + 1);
        fill<int>(cell_count, 0, ncell + 1, s);
        k_cell_hist<<<grid_for(n), BLOCK, 0, s>>>(q, n, g, key, cell_count);
        LAUNCH_CHECK();
        scan_i32(cell_count, cell_start, ncell, s, sc);
        HIP_TRY(hipMemcpyAsync(cell_count, cell_start, sizeof(int) * ncell, hipMemcpyDeviceToDevice, s));
        int4 *tmp_atom = sc.get<int4>(n);
        int *tmp_perm = sc.get<int>(n);
        k_scatter<<<grid_for(n), BLOCK, 0, s>>>(q, key, n, cell_count, tmp_atom, tmp_perm);
        LAUNCH_CHECK();
        int4 *atom = sc.get<int4>(n);
        int *perm = sc.get<int>(n);
        k_cell_order<<<grid_for(n), BLOCK, 0, s>>>(tmp_atom, tmp_perm, n, g, cell_start, atom, perm, cnt);
        LAUNCH_CHECK();

        // ---- neighbours and candidate edges ----
        int *deg_n = sc.get<int>(n), *deg_up = sc.get<int>(n);
        int *nbr_start = sc.get<int>(n + 1), *up_start = sc.get<int>(n + 1);
        tm.mark(ST_NBR_COUNT);
        k_neighbours<false><<<grid_for(n), BLOCK, 0, s>>>(atom, n, g, cell_start, pp, deg_n, deg_up, nullptr, nullptr,
                                                         nullptr, nullptr, nullptr, cnt);
        LAUNCH_CHECK();
        tm.mark(ST_NBR_SCAN);
        scan_i32(deg_n, nbr_start, n, s, sc);
        scan_i32(deg_up, up_start, n, s, sc);
        const Counters c0 = read_one(cnt, s);
        if (c0.dup) throw HipError{AC_E_DUPLICATE, "two balls have equal quantised centres"};
        const int Nn = read_one(nbr_start + n, s);
        const int E = read_one(up_start + n, s);
        int *nbr = sc.get<int>(Nn > 0 ? Nn : 1);
        int *up = sc.get<int>(E > 0 ? E : 1);
        int *edge_i = sc.get<int>(E > 0 ? E : 1);
        tm.mark(ST_NBR_FILL);
        k_neighbours<true><<<grid_for(n), BLOCK, 0, s>>>(atom, n, g, cell_start, pp, nullptr, nullptr, nbr_start,
                                                        up_start, nbr, up, edge_i, cnt);
        LAUNCH_CHECK();

        // ---- candidate triangles ----
        int *tri_cnt = sc.get<int>(E > 0 ? E : 1);
        int *tri_start = sc.get<int>(E + 1);
        tm.mark(ST_TRI_COUNT);
        if (E > 0) {
            k_triangles<false><<<grid_for(E), BLOCK, 0, s>>>(atom, up_start, up, edge_i, E, pp, tri_cnt, nullptr,
                                                            nullptr, nullptr, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TRI_SCAN);
        scan_i32(tri_cnt, tri_start, E, s, sc);
        const int T = read_one(tri_start + E, s);
        int *tri_k = sc.get<int>(T > 0 ? T : 1);
        int *tri_e = sc.get<int>(T > 0 ? T : 1);
        tm.mark(ST_TRI_FILL);
        if (T > 0) {
            k_triangles<true><<<grid_for(E), BLOCK, 0, s>>>(atom, up_start, up, edge_i, E, pp, nullptr, tri_start, tri_k,
                                                           tri_e, cnt);
            LAUNCH_CHECK();
        }

        // ---- pruning: tetrahedra, triangles, edges, vertices ----
        int *tri_att = sc.get<int>(T > 0 ? T : 1);
        long long *tri_min = sc.get<long long>(T > 0 ? T : 1);
        int *edge_att = sc.get<int>(E > 0 ? E : 1);
        long long *edge_min = sc.get<long long>(E > 0 ? E : 1);
        int *vert_att = sc.get<int>(n);
        long long *vert_min = sc.get<long long>(n);
        fill<int>(tri_att, 0, T, s);
        fill<long long>(tri_min, ORDERED_POS_INF, T, s);
        fill<int>(edge_att, 0, E, s);
        fill<long long>(edge_min, ORDERED_POS_INF, E, s);
        fill<int>(vert_att, 0, n, s);
        fill<long long>(vert_min, ORDERED_POS_INF, n, s);
        // a triangle has at most two tetrahedra in K, each tetrahedron four facets
        const int cap3 = T / 2 + 1;
        int4 *k3 = sc.get<int4>(cap3);
        double *k3_size = sc.get<double>(cap3);
        int4 *k2 = sc.get<int4>(T > 0 ? T : 1);
        double *k2_size = sc.get<double>(T > 0 ? T : 1);
        int2 *k1 = sc.get<int2>(E > 0 ? E : 1);
        double *k1_size = sc.get<double>(E > 0 ? E : 1);
        int *k0 = sc.get<int>(n);
        double *k0_size = sc.get<double>(n);
        tm.mark(ST_TETRA);
        if (T > 0) {
            k_tetrahedra<<<grid_for(T), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr, up_start, up, edge_i, tri_start,
                                                      tri_k, tri_e, T, pp, tri_att, tri_min, k3, k3_size, cap3, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_TRI_FINAL);
        if (T > 0) {
            k_tri_final<<<grid_for(T), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr, up_start, up, edge_i, tri_k, tri_e, T,
                                                     pp, tri_att, tri_min, edge_att, edge_min, k2, k2_size, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_EDGE_FINAL);
        if (E > 0) {
            k_edge_final<<<grid_for(E), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr, up, edge_i, E, edge_att, edge_min,
                                                      vert_att, vert_min, k1, k1_size, cnt);
            LAUNCH_CHECK();
        }
        tm.mark(ST_VERT_FINAL);
        k_vert_final<<<grid_for(n), BLOCK, 0, s>>>(atom, perm, nbr_start, nbr, n, pp, o.vertex_shortcut, vert_att,
                                                  vert_min, k0, k0_size, cnt);
        LAUNCH_CHECK();
        tm.mark(ST_EMIT);
        const Counters cf = read_one(cnt, s);
        if (cf.lookup) throw HipError{AC_E_DEVICE, "internal error: a facet of a kept simplex is not a candidate"};
        if (cf.k3 > cap3) throw HipError{AC_E_CAPACITY, "tetrahedron list overflow"};
        res->cand[0] = n;  // refined below to active balls
        res->cand[1] = E;
        res->cand[2] = T;
        res->cand[3] = cf.k3;  // candidates that reached AC2 are not counted separately
        res->fallbacks = (int64_t)cf.exact_fallbacks;

        // ---- emit ----
        emit_dim<1>(k0, k0_size, cf.k0, perm, n, s, sc, res, 0);
        emit_dim<2>(reinterpret_cast<const int *>(k1), k1_size, cf.k1, perm, n, s, sc, res, 1);
        emit_dim<3>(reinterpret_cast<const int *>(k2), k2_size, cf.k2, perm, n, s, sc, res, 2);
        emit_dim<4>(reinterpret_cast<const int *>(k3), k3_size, cf.k3, perm, n, s, sc, res, 3);
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
