// HIP kernels of the alpha-complex pipeline for gfx950.
//
// Stages (Masood, Ray, Natarajan, Sec. 3.1 Steps 1-5 and Sec. 4.2-4.5):
//   quantise  -> integer milli-angstrom balls, bounding box, validation
//   binning   -> counting sort of the balls by uniform-grid cell (Sec. 4.2)
//   neighbours-> per ball: every ball whose grown ball (radius^2 W + alpha)
//                meets its own (the only possible AC2 violators of any
//                candidate it belongs to), and the upper candidate edges,
//                Sigma_ortho^1 (Sec. 4.3)
//   triangles -> Sigma_ortho^2 from pairs of candidate edges (Sec. 4.3)
//   tetrahedra-> Sigma_ortho^3 from candidate triangles, each tested at once
//                with AC2 at its ortho-centre (Step 2); survivors mark their
//                facets attached (Step 3, first half)
//   finalise  -> triangles, edges, vertices: a candidate is in K_alpha iff it
//                passes AC2 at its own ortho-centre or is a face of a kept
//                coface (Steps 3-5, Lemmas 1-2); Size is its OrthoSize when it
//                passes AC2, else the least Size of a kept coface (Sec. 2.3)
//   emit      -> input ids, sorted within a row, rows sorted (bucket by the
//                first id, then each bucket sorted in place)
#pragma once
#include "common.hpp"
#include "predicates.hpp"
#include "radix.hpp"
#include "emit.hpp"

namespace acx {

struct Stats {
    int minx, miny, minz, maxx, maxy, maxz;
    int wmax, flags;  // flags: 1 invalid value, 2 out of range
};

// Uniform grid (Sec. 4.2). Cells are numbered in row-major order (x fastest;
// the cells of one grid row are then contiguous in the sorted order), or
// along a Morton (Z-order) curve, the space-filling alternative Sec. 4.2
// names: the bits of the three cell coordinates interleaved, over a cube of
// 2^L cells a side. A batch of molecules has one grid per molecule; their
// cells are numbered one after the other in a single table, so no ball ever
// sees another molecule's balls.
// ORDER_STOP: the grid of a molecule a recorded build could not take (ball k
// of the molecule alone in its cell k, no neighbour scan); see plan.hpp.
enum { ORDER_ROW = 0, ORDER_MORTON = 1, ORDER_STOP = 2 };
constexpr int MORTON_MAX_BITS = 10;  // cell coordinates below 1024: 30-bit codes

struct Grid {
    int ox, oy, oz;   // low corner (mA)
    int s;            // cell side (mA)
    int nx, ny, nz;
    int reach;        // cells to scan on each side for neighbours
    long long base;   // first cell of this grid in the shared cell table
    int a0, a1;       // the molecule's balls: [a0, a1) in input and in sorted order
    int order;        // ORDER_ROW or ORDER_MORTON
};

// v (< 2^10) with two zero bits after each of its bits
__device__ __forceinline__ unsigned spread3(unsigned v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Molecule of ball i (input or sorted index): the last grid with a0 <= i.
__device__ __forceinline__ int mol_of(const Grid *__restrict__ grids, int n_mol, int i) {
    int lo = 0, hi = n_mol - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (grids[mid].a0 <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

constexpr int BLOCK = 256;

// ---------------------------------------------------------------------------
// Quantise: x -> rint(1000 x) (round half to even), W = R^2. Block b handles
// the balls [tiles[b].x, tiles[b].y) (at most QTILE, all of one molecule) and
// writes their bounding box and flags; k_stats_reduce folds each molecule's
// tiles. Every load of a thread is issued before the first conversion.
constexpr int QTILE = 1024;  // balls per block
__global__ void __launch_bounds__(BLOCK) k_quantise(const double *__restrict__ xyz, const double *__restrict__ r,
                                                     const int2 *__restrict__ tiles, int4 *__restrict__ q,
                                                     Stats *__restrict__ part) {
    constexpr int PT = QTILE / BLOCK;
    int mn[3] = {INT_MAX, INT_MAX, INT_MAX}, mx[3] = {INT_MIN, INT_MIN, INT_MIN}, wmax = 0, flags = 0;
    const int2 tile = tiles[blockIdx.x];
    double vx[PT][3], vr[PT];
#pragma unroll
    for (int u = 0; u < PT; u++) {
        const int i = tile.x + (int)threadIdx.x + u * BLOCK;
        const long long k = i < tile.y ? i : tile.x;  // past the tile: any ball of it, not used
#pragma unroll
        for (int a = 0; a < 3; a++) vx[u][a] = xyz[3 * k + a];
        vr[u] = r[k];
    }
#pragma unroll
    for (int u = 0; u < PT; u++) {
        const int i = tile.x + (int)threadIdx.x + u * BLOCK;
        if (i >= tile.y) break;
        int c[3];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const double v = vx[u][a];
            c[a] = 0;
            if (!isfinite(v)) { flags |= 1; continue; }
            const double s = v * 1000.0;
            if (!(fabs(s) < 524288.0)) { flags |= 2; continue; }
            c[a] = (int)rint(s);
            if (c[a] >= 524288 || c[a] <= -524288) flags |= 2;
            mn[a] = min(mn[a], c[a]);
            mx[a] = max(mx[a], c[a]);
        }
        const double rv = vr[u];
        int W = 0;
        if (!isfinite(rv) || !(rv > 0.0)) {
            flags |= 1;
        } else {
            const double rs = rv * 1000.0;
            if (!(rs < 8192.0)) {
                flags |= 2;
            } else {
                const int R = (int)rint(rs);
                if (R < 1) flags |= 1;
                W = R * R;
            }
        }
        wmax = max(wmax, W);
        q[i] = make_int4(c[0], c[1], c[2], W);
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
#pragma unroll
        for (int a = 0; a < 3; a++) {
            mn[a] = min(mn[a], __shfl_xor(mn[a], off, WAVE));
            mx[a] = max(mx[a], __shfl_xor(mx[a], off, WAVE));
        }
        wmax = max(wmax, __shfl_xor(wmax, off, WAVE));
        flags |= __shfl_xor(flags, off, WAVE);
    }
    __shared__ Stats ws[BLOCK / WAVE];
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) ws[w] = Stats{mn[0], mn[1], mn[2], mx[0], mx[1], mx[2], wmax, flags};
    __syncthreads();
    if (threadIdx.x == 0) {
        Stats b = ws[0];
        for (int k = 1; k < BLOCK / WAVE; k++) {
            const Stats &o = ws[k];
            b.minx = min(b.minx, o.minx); b.miny = min(b.miny, o.miny); b.minz = min(b.minz, o.minz);
            b.maxx = max(b.maxx, o.maxx); b.maxy = max(b.maxy, o.maxy); b.maxz = max(b.maxz, o.maxz);
            b.wmax = max(b.wmax, o.wmax); b.flags |= o.flags;
        }
        part[blockIdx.x] = b;
    }
}

// Block m folds the partials of molecule m's tiles [tile_first[m],
// tile_first[m+1]) into st[m].
__global__ void __launch_bounds__(BLOCK) k_stats_reduce(const Stats *__restrict__ part, const int *__restrict__ tile_first,
                                                         Stats *st) {
    Stats b{INT_MAX, INT_MAX, INT_MAX, INT_MIN, INT_MIN, INT_MIN, 0, 0};
    for (int k = tile_first[blockIdx.x] + threadIdx.x; k < tile_first[blockIdx.x + 1]; k += BLOCK) {
        const Stats &o = part[k];
        b.minx = min(b.minx, o.minx); b.miny = min(b.miny, o.miny); b.minz = min(b.minz, o.minz);
        b.maxx = max(b.maxx, o.maxx); b.maxy = max(b.maxy, o.maxy); b.maxz = max(b.maxz, o.maxz);
        b.wmax = max(b.wmax, o.wmax); b.flags |= o.flags;
    }
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        b.minx = min(b.minx, __shfl_xor(b.minx, off, WAVE));
        b.miny = min(b.miny, __shfl_xor(b.miny, off, WAVE));
        b.minz = min(b.minz, __shfl_xor(b.minz, off, WAVE));
        b.maxx = max(b.maxx, __shfl_xor(b.maxx, off, WAVE));
        b.maxy = max(b.maxy, __shfl_xor(b.maxy, off, WAVE));
        b.maxz = max(b.maxz, __shfl_xor(b.maxz, off, WAVE));
        b.wmax = max(b.wmax, __shfl_xor(b.wmax, off, WAVE));
        b.flags |= __shfl_xor(b.flags, off, WAVE);
    }
    __shared__ Stats ws[BLOCK / WAVE];
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < BLOCK / WAVE; k++) {
            const Stats &o = ws[k];
            b.minx = min(b.minx, o.minx); b.miny = min(b.miny, o.miny); b.minz = min(b.minz, o.minz);
            b.maxx = max(b.maxx, o.maxx); b.maxy = max(b.maxy, o.maxy); b.maxz = max(b.maxz, o.maxz);
            b.wmax = max(b.wmax, o.wmax); b.flags |= o.flags;
        }
        st[blockIdx.x] = b;
    }
}

template <class T>
__global__ void __launch_bounds__(BLOCK) k_fill(T *__restrict__ p, T v, long long n) {
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) p[i] = v;
}

// Start values of the pruning stage's attachment flags (0) and minima (+inf
// in the ordered-integer encoding) for T triangles, E edges and n vertices.
__global__ void __launch_bounds__(BLOCK) k_prune_init(long long T, long long E, long long n, int *__restrict__ tri_att,
                                                       long long *__restrict__ tri_min, int *__restrict__ edge_att,
                                                       long long *__restrict__ edge_min, int *__restrict__ vert_att,
                                                       long long *__restrict__ vert_min) {
    const long long stride = (long long)gridDim.x * BLOCK;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < T; i += stride) {
        tri_att[i] = 0;
        tri_min[i] = ORDERED_POS_INF;
    }
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < E; i += stride) {
        edge_att[i] = 0;
        edge_min[i] = ORDERED_POS_INF;
    }
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += stride) {
        vert_att[i] = 0;
        vert_min[i] = ORDERED_POS_INF;
    }
}

// ---------------------------------------------------------------------------
// Binning (Sec. 4.2): cell key per ball, a stable radix sort by key (inside a
// cell the balls keep input order), then the dense cell table.
__device__ __forceinline__ long long cell_id(const Grid &g, int cx, int cy, int cz) {
    if (g.order == ORDER_MORTON)
        return (long long)(spread3((unsigned)cx) | (spread3((unsigned)cy) << 1) | (spread3((unsigned)cz) << 2));
    return ((long long)cz * g.ny + cy) * g.nx + cx;
}

__device__ __forceinline__ long long cell_of(const Grid &g, int x, int y, int z) {
    return cell_id(g, (x - g.ox) / g.s, (y - g.oy) / g.s, (z - g.oz) / g.s);
}

__global__ void __launch_bounds__(BLOCK) k_cell_key(const int4 *__restrict__ q, int n, const Grid *__restrict__ grids,
                                                     int n_mol, unsigned *__restrict__ key, unsigned *__restrict__ idx) {
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    const int4 a = q[i];
    const Grid &g = grids[mol_of(grids, n_mol, i)];
    key[i] = (unsigned)(g.base + (g.order == ORDER_STOP ? i - g.a0 : cell_of(g, a.x, a.y, a.z)));
    idx[i] = (unsigned)i;
}

// After the stable sort by cell: the first ball of each cell writes the
// cell's population (cells are short runs of equal keys).
__global__ void __launch_bounds__(BLOCK) k_cell_runs(const unsigned *__restrict__ key, int n,
                                                      int *__restrict__ cell_count) {
    const int p = blockIdx.x * BLOCK + threadIdx.x;
    if (p >= n) return;
    const unsigned c = key[p];
    if (p > 0 && key[p - 1] == c) return;
    int e = p + 1;
    while (e < n && key[e] == c) e++;
    cell_count[c] = e - p;
}

// Sorted balls and their input indices (one gather per ball), and the check
// for equal centres: they share a cell, so they are adjacent in the sorted
// order; each ball compares itself with the following balls of its cell (of
// this block from LDS, past its end from their inputs).
__global__ void __launch_bounds__(BLOCK) k_gather_atoms(const int4 *__restrict__ q, const unsigned *__restrict__ idx,
                                                         const unsigned *__restrict__ key, int n,
                                                         int4 *__restrict__ atom, int *__restrict__ perm, Counters *cnt) {
    __shared__ int4 sa[BLOCK];
    __shared__ unsigned sk[BLOCK];
    const int b0 = blockIdx.x * BLOCK;
    const int p = b0 + threadIdx.x;
    int4 a = make_int4(0, 0, 0, 0);
    unsigned c = 0;
    if (p < n) {
        const int me = (int)idx[p];
        a = q[me];
        c = key[p];
        atom[p] = a;
        perm[p] = me;
    }
    sa[threadIdx.x] = a;
    sk[threadIdx.x] = c;
    __syncthreads();
    if (p >= n) return;
    bool dup = false;
    for (int k = p + 1; k < n; k++) {
        const int t = k - b0;
        if ((t < BLOCK ? sk[t] : key[k]) != c) break;
        const int4 o = t < BLOCK ? sa[t] : q[idx[k]];
        dup |= o.x == a.x && o.y == a.y && o.z == a.z;
    }
    if (dup) cnt->dup = 1;
}

// ---------------------------------------------------------------------------
// Neighbour lists and candidate edges (Sec. 4.3, first step). A thread per
// ball scans the cells within `reach`; cells of one grid row are contiguous
// in the sorted order, so each (dz, dy) row is one contiguous range. The fill
// pass also decides AC2 for the ball as a vertex (Step 5): every ball that
// could be strictly closer in power to its centre is in its neighbour list.
// MODE: NB_ONEPASS writes each ball's neighbour row into an LDS slot of
// SLOT entries and marks in a 32-bit mask which of them are upper
// candidate edges (the upper row is a filtered part of the neighbour row);
// the block packs the rows into a slab of its own, and k_nbr_compact writes
// both rows into place once the block totals are scanned. Exact counts are
// kept; a ball with more than SLOT neighbours sets cnt->overflow, after
// which the host runs NB_FILL over the scanned counts instead (same result).
// NB_FILL writes the rows into the CSR rows the counts sized (each thread's
// row contiguous, consecutive rows adjacent).
enum { NB_ONEPASS = 0, NB_FILL = 1 };
// Slot sizes: 16 holds every row of the van der Waals workloads at alpha = 0
// (largest degree 14); 32 serves grown radii up to about 2.6 A.
constexpr int NB_SLOT = 16;
constexpr int NB_SLOT_WIDE = 32;

// FAST: the pair test without clamping and with full-rate arithmetic, for
// grids where it is exact (the launch checks: every scanned offset below
// 26 A per axis, s_g^2 < 2^25 mA^2, alpha >= 0): offsets of balls of cells
// within `reach` are below (reach + 1) s, so d^2 < 2^31 and each square is a
// 24-bit product; the grown balls meet iff L = d^2 - rho_a^2 - rho_b^2 <= 0
// or L^2 <= 4 rho_a^2 rho_b^2, and in float64 4 rho_a^2 rho_b^2 < 2^52 is
// exact while L^2 is exact below 2^53 and, above, rounds to at least 2^53:
// the comparison is decided exactly either way.
// The one-pass kernel with 16-entry slots runs eight waves per SIMD (64
// registers, a few values spilled; its LDS allows eight blocks per CU): the
// eighth wave hides more of the latency of the cell-row loads than the
// spills cost (0.259 ms against 0.268 at the compiler's 66 registers and
// seven waves, on the 3M-atom shell). The other forms are held to fewer
// waves by their LDS.
template <int MODE, int SLOT>
constexpr int nb_waves() { return MODE == NB_ONEPASS && SLOT == NB_SLOT ? 8 : 1; }
template <int MODE, int SLOT, bool FAST = false>
__global__ void __launch_bounds__(BLOCK, (nb_waves<MODE, SLOT>()))
k_neighbours(const int4 *__restrict__ atom, const int *__restrict__ perm, int n,
             const Grid *__restrict__ grids, int n_mol,
             const int *__restrict__ cell_start, PredParams pp,
             int *__restrict__ deg_n, int *__restrict__ deg_up,
             unsigned *__restrict__ upmask, int *__restrict__ nslab,
             int *__restrict__ block_tot,
             const int *__restrict__ nbr_start, const int *__restrict__ up_start,
             int *__restrict__ nbr, int *__restrict__ up,
             int *__restrict__ edge_i, unsigned char *__restrict__ vgab,
             long long *__restrict__ vert_min, Counters *cnt) {
    static_assert(SLOT <= 32, "one mask bit per slot entry");
    constexpr int NB_SLAB = BLOCK * SLOT;
    constexpr bool ONE = MODE == NB_ONEPASS;
    // NB_FILL stages the block's rows in LDS and writes them out as one
    // contiguous range (the block's rows are adjacent in the CSR arrays);
    // rows written straight from the scan would be partial-line scattered
    // stores. A block whose rows exceed the LDS buffers writes directly.
    constexpr int LDS_N = ONE ? NB_SLAB : 4096, LDS_U = ONE ? 1 : 2048;
    __shared__ int sn[LDS_N];
    __shared__ int su[LDS_U];
    const int b = xcd_block();
    const int b0 = b * BLOCK;
    const int i = b0 + threadIdx.x;
    const bool valid = i < n;
    int bn = 0, bu = 0, en = 0, eu = 0;
    bool staged = false;
    if (!ONE) {
        const int last = min(b0 + BLOCK, n);
        bn = nbr_start[b0]; en = nbr_start[last];
        bu = up_start[b0]; eu = up_start[last];
        staged = en - bn <= LDS_N && eu - bu <= LDS_U;
    }
    const int4 a = valid ? atom[i] : make_int4(0, 0, 0, 0);
    const int ra = valid ? a.w + (int)pp.aq : -1;  // |aq| < 2^26 and W < 2^26
    int cn = 0, cu = 0;
    unsigned mask = 0;
    bool gab = true;
    if (ra >= 0) {
        // where this ball's rows go: its LDS slot (entry k at k * BLOCK, so
        // that a wave's lanes hit distinct banks), or its CSR rows
        constexpr int RS = ONE ? BLOCK : 1;
        int *const rn = ONE ? sn + threadIdx.x : (staged ? sn + (nbr_start[i] - bn) : nbr + nbr_start[i]);
        int *const ru = ONE ? nullptr : (staged ? su + (up_start[i] - bu) : up + up_start[i]);
        const int capn = ONE ? SLOT : INT_MAX;
        const Grid g = grids[mol_of(grids, n_mol, i)];
        const int cx = (a.x - g.ox) / g.s, cy = (a.y - g.oy) / g.s, cz = (a.z - g.oz) / g.s;
        const int x0 = max(cx - g.reach, 0), x1 = min(cx + g.reach, g.nx - 1);
        const int y0 = max(cy - g.reach, 0), y1 = min(cy + g.reach, g.ny - 1);
        const int z0 = max(cz - g.reach, 0), z1 = min(cz + g.reach, g.nz - 1);
        const int lim = 4 * (int)pp.sg2;     // (2 s_g)^2 < 2^28
        const int reach1 = 2 * (int)pp.sgc;  // 2 ceil(s_g) <= 2^14
        const double ra4 = 4.0 * (double)ra;
        // the balls whose grown balls meet this one's, in cell order
        auto scan = [&](auto &&on_meet) {
            for (int z = z0; z <= z1; z++) {
                // rows whose cells all lie farther than 2 s_g are skipped
                const int zlo = g.oz + z * g.s, zhi = zlo + g.s - 1;
                const int dzm = a.z < zlo ? zlo - a.z : (a.z > zhi ? a.z - zhi : 0);
                if (dzm > reach1) continue;
                const int rz = lim - dzm * dzm;
                if (rz < 0) continue;
                for (int y = y0; y <= y1; y++) {
                    const int ylo = g.oy + y * g.s, yhi = ylo + g.s - 1;
                    const int dym = a.y < ylo ? ylo - a.y : (a.y > yhi ? a.y - yhi : 0);
                    if (dym > reach1 || rz - dym * dym < 0) continue;
                    // the row's balls: one range (row-major), or one per cell
                    // (Morton; the row is sorted after the scan)
                    const bool morton = g.order == ORDER_MORTON;
                    const long long rb = g.base + ((long long)z * g.ny + y) * g.nx;
                    for (int xc = x0; xc <= (morton ? x1 : x0); xc++) {
                        const long long c0 = morton ? g.base + cell_id(g, xc, y, z) : rb + x0;
                        const int s = cell_start[c0], e = cell_start[morton ? c0 + 1 : rb + x1 + 1];
                        for (int j = s; j < e; j++) {
                            const int4 bb = atom[j];
                            // one combined test (a branch per condition costs more
                            // exec-mask work than the arithmetic it would skip)
                            bool meet;
                            if constexpr (FAST) {
                                const int dx = bb.x - a.x, dy = bb.y - a.y, dz = bb.z - a.z;
                                const int d2 = __mul24(dx, dx) + __mul24(dy, dy) + __mul24(dz, dz);
                                const int rb2 = bb.w + (int)pp.aq;
                                const int L = d2 - ra - rb2;
                                // d2 == 0: the ball itself (equal centres are reported by k_gather_atoms)
                                meet = (d2 <= lim) & (d2 != 0) &
                                       ((L <= 0) | ((double)L * (double)L <= ra4 * (double)rb2));
                            } else {
                                // offsets clamped to reach1 + 1: d2 then fits int32, and
                                // a clamped offset alone gives d2 > (2 ceil s_g)^2 >= lim
                                const int dx = min(max(bb.x - a.x, -reach1 - 1), reach1 + 1);
                                const int dy = min(max(bb.y - a.y, -reach1 - 1), reach1 + 1);
                                const int dz = min(max(bb.z - a.z, -reach1 - 1), reach1 + 1);
                                const int d2 = dx * dx + dy * dy + dz * dz;
                                const int rb2 = bb.w + (int)pp.aq;
                                const int L = d2 - ra - rb2;
                                // grown balls meet: d <= rho_a + rho_b; equal centres are reported by k_gather_atoms
                                meet = (j != i) & (d2 <= lim) & (d2 != 0) & (rb2 >= 0) &
                                       ((L <= 0) | ((i64)L * L <= 4 * (i64)ra * rb2));
                            }
                            if (meet) on_meet(j, bb);
                        }
                    }
                }
            }
        };
        // AC2 of the vertex and AC3 of the edge for neighbour number k
        auto tests = [&](int j, int4 bb, int k) {
            if (gab && vertex_violation_sign(a, i, bb, j, perm) < 0) gab = false;
            if (j > i && edge_ac3(edge_setup(a, bb), pp.aq)) {
                if (ONE) {
                    if (k < 32) mask |= 1u << k;
                } else {
                    ru[cu] = j;
                }
                cu++;
            }
        };
        // the scan only collects the row; the float64 tests then run over the
        // row, where a wave's lanes are mostly busy (inside the scan they would
        // run whenever any lane of the wave met a ball)
        scan([&](int j, int4) {
            if (cn < capn) rn[cn * RS] = j;
            cn++;
        });
        const int kn = min(cn, capn);
        if (g.order == ORDER_MORTON) {
            // rows must ascend in sorted order (upper rows are merged and
            // searched); a Morton scan visits the cells of a row out of order
            for (int a = 1; a < kn; a++) {
                const int v = rn[a * RS];
                int b = a;
                for (; b > 0 && rn[(b - 1) * RS] > v; b--) rn[b * RS] = rn[(b - 1) * RS];
                rn[b * RS] = v;
            }
        }
        for (int k = 0; k < kn; k++) {
            const int j = rn[k * RS];
            tests(j, atom[j], k);
        }
        if (cn > capn) {
            // one-pass mode, row longer than the slot: the exact counts still
            // need the tests of the rest (the fill pass redoes this row)
            int k = 0;
            scan([&](int j, int4 bb) {
                if (k >= capn) tests(j, bb, k);
                k++;
            });
        }
    }
    if (valid) {
        vgab[i] = (unsigned char)(ra >= 0 && gab);
        // start of the least Size of a kept incident edge (only read for a
        // ball that fails AC2 at its own centre)
        if (ONE && !(ra >= 0 && gab)) vert_min[i] = ORDERED_POS_INF;
    }
    if (ONE) {
        if (valid) {
            deg_n[i] = cn;
            deg_up[i] = cu;
            upmask[i] = mask;
        }
        if (cn > SLOT) cnt->overflow = 1;
        const int kn = min(cn, SLOT);
        int totn, totu;
        const int offn = block_exclusive_scan<BLOCK>(kn, &totn);
        (void)block_exclusive_scan<BLOCK>(cu, &totu);
        if (threadIdx.x == 0) {
            block_tot[b] = totn;             // neighbour entries of the block
            block_tot[gridDim.x + b] = totu;  // upper entries of the block
        }
        int *dn = nslab + (long long)b * NB_SLAB + offn;
        for (int k = 0; k < kn; k++) dn[k] = sn[k * BLOCK + threadIdx.x];
        return;
    }
    if (!staged) {
        // rows went straight to nbr / up; the upper rows' owner ids remain
        if (valid) {
            const int pu = up_start[i];
            for (int k = 0; k < cu; k++) edge_i[pu + k] = i;
        }
        return;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < en - bn; k += BLOCK) nbr[bn + k] = sn[k];
    for (int k = threadIdx.x; k < eu - bu; k += BLOCK) up[bu + k] = su[k];
    __syncthreads();
    // owner of each upper-row slot: a ball writes its id over its own slots
    if (valid) {
        const int pu = up_start[i] - bu;
        for (int k = 0; k < cu; k++) su[pu + k] = i;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < eu - bu; k += BLOCK) edge_i[bu + k] = su[k];
}

// After a one-pass neighbour search: the neighbour rows stay where the pass
// packed them, in the block's slab (nbr_start[i] points there; the rows of a
// ball are read with its count deg_n[i], so they need not be adjacent across
// blocks). The upper rows, whose entries are the dense candidate-edge ids,
// are written into place (uoff: exclusive scan of the blocks' upper totals)
// with the owner of every upper entry.
template <int SLOT>
__global__ void __launch_bounds__(BLOCK) k_nbr_compact(const int *__restrict__ deg_n, const int *__restrict__ deg_up,
                                                        const unsigned *__restrict__ upmask, int n,
                                                        const int *__restrict__ nslab, const int *__restrict__ uoff,
                                                        int *__restrict__ nbr_start, int *__restrict__ up_start,
                                                        int *__restrict__ up, int *__restrict__ edge_i,
                                                        const int *__restrict__ stop = nullptr) {
    if (stop && *stop) return;  // a recorded build stopped: the upper rows may not fit
    // the block's upper entries are one contiguous range [gu, gu + totu):
    // they and their owners are gathered in LDS and written with coalesced
    // stores (each thread writing its own few entries would leave partial
    // lines)
    __shared__ int s_up[BLOCK * SLOT];
    __shared__ unsigned char s_own[BLOCK * SLOT];
    const int b = blockIdx.x;
    const int i = b * BLOCK + threadIdx.x;
    const int cn = i < n ? deg_n[i] : 0, cu = i < n ? deg_up[i] : 0;
    int totn, totu;
    const int offn = block_exclusive_scan<BLOCK>(cn, &totn);
    const int offu = block_exclusive_scan<BLOCK>(cu, &totu);
    const int gu = uoff[b];
    const int base = b * (BLOCK * SLOT);  // the block's slab
    if (i < n) {
        nbr_start[i] = base + offn;
        up_start[i] = gu + offu;
        if (i == n - 1) up_start[n] = gu + offu + cu;
        unsigned m = upmask[i];
        int q = offu;
        while (m) {
            const int k = __ffs((int)m) - 1;
            m &= m - 1;
            s_up[q] = nslab[base + offn + k];
            s_own[q] = (unsigned char)threadIdx.x;
            q++;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < totu; k += BLOCK) {
        up[gu + k] = s_up[k];
        edge_i[gu + k] = b * BLOCK + s_own[k];
    }
}

// 64-bit sum of n int32 counts: each block writes its partial to
// out[blockIdx.x]; k_fold_i64 then adds the partials in block order.
__global__ void __launch_bounds__(BLOCK) k_sum_i64(const int *__restrict__ x, long long n, long long *__restrict__ out) {
    __shared__ long long ws[BLOCK / WAVE];
    long long v = 0;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) v += x[i];
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_down(v, off, WAVE);
    if (lane_id() == 0) ws[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int k = 0; k < BLOCK / WAVE; k++) t += ws[k];
        out[blockIdx.x] = t;
    }
}

__global__ void k_fold_i64(const long long *__restrict__ part, int nb, long long *__restrict__ out) {
    long long t = 0;
    for (int k = 0; k < nb; k++) t += part[k];
    *out = t;
}

// Position of b in the (sorted) upper-edge list of a, i.e. the edge id; -1 if absent.
__device__ __forceinline__ int find_edge(const int *__restrict__ up_start, const int *__restrict__ up, int a, int b) {
    int lo = up_start[a], hi = up_start[a + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = up[mid];
        if (v == b) return mid;
        if (v < b) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// Triangle id of (a < b < c); -1 if absent.
__device__ __forceinline__ int find_tri(const int *__restrict__ up_start, const int *__restrict__ up,
                                        const int *__restrict__ tri_start, const int *__restrict__ tri_k, int a, int b,
                                        int c) {
    const int e = find_edge(up_start, up, a, b);
    if (e < 0) return -1;
    int lo = tri_start[e], hi = tri_start[e + 1] - 1;
    while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = tri_k[mid];
        if (v == c) return mid;
        if (v < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Candidate triangles (Sec. 4.3): for an edge (i, j), every k > j adjacent to
// both by a candidate edge, not collinear, with OrthoSize <= alpha. The first
// pass also decides AC2 for the edge at its own ortho-centre (violators of any
// candidate lie in the neighbour list of each of its vertices).
//
// MODE TRI_ONEPASS: one pass writes each edge's row into an LDS slot of
// TRI_SLOT entries, the block packs its rows into its own slab of TRI_SLAB
// entries of a staging array, and k_tri_compact moves every slab to its
// final place once the block totals are scanned. Exact counts are written
// either way; if a row or a block does not fit, cnt->overflow is set and the
// host runs the TRI_FILL pass over scanned counts instead (same result).
enum { TRI_ONEPASS = 0, TRI_FILL = 1 };
constexpr int TRI_SLOT = 8;
constexpr int AC2_GROUP = 4;  // neighbours loaded together in the edge AC2 loop
// Neighbour arrays are allocated AC2_GROUP entries longer, so that a group
// that starts inside a row (or at its end) can be loaded whole (entries past
// the row are replaced, not used).
constexpr int NBR_PAD = AC2_GROUP;
constexpr int TRI_SLAB = 1024;

// AC2 of candidate edge e = (i, j) at its own ortho-centre (Step 4): every
// violator meets the ortho-centre, so it is in i's neighbour row. Writes
// egab[e], and starts edge_min[e] (the least Size of a kept coface) for an
// edge that fails. Every neighbour is tested (no early exit: most edges pass,
// and the loop stays convergent); only filter-undecided ones branch.
// Neighbours go in groups of AC2_GROUP whose loads are all issued before the
// first test, so a wave has several in flight.
__device__ __forceinline__ void edge_ac2(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                         const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                         const int *__restrict__ nbr, const PredParams &pp, int e, int i, int j,
                                         int4 vi, int4 vj, unsigned char *__restrict__ egab,
                                         long long *__restrict__ edge_min) {
    const int ns = nbr_start[i], ne = ns + nbr_cnt[i];
    const Edge ed = edge_setup(vi, vj);
    bool viol = false;
    // the next group's indices are loaded while this group is tested
    int nx[AC2_GROUP];
#pragma unroll
    for (int u = 0; u < AC2_GROUP; u++) nx[u] = nbr[ns + u];  // in bounds: NBR_PAD
    for (int p0 = ns; p0 < ne; p0 += AC2_GROUP) {
        int qs[AC2_GROUP];
        int4 aqs[AC2_GROUP];
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) qs[u] = p0 + u < ne ? nx[u] : j;
        const int pn = p0 + AC2_GROUP < ne ? p0 + AC2_GROUP : p0;  // the last group reloads itself
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) nx[u] = nbr[pn + u];
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) aqs[u] = atom[qs[u]];
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) {
            const int q = qs[u];  // padding entries repeat j, which is never tested
            int sg = pp.force_exact ? 0 : edge_violation_filter(ed, aqs[u]);
            if (sg == 0 && q != j) sg = edge_violation_sign(ed, i, j, aqs[u], q, perm, 1);
            viol |= (sg < 0) & (q != j);
        }
    }
    egab[e] = (unsigned char)!viol;
    if (viol) edge_min[e] = ORDERED_POS_INF;
}

// AC2: whether the one-pass kernel also decides the edges' AC2 (the build
// does; a profiled build run for a per-step breakdown times k_edge_ac2 apart).
template <int MODE, bool AC2 = true>
__global__ void __launch_bounds__(BLOCK) k_triangles(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                      const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                                      const int *__restrict__ nbr,
                                                      const int *__restrict__ up_start, const int *__restrict__ up,
                                                      const int *__restrict__ edge_i, int E, PredParams pp,
                                                      int *__restrict__ tri_cnt, unsigned char *__restrict__ egab,
                                                      long long *__restrict__ edge_min,
                                                      int *__restrict__ slab, int *__restrict__ block_tot,
                                                      const int *__restrict__ tri_start, int *__restrict__ tri_k,
                                                      int *__restrict__ tri_e, Counters *cnt,
                                                      const int *__restrict__ live = nullptr) {
    constexpr bool ONE = MODE == TRI_ONEPASS;
    E = live_count(E, live);
    __shared__ int slot[ONE ? BLOCK * TRI_SLOT : 1];
    __shared__ int cand[BLOCK * TRI_SLOT];
    const int b = xcd_block(E / BLOCK + (E % BLOCK != 0));
    const int e = b * BLOCK + threadIdx.x;
    int c = 0;
    if (e < E) {
        const int i = edge_i[e], j = up[e];
        const int4 vi = atom[i], vj = atom[j];
        if (ONE && AC2) edge_ac2(atom, perm, nbr_start, nbr_cnt, nbr, pp, e, i, j, vi, vj, egab, edge_min);
        int pa = e + 1;
        const int ea = up_start[i + 1];
        int pb = up_start[j];
        const int eb = up_start[j + 1];
        const int out = ONE ? 0 : tri_start[e];
        // merge of the two upper rows without divergent branches (advance the
        // smaller side, both when equal). The common entries are collected in
        // rounds of up to TRI_SLOT and tested after each round, so that the
        // float64 test runs with the wave's lanes mostly busy.
        int *const lst = cand + threadIdx.x;  // entry u at u * BLOCK
        for (;;) {
            int m = 0;
            while (pa < ea && pb < eb && m < TRI_SLOT) {
                const int ka = up[pa], kb = up[pb];
                pa += ka <= kb;
                pb += kb <= ka;
                if (ka == kb) lst[(m++) * BLOCK] = ka;
            }
            for (int u = 0; u < m; u++) {
                const int ka = lst[u * BLOCK];
                if (!tri_candidate(vi, vj, atom[ka], pp, cnt)) continue;
                if (ONE) {
                    if (c < TRI_SLOT) slot[c * BLOCK + threadIdx.x] = ka;
                } else {
                    tri_k[out + c] = ka;
                    tri_e[out + c] = e;
                }
                c++;
            }
            if (m < TRI_SLOT) break;
        }
        if (ONE) tri_cnt[e] = c;
    }
    if (!ONE) return;
    if (c > TRI_SLOT) cnt->overflow = 1;
    const int kept = min(c, TRI_SLOT);
    int total;
    const int off = block_exclusive_scan<BLOCK>(kept, &total);
    if (threadIdx.x == 0) {
        block_tot[b] = total;
        if (total > TRI_SLAB) cnt->overflow = 1;
    }
    if (total > TRI_SLAB) return;
    int *dst = slab + (long long)b * TRI_SLAB + off;
    for (int u = 0; u < kept; u++) dst[u] = slot[u * BLOCK + threadIdx.x];
}

// Moves the slabs of TRI_CB consecutive blocks of the triangle pass to their
// final place (block_off = exclusive scan of the block totals: the slabs'
// outputs are consecutive) and writes the row starts; a thread takes
// TRI_CB consecutive edges (one 16-byte load of counts and one store of
// starts), so that the block scan and its barriers serve 4 * BLOCK edges.
constexpr int TRI_CB = 4;
__global__ void __launch_bounds__(BLOCK) k_tri_compact(const int *__restrict__ tri_cnt, int E,
                                                        const int *__restrict__ slab, const int *__restrict__ block_off,
                                                        int *__restrict__ tri_start, int *__restrict__ tri_k,
                                                        int *__restrict__ tri_e, const int *__restrict__ live = nullptr) {
    static_assert(TRI_CB == 4, "one int4 of counts per thread");
    E = live_count(E, live);
    const int nb = E / BLOCK + (E % BLOCK != 0);  // blocks of the triangle pass
    const int b0 = blockIdx.x * TRI_CB;            // its first block here
    const long long e0 = (long long)blockIdx.x * (TRI_CB * BLOCK) + (long long)threadIdx.x * TRI_CB;
    int c[TRI_CB];
    if (e0 + TRI_CB <= E) {
        const int4 v = *reinterpret_cast<const int4 *>(tri_cnt + e0);
        c[0] = v.x; c[1] = v.y; c[2] = v.z; c[3] = v.w;
    } else {
#pragma unroll
        for (int u = 0; u < TRI_CB; u++) c[u] = e0 + u < E ? tri_cnt[e0 + u] : 0;
    }
    const int mine = c[0] + c[1] + c[2] + c[3];
    int total;
    const int off = block_exclusive_scan<BLOCK>(mine, &total);
    const int g0 = b0 < nb ? block_off[b0] : 0;
    // owner edge (index in this block's TRI_CB * BLOCK edges) of each entry
    __shared__ unsigned short s_own[TRI_CB * TRI_SLAB];
    __shared__ int sub[TRI_CB + 1];  // entries before each of the blocks' slabs
    if (threadIdx.x <= TRI_CB) sub[threadIdx.x] = block_off[min(b0 + (int)threadIdx.x, nb)] - g0;
    int st[TRI_CB], o = off;
#pragma unroll
    for (int u = 0; u < TRI_CB; u++) {
        st[u] = g0 + o;
        for (int w = 0; w < c[u] && o + w < TRI_CB * TRI_SLAB; w++)
            s_own[o + w] = (unsigned short)(threadIdx.x * TRI_CB + u);
        o += c[u];
    }
    if (e0 + TRI_CB <= E) {
        *reinterpret_cast<int4 *>(tri_start + e0) = make_int4(st[0], st[1], st[2], st[3]);
    } else {
#pragma unroll
        for (int u = 0; u < TRI_CB; u++)
            if (e0 + u < E) tri_start[e0 + u] = st[u];
    }
    if (e0 <= E - 1 && E - 1 < e0 + TRI_CB) tri_start[E] = g0 + off + mine;
    __syncthreads();
    const long long ebase = (long long)blockIdx.x * (TRI_CB * BLOCK);
    for (int k = threadIdx.x; k < total; k += BLOCK) {
        int j = 0;
#pragma unroll
        for (int q = 1; q < TRI_CB; q++) j += k >= sub[q];
        tri_k[g0 + k] = slab[(long long)(b0 + j) * TRI_SLAB + (k - sub[j])];
        tri_e[g0 + k] = (int)(ebase + s_own[k]);
    }
}

// OrthoSize evaluated with the vertices in lexicographic order of their
// integer centres (a total order: equal centres are rejected). The rounded
// float64 value then depends only on the balls, not on the grid, the sorted
// order or the other molecules of a batch, so reported Sizes are
// bit-identical whatever the cell size; no input-index gather is needed.
__device__ __forceinline__ bool centre_less(const int4 &a, const int4 &b) {
    return a.x != b.x ? a.x < b.x : (a.y != b.y ? a.y < b.y : a.z < b.z);
}

__device__ __forceinline__ double edge_size_canon(int4 a, int4 b) {
    return centre_less(a, b) ? edge_orthosize(edge_setup(a, b)) : edge_orthosize(edge_setup(b, a));
}

template <int K>
__device__ __forceinline__ void sort_centres(int4 (&v)[K]) {
#pragma unroll
    for (int a = 1; a < K; a++)
#pragma unroll
        for (int b = a; b > 0; b--)
            if (centre_less(v[b], v[b - 1])) {
                const int4 u = v[b]; v[b] = v[b - 1]; v[b - 1] = u;
            }
}

__device__ __forceinline__ double tri_size_canon(int4 a, int4 b, int4 c, const PredParams &pp) {
    int4 v[3] = {a, b, c};
    sort_centres<3>(v);
    return tri_orthosize(tri_setup(v[0], v[1], v[2], pp));
}

__device__ __forceinline__ double tet_size_canon(int4 a, int4 b, int4 c, int4 d, const PredParams &pp) {
    int4 v[4] = {a, b, c, d};
    sort_centres<4>(v);
    return tet_orthosize(tet_setup(v[0], v[1], v[2], v[3], pp));
}

// ---------------------------------------------------------------------------
// Candidate tetrahedra (Step 1, d = 3): for a triangle (i, j, k), every l > k
// adjacent to all three by candidate edges (all six edges in Sigma_ortho^1
// suffice, since OrthoSize grows from face to coface, Sec. 4.3), not flat,
// with OrthoSize <= alpha, as (triangle, l) pairs.
//
// MODE TET_ONEPASS (one thread per triangle) also decides AC2 for the
// triangle at its own ortho-centre and its OrthoSize, and writes the pairs
// through LDS slots and per-block slabs like k_triangles; TET_FILL is the
// second pass of the two-pass path, over scanned exact counts.
enum { TET_ONEPASS = 0, TET_FILL = 1 };
constexpr int TET_SLOT = 4;
constexpr int TET_SLAB = 256;
constexpr int TRI_AC2_GROUP = 2;  // neighbours loaded together in the triangle AC2 loop (<= AC2_GROUP)

// AC2 of candidate triangle t = (i, j, k) at its own ortho-centre (Step 3;
// violators are in i's neighbour row) and its OrthoSize. Writes tgab[t],
// tsize[t], and starts tri_min[t] for a triangle that fails. Every neighbour
// is tested (no early exit, convergent loop); only filter-undecided ones take
// the exact branch.
__device__ __forceinline__ void tri_ac2(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                        const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                        const int *__restrict__ nbr, const PredParams &pp, int t, int i, int j, int k,
                                        int4 vi, int4 vj, int4 vk, unsigned char *__restrict__ tgab,
                                        double *__restrict__ tsize, long long *__restrict__ tri_min, Counters *cnt) {
    const Tri tr = tri_setup(vi, vj, vk, pp);
    bool viol = false;
    const int ns = nbr_start[i], ne = ns + nbr_cnt[i];
    // neighbours in pairs, both loads issued before the first test (the
    // index pair is one load: the arrays are padded), the next pair's
    // indices loaded while this pair is tested
    int nx[TRI_AC2_GROUP];
#pragma unroll
    for (int u = 0; u < TRI_AC2_GROUP; u++) nx[u] = nbr[ns + u];  // in bounds: NBR_PAD
    for (int p0 = ns; p0 < ne; p0 += TRI_AC2_GROUP) {
        int qs[TRI_AC2_GROUP];
        int4 aqs[TRI_AC2_GROUP];
#pragma unroll
        for (int u = 0; u < TRI_AC2_GROUP; u++) qs[u] = p0 + u < ne ? nx[u] : j;  // padding repeats j, never tested
        const int pn = p0 + TRI_AC2_GROUP < ne ? p0 + TRI_AC2_GROUP : p0;  // the last pair reloads itself
#pragma unroll
        for (int u = 0; u < TRI_AC2_GROUP; u++) nx[u] = nbr[pn + u];
#pragma unroll
        for (int u = 0; u < TRI_AC2_GROUP; u++) aqs[u] = atom[qs[u]];
#pragma unroll
        for (int u = 0; u < TRI_AC2_GROUP; u++) {
            const int q = qs[u];
            const bool other = (q != j) & (q != k);
            int sg = pp.force_exact ? 0 : tri_violation_filter(tr, aqs[u]);
            if (sg == 0 && other) {
                if (!pp.force_exact) note_fallback(cnt);
                sg = tri_violation_exact(tr, i, j, k, aqs[u], q, perm);
            }
            viol |= (sg < 0) & other;
        }
    }
    tgab[t] = (unsigned char)!viol;
    if (viol) tri_min[t] = ORDERED_POS_INF;
    tsize[t] = tri_size_canon(vi, vj, vk, pp);
}

// AC2: whether the one-pass kernel also decides the triangles' AC2 and
// OrthoSize (the build does; a profiled build for a per-step breakdown times
// k_tri_ac2 apart).
template <int MODE, bool AC2 = true>
__global__ void __launch_bounds__(BLOCK, 4) k_tet_candidates(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                           const int *__restrict__ nbr_start,
                                                           const int *__restrict__ nbr_cnt, const int *__restrict__ nbr,
                                                           const int *__restrict__ up_start, const int *__restrict__ up,
                                                           const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                           const int *__restrict__ tri_e, int T, PredParams pp,
                                                           unsigned char *__restrict__ tgab, double *__restrict__ tsize,
                                                           long long *__restrict__ tri_min,
                                                           int *__restrict__ tet_cnt, int *__restrict__ slab,
                                                           int *__restrict__ block_tot,
                                                           const int *__restrict__ tet_start, int *__restrict__ tet_t,
                                                           int *__restrict__ tet_l, Counters *cnt,
                                                           const int *__restrict__ live = nullptr) {
    constexpr bool ONE = MODE == TET_ONEPASS;
    T = live_count(T, live);
    __shared__ int slot[ONE ? BLOCK * TET_SLOT : 1];
    __shared__ int cand[BLOCK * TET_SLOT];
    const int b = xcd_block(T / BLOCK + (T % BLOCK != 0));
    const int t = b * BLOCK + threadIdx.x;
    int c = 0;
    if (t < T) {
        const int e = tri_e[t];
        const int i = edge_i[e], j = up[e], k = tri_k[t];
        const int4 vi = atom[i], vj = atom[j], vk = atom[k];
        if (ONE && AC2) tri_ac2(atom, perm, nbr_start, nbr_cnt, nbr, pp, t, i, j, k, vi, vj, vk, tgab, tsize, tri_min, cnt);
        int pa = e + 1;
        const int ea = up_start[i + 1];
        int pb = up_start[j];
        const int eb = up_start[j + 1];
        int pc = up_start[k];
        const int ec = up_start[k + 1];
        const int out = ONE ? 0 : tet_start[t];
        // three-way merge step without divergent branches; the common entries
        // are collected in rounds of up to TET_SLOT and tested after each
        // round (the float64 test then runs with the wave's lanes mostly busy)
        int *const lst = cand + threadIdx.x;  // entry u at u * BLOCK
        for (;;) {
            int mc = 0;
            while (pa < ea && pb < eb && pc < ec && mc < TET_SLOT) {
                const int la = up[pa], lb = up[pb], lc = up[pc];
                const int m = max(la, max(lb, lc));
                const bool all = (la == m) & (lb == m) & (lc == m);
                pa += (la < m) | all;
                pb += (lb < m) | all;
                pc += (lc < m) | all;
                if (all) lst[(mc++) * BLOCK] = m;
            }
            for (int u = 0; u < mc; u++) {
                const int l = lst[u * BLOCK];
                const Tet te = tet_setup(vi, vj, vk, atom[l], pp);
                if (te.D == 0 || !tet_ac3(te, pp, cnt)) continue;
                if (ONE) {
                    if (c < TET_SLOT) slot[c * BLOCK + threadIdx.x] = l;
                } else {
                    tet_t[out + c] = t;
                    tet_l[out + c] = l;
                }
                c++;
            }
            if (mc < TET_SLOT) break;
        }
        if (ONE) tet_cnt[t] = c;
    }
    if (!ONE) return;
    if (c > TET_SLOT) cnt->overflow = 1;
    const int kept = min(c, TET_SLOT);
    int total;
    const int off = block_exclusive_scan<BLOCK>(kept, &total);
    if (threadIdx.x == 0) {
        block_tot[b] = total;
        if (total > TET_SLAB) cnt->overflow = 1;
    }
    if (total > TET_SLAB) return;
    int *dst = slab + (long long)b * TET_SLAB + off;
    for (int u = 0; u < kept; u++) dst[u] = slot[u * BLOCK + threadIdx.x];
}

// Moves block b's slab of tetrahedron candidates to its final place.
__global__ void __launch_bounds__(BLOCK) k_tet_compact(const int *__restrict__ tet_cnt, int T,
                                                        const int *__restrict__ slab, const int *__restrict__ block_off,
                                                        int *__restrict__ tet_t, int *__restrict__ tet_l,
                                                        const int *__restrict__ live = nullptr) {
    T = live_count(T, live);
    const int b = blockIdx.x;
    const int t = b * BLOCK + threadIdx.x;
    const int c = t < T ? tet_cnt[t] : 0;
    int total;
    const int off = block_exclusive_scan<BLOCK>(c, &total);
    const int g0 = block_off[b];
    __shared__ unsigned char s_own[TET_SLAB];  // owner triangle of each entry of the block (coalesced stores)
    if (t < T)
        for (int u = 0; u < c && off + u < TET_SLAB; u++) s_own[off + u] = (unsigned char)threadIdx.x;
    __syncthreads();
    const int *src = slab + (long long)b * TET_SLAB;
    for (int k = threadIdx.x; k < total; k += BLOCK) {
        tet_l[g0 + k] = src[k];
        tet_t[g0 + k] = b * BLOCK + s_own[k];
    }
}

// The AC2 tests of candidate edges and triangles as kernels of their own
// (same results as inside the one-pass kernels), for a profiled per-step
// breakdown.
__global__ void __launch_bounds__(BLOCK) k_edge_ac2(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                     const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                                     const int *__restrict__ nbr, const int *__restrict__ up,
                                                     const int *__restrict__ edge_i, int E, PredParams pp,
                                                     unsigned char *__restrict__ egab, long long *__restrict__ edge_min) {
    const int e = xcd_block() * BLOCK + threadIdx.x;
    if (e >= E) return;
    const int i = edge_i[e], j = up[e];
    edge_ac2(atom, perm, nbr_start, nbr_cnt, nbr, pp, e, i, j, atom[i], atom[j], egab, edge_min);
}

__global__ void __launch_bounds__(BLOCK) k_tri_ac2(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                    const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                                    const int *__restrict__ nbr, const int *__restrict__ up,
                                                    const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                    const int *__restrict__ tri_e, int T, PredParams pp,
                                                    unsigned char *__restrict__ tgab, double *__restrict__ tsize,
                                                    long long *__restrict__ tri_min, Counters *cnt) {
    const int t = xcd_block() * BLOCK + threadIdx.x;
    if (t >= T) return;
    const int e = tri_e[t];
    const int i = edge_i[e], j = up[e], k = tri_k[t];
    tri_ac2(atom, perm, nbr_start, nbr_cnt, nbr, pp, t, i, j, k, atom[i], atom[j], atom[k], tgab, tsize, tri_min, cnt);
}

// A face that passes AC2 itself is in K with Size = OrthoSize whatever its
// cofaces do, so only faces failing AC2 record the kept coface: the least
// Size of their kept cofaces (order-preserving integer; +inf while none), so
// such a face is kept iff that minimum is finite.
__device__ __forceinline__ void mark_face(const unsigned char *gab, long long *mins, int f, long long key,
                                          Counters *cnt) {
    if (f < 0) { atomicOr(&cnt->lookup, 1); return; }
    if (gab[f]) return;
    atomicMin(&mins[f], key);
}

// Tetrahedra (Step 2): kept iff no ball is strictly closer in power to the
// ortho-centre; a kept tetrahedron records itself on its facets (Step 3) and
// gets its emit key and payload (input ids; not kept: the drop key).
// SWEEP (candidates of several alpha values): qin holds AC2 alone, and the
// facet ids go to tface for the per-alpha passes instead of being marked.
template <bool SWEEP>
__global__ void __launch_bounds__(BLOCK) k_tet_ac2(const int4 *__restrict__ atom, const int *__restrict__ perm,
                                                    const int *__restrict__ nbr_start, const int *__restrict__ nbr_cnt,
                                                      const int *__restrict__ nbr,
                                                    const int *__restrict__ up_start, const int *__restrict__ up,
                                                    const int *__restrict__ edge_i, const int *__restrict__ tri_start,
                                                    const int *__restrict__ tri_k, const int *__restrict__ tri_e,
                                                    const int *__restrict__ tet_t, const int *__restrict__ tet_l, int Q,
                                                    PredParams pp, const unsigned char *__restrict__ tgab,
                                                    long long *__restrict__ tri_min,
                                                    unsigned char *__restrict__ qin, double *__restrict__ qsize,
                                                    int4 *__restrict__ tface, unsigned drop, unsigned *__restrict__ qkey,
                                                    typename EmitPay<4>::type *__restrict__ qpay, Counters *cnt,
                                                    const int *__restrict__ live = nullptr) {
    const int Ql = live_count(Q, live);
    const int c = xcd_block(Ql / BLOCK + (Ql % BLOCK != 0)) * BLOCK + threadIdx.x;
    if (c >= Ql) return;
    const int t = tet_t[c], l = tet_l[c];
    const int e = tri_e[t];
    const int i = edge_i[e], j = up[e], k = tri_k[t];
    const Tet te = tet_setup(atom[i], atom[j], atom[k], atom[l], pp);
    bool keep = true;
    const int ns = nbr_start[i], ne = ns + nbr_cnt[i];
    // neighbours in groups whose loads are all issued before the first test
    // (few tetrahedra: a thread's chain of dependent loads is the kernel's
    // time); the index group is one load (the arrays are padded)
    for (int p0 = ns; p0 < ne && keep; p0 += AC2_GROUP) {
        int qs[AC2_GROUP];
        int4 aqs[AC2_GROUP];
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) {
            const int r = nbr[p0 + u];  // in bounds: NBR_PAD
            qs[u] = p0 + u < ne ? r : j;  // padding repeats j, which is never tested
        }
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) aqs[u] = atom[qs[u]];
#pragma unroll
        for (int u = 0; u < AC2_GROUP; u++) {
            const int q = qs[u];
            if (!keep || q == j || q == k || q == l) continue;
            if (tet_violation_sign(te, i, j, k, l, aqs[u], q, perm, pp, cnt) < 0) keep = false;
        }
    }
    if (SWEEP) qin[c] = (unsigned char)keep;
    if (!keep) {
        if (!SWEEP) {
            int v[4] = {0, 0, 0, 0};
            emit_pack<4>(false, v, 0.0, c, drop, qkey[c], qpay[c]);
        }
        return;
    }
    const double sz = tet_size_canon(atom[i], atom[j], atom[k], atom[l], pp);
    qsize[c] = sz;
    const int f1 = find_tri(up_start, up, tri_start, tri_k, i, j, l);
    const int f2 = find_tri(up_start, up, tri_start, tri_k, i, k, l);
    const int f3 = find_tri(up_start, up, tri_start, tri_k, j, k, l);
    if (SWEEP) {
        tface[c] = make_int4(t, f1, f2, f3);
        return;
    }
    int v[4] = {perm[i], perm[j], perm[k], perm[l]};
    emit_pack<4>(true, v, sz, c, drop, qkey[c], qpay[c]);
    const long long key = ordered_from_double(sz);
    mark_face(tgab, tri_min, t, key, cnt);
    mark_face(tgab, tri_min, f1, key, cnt);
    mark_face(tgab, tri_min, f2, key, cnt);
    mark_face(tgab, tri_min, f3, key, cnt);
}

// Triangles (Step 3): kept iff AC2 holds at the ortho-centre or a kept
// tetrahedron has it as a facet; Size is then the OrthoSize or the least Size
// of a kept tetrahedron. Kept triangles record themselves on their edges;
// every triangle gets its emit key and payload (not kept: the drop key).
__global__ void __launch_bounds__(BLOCK) k_tri_final(const int *__restrict__ up_start, const int *__restrict__ up,
                                                      const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                      const int *__restrict__ tri_e, int T,
                                                      const unsigned char *__restrict__ tgab,
                                                      const double *__restrict__ tsize,
                                                      const long long *__restrict__ tri_min,
                                                      const unsigned char *__restrict__ egab,
                                                      long long *__restrict__ edge_min, const int *__restrict__ perm,
                                                      unsigned drop, unsigned *__restrict__ tkey,
                                                      typename EmitPay<3>::type *__restrict__ tpay, Counters *cnt,
                                                      const int *__restrict__ live = nullptr) {
    const int Tl = live_count(T, live);
    const int t = xcd_block(Tl / BLOCK + (Tl % BLOCK != 0)) * BLOCK + threadIdx.x;
    if (t >= Tl) return;
    const bool gab = tgab[t];
    const long long mn = gab ? ORDERED_POS_INF : tri_min[t];
    const bool in = gab || mn != ORDERED_POS_INF;
    int v[4] = {0, 0, 0, 0};
    if (!in) {
        emit_pack<3>(false, v, 0.0, t, drop, tkey[t], tpay[t]);
        return;
    }
    const double sz = gab ? tsize[t] : double_from_ordered(mn);
    const int e = tri_e[t];
    const int i = edge_i[e], j = up[e], k = tri_k[t];
    v[0] = perm[i]; v[1] = perm[j]; v[2] = perm[k];
    emit_pack<3>(true, v, sz, t, drop, tkey[t], tpay[t]);
    const long long key = ordered_from_double(sz);
    mark_face(egab, edge_min, e, key, cnt);
    mark_face(egab, edge_min, find_edge(up_start, up, i, k), key, cnt);
    mark_face(egab, edge_min, find_edge(up_start, up, j, k), key, cnt);
}

// Edge ids (i, k) and (j, k) of every candidate triangle (i, j, k), once per
// sweep.
__global__ void __launch_bounds__(BLOCK) k_tri_edges(const int *__restrict__ up_start, const int *__restrict__ up,
                                                      const int *__restrict__ edge_i, const int *__restrict__ tri_k,
                                                      const int *__restrict__ tri_e, int T, int2 *__restrict__ tedge) {
    const int t = xcd_block() * BLOCK + threadIdx.x;
    if (t >= T) return;
    const int e = tri_e[t];
    const int i = edge_i[e], j = up[e], k = tri_k[t];
    tedge[t] = make_int2(find_edge(up_start, up, i, k), find_edge(up_start, up, j, k));
}

// Edges (Step 4), with their emit keys and payloads (not kept: the drop key).
__global__ void __launch_bounds__(BLOCK) k_edge_final(const int4 *__restrict__ atom, const int *__restrict__ up,
                                                       const int *__restrict__ edge_i, int E,
                                                       const unsigned char *__restrict__ egab,
                                                       const long long *__restrict__ edge_min,
                                                       const unsigned char *__restrict__ vgab,
                                                       long long *__restrict__ vert_min, const int *__restrict__ perm,
                                                       unsigned drop, unsigned *__restrict__ ekey,
                                                       typename EmitPay<2>::type *__restrict__ epay,
                                                       const int *__restrict__ live = nullptr) {
    const int El = live_count(E, live);
    const int e = xcd_block(El / BLOCK + (El % BLOCK != 0)) * BLOCK + threadIdx.x;
    if (e >= El) return;
    const bool gab = egab[e];
    const long long mn = gab ? ORDERED_POS_INF : edge_min[e];
    const bool in = gab || mn != ORDERED_POS_INF;
    int v[4] = {0, 0, 0, 0};
    if (!in) {
        emit_pack<2>(false, v, 0.0, e, drop, ekey[e], epay[e]);
        return;
    }
    const int i = edge_i[e], j = up[e];
    const double sz = gab ? edge_size_canon(atom[i], atom[j]) : double_from_ordered(mn);
    v[0] = perm[i]; v[1] = perm[j];
    emit_pack<2>(true, v, sz, e, drop, ekey[e], epay[e]);
    const long long key = ordered_from_double(sz);
    if (!vgab[i]) atomicMin(&vert_min[i], key);
    if (!vgab[j]) atomicMin(&vert_min[j], key);
}

// Vertices (Step 5): a ball with -W <= alpha is kept iff no ball is strictly
// closer in power to its own centre (decided in k_neighbours), or it ends a
// kept edge. With `shortcut`, every such ball is kept with Size -W (the
// paper's implementation shortcut). One float64 per ball goes to its input
// position: the Size in mA^2, NaN when not kept.
__global__ void __launch_bounds__(BLOCK) k_vert_final(const int4 *__restrict__ atom, const int *__restrict__ perm, int n,
                                                       PredParams pp, int shortcut,
                                                       const unsigned char *__restrict__ vgab,
                                                       const long long *__restrict__ vert_min,
                                                       double *__restrict__ vsize_in) {
    const int v = xcd_block() * BLOCK + threadIdx.x;
    if (v >= n) return;
    const int w = atom[v].w;
    double sz = __longlong_as_double(0x7ff8000000000000LL);  // NaN: not kept
    if ((i64)w + pp.aq >= 0) {
        const bool gab = shortcut || vgab[v];
        if (gab) {
            sz = -(double)w;
        } else {
            const long long mn = vert_min[v];
            if (mn != ORDERED_POS_INF) sz = double_from_ordered(mn);
        }
    }
    vsize_in[perm[v]] = sz;
}

// ---------------------------------------------------------------------------
// Output order of a sweep.
// Row of candidate c (sorted-order indices) for d = 1, 2, 3.
template <int K>
__device__ __forceinline__ void candidate_row(int c, const int *__restrict__ up, const int *__restrict__ edge_i,
                                              const int *__restrict__ tri_k, const int *__restrict__ tri_e,
                                              const int *__restrict__ tet_t, const int *__restrict__ tet_l,
                                              int (&v)[4]) {
    v[3] = 0;
    if (K == 2) {
        v[0] = edge_i[c]; v[1] = up[c]; v[2] = 0;
    } else if (K == 3) {
        const int e = tri_e[c];
        v[0] = edge_i[e]; v[1] = up[e]; v[2] = tri_k[c];
    } else {
        const int t = tet_t[c];
        const int e = tri_e[t];
        v[0] = edge_i[e]; v[1] = up[e]; v[2] = tri_k[t]; v[3] = tet_l[c];
    }
}

// Payload of the output-order sort of a sweep (every candidate, no Size):
// the ids after the least, then the candidate index.
template <int K> struct OrderPay;
template <> struct OrderPay<2> { typedef uint2 type; };
template <> struct OrderPay<3> { typedef uint3 type; };
template <> struct OrderPay<4> { typedef uint4 type; };

// Output-order keys of a sweep: every candidate c, kept at some alpha or
// not, keyed by the least input id of its row, payload (other ids, c).
template <int K>
__global__ void __launch_bounds__(BLOCK) k_order_keys(int M, const int *__restrict__ up, const int *__restrict__ edge_i,
                                                       const int *__restrict__ tri_k, const int *__restrict__ tri_e,
                                                       const int *__restrict__ tet_t, const int *__restrict__ tet_l,
                                                       const int *__restrict__ perm, unsigned *__restrict__ key,
                                                       typename OrderPay<K>::type *__restrict__ pay) {
    const int c = xcd_block() * BLOCK + threadIdx.x;
    if (c >= M) return;
    int v[4];
    candidate_row<K>(c, up, edge_i, tri_k, tri_e, tet_t, tet_l, v);
#pragma unroll
    for (int u = 0; u < K; u++) v[u] = perm[v[u]];
#pragma unroll
    for (int a = 1; a < K; a++)
#pragma unroll
        for (int b = a; b > 0; b--)
            if (v[b - 1] > v[b]) { const int t = v[b]; v[b] = v[b - 1]; v[b - 1] = t; }
    key[c] = (unsigned)v[0];
    if constexpr (K == 2) pay[c] = make_uint2((unsigned)v[1], (unsigned)c);
    else if constexpr (K == 3) pay[c] = make_uint3((unsigned)v[1], (unsigned)v[2], (unsigned)c);
    else pay[c] = make_uint4((unsigned)v[1], (unsigned)v[2], (unsigned)v[3], (unsigned)c);
}

// After the sort of a sweep's candidates by least id, each row finds its
// bucket (equal keys are adjacent; buckets are short) and its rank in the
// bucket by the remaining ids, and writes the sorted row to rows_s and each
// candidate's place to spos. A block stages its 256 rows and RANK_HALO rows
// on each side in LDS, so the bucket walks are LDS reads; a bucket reaching
// past the halo is finished from global memory.
constexpr int RANK_HALO = 64;

template <int K>
__global__ void __launch_bounds__(BLOCK) k_order_rank(const unsigned *__restrict__ key,
                                                       const typename OrderPay<K>::type *__restrict__ pay, int m,
                                                       int *__restrict__ rows_s, int *__restrict__ spos) {
    typedef typename OrderPay<K>::type P;
    constexpr int SPAN = BLOCK + 2 * RANK_HALO;
    __shared__ unsigned sk[SPAN];
    __shared__ P sp[SPAN];
    const int b0 = blockIdx.x * BLOCK;
    const int lo = b0 - RANK_HALO;
    for (int t = threadIdx.x; t < SPAN; t += BLOCK) {
        const int g = lo + t;
        if (g >= 0 && g < m) {
            sk[t] = key[g];
            sp[t] = pay[g];
        } else {
            sk[t] = 0xffffffffu;
        }
    }
    __syncthreads();
    const int p = b0 + threadIdx.x;
    if (p >= m) return;
    const int lp = p - lo;
    const unsigned u0 = sk[lp];
    auto ids = [](const P &q, unsigned (&r)[3]) {
        if constexpr (K == 2) { r[0] = q.x; r[1] = 0; r[2] = 0; }
        else if constexpr (K == 3) { r[0] = q.x; r[1] = q.y; r[2] = 0; }
        else { r[0] = q.x; r[1] = q.y; r[2] = q.z; }
    };
    const P me = sp[lp];
    unsigned r[3];
    ids(me, r);
    auto before = [&](const P &x) -> int {
        unsigned o[3];
        ids(x, o);
        return o[0] != r[0] ? o[0] < r[0] : (o[1] != r[1] ? o[1] < r[1] : o[2] < r[2]);
    };
    // the bucket inside the staged span, else walked in global memory
    int ls = lp;
    while (ls > 0 && sk[ls - 1] == u0) ls--;
    int le = lp + 1;
    while (le < SPAN && sk[le] == u0) le++;
    int s, rank = 0;
    if ((ls > 0 || lo + ls == 0) && (le < SPAN || lo + le == m)) {
        s = lo + ls;
        for (int w = ls; w < le; w++) rank += (w != lp) && before(sp[w]);
    } else {
        s = p;
        while (s > 0 && key[s - 1] == u0) s--;
        int e = p + 1;
        while (e < m && key[e] == u0) e++;
        for (int w = s; w < e; w++) rank += (w != p) && before(pay[w]);
    }
    const int pos = s + rank;
    const long long q = (long long)pos * K;
    rows_s[q] = (int)u0;
#pragma unroll
    for (int u = 1; u < K; u++) rows_s[q + u] = (int)r[u - 1];
    unsigned c;
    if constexpr (K == 2) c = me.y;
    else if constexpr (K == 3) c = me.z;
    else c = me.w;
    spos[c] = pos;
}

// Rows of a simplex array sorted by least id (K ids per row): out[j] = first
// row whose least id is >= bound[j]; the rows of molecule m of a batch are
// [out[m], out[m+1]) when bound holds the molecules' first balls.
template <int K>
__global__ void __launch_bounds__(BLOCK) k_row_lower_bound(const int *__restrict__ simp, const int *__restrict__ m,
                                                            const long long *__restrict__ bound, int nb,
                                                            long long *__restrict__ out) {
    const int j = blockIdx.x * BLOCK + threadIdx.x;
    if (j >= nb) return;
    const long long b = bound[j];
    long long lo = 0, hi = *m;
    while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((long long)simp[mid * K] < b) lo = mid + 1; else hi = mid;
    }
    out[j] = lo;
}

}  // namespace acx
