// Kernels of a recorded build: the pipeline with every size fixed in advance
// (grid cells per molecule, candidate capacities), so that a whole build is a
// fixed sequence of launches with no value read back by the host, and can be
// captured once in a HIP graph and replayed on new coordinates. Each launch
// that depends on a count takes it from device memory (the live counts of
// Counters); when the input does not fit what was recorded, the build stops
// (every later count 0, reason in Counters::stop) and the host builds again
// the ordinary way.
#pragma once
#include "kernels.hpp"

namespace acx {

enum {
    STOP_INPUT = 1,     // invalid or out-of-range value, or a radius above the recorded largest
    STOP_CELLS = 2,     // a molecule's grid needs more cells than recorded
    STOP_DUP = 4,       // equal quantised centres
    STOP_SLOT = 8,      // a row outgrew its single-pass slot (the ordinary build takes two passes there)
    STOP_CAPACITY = 16  // a candidate total above its recorded capacity
};

// Grid of molecule m (one thread each) from the bounding box of this run, with
// the recorded cell side, reach, order and first cell (tmpl), and at most
// cap[m] cells. A molecule that does not fit, or a value the recorded build
// cannot take, stops the build; a stopped molecule's grid puts every ball in
// a cell of its own and scans no neighbours, so the remaining launches stay in
// bounds and do no work.
__global__ void __launch_bounds__(BLOCK) k_plan_grids(const Stats *__restrict__ st, int n_mol,
                                                       const Grid *__restrict__ tmpl, const long long *__restrict__ cap,
                                                       int wmax_rec, Grid *__restrict__ grids, Counters *cnt) {
    const int m = blockIdx.x * BLOCK + threadIdx.x;
    if (m >= n_mol) return;
    const Stats h = st[m];
    Grid g = tmpl[m];
    int why = (h.flags || h.wmax > wmax_rec) ? STOP_INPUT : 0;
    if (!why) {
        const long long s = g.s;
        const long long nx = ((long long)h.maxx - h.minx + s) / s, ny = ((long long)h.maxy - h.miny + s) / s,
                        nz = ((long long)h.maxz - h.minz + s) / s;
        long long cells = nx * ny * nz;
        if (g.order == ORDER_MORTON) {
            int L = 0;
            while ((1LL << L) < max(nx, max(ny, nz))) L++;
            cells = L > MORTON_MAX_BITS ? LLONG_MAX : 1LL << (3 * L);
        }
        if (cells > cap[m]) {
            why = STOP_CELLS;
        } else {
            g.ox = h.minx; g.oy = h.miny; g.oz = h.minz;
            g.nx = (int)nx; g.ny = (int)ny; g.nz = (int)nz;
        }
    }
    if (why) {
        g.ox = g.oy = g.oz = 0;
        g.nx = g.ny = g.nz = 1;
        g.reach = -1;  // empty neighbour scan
        g.order = ORDER_STOP;
        atomicOr(&cnt->stop, why);
    }
    grids[m] = g;
}

// After a stage's totals (stage 0: neighbours -> candidate edges; 1:
// triangles; 2: tetrahedra): the stage's live count, or 0 for every later
// stage once the build has stopped.
__global__ void k_plan_guard(Counters *cnt, int stage, int cap) {
    if (threadIdx.x != 0) return;
    const int tot = stage == 0 ? cnt->E : (stage == 1 ? cnt->T : cnt->Q);
    int why = cnt->stop;
    if (cnt->overflow) why |= STOP_SLOT;
    if (cnt->dup) why |= STOP_DUP;
    if (tot > cap) why |= STOP_CAPACITY;
    cnt->stop = why;
    if (why) {
        cnt->El = 0;
        cnt->Tl = 0;
        cnt->Ql = 0;
    } else if (stage == 0) {
        cnt->El = tot;
    } else if (stage == 1) {
        cnt->Tl = tot;
    } else {
        cnt->Ql = tot;
    }
}

__global__ void k_copy_int(const int *__restrict__ src, int *__restrict__ dst) {
    if (threadIdx.x == 0) *dst = *src;
}

}  // namespace acx
