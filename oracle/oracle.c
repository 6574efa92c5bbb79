/*
 * CPU oracle: alpha complex of weighted points through the weighted Delaunay
 * (regular) triangulation. Test infrastructure only; see oracle.h.
 *
 * Plan, following the paper's definitions (Masood, Ray, Natarajan,
 * "Parallel Computation of Alpha Complexes for Biomolecules"):
 *   1. Quantise to integer milli-angstrom; power distance pi(p,b) =
 *      |p - p_b|^2 - r_b^2 (Sec. 2.2).
 *   2. Build D, the regular triangulation (Sec. 2.2 definition DT1/DT2), by
 *      incremental Bowyer-Watson insertion (cited in Sec. 1.1) with an
 *      infinite vertex. A ball whose power cell is empty is "hidden" and is
 *      not a vertex of D (Sec. 2.2 remark on empty Voronoi regions).
 *   3. Every simplex of D gets its Size (Sec. 2.3): the smallest power
 *      distance over its witnesses. The ortho-centre minimises the power
 *      distance over the points satisfying DT1 (OrthoSize); if it is itself a
 *      witness the Size equals the OrthoSize, otherwise the minimum lies on
 *      the boundary of the simplex's dual power face, whose facets are the
 *      duals of its cofaces, so the Size is the least Size of a coface.
 *   4. K_alpha = { sigma in D : Size(sigma) <= alpha } (Sec. 2.4).
 *
 * Arithmetic is exact: every predicate is an integer polynomial evaluated in
 * __int128; Sizes are exact rationals (converted to floating point only for
 * output). Ties are broken by simulation of simplicity on the weights: weight
 * W_i becomes W_i + eps_i with eps_0 >> eps_1 >> ... (input index order), and
 * since every predicate is affine in the weights, a zero value takes the sign
 * of the first non-zero partial derivative in that order.
 *
 * Bit budget: coordinates |x| < 2^19 mA, so differences < 2^20; radii and
 * alpha with W_max + alpha_q < 2^26. Simplices whose Size could be <= alpha
 * have every edge passing the edge OrthoSize test, hence edge length
 * <= 2 sqrt(W_max + alpha_q) < 2^14 (a face's OrthoSize never exceeds its
 * coface's, Sec. 4.3); only for those are ortho-centres formed.
 */
#define _GNU_SOURCE /* qsort_r: comparators take their context as an argument (thread safety) */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;
typedef int64_t i64;

typedef struct { i64 x, y, z, w; } opt;

#define INF_V (-1)

static int sgn(i128 v) { return (v > 0) - (v < 0); }

/* ---------------------------------------------------------------------- */
/* Simulation of simplicity: ids[] are the balls a predicate depends on,     */
/* coef[] its partial derivatives by their weights.                          */
static int sos_sign(int k, const int *ids, const i128 *coef) {
    int used[8] = {0};
    for (int step = 0; step < k; step++) {
        int best = -1;
        for (int t = 0; t < k; t++)
            if (!used[t] && (best < 0 || ids[t] < ids[best])) best = t;
        used[best] = 1;
        if (coef[best] != 0) return sgn(coef[best]);
    }
    return 0;
}

static i128 det3(i64 a0, i64 a1, i64 a2, i64 b0, i64 b1, i64 b2, i64 c0, i64 c1, i64 c2) {
    return (i128)a0 * ((i128)b1 * c2 - (i128)b2 * c1) - (i128)a1 * ((i128)b0 * c2 - (i128)b2 * c0) +
           (i128)a2 * ((i128)b0 * c1 - (i128)b1 * c0);
}

/* Sign of det[b-a; c-a; d-a]; positive for a right-handed tetrahedron. */
static int orient(const opt *P, int a, int b, int c, int d) {
    const opt *A = P + a, *B = P + b, *C = P + c, *D = P + d;
    return sgn(det3(B->x - A->x, B->y - A->y, B->z - A->z, C->x - A->x, C->y - A->y, C->z - A->z, D->x - A->x,
                    D->y - A->y, D->z - A->z));
}

/*
 * Lifted power test for a positively oriented tetrahedron v[0..3] and a ball q:
 * PT = det [ p_i - q , |p_i - q|^2 - W_i + W_q ]_{i=0..3}. PT equals
 * orient(v) times (pi(c,q) - pi(c,v_0)) with c the ortho-centre, so a negative
 * value means q is strictly closer in power to c than the tetrahedron's balls.
 * Never returns 0 (the W_q partial, -orient, is non-zero).
 */
static int power_sign(const opt *P, const int *v, int q) {
    i64 u[4][3];
    i128 l[4];
    for (int i = 0; i < 4; i++) {
        u[i][0] = P[v[i]].x - P[q].x;
        u[i][1] = P[v[i]].y - P[q].y;
        u[i][2] = P[v[i]].z - P[q].z;
        l[i] = (i128)(u[i][0] * u[i][0] + u[i][1] * u[i][1] + u[i][2] * u[i][2]) - P[v[i]].w + P[q].w;
    }
    i128 C[4];
    for (int i = 0; i < 4; i++) {
        int r[3], m = 0;
        for (int j = 0; j < 4; j++)
            if (j != i) r[m++] = j;
        i128 M = det3(u[r[0]][0], u[r[0]][1], u[r[0]][2], u[r[1]][0], u[r[1]][1], u[r[1]][2], u[r[2]][0], u[r[2]][1],
                      u[r[2]][2]);
        C[i] = ((i + 3) & 1) ? -M : M; /* cofactor of entry (i, 3) */
    }
    i128 pt = 0;
    for (int i = 0; i < 4; i++) pt += l[i] * C[i];
    if (pt != 0) return sgn(pt);
    int ids[5] = {v[0], v[1], v[2], v[3], q};
    i128 coef[5] = {-C[0], -C[1], -C[2], -C[3], C[0] + C[1] + C[2] + C[3]};
    return sos_sign(5, ids, coef);
}

/* ---------------------------------------------------------------------- */
/* Triangulation with an infinite vertex. Cell c has vertices v[0..3] and     */
/* nb[i] is the cell across the face opposite v[i]. Finite cells are          */
/* positively oriented; in an infinite cell, putting a point beyond its hull  */
/* facet in place of the infinite vertex gives a positive orientation.       */

typedef struct { int v[4]; int nb[4]; } ocell;

static int64_t edge_lookup(const int64_t *vstart, const int64_t *adj_v, const int64_t *adj_e, int64_t u, int64_t w);

typedef struct {
    const opt *P;
    int n;
    ocell *cell;
    int ncell, cap;
    int *freel;
    int nfree, freecap;
    uint32_t *mark;
    uint32_t stamp;
    int last;
    uint64_t rng;
    /* per-insertion scratch */
    int *queue, qcap;
    int *bc, *bf, bcap, bfcap; /* boundary (cavity cell, face) */
    int *nc, nccap;            /* new cells */
    int *hk0, *hk1, *hc, *hf, hcap;
    int oom;
} otri;

static uint64_t orng_next(uint64_t *s) { /* xorshift64* */
    uint64_t x = *s;
    x ^= x >> 12;
    x ^= x << 25;
    x ^= x >> 27;
    *s = x;
    return x * 0x2545F4914F6CDD1Dull;
}

static int cell_alloc(otri *T) {
    if (T->nfree > 0) return T->freel[--T->nfree];
    if (T->ncell == T->cap) {
        int nc = T->cap ? T->cap * 2 : 1024;
        ocell *c = (ocell *)realloc(T->cell, (size_t)nc * sizeof(ocell));
        uint32_t *m = (uint32_t *)realloc(T->mark, (size_t)nc * sizeof(uint32_t));
        if (!c || !m) {
            if (c) T->cell = c;
            if (m) T->mark = m;
            T->oom = 1;
            return -1;
        }
        memset(m + T->cap, 0, (size_t)(nc - T->cap) * sizeof(uint32_t));
        T->cell = c;
        T->mark = m;
        T->cap = nc;
    }
    return T->ncell++;
}

static void cell_free(otri *T, int c) {
    if (T->nfree == T->freecap) {
        int nc = T->freecap ? T->freecap * 2 : 1024;
        int *f = (int *)realloc(T->freel, (size_t)nc * sizeof(int));
        if (!f) { T->oom = 1; return; }
        T->freel = f;
        T->freecap = nc;
    }
    T->cell[c].v[0] = -2; /* dead */
    T->freel[T->nfree++] = c;
}

static int inf_pos(const ocell *c) {
    for (int i = 0; i < 4; i++)
        if (c->v[i] == INF_V) return i;
    return -1;
}

/* Does ball q conflict with cell c, i.e. is c destroyed when q is inserted? */
static int in_conflict(const otri *T, int c, int q) {
    const ocell *C = &T->cell[c];
    int k = inf_pos(C);
    if (k < 0) return power_sign(T->P, C->v, q) < 0;
    int p[4];
    memcpy(p, C->v, sizeof p);
    p[k] = q;
    int o = orient(T->P, p[0], p[1], p[2], p[3]);
    if (o != 0) return o > 0;
    /* q on the hull plane: restricted to that plane both cells sharing the
     * facet test the facet's own ortho-circle, so ask the finite one. */
    return power_sign(T->P, T->cell[C->nb[k]].v, q) < 0;
}

static int grow(int **a, int *cap, int need) {
    if (need <= *cap) return 1;
    int nc = *cap ? *cap : 64;
    while (nc < need) nc *= 2;
    int *t = (int *)realloc(*a, (size_t)nc * sizeof(int));
    if (!t) return 0;
    *a = t;
    *cap = nc;
    return 1;
}

/* 1 inserted, 0 hidden, -1 out of memory. */
static int insert_point(otri *T, int q) {
    const opt *P = T->P;
    /* Locate q by a randomised visibility walk. */
    int c = T->last;
    if (inf_pos(&T->cell[c]) >= 0) c = T->cell[c].nb[inf_pos(&T->cell[c])];
    int seed = -1;
    for (;;) {
        const ocell *C = &T->cell[c];
        if (inf_pos(C) >= 0) { seed = c; break; } /* stepped out through a hull facet */
        int start = (int)(orng_next(&T->rng) & 3), moved = 0;
        for (int t = 0; t < 4; t++) {
            int i = (start + t) & 3;
            int p[4];
            memcpy(p, C->v, sizeof p);
            p[i] = q;
            if (orient(P, p[0], p[1], p[2], p[3]) < 0) {
                c = C->nb[i];
                moved = 1;
                break;
            }
        }
        if (!moved) {
            if (!in_conflict(T, c, q)) return 0; /* power cell of q is empty */
            seed = c;
            break;
        }
    }
    /* Cavity: all cells in conflict with q, found by breadth-first search. */
    T->stamp += 2;
    const uint32_t IN = T->stamp, OUT = T->stamp + 1;
    int nq = 0, head = 0, nb = 0;
    if (!grow(&T->queue, &T->qcap, 1)) return -1;
    T->queue[nq++] = seed;
    T->mark[seed] = IN;
    while (head < nq) {
        int cc = T->queue[head++];
        for (int i = 0; i < 4; i++) {
            int d = T->cell[cc].nb[i];
            if (T->mark[d] == IN) continue;
            if (T->mark[d] != OUT && in_conflict(T, d, q)) {
                T->mark[d] = IN;
                if (!grow(&T->queue, &T->qcap, nq + 1)) return -1;
                T->queue[nq++] = d;
            } else {
                T->mark[d] = OUT;
                if (!grow(&T->bc, &T->bcap, nb + 1) || !grow(&T->bf, &T->bfcap, nb + 1)) return -1;
                T->bc[nb] = cc;
                T->bf[nb] = i;
                nb++;
            }
        }
    }
    /* Star the cavity boundary from q. */
    if (!grow(&T->nc, &T->nccap, nb)) return -1;
    for (int b = 0; b < nb; b++) {
        int n = cell_alloc(T);
        if (n < 0) return -1;
        int cc = T->bc[b], i = T->bf[b];
        ocell *N = &T->cell[n];
        memcpy(N->v, T->cell[cc].v, sizeof N->v);
        N->v[i] = q;
        int d = T->cell[cc].nb[i];
        N->nb[i] = d;
        N->nb[(i + 1) & 3] = N->nb[(i + 2) & 3] = N->nb[(i + 3) & 3] = -1;
        for (int j = 0; j < 4; j++)
            if (T->cell[d].nb[j] == cc) { T->cell[d].nb[j] = n; break; }
        T->mark[n] = 0;
        T->nc[b] = n;
    }
    /* Glue new cells to each other across faces containing q: the two cells
     * sharing such a face share the boundary edge opposite it. */
    int hsz = 16;
    while (hsz < 4 * nb) hsz *= 2;
    if (hsz > T->hcap) {
        int *a = (int *)realloc(T->hk0, (size_t)hsz * sizeof(int)), *b2 = NULL, *c2 = NULL, *d2 = NULL;
        if (a) T->hk0 = a;
        b2 = (int *)realloc(T->hk1, (size_t)hsz * sizeof(int));
        if (b2) T->hk1 = b2;
        c2 = (int *)realloc(T->hc, (size_t)hsz * sizeof(int));
        if (c2) T->hc = c2;
        d2 = (int *)realloc(T->hf, (size_t)hsz * sizeof(int));
        if (d2) T->hf = d2;
        if (!a || !b2 || !c2 || !d2) return -1;
        T->hcap = hsz;
    }
    for (int h = 0; h < hsz; h++) T->hc[h] = -1;
    for (int b = 0; b < nb; b++) {
        int n = T->nc[b], i = T->bf[b];
        for (int j = 0; j < 4; j++) {
            if (j == i) continue;
            int e[2], m = 0;
            for (int k = 0; k < 4; k++)
                if (k != i && k != j) e[m++] = T->cell[n].v[k];
            int k0 = e[0] < e[1] ? e[0] : e[1], k1 = e[0] < e[1] ? e[1] : e[0];
            uint64_t hv = ((uint64_t)(uint32_t)(k0 + 1) * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)(uint32_t)(k1 + 1) * 0xC2B2AE3D27D4EB4Full);
            int h = (int)((hv >> 17) & (uint64_t)(hsz - 1));
            for (;;) {
                if (T->hc[h] == -1) { /* empty: first face with this edge */
                    T->hk0[h] = k0; T->hk1[h] = k1; T->hc[h] = n; T->hf[h] = j;
                    break;
                }
                if (T->hc[h] >= 0 && T->hk0[h] == k0 && T->hk1[h] == k1) {
                    int o = T->hc[h], of = T->hf[h];
                    T->cell[n].nb[j] = o;
                    T->cell[o].nb[of] = n;
                    T->hc[h] = -2; /* matched; the slot stays occupied for probing */
                    break;
                }
                h = (h + 1) & (hsz - 1);
            }
        }
    }
    for (int t = 0; t < nq; t++) cell_free(T, T->queue[t]);
    if (T->oom) return -1;
    T->last = T->nc[0];
    for (int b = 0; b < nb; b++)
        if (inf_pos(&T->cell[T->nc[b]]) < 0) { T->last = T->nc[b]; break; }
    return 1;
}

/* Build the first tetrahedron from the first four affinely independent
 * points in insertion order; the rest of order[] is inserted afterwards. */
static int init_simplex(otri *T, const int *order, int n, int *used) {
    const opt *P = T->P;
    int a = order[0], b = order[1], c = -1, d = -1, ia = 0, ib = 1, ic = -1, id = -1;
    for (int t = 2; t < n && c < 0; t++) {
        int x = order[t];
        i64 ux = P[b].x - P[a].x, uy = P[b].y - P[a].y, uz = P[b].z - P[a].z;
        i64 vx = P[x].x - P[a].x, vy = P[x].y - P[a].y, vz = P[x].z - P[a].z;
        i128 cx = (i128)uy * vz - (i128)uz * vy, cy = (i128)uz * vx - (i128)ux * vz, cz = (i128)ux * vy - (i128)uy * vx;
        if (cx != 0 || cy != 0 || cz != 0) { c = x; ic = t; }
    }
    if (c < 0) return 0;
    for (int t = 2; t < n && d < 0; t++) {
        if (t == ic) continue;
        if (orient(P, a, b, c, order[t]) != 0) { d = order[t]; id = t; }
    }
    if (d < 0) return 0;
    used[ia] = used[ib] = used[ic] = used[id] = 1;
    if (orient(P, a, b, c, d) < 0) { int s = a; a = b; b = s; }
    int f = cell_alloc(T);
    if (f < 0) return -1;
    int vv[4] = {a, b, c, d};
    memcpy(T->cell[f].v, vv, sizeof vv);
    int ic4[4];
    for (int i = 0; i < 4; i++) {
        int g = cell_alloc(T);
        if (g < 0) return -1;
        int w[4];
        memcpy(w, vv, sizeof w);
        w[i] = INF_V;
        /* swap two finite entries so the infinite cell is positively oriented */
        int s0 = (i + 1) & 3, s1 = (i + 2) & 3;
        int tmp = w[s0]; w[s0] = w[s1]; w[s1] = tmp;
        memcpy(T->cell[g].v, w, sizeof w);
        ic4[i] = g;
    }
    /* adjacency by shared faces, brute force over the five cells */
    int all[5] = {f, ic4[0], ic4[1], ic4[2], ic4[3]};
    for (int x = 0; x < 5; x++)
        for (int i = 0; i < 4; i++) {
            int cx = all[x];
            T->cell[cx].nb[i] = -1;
            for (int y = 0; y < 5; y++) {
                if (y == x) continue;
                int cy = all[y], shared = 0;
                for (int k = 0; k < 4; k++) {
                    if (k == i) continue;
                    for (int m = 0; m < 4; m++)
                        if (T->cell[cy].v[m] == T->cell[cx].v[k]) { shared++; break; }
                }
                if (shared == 3) { T->cell[cx].nb[i] = cy; break; }
            }
        }
    for (int i = 0; i < 4; i++) T->mark[all[i]] = 0;
    T->mark[ic4[3]] = 0;
    T->last = f;
    return 1;
}

static void tri_destroy(otri *T) {
    free(T->cell); free(T->freel); free(T->mark); free(T->queue); free(T->bc); free(T->bf); free(T->nc);
    free(T->hk0); free(T->hk1); free(T->hc); free(T->hf);
}

/* ---------------------------------------------------------------------- */
/* Insertion order: biased randomised rounds, each sorted along a Morton     */
/* curve (only for speed; the result does not depend on the order).         */

static uint64_t morton_key(const opt *p) {
    uint64_t k = 0;
    uint64_t x = (uint64_t)(p->x + (1 << 19)), y = (uint64_t)(p->y + (1 << 19)), z = (uint64_t)(p->z + (1 << 19));
    for (int b = 19; b >= 0; b--) k = (k << 3) | (((x >> b) & 1) << 2) | (((y >> b) & 1) << 1) | ((z >> b) & 1);
    return k;
}

typedef struct { uint64_t key; int id; } kid;

static int cmp_kid(const void *a, const void *b) {
    const kid *x = (const kid *)a, *y = (const kid *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return (x->id > y->id) - (x->id < y->id);
}

static int make_order(const opt *P, int n, uint64_t seed, int *order) {
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    if (s == 0) s = 1;
    for (int i = 0; i < n; i++) order[i] = i;
    for (int i = n - 1; i > 0; i--) {
        int j = (int)(orng_next(&s) % (uint64_t)(i + 1));
        int t = order[i]; order[i] = order[j]; order[j] = t;
    }
    kid *tmp = (kid *)malloc((size_t)n * sizeof(kid));
    if (!tmp) return 0;
    int end = n;
    while (end > 0) {
        int start = end / 2;
        if (end - start < 64) start = 0;
        if (start > 0) { /* the first (smallest) round keeps its random order */
            for (int i = start; i < end; i++) { tmp[i].key = morton_key(P + order[i]); tmp[i].id = order[i]; }
            qsort(tmp + start, (size_t)(end - start), sizeof(kid), cmp_kid);
            for (int i = start; i < end; i++) order[i] = tmp[i].id;
        }
        end = start;
    }
    free(tmp);
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Exact ortho-centre quantities (origin at the simplex's first vertex).     */

typedef struct { i128 num, den; } rat; /* den > 0 */

static long double rat_ld(rat r) { return (long double)r.num / (long double)r.den; }
static int rat_le(rat r, i64 a) { return r.num <= (i128)a * r.den; }

/* OrthoSize of edge (p0,p1) <= alpha_q ? Exact; symmetric in the endpoints. */
static int edge_passes(const opt *P, int i, int j, i64 aq) {
    i64 ax = P[j].x - P[i].x, ay = P[j].y - P[i].y, az = P[j].z - P[i].z;
    i64 den = ax * ax + ay * ay + az * az;
    i128 beta = (i128)den - P[j].w + P[i].w;
    i128 rhs = (i128)4 * den * (i128)(P[i].w + aq);
    return beta * beta <= rhs;
}

/* OrthoSize of vertex v: the power distance of p_v to its own ball. */
static rat os_vertex(const opt *P, int v) { rat r = {-(i128)P[v].w, 1}; return r; }

/* OrthoSize of an edge: c = p0 + lambda a with 2 a.c' = beta, so
 * |c - p0|^2 = beta^2 / (4 |a|^2). */
static rat os_edge(const opt *P, int p0, int p1) {
    i64 ax = P[p1].x - P[p0].x, ay = P[p1].y - P[p0].y, az = P[p1].z - P[p0].z;
    i64 den = ax * ax + ay * ay + az * az;
    i128 beta = (i128)den - P[p1].w + P[p0].w;
    rat r = {beta * beta - (i128)4 * den * P[p0].w, (i128)4 * den};
    return r;
}

typedef struct { i64 a1[3], a2[3]; i128 g11, g12, g22, den, b1, b2; } tri_frame;

static void tri_setup(const opt *P, int p0, int p1, int p2, tri_frame *F) {
    F->a1[0] = P[p1].x - P[p0].x; F->a1[1] = P[p1].y - P[p0].y; F->a1[2] = P[p1].z - P[p0].z;
    F->a2[0] = P[p2].x - P[p0].x; F->a2[1] = P[p2].y - P[p0].y; F->a2[2] = P[p2].z - P[p0].z;
    F->g11 = (i128)F->a1[0] * F->a1[0] + (i128)F->a1[1] * F->a1[1] + (i128)F->a1[2] * F->a1[2];
    F->g12 = (i128)F->a1[0] * F->a2[0] + (i128)F->a1[1] * F->a2[1] + (i128)F->a1[2] * F->a2[2];
    F->g22 = (i128)F->a2[0] * F->a2[0] + (i128)F->a2[1] * F->a2[1] + (i128)F->a2[2] * F->a2[2];
    F->den = F->g11 * F->g22 - F->g12 * F->g12; /* Gram determinant */
    F->b1 = F->g11 - P[p1].w + P[p0].w;
    F->b2 = F->g22 - P[p2].w + P[p0].w;
}

/* OrthoSize of a triangle: c - p0 = l1 a1 + l2 a2 with G l = beta / 2, so
 * |c - p0|^2 = l^T G l = beta^T adj(G) beta / (4 det G). */
static rat os_tri(const opt *P, int p0, int p1, int p2) {
    tri_frame F;
    tri_setup(P, p0, p1, p2, &F);
    i128 q = F.g22 * F.b1 * F.b1 - 2 * F.g12 * F.b1 * F.b2 + F.g11 * F.b2 * F.b2;
    rat r = {q - 4 * F.den * P[p0].w, 4 * F.den};
    return r;
}

/* OrthoSize of a tetrahedron: A (c - p0) = beta / 2 with rows a_k, solved by
 * Cramer's rule: (c - p0)_j = N_j / (2 det A), N_j = det A with column j
 * replaced by beta. */
static rat os_tet(const opt *P, const int *v) {
    i64 a[3][3];
    i128 b[3];
    for (int k = 0; k < 3; k++) {
        a[k][0] = P[v[k + 1]].x - P[v[0]].x;
        a[k][1] = P[v[k + 1]].y - P[v[0]].y;
        a[k][2] = P[v[k + 1]].z - P[v[0]].z;
        b[k] = (i128)(a[k][0] * a[k][0] + a[k][1] * a[k][1] + a[k][2] * a[k][2]) - P[v[k + 1]].w + P[v[0]].w;
    }
    i128 D = det3(a[0][0], a[0][1], a[0][2], a[1][0], a[1][1], a[1][2], a[2][0], a[2][1], a[2][2]);
    i128 N[3];
    for (int j = 0; j < 3; j++) {
        /* expand det with column j replaced by b along that column */
        i128 s = 0;
        for (int k = 0; k < 3; k++) {
            int r0 = (k + 1) % 3, r1 = (k + 2) % 3;
            int c0 = (j + 1) % 3, c1 = (j + 2) % 3;
            i128 minor = (i128)a[r0][c0] * a[r1][c1] - (i128)a[r0][c1] * a[r1][c0];
            s += b[k] * minor;
        }
        N[j] = s;
    }
    rat r = {N[0] * N[0] + N[1] * N[1] + N[2] * N[2] - 4 * D * D * P[v[0]].w, 4 * D * D};
    return r;
}

/* Violation tests at a simplex's own ortho-centre c: sign of a positive
 * multiple of pi(c, q) - pi(c, p0) with weights perturbed; < 0 means q is
 * strictly closer in power to c than the simplex's balls. */
static int viol_vertex(const opt *P, int v, int q) {
    i64 bx = P[q].x - P[v].x, by = P[q].y - P[v].y, bz = P[q].z - P[v].z;
    i128 g = (i128)(bx * bx + by * by + bz * bz) - P[q].w + P[v].w;
    if (g) return sgn(g);
    int ids[2] = {q, v};
    i128 coef[2] = {-1, 1};
    return sos_sign(2, ids, coef);
}

static int viol_edge(const opt *P, int p0, int p1, int q) {
    i64 ax = P[p1].x - P[p0].x, ay = P[p1].y - P[p0].y, az = P[p1].z - P[p0].z;
    i64 bx = P[q].x - P[p0].x, by = P[q].y - P[p0].y, bz = P[q].z - P[p0].z;
    i128 den = (i128)(ax * ax + ay * ay + az * az);
    i128 beta = den - P[p1].w + P[p0].w;
    i128 gam = (i128)(bx * bx + by * by + bz * bz) - P[q].w + P[p0].w;
    i128 t = (i128)ax * bx + (i128)ay * by + (i128)az * bz;
    i128 val = den * gam - beta * t; /* den * (gamma - 2 lambda a.b), lambda = beta / (2 den) */
    if (val) return sgn(val);
    int ids[3] = {q, p1, p0};
    i128 coef[3] = {-den, t, den - t};
    return sos_sign(3, ids, coef);
}

static int viol_tri(const opt *P, int p0, int p1, int p2, int q) {
    tri_frame F;
    tri_setup(P, p0, p1, p2, &F);
    i64 bx = P[q].x - P[p0].x, by = P[q].y - P[p0].y, bz = P[q].z - P[p0].z;
    i128 t1 = (i128)F.a1[0] * bx + (i128)F.a1[1] * by + (i128)F.a1[2] * bz;
    i128 t2 = (i128)F.a2[0] * bx + (i128)F.a2[1] * by + (i128)F.a2[2] * bz;
    i128 gam = (i128)(bx * bx + by * by + bz * bz) - P[q].w + P[p0].w;
    /* 2 den l = adj(G) beta */
    i128 m1 = F.g22 * F.b1 - F.g12 * F.b2, m2 = F.g11 * F.b2 - F.g12 * F.b1;
    i128 val = F.den * gam - (m1 * t1 + m2 * t2);
    if (val) return sgn(val);
    int ids[4] = {q, p1, p2, p0};
    i128 coef[4] = {-F.den, F.g22 * t1 - F.g12 * t2, F.g11 * t2 - F.g12 * t1,
                    F.den - ((F.g22 - F.g12) * t1 + (F.g11 - F.g12) * t2)};
    return sos_sign(4, ids, coef);
}

/* ---------------------------------------------------------------------- */
/* Sorting helpers                                                           */

typedef struct { int v[4]; long double s; } orow;
/* ctx: the dimension of the rows (compared on their first dim + 1 ids) */
static int cmp_row(const void *a, const void *b, void *ctx) {
    const orow *x = (const orow *)a, *y = (const orow *)b;
    const int dim = *(const int *)ctx;
    for (int k = 0; k <= dim; k++)
        if (x->v[k] != y->v[k]) return x->v[k] < y->v[k] ? -1 : 1;
    return 0;
}

static void sort3(int *v) {
    int a = v[0], b = v[1], c = v[2], t;
    if (a > b) { t = a; a = b; b = t; }
    if (b > c) { t = b; b = c; c = t; }
    if (a > b) { t = a; a = b; b = t; }
    v[0] = a; v[1] = b; v[2] = c;
}
static void sort4(int *v) {
    for (int i = 1; i < 4; i++)
        for (int j = i; j > 0 && v[j - 1] > v[j]; j--) { int t = v[j]; v[j] = v[j - 1]; v[j - 1] = t; }
}

typedef struct { int64_t a, b; } epair;
static int cmp_epair(const void *x, const void *y) {
    const epair *p = (const epair *)x, *q = (const epair *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    return (p->b > q->b) - (p->b < q->b);
}

/* ---------------------------------------------------------------------- */

static int quantise(int64_t n, const double *xyz, const double *radii, double alpha, opt *P, i64 *aq) {
    if (n < 1 || !isfinite(alpha)) return ORACLE_E_INVALID;
    i64 wmax = 0;
    for (int64_t i = 0; i < n; i++) {
        i64 c[3];
        for (int a = 0; a < 3; a++) {
            double v = xyz[3 * i + a];
            if (!isfinite(v)) return ORACLE_E_INVALID;
            double s = v * 1000.0;
            if (!(fabs(s) < 524288.0)) return ORACLE_E_RANGE;
            c[a] = (i64)nearbyint(s);
            if (c[a] >= 524288 || c[a] <= -524288) return ORACLE_E_RANGE;
        }
        double r = radii[i];
        if (!isfinite(r) || !(r > 0)) return ORACLE_E_INVALID;
        double rs = r * 1000.0;
        if (!(rs < 8192.0)) return ORACLE_E_RANGE;
        i64 R = (i64)nearbyint(rs);
        if (R < 1) return ORACLE_E_INVALID;
        P[i].x = c[0]; P[i].y = c[1]; P[i].z = c[2]; P[i].w = R * R;
        if (P[i].w > wmax) wmax = P[i].w;
    }
    double as = alpha * 1e6;
    if (!(fabs(as) < 67108864.0)) return ORACLE_E_RANGE;
    *aq = (i64)nearbyint(as);
    if (wmax + *aq >= 67108864) return ORACLE_E_RANGE;
    return ORACLE_OK;
}

/* ctx: the point array the indices refer to */
static int cmp_pt(const void *a, const void *b, void *ctx) {
    const opt *P = (const opt *)ctx;
    const opt *p = P + *(const int *)a, *q = P + *(const int *)b;
    if (p->x != q->x) return p->x < q->x ? -1 : 1;
    if (p->y != q->y) return p->y < q->y ? -1 : 1;
    return (p->z > q->z) - (p->z < q->z);
}

static int emit(oracle_result *out, int d, orow *rows, int64_t m) {
    qsort_r(rows, (size_t)m, sizeof(orow), cmp_row, &d);
    out->count[d] = m;
    out->simp[d] = (int32_t *)malloc((size_t)(m ? m : 1) * (d + 1) * sizeof(int32_t));
    out->size[d] = (double *)malloc((size_t)(m ? m : 1) * sizeof(double));
    if (!out->simp[d] || !out->size[d]) return 0;
    for (int64_t i = 0; i < m; i++) {
        for (int k = 0; k <= d; k++) out->simp[d][i * (d + 1) + k] = rows[i].v[k];
        out->size[d][i] = (double)(rows[i].s / 1.0e6L);
    }
    return 1;
}

#define SMALL_ROUTE_MAX 4096 /* largest input taken by the low-dimensional route */
static int small_route(const opt *P, int n, i64 aq, oracle_result *out);

int oracle_alpha_complex(int64_t n64, const double *xyz, const double *radii, double alpha, uint64_t order_seed,
                         oracle_result *out) {
    memset(out, 0, sizeof *out);
    if (n64 < 1 || n64 > (1 << 26)) return ORACLE_E_INVALID;
    int n = (int)n64;
    opt *P = (opt *)malloc((size_t)n * sizeof(opt));
    if (!P) return ORACLE_E_NOMEM;
    i64 aq = 0;
    int st = quantise(n64, xyz, radii, alpha, P, &aq);
    if (st) { free(P); return st; }
    {   /* duplicate centres */
        int *ix = (int *)malloc((size_t)n * sizeof(int));
        if (!ix) { free(P); return ORACLE_E_NOMEM; }
        for (int i = 0; i < n; i++) ix[i] = i;
        qsort_r(ix, (size_t)n, sizeof(int), cmp_pt, P);
        for (int i = 1; i < n; i++)
            if (cmp_pt(ix + i - 1, ix + i, P) == 0) { free(ix); free(P); return ORACLE_E_DUPLICATE; }
        free(ix);
    }

    otri T;
    memset(&T, 0, sizeof T);
    T.P = P;
    T.n = n;
    T.rng = order_seed * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull;
    if (T.rng == 0) T.rng = 1;
    int *order = (int *)malloc((size_t)n * sizeof(int));
    int *used = (int *)calloc((size_t)n, sizeof(int));
    if (!order || !used) { free(order); free(used); free(P); return ORACLE_E_NOMEM; }
    if (n >= 4 && !make_order(P, n, order_seed, order)) {
        free(order); free(used); free(P);
        return ORACLE_E_NOMEM;
    }
    /* init_simplex fails (0) only when no four centres span a tetrahedron */
    int init = n >= 4 ? init_simplex(&T, order, n, used) : 0;
    if (init <= 0) {
        free(order); free(used); tri_destroy(&T);
        if (init < 0) { free(P); return ORACLE_E_NOMEM; }
        st = (n <= SMALL_ROUTE_MAX) ? small_route(P, n, aq, out) : ORACLE_E_DEGENERATE;
        free(P);
        return st;
    }
    for (int t = 0; t < n; t++) {
        if (used[t]) continue;
        if (insert_point(&T, order[t]) < 0) {
            free(order); free(used); tri_destroy(&T); free(P);
            return ORACLE_E_NOMEM;
        }
    }
    free(order);
    free(used);

    /* ---- simplices of D ---- */
    int ncell = T.ncell;
    /* finite cells */
    int64_t nt = 0;
    for (int c = 0; c < ncell; c++)
        if (T.cell[c].v[0] != -2 && inf_pos(&T.cell[c]) < 0) nt++;
    /* unique edges of D from finite cells */
    epair *ep = (epair *)malloc((size_t)(nt * 6 + 1) * sizeof(epair));
    if (!ep) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    int64_t ne = 0;
    for (int c = 0; c < ncell; c++) {
        const ocell *C = &T.cell[c];
        if (C->v[0] == -2 || inf_pos(C) >= 0) continue;
        for (int i = 0; i < 4; i++)
            for (int j = i + 1; j < 4; j++) {
                int a = C->v[i], b = C->v[j];
                ep[ne].a = a < b ? a : b;
                ep[ne].b = a < b ? b : a;
                ne++;
            }
    }
    qsort(ep, (size_t)ne, sizeof(epair), cmp_epair);
    int64_t nu = 0;
    for (int64_t i = 0; i < ne; i++)
        if (nu == 0 || ep[i].a != ep[nu - 1].a || ep[i].b != ep[nu - 1].b) ep[nu++] = ep[i];
    ne = nu;
    /* per-vertex edge index: both directions, sorted, for lookups */
    int64_t *vstart = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *adj_v = (int64_t *)malloc((size_t)(2 * ne + 1) * sizeof(int64_t));
    int64_t *adj_e = (int64_t *)malloc((size_t)(2 * ne + 1) * sizeof(int64_t));
    unsigned char *epass = (unsigned char *)malloc((size_t)(ne + 1));
    unsigned char *ein = (unsigned char *)calloc((size_t)(ne + 1), 1);
    unsigned char *egab = (unsigned char *)calloc((size_t)(ne + 1), 1);
    long double *esize = (long double *)malloc((size_t)(ne + 1) * sizeof(long double));
    if (!vstart || !adj_v || !adj_e || !epass || !ein || !egab || !esize) {
        free(ep); free(vstart); free(adj_v); free(adj_e); free(epass); free(ein); free(egab); free(esize);
        tri_destroy(&T); free(P);
        return ORACLE_E_NOMEM;
    }
    for (int64_t e = 0; e < ne; e++) { vstart[ep[e].a + 1]++; vstart[ep[e].b + 1]++; }
    for (int i = 0; i < n; i++) vstart[i + 1] += vstart[i];
    {
        int64_t *fill = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
        if (!fill) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
        memcpy(fill, vstart, (size_t)(n + 1) * sizeof(int64_t));
        for (int64_t e = 0; e < ne; e++) { /* edges sorted, so lists come out sorted */
            adj_v[fill[ep[e].a]] = ep[e].b; adj_e[fill[ep[e].a]++] = e;
        }
        for (int64_t e = 0; e < ne; e++) { adj_v[fill[ep[e].b]] = ep[e].a; adj_e[fill[ep[e].b]++] = e; }
        free(fill);
        /* second pass entries are appended after the first; re-sort each list */
        for (int v = 0; v < n; v++) {
            int64_t s = vstart[v], t = vstart[v + 1];
            for (int64_t i = s + 1; i < t; i++)
                for (int64_t j = i; j > s && adj_v[j - 1] > adj_v[j]; j--) {
                    int64_t tv = adj_v[j]; adj_v[j] = adj_v[j - 1]; adj_v[j - 1] = tv;
                    int64_t te = adj_e[j]; adj_e[j] = adj_e[j - 1]; adj_e[j - 1] = te;
                }
        }
    }
    for (int64_t e = 0; e < ne; e++) epass[e] = (unsigned char)edge_passes(P, (int)ep[e].a, (int)ep[e].b, aq);
#define EDGE_ID(u, w) edge_lookup(vstart, adj_v, adj_e, (u), (w))

    /* ---- tetrahedra ---- */
    unsigned char *tin = (unsigned char *)calloc((size_t)ncell + 1, 1);
    long double *tsize = (long double *)malloc((size_t)(ncell + 1) * sizeof(long double));
    if (!tin || !tsize) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    for (int c = 0; c < ncell; c++) {
        const ocell *C = &T.cell[c];
        if (C->v[0] == -2 || inf_pos(C) >= 0) continue;
        int allpass = 1;
        for (int i = 0; i < 4 && allpass; i++)
            for (int j = i + 1; j < 4; j++)
                if (!epass[EDGE_ID(C->v[i], C->v[j])]) { allpass = 0; break; }
        if (!allpass) continue;
        rat os = os_tet(P, C->v);
        if (rat_le(os, aq)) { tin[c] = 1; tsize[c] = rat_ld(os); }
    }

    /* ---- triangles: one record per (triangle, edge) for the edge pass ---- */
    typedef struct { int64_t e; int w; unsigned char in; long double s; } erec;
    int64_t nf = 0, nrec = 0, reccap = 1024, nkt = 0, ktcap = 1024;
    erec *rec = (erec *)malloc((size_t)reccap * sizeof(erec));
    orow *kt = (orow *)malloc((size_t)ktcap * sizeof(orow)); /* K^2 */
    if (!rec || !kt) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    for (int c = 0; c < ncell; c++) {
        const ocell *C = &T.cell[c];
        if (C->v[0] == -2 || inf_pos(C) >= 0) continue;
        for (int i = 0; i < 4; i++) {
            int d = C->nb[i];
            int dfin = inf_pos(&T.cell[d]) < 0;
            if (dfin && d < c) continue; /* visit each face once */
            nf++;
            int f[3], m = 0;
            for (int k = 0; k < 4; k++)
                if (k != i) f[m++] = C->v[k];
            sort3(f);
            int opp[2] = {C->v[i], -1}, cof[2] = {c, -1};
            if (dfin) {
                for (int k = 0; k < 4; k++)
                    if (T.cell[d].nb[k] == c) { opp[1] = T.cell[d].v[k]; cof[1] = d; break; }
            }
            int64_t e01 = EDGE_ID(f[0], f[1]), e02 = EDGE_ID(f[0], f[2]), e12 = EDGE_ID(f[1], f[2]);
            unsigned char in = 0;
            long double sz = 0;
            if (epass[e01] && epass[e02] && epass[e12]) {
                rat os = os_tri(P, f[0], f[1], f[2]);
                int gab = 1;
                for (int k = 0; k < 2; k++)
                    if (opp[k] >= 0 && viol_tri(P, f[0], f[1], f[2], opp[k]) < 0) gab = 0;
                if (gab) {
                    if (rat_le(os, aq)) { in = 1; sz = rat_ld(os); }
                } else {
                    for (int k = 0; k < 2; k++)
                        if (cof[k] >= 0 && tin[cof[k]] && (!in || tsize[cof[k]] < sz)) { in = 1; sz = tsize[cof[k]]; }
                }
            }
            if (in) {
                if (nkt == ktcap) {
                    ktcap *= 2;
                    orow *t2 = (orow *)realloc(kt, (size_t)ktcap * sizeof(orow));
                    if (!t2) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
                    kt = t2;
                }
                kt[nkt].v[0] = f[0]; kt[nkt].v[1] = f[1]; kt[nkt].v[2] = f[2]; kt[nkt].v[3] = 0; kt[nkt].s = sz;
                nkt++;
            }
            int64_t es[3] = {e01, e02, e12};
            int ws[3] = {f[2], f[1], f[0]};
            for (int k = 0; k < 3; k++) {
                if (!epass[es[k]]) continue;
                if (nrec == reccap) {
                    reccap *= 2;
                    erec *r2 = (erec *)realloc(rec, (size_t)reccap * sizeof(erec));
                    if (!r2) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
                    rec = r2;
                }
                rec[nrec].e = es[k]; rec[nrec].w = ws[k]; rec[nrec].in = in; rec[nrec].s = sz;
                nrec++;
            }
        }
    }

    /* ---- edges: group records by edge (counting sort) ---- */
    int64_t *rs = (int64_t *)calloc((size_t)ne + 1, sizeof(int64_t));
    erec *rsorted = (erec *)malloc((size_t)(nrec + 1) * sizeof(erec));
    if (!rs || !rsorted) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    for (int64_t r = 0; r < nrec; r++) rs[rec[r].e + 1]++;
    for (int64_t e = 0; e < ne; e++) rs[e + 1] += rs[e];
    {
        int64_t *fill = (int64_t *)malloc((size_t)(ne + 1) * sizeof(int64_t));
        if (!fill) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
        memcpy(fill, rs, (size_t)(ne + 1) * sizeof(int64_t));
        for (int64_t r = 0; r < nrec; r++) rsorted[fill[rec[r].e]++] = rec[r];
        free(fill);
    }
    free(rec);
    for (int64_t e = 0; e < ne; e++) {
        if (!epass[e]) continue;
        int a = (int)ep[e].a, b = (int)ep[e].b;
        int gab = 1;
        for (int64_t r = rs[e]; r < rs[e + 1]; r++)
            if (viol_edge(P, a, b, rsorted[r].w) < 0) { gab = 0; break; }
        egab[e] = (unsigned char)gab;
        if (gab) {
            rat os = os_edge(P, a, b);
            if (rat_le(os, aq)) { ein[e] = 1; esize[e] = rat_ld(os); }
        } else {
            for (int64_t r = rs[e]; r < rs[e + 1]; r++)
                if (rsorted[r].in && (!ein[e] || rsorted[r].s < esize[e])) { ein[e] = 1; esize[e] = rsorted[r].s; }
        }
    }
    free(rs);
    free(rsorted);

    /* ---- vertices ---- */
    int64_t nkv = 0;
    orow *kv = (orow *)malloc((size_t)n * sizeof(orow));
    if (!kv) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    int64_t nvert = 0;
    for (int v = 0; v < n; v++) {
        if (vstart[v + 1] == vstart[v]) continue; /* hidden: no edge of D */
        nvert++;
        int gab = 1;
        for (int64_t t = vstart[v]; t < vstart[v + 1]; t++)
            if (viol_vertex(P, v, (int)adj_v[t]) < 0) { gab = 0; break; }
        unsigned char in = 0;
        long double sz = 0;
        if (gab) {
            rat os = os_vertex(P, v);
            if (rat_le(os, aq)) { in = 1; sz = rat_ld(os); }
        } else {
            for (int64_t t = vstart[v]; t < vstart[v + 1]; t++) {
                int64_t e = adj_e[t];
                if (ein[e] && (!in || esize[e] < sz)) { in = 1; sz = esize[e]; }
            }
        }
        if (in) { kv[nkv].v[0] = v; kv[nkv].s = sz; nkv++; }
    }

    /* ---- collect K^1 and K^3 ---- */
    int64_t nke = 0;
    for (int64_t e = 0; e < ne; e++) nke += ein[e];
    orow *ke = (orow *)malloc((size_t)(nke + 1) * sizeof(orow));
    int64_t nktet = 0;
    for (int c = 0; c < ncell; c++) nktet += tin[c];
    orow *ktet = (orow *)malloc((size_t)(nktet + 1) * sizeof(orow));
    if (!ke || !ktet) { tri_destroy(&T); free(P); return ORACLE_E_NOMEM; }
    nke = 0;
    for (int64_t e = 0; e < ne; e++)
        if (ein[e]) { ke[nke].v[0] = (int)ep[e].a; ke[nke].v[1] = (int)ep[e].b; ke[nke].s = esize[e]; nke++; }
    nktet = 0;
    for (int c = 0; c < ncell; c++)
        if (tin[c]) {
            memcpy(ktet[nktet].v, T.cell[c].v, sizeof(int) * 4);
            sort4(ktet[nktet].v);
            ktet[nktet].s = tsize[c];
            nktet++;
        }

    out->n_hidden = n - nvert;
    out->d_count[0] = nvert;
    out->d_count[1] = ne;
    out->d_count[2] = nf;
    out->d_count[3] = nt;
    int okm = emit(out, 0, kv, nkv) && emit(out, 1, ke, nke) && emit(out, 2, kt, nkt) && emit(out, 3, ktet, nktet);
    free(kv); free(ke); free(kt); free(ktet);
    free(ep); free(vstart); free(adj_v); free(adj_e); free(epass); free(ein); free(egab); free(esize);
    free(tin); free(tsize);
    tri_destroy(&T);
    free(P);
    if (!okm) { oracle_free(out); return ORACLE_E_NOMEM; }
    return ORACLE_OK;
}

static int64_t edge_lookup(const int64_t *vstart, const int64_t *adj_v, const int64_t *adj_e, int64_t u, int64_t w) {
    int64_t lo = vstart[u], hi = vstart[u + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (adj_v[mid] == w) return adj_e[mid];
        if (adj_v[mid] < w) lo = mid + 1; else hi = mid - 1;
    }
    abort(); /* every edge of a cell of D is in the edge table */
}

/* ---------------------------------------------------------------------- */

static int contains_all(const int *big, int nb, const int *small, int ns) {
    for (int i = 0; i < ns; i++) {
        int f = 0;
        for (int j = 0; j < nb; j++) f |= big[j] == small[i];
        if (!f) return 0;
    }
    return 1;
}

/* Appends row v (k ids, ascending) with Size s to the rows of dimension d. */
static int push_row(orow **rows, int64_t *cnt, int64_t *cap, int d, const int *v, int k, long double s) {
    if (cnt[d] == cap[d]) {
        int64_t nc = cap[d] ? 2 * cap[d] : 64;
        orow *r = (orow *)realloc(rows[d], (size_t)nc * sizeof(orow));
        if (!r) return 0;
        rows[d] = r;
        cap[d] = nc;
    }
    orow *r = &rows[d][cnt[d]++];
    for (int i = 0; i < 4; i++) r->v[i] = i < k ? v[i] : 0;
    r->s = s;
    return 1;
}

static int collinear(const opt *P, int a, int b, int c) {
    i64 ux = P[b].x - P[a].x, uy = P[b].y - P[a].y, uz = P[b].z - P[a].z;
    i64 wx = P[c].x - P[a].x, wy = P[c].y - P[a].y, wz = P[c].z - P[a].z;
    return (i128)uy * wz - (i128)uz * wy == 0 && (i128)uz * wx - (i128)ux * wz == 0 &&
           (i128)ux * wy - (i128)uy * wx == 0;
}

/* Membership and Size of the k-subset v (k = 1..3, ascending ids) whose edges
 * all pass the edge OrthoSize test, given the kept (k+1)-subsets cof[0..ncof).
 * In K_alpha iff its ortho-centre is a witness (no other ball strictly closer
 * in power, ties by the perturbation) with OrthoSize <= alpha, or an
 * immediate coface is in K_alpha; the Size is then the least Size of such a
 * coface (Sec. 2.3). */
static int decide_low(const opt *P, int n, i64 aq, const int *v, int k, const orow *cof, int64_t ncof,
                      long double *sz) {
    int gab = 1;
    for (int q = 0; q < n && gab; q++) {
        if (contains_all(v, k, &q, 1)) continue;
        int sg = k == 1 ? viol_vertex(P, v[0], q)
                        : (k == 2 ? viol_edge(P, v[0], v[1], q) : viol_tri(P, v[0], v[1], v[2], q));
        if (sg < 0) gab = 0;
    }
    if (gab) {
        rat os = k == 1 ? os_vertex(P, v[0]) : (k == 2 ? os_edge(P, v[0], v[1]) : os_tri(P, v[0], v[1], v[2]));
        if (!rat_le(os, aq)) return 0;
        *sz = rat_ld(os);
        return 1;
    }
    int in = 0;
    for (int64_t t = 0; t < ncof; t++)
        if (contains_all(cof[t].v, k + 1, v, k) && (!in || cof[t].s < *sz)) {
            in = 1;
            *sz = cof[t].s;
        }
    return in;
}

/* Inputs whose D is not three-dimensional: fewer than four balls, or every
 * centre on one plane. No four centres then span a tetrahedron, so D has no
 * tetrahedra, and every triple, pair and single ball is examined directly
 * (n <= SMALL_ROUTE_MAX) by decide_low, triangles first. A subset with an edge
 * failing the edge OrthoSize test is skipped: its OrthoSize, and so its Size
 * and that of any coface, exceeds alpha (a face's OrthoSize never exceeds its
 * coface's, Sec. 4.3). Counts of D are not produced on this route (-1). */
static int small_route(const opt *P, int n, i64 aq, oracle_result *out) {
    orow *rows[4] = {NULL, NULL, NULL, NULL};
    int64_t cnt[4] = {0, 0, 0, 0}, cap[4] = {0, 0, 0, 0};
    int ok = 1;
    long double sz = 0;
    for (int a = 0; a < n && ok; a++)
        for (int b = a + 1; b < n && ok; b++) {
            if (!edge_passes(P, a, b, aq)) continue;
            for (int c = b + 1; c < n && ok; c++) {
                if (!edge_passes(P, a, c, aq) || !edge_passes(P, b, c, aq) || collinear(P, a, b, c)) continue;
                int v[3] = {a, b, c};
                if (decide_low(P, n, aq, v, 3, rows[3], cnt[3], &sz)) ok = push_row(rows, cnt, cap, 2, v, 3, sz);
            }
        }
    for (int a = 0; a < n && ok; a++)
        for (int b = a + 1; b < n && ok; b++) {
            if (!edge_passes(P, a, b, aq)) continue;
            int v[2] = {a, b};
            if (decide_low(P, n, aq, v, 2, rows[2], cnt[2], &sz)) ok = push_row(rows, cnt, cap, 1, v, 2, sz);
        }
    for (int a = 0; a < n && ok; a++) {
        int v[1] = {a};
        if (decide_low(P, n, aq, v, 1, rows[1], cnt[1], &sz)) ok = push_row(rows, cnt, cap, 0, v, 1, sz);
    }
    for (int d = 0; d < 4 && ok; d++) {
        out->d_count[d] = -1;
        ok = emit(out, d, rows[d], cnt[d]);
    }
    for (int d = 0; d < 4; d++) free(rows[d]);
    if (!ok) {
        oracle_free(out);
        return ORACLE_E_NOMEM;
    }
    out->n_hidden = -1;
    return ORACLE_OK;
}

void oracle_free(oracle_result *r) {
    for (int d = 0; d < 4; d++) {
        free(r->simp[d]);
        free(r->size[d]);
        r->simp[d] = NULL;
        r->size[d] = NULL;
        r->count[d] = 0;
    }
}
