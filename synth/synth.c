/*
 * Seeded synthetic molecules: random sequential adsorption (dart throwing with
 * a minimum centre separation) on the integer milli-angstrom lattice inside a
 * ball or a spherical shell, plus element draws, Gaussian jitter and batch
 * size draws.
 *
 * This module holds input generation only; it computes nothing of the alpha
 * complex. Both the HIP path and the CPU oracle are fed from it.
 *
 * Random numbers: xoshiro256** seeded through splitmix64 (Blackman and Vigna,
 * "Scrambled linear pseudorandom number generators", 2018), written from
 * their published descriptions.
 *
 * Sampling: the next accepted centre of plain dart throwing is uniform over
 * the part of the domain that no accepted centre excludes yet. Darts are drawn
 * uniformly from a set of equal-sized "active" cubes that always covers that
 * part (cubes wholly excluded, or wholly outside the domain, are dropped; all
 * remaining cubes are halved together when the hit rate falls), so the
 * accepted sequence has the same law as plain dart throwing (Ebeida et al.,
 * "Efficient maximal Poisson-disk sampling", SIGGRAPH 2011/2012), only with
 * far fewer wasted darts.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64_next(uint64_t *state) {
    uint64_t z = (*state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static void rng_seed(rng_t *r, uint64_t seed) {
    uint64_t st = seed;
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64_next(&st);
}

static inline uint64_t rotl64(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    const uint64_t out = rotl64(s[1] * 5, 7) * 9;
    const uint64_t t = s[1] << 17;
    s[2] ^= s[0];
    s[3] ^= s[1];
    s[1] ^= s[2];
    s[0] ^= s[3];
    s[2] ^= t;
    s[3] = rotl64(s[3], 45);
    return out;
}

/* Uniform integer in [0, m), m >= 1, by multiply-shift with rejection
 * (Lemire, "Fast random integer generation in an interval", 2019). */
static inline uint64_t rng_below(rng_t *r, uint64_t m) {
    uint64_t x = rng_next(r);
    unsigned __int128 p = (unsigned __int128)x * m;
    uint64_t lo = (uint64_t)p;
    if (lo < m) {
        uint64_t thresh = (0 - m) % m;
        while (lo < thresh) {
            x = rng_next(r);
            p = (unsigned __int128)x * m;
            lo = (uint64_t)p;
        }
    }
    return (uint64_t)(p >> 64);
}

/* Uniform double in [0, 1) with 53 random bits. */
static inline double rng_unit(rng_t *r) { return (double)(rng_next(r) >> 11) * 0x1.0p-53; }

/* ---------------------------------------------------------------------- */
/* Occupancy grid: at most one centre per cell, since the cell diagonal is   */
/* below the minimum separation.                                            */

typedef struct {
    int64_t lo;        /* lattice coordinate of the grid's low corner (all axes) */
    int64_t side;
    int64_t dim;       /* cells per axis */
    int32_t *cell;     /* dim^3, -1 = empty, else point index */
    int64_t reach;     /* cells to scan on each side */
} occ_t;

static inline int64_t occ_coord(const occ_t *g, int64_t x) { return (x - g->lo) / g->side; }

/* 1 if some accepted centre lies strictly closer than sep to (x,y,z). */
static int occ_conflict(const occ_t *g, const int32_t *pts, int64_t x, int64_t y, int64_t z, int64_t sep2) {
    int64_t cx = occ_coord(g, x), cy = occ_coord(g, y), cz = occ_coord(g, z);
    int64_t r = g->reach;
    int64_t z0 = cz - r < 0 ? 0 : cz - r, z1 = cz + r >= g->dim ? g->dim - 1 : cz + r;
    int64_t y0 = cy - r < 0 ? 0 : cy - r, y1 = cy + r >= g->dim ? g->dim - 1 : cy + r;
    int64_t x0 = cx - r < 0 ? 0 : cx - r, x1 = cx + r >= g->dim ? g->dim - 1 : cx + r;
    for (int64_t k = z0; k <= z1; k++)
        for (int64_t j = y0; j <= y1; j++) {
            const int32_t *row = g->cell + (k * g->dim + j) * g->dim;
            for (int64_t i = x0; i <= x1; i++) {
                int32_t p = row[i];
                if (p < 0) continue;
                int64_t dx = pts[3 * p] - x, dy = pts[3 * p + 1] - y, dz = pts[3 * p + 2] - z;
                if (dx * dx + dy * dy + dz * dz < sep2) return 1;
            }
        }
    return 0;
}

/* Gathers into near[] (at most cap) the centres that could exclude a point of
 * the lattice cube [x,x+h-1]^3; returns how many. */
static int occ_gather(const occ_t *g, const int32_t *pts, int64_t x, int64_t y, int64_t z, int64_t h, int64_t sep,
                      int32_t *near, int cap) {
    int64_t lo[3] = {x - sep, y - sep, z - sep}, hi[3] = {x + h - 1 + sep, y + h - 1 + sep, z + h - 1 + sep};
    int64_t c0[3], c1[3];
    for (int a = 0; a < 3; a++) {
        c0[a] = lo[a] < g->lo ? 0 : (lo[a] - g->lo) / g->side;
        c1[a] = (hi[a] - g->lo) / g->side;
        if (c1[a] >= g->dim) c1[a] = g->dim - 1;
    }
    int m = 0;
    for (int64_t k = c0[2]; k <= c1[2]; k++)
        for (int64_t j = c0[1]; j <= c1[1]; j++) {
            const int32_t *row = g->cell + (k * g->dim + j) * g->dim;
            for (int64_t i = c0[0]; i <= c1[0]; i++)
                if (row[i] >= 0 && m < cap) near[m++] = row[i];
        }
    return m;
}

/* 1 if the whole lattice cube [x,x+h-1]^3 is excluded by a single centre of near[]
 * (all eight corners strictly within the separation; a ball is convex). */
static int covers_cube(const int32_t *pts, const int32_t *near, int m, int64_t x, int64_t y, int64_t z, int64_t h,
                       int64_t sep2) {
    const int32_t x0 = (int32_t)x, y0 = (int32_t)y, z0 = (int32_t)z, x1 = (int32_t)(x + h - 1),
                  y1 = (int32_t)(y + h - 1), z1 = (int32_t)(z + h - 1);
    int hit = 0;
    for (int t = 0; t < m; t++) {
        const int32_t *p = pts + 3 * near[t];
        int32_t ax = abs(x0 - p[0]), bx = abs(x1 - p[0]);
        int32_t ay = abs(y0 - p[1]), by = abs(y1 - p[1]);
        int32_t az = abs(z0 - p[2]), bz = abs(z1 - p[2]);
        int64_t dx = ax > bx ? ax : bx, dy = ay > by ? ay : by, dz = az > bz ? az : bz;
        hit |= (dx * dx + dy * dy + dz * dz < sep2);
    }
    return hit;
}

/* 0: cube misses the shell, 1: cube may meet it, 2: cube lies wholly inside it. */
static int cube_shell_state(int64_t x, int64_t y, int64_t z, int64_t h, int64_t rin2, int64_t rout2) {
    int64_t c[3] = {x, y, z};
    int64_t dmin = 0, dmax = 0;
    for (int a = 0; a < 3; a++) {
        int64_t l = c[a], u = c[a] + h - 1;
        int64_t near = (l > 0) ? l : (u < 0 ? -u : 0);
        int64_t far = llabs(l) > llabs(u) ? llabs(l) : llabs(u);
        dmin += near * near;
        dmax += far * far;
    }
    if (dmin > rout2 || dmax < rin2) return 0;
    return (dmin >= rin2 && dmax <= rout2) ? 2 : 1;
}

/*
 * Random sequential adsorption of n centres on Z^3 with rin_mA <= |p| <= rout_mA
 * (rin_mA = 0 for a ball) and pairwise squared distance >= min_sep^2.
 * Writes xyz[3n] in acceptance order (which is the input order).
 * Returns 0 on success, -1 if the domain jammed before n centres, -2 on
 * allocation failure, -3 on bad arguments. *darts_out gets the darts thrown.
 */
int synth_rsa(int64_t n, uint64_t seed, int64_t rin_mA, int64_t rout_mA, int64_t min_sep, int32_t *xyz,
              int64_t *darts_out) {
    if (n < 0 || rout_mA <= 0 || rin_mA < 0 || rin_mA >= rout_mA || min_sep <= 0 || rout_mA > (1 << 20))
        return -3;
    if (n == 0) { if (darts_out) *darts_out = 0; return 0; }
    rng_t rng;
    rng_seed(&rng, seed);
    const int64_t sep2 = min_sep * min_sep;
    const int64_t rin2 = rin_mA * rin_mA, rout2 = rout_mA * rout_mA;

    occ_t g;
    g.side = (int64_t)floor((double)min_sep / sqrt(3.0));
    while (3 * g.side * g.side >= sep2) g.side--;
    g.lo = -rout_mA - 1;
    g.dim = (2 * rout_mA + 3) / g.side + 2;
    g.reach = (min_sep + g.side - 1) / g.side;
    size_t ncell = (size_t)g.dim * g.dim * g.dim;
    g.cell = (int32_t *)malloc(ncell * sizeof(int32_t));
    if (!g.cell) return -2;
    memset(g.cell, 0xff, ncell * sizeof(int32_t));

    /* Active cubes: side h, a power of two no larger than the occupancy cell,
     * so a cube holding a centre is wholly excluded. */
    int64_t h = 1;
    while (2 * h <= g.side) h *= 2;
    const int64_t base = -rout_mA - 1;
    int64_t per_axis = (2 * rout_mA + 3 + h - 1) / h;
    int64_t cap = 1 << 20, na = 0;
    int32_t *act = (int32_t *)malloc((size_t)cap * 3 * sizeof(int32_t));
    if (!act) { free(g.cell); return -2; }
    for (int64_t k = 0; k < per_axis; k++)
        for (int64_t j = 0; j < per_axis; j++)
            for (int64_t i = 0; i < per_axis; i++) {
                int64_t x = base + i * h, y = base + j * h, z = base + k * h;
                if (!cube_shell_state(x, y, z, h, rin2, rout2)) continue;
                if (na == cap) {
                    cap *= 2;
                    int32_t *t = (int32_t *)realloc(act, (size_t)cap * 3 * sizeof(int32_t));
                    if (!t) { free(act); free(g.cell); return -2; }
                    act = t;
                }
                act[3 * na] = (int32_t)x; act[3 * na + 1] = (int32_t)y; act[3 * na + 2] = (int32_t)z;
                na++;
            }

    int64_t got = 0, darts = 0;
    int rc = 0;
    while (got < n) {
        if (na == 0) { rc = -1; break; }
        /* A phase: darts until the recent hit rate drops, then refine. */
        int64_t window = 0, hits = 0;
        const int64_t win = na / 16 < 4096 ? 4096 : na / 16;
        for (;;) {
            uint64_t a = rng_below(&rng, (uint64_t)na);
            int64_t x = act[3 * a] + (int64_t)rng_below(&rng, (uint64_t)h);
            int64_t y = act[3 * a + 1] + (int64_t)rng_below(&rng, (uint64_t)h);
            int64_t z = act[3 * a + 2] + (int64_t)rng_below(&rng, (uint64_t)h);
            darts++;
            window++;
            int64_t r2 = x * x + y * y + z * z;
            if (r2 >= rin2 && r2 <= rout2 && !occ_conflict(&g, xyz, x, y, z, sep2)) {
                xyz[3 * got] = (int32_t)x; xyz[3 * got + 1] = (int32_t)y; xyz[3 * got + 2] = (int32_t)z;
                g.cell[(occ_coord(&g, z) * g.dim + occ_coord(&g, y)) * g.dim + occ_coord(&g, x)] = (int32_t)got;
                got++;
                hits++;
                if (got == n) break;
            }
            if (window >= win) {
                if (hits * 4 < window) break; /* hit rate below 1/4: refine */
                window = 0; hits = 0;
            }
        }
        if (got == n) break;
        /* Refine: drop excluded cubes, halve the rest (while h > 1). Each parent
         * gets an 8-bit mask of surviving children (bit 0 alone when h == 1);
         * the masks are decided in parallel and compacted in parent order, so
         * the result does not depend on the thread count. */
        int64_t nh = h > 1 ? h / 2 : 1;
        uint8_t *mask = (uint8_t *)malloc((size_t)na);
        if (!mask) { rc = -2; break; }
#pragma omp parallel for schedule(static, 4096)
        for (int64_t a = 0; a < na; a++) {
            int32_t near[512];
            int64_t x = act[3 * a], y = act[3 * a + 1], z = act[3 * a + 2];
            int m = occ_gather(&g, xyz, x, y, z, h, min_sep, near, 512);
            uint8_t mk = 0;
            if (!covers_cube(xyz, near, m, x, y, z, h, sep2)) {
                if (h == 1) {
                    mk = 1;
                } else {
                    const int inside = cube_shell_state(x, y, z, h, rin2, rout2) == 2;
                    for (int c = 0; c < 8; c++) {
                        int64_t cx = x + (c & 1) * nh, cy = y + ((c >> 1) & 1) * nh, cz = z + ((c >> 2) & 1) * nh;
                        if (!inside && !cube_shell_state(cx, cy, cz, nh, rin2, rout2)) continue;
                        if (covers_cube(xyz, near, m, cx, cy, cz, nh, sep2)) continue;
                        mk |= (uint8_t)(1u << c);
                    }
                }
            }
            mask[a] = mk;
        }
        int64_t nn = 0;
        for (int64_t a = 0; a < na; a++) nn += __builtin_popcount(mask[a]);
        int32_t *nact = (int32_t *)malloc((size_t)(nn > 0 ? nn : 1) * 3 * sizeof(int32_t));
        if (!nact) { free(mask); rc = -2; break; }
        int64_t w = 0;
        for (int64_t a = 0; a < na; a++) {
            uint8_t mk = mask[a];
            if (!mk) continue;
            int64_t x = act[3 * a], y = act[3 * a + 1], z = act[3 * a + 2];
            for (int c = 0; c < 8; c++) {
                if (!(mk & (1u << c))) continue;
                nact[3 * w] = (int32_t)(x + (c & 1) * nh);
                nact[3 * w + 1] = (int32_t)(y + ((c >> 1) & 1) * nh);
                nact[3 * w + 2] = (int32_t)(z + ((c >> 2) & 1) * nh);
                w++;
            }
        }
        free(mask);
        free(act);
        act = nact;
        na = nn;
        h = nh;
    }
    free(act);
    free(g.cell);
    if (darts_out) *darts_out = darts;
    return rc;
}

/* Element radii (mA) in input order: C 1700 (p .62), N 1550 (.17), O 1520 (.19), S 1800 (.02). */
void synth_radii(int64_t n, uint64_t seed, int32_t *R) {
    rng_t rng;
    rng_seed(&rng, seed);
    for (int64_t i = 0; i < n; i++) {
        uint64_t u = rng_below(&rng, 100);
        R[i] = u < 62 ? 1700 : (u < 79 ? 1550 : (u < 98 ? 1520 : 1800));
    }
}

/* n standard normal deviates by the Box-Muller transform. */
void synth_normal(int64_t n, uint64_t seed, double *out) {
    rng_t rng;
    rng_seed(&rng, seed);
    for (int64_t i = 0; i < n; i += 2) {
        double u1 = rng_unit(&rng), u2 = rng_unit(&rng);
        if (u1 <= 0.0) u1 = 0x1.0p-53;
        double rad = sqrt(-2.0 * log(u1)), th = 6.283185307179586 * u2;
        out[i] = rad * cos(th);
        if (i + 1 < n) out[i + 1] = rad * sin(th);
    }
}

/* n uniform doubles in [0,1). */
void synth_uniform(int64_t n, uint64_t seed, double *out) {
    rng_t rng;
    rng_seed(&rng, seed);
    for (int64_t i = 0; i < n; i++) out[i] = rng_unit(&rng);
}

/* n uniform integers in [0, m). */
void synth_below(int64_t n, uint64_t seed, uint64_t m, int64_t *out) {
    rng_t rng;
    rng_seed(&rng, seed);
    for (int64_t i = 0; i < n; i++) out[i] = (int64_t)rng_below(&rng, m);
}
