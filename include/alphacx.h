/*
 * alphacx: alpha complex of weighted points (atoms as balls) on AMD MI355X.
 *
 * C ABI of libalphacx.so. Every call returns an ac_status; no C++ exception
 * crosses this boundary. All pointers are plain host or device pointers as
 * stated per argument; no framework types appear here.
 *
 * What is computed (Masood, Ray, Natarajan, "Parallel Computation of Alpha
 * Complexes for Biomolecules", SoCG 2020):
 *   - balls b_i = (p_i, r_i) with weight r_i^2, power distance
 *     pi(p, b_i) = |p - p_i|^2 - r_i^2 (Sec. 2.2);
 *   - the alpha complex K_alpha = { sigma in D : Size(sigma) <= alpha }, with D
 *     the weighted Delaunay triangulation and Size the least power distance of
 *     a witness of sigma (Sec. 2.3, 2.4), computed without building D by the
 *     two-stage method of Sec. 3 (Steps 1-5) on a uniform grid (Sec. 4.2-4.4).
 *
 * Units and quantisation: coordinates and radii in angstrom are rounded to
 * integer milli-angstrom (round half to even) and alpha to integer
 * milli-angstrom squared; every membership decision is then exact (floating
 * point filter with an exact 128-bit integer fallback). Degenerate inputs are
 * resolved by simulation of simplicity on the weights, ranked by input index
 * (lower index dominates), which the paper names for degeneracies (Sec. 2).
 *
 * Output: for each dimension d = 0..3, the simplices of K_alpha as rows of
 * d+1 input indices (0-based), ascending within a row, rows in lexicographic
 * order, and each simplex's Size in square angstrom (float64).
 */
#ifndef ALPHACX_H
#define ALPHACX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AC_OK = 0,
    AC_E_INVALID = 1,   /* n < 1, a non-finite value, a radius <= 0 (or below 0.0005 A), non-finite alpha, bad dim */
    AC_E_DUPLICATE = 2, /* two equal quantised centres */
    AC_E_RANGE = 3,     /* |coordinate| >= 524.288 A, radius >= 8.192 A, or r_max^2 + alpha >= 67.108864 A^2 */
    AC_E_NOMEM = 4,     /* device or host allocation failed */
    AC_E_DEVICE = 5,    /* a HIP runtime error; ac_last_error() has the detail */
    AC_E_CAPACITY = 6   /* a candidate list outgrew its buffer even after the internal retry */
} ac_status;

/* Opaque result; owned by the library until ac_free(). */
typedef struct ac_complex ac_complex;

/* Tuning knobs; a zeroed struct (or NULL) selects the defaults. None of them
 * changes the result. */
typedef struct {
    int32_t cell_mA;         /* uniform-grid cell side in milli-angstrom; 0 = ceil(sqrt(r_max^2 + alpha)) */
    int32_t wave_tile;       /* reserved for the batched path; 0 = default */
    int32_t force_exact;     /* 1 = skip the floating-point filter, decide every predicate in exact integers */
    int32_t vertex_shortcut; /* 1 = take every ball whose OrthoSize -r^2 <= alpha as a vertex without testing
                                its own centre (the paper's implementation shortcut, Sec. 4.4); exact
                                only when no centre lies inside another ball's power cell */
    int64_t capacity_hint;   /* expected simplices per atom for buffer sizing; 0 = adaptive */
    int32_t profile;         /* 1 = record HIP events between pipeline stages (see ac_stage_ms) */
    int32_t reserved;        /* must be 0 */
} ac_options;

/*
 * Alpha complex from host arrays.
 *   xyz    host, n x 3 float64 row-major, angstrom (read during the call only)
 *   radii  host, n float64, angstrom
 *   n      number of balls, 1 <= n < 2^26
 *   alpha  square angstrom (the power-distance parameter of Sec. 2.4)
 *   opt    may be NULL
 *   out    receives a new result (NULL on error; nothing leaks)
 * Runs on the current HIP device and its null stream; host-to-device and
 * device-to-host copies are included. Result arrays are host memory.
 */
ac_status ac_alpha_complex(const double *xyz, const double *radii, int64_t n, double alpha, const ac_options *opt,
                           ac_complex **out);

/*
 * Same computation from device arrays, on the given HIP stream (hipStream_t,
 * NULL = the null stream). d_xyz / d_radii are device pointers with the
 * layout above and must stay valid until the call returns. The call returns
 * once the counts are known; the sorted device arrays (ac_simplices_device,
 * ac_sizes_device) are complete when `stream` reaches the point of return.
 * Host copies are made only on the first ac_simplices / ac_sizes access.
 */
ac_status ac_alpha_complex_device(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                  const ac_options *opt, void *stream, ac_complex **out);

/* Number of d-simplices in K_alpha (d = 0..3); -1 for a NULL result or bad d. */
int64_t ac_count(const ac_complex *c, int dim);

/* Host pointers (count x (dim+1) int32 input ids / count float64 Sizes in A^2),
 * valid until ac_free; NULL for a bad dim or on a failed copy. */
const int32_t *ac_simplices(ac_complex *c, int dim);
const double *ac_sizes(ac_complex *c, int dim);

/* Device pointers to the same arrays (device results only; NULL otherwise). */
const int32_t *ac_simplices_device(const ac_complex *c, int dim);
const double *ac_sizes_device(const ac_complex *c, int dim);

/* Candidate counts of the estimation stage (Sigma_ortho^d, d = 1..3; d = 0
 * gives the balls with -r^2 <= alpha) and the number of exact fallbacks taken
 * by the floating-point filter; for diagnostics and benchmarking. */
int64_t ac_candidate_count(const ac_complex *c, int dim);
int64_t ac_exact_fallbacks(const ac_complex *c);

/* Per-stage device time of a call made with opt->profile = 1, from HIP events
 * recorded on the call's stream between stages (milliseconds; -1 if not
 * profiled or i out of range). Stage i is named by ac_stage_name(i), for
 * 0 <= i < ac_stage_count(). */
int ac_stage_count(void);
const char *ac_stage_name(int i);
double ac_stage_ms(const ac_complex *c, int i);

/* Releases a result (NULL is allowed). */
void ac_free(ac_complex *c);

/* Releases the library's cached device workspace on the current device. */
ac_status ac_release_workspace(void);

const char *ac_status_str(ac_status s);

/* Detail of the last error on the calling thread ("" if none). */
const char *ac_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
