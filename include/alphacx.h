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

/* Largest number of alpha values of one ac_alpha_sweep_device call. */
#define AC_MAX_SWEEP 1024

/* Opaque result; owned by the library until ac_free(). */
typedef struct ac_complex ac_complex;

/* Tuning knobs; a zeroed struct (or NULL) selects the defaults. None of them
 * changes the result. Every field is checked: a value outside its stated
 * range makes the call return AC_E_INVALID before any device work. */
typedef struct {
    int32_t cell_mA;         /* uniform-grid cell side in milli-angstrom, >= 0; 0 = ceil(sqrt(r_max^2 + alpha)) */
    int32_t wave_tile;       /* must be 0: every kernel maps one work item (ball, edge, triangle, tetrahedron,
                                simplex corner) to one lane, so there is no tile to choose */
    int32_t force_exact;     /* 0 or 1; 1 = skip the floating-point filter, decide every predicate in exact integers */
    int32_t vertex_shortcut; /* 0 or 1; 1 = take every ball whose OrthoSize -r^2 <= alpha as a vertex without
                                testing its own centre (the paper's implementation shortcut, Sec. 4.4); exact
                                only when no centre lies inside another ball's power cell */
    int64_t capacity_hint;   /* must be 0: candidate and output buffers are sized from exact counts */
    int32_t profile;         /* 0, 1, 2 + i (0 <= i < ac_stage_count()) or 2 + ac_stage_count(); 1 = record HIP
                                events between pipeline stages (see ac_stage_ms); 2 + i = record only the two
                                events around stage i (each event adds a few microseconds of device idle time);
                                2 + ac_stage_count() = every stage, with the AC2 tests of candidate edges and
                                triangles run as kernels of their own ("edges_ac2", "triangles_ac2": the same
                                result, for a per-step breakdown that separates them as the paper's Table 2
                                does) */
    int32_t cell_order;      /* numbering of the grid cells, which orders the balls in memory: 0 = row-major
                                (x fastest), 1 = Morton / Z-order curve (Sec. 4.2 names space-filling curves) */
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

/* ---- Build without allocation ----
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * computation of ac_alpha_complex_device, with every intermediate buffer
 * taken from a fixed scratch array of AC_NOALLOC_SCRATCH_MIB MiB that the
 * library holds on each device it runs on until the process ends, and the
 * result written into caller buffers. The call makes no device or pinned-host
 * allocation (no hipMalloc, hipFree, hipHostMalloc, HIP event or pool block).
 *   d_xyz, d_radii, n, alpha, opt, stream  as ac_alpha_complex_device;
 *            opt->profile must be 0
 *   d_simp   host array of 4 device pointers: d_simp[d] has room for
 *            capacity[d] rows of d + 1 int32 (row-major)
 *   d_size   host array of 4 device pointers: d_size[d] has room for
 *            capacity[d] float64
 *   capacity host array of 4 row capacities (>= 0; a pointer may be NULL
 *            when its capacity is 0)
 *   counts   host array of 4: receives the number of d-simplices of K_alpha
 *            (also when AC_E_CAPACITY reports a too small output buffer; -1
 *            when the build did not finish)
 * On AC_OK the rows and Sizes are exactly those of ac_alpha_complex_device
 * (same layout, order and values) and are complete on return: the call
 * synchronises `stream` before it returns. Calls on one device share its
 * scratch array; the library serialises them (a call holds the device's
 * scratch until its work on the stream has finished), and a call's scratch
 * contents are not kept for the next.
 * Errors as ac_alpha_complex_device, plus AC_E_CAPACITY when the build needs
 * more than the fixed scratch (n above AC_NOALLOC_SCRATCH_MIB MiB / 128 B is
 * refused before any device work; measured on synthetic molecules at alpha = 0:
 * 250,000 balls with van der Waals radii fit, and 12,000 but not 16,000 with
 * solvent-accessible radii, whose candidates per ball are about ten times as
 * many) or when an output buffer is
 * smaller than the result (nothing is written to the outputs then). The
 * pointers of d_simp / d_size are not written on any error. */
#define AC_NOALLOC_SCRATCH_MIB 256
ac_status ac_alpha_complex_noalloc(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                   const ac_options *opt, void *stream, int32_t *const *d_simp,
                                   double *const *d_size, const int64_t *capacity, int64_t *counts);

/* ---- Partitioned build ----
 *
 * The same complex built slab by slab: the balls are cut into `parts` slabs
 * of equal width along x; each slab is built with every ball within
 * 4 sqrt(r_max^2 + alpha) + 2 A of it, and keeps the simplices whose owner
 * vertex (least quantised x, ties to the least input id) lies in it; the
 * kept rows of all slabs are then merged into output order. Membership and
 * Size of a simplex depend only on balls within 4 sqrt(r_max^2 + alpha) of
 * any of its vertices (Sec. 3.1 Steps 1-5 with the neighbour bound of
 * Sec. 4.3), so the result equals ac_alpha_complex_device bit for bit, while
 * the scratch memory of a call is that of one slab's build. This is the
 * split the library would use across GPUs, and for inputs whose build does
 * not fit at once (the paper processes chunks of the sorted atom list,
 * Sec. 4.6).
 *   parts    1 <= parts <= 64
 * Other arguments and errors as ac_alpha_complex_device. ac_candidate_count
 * and ac_work_count report -1; ac_exact_fallbacks sums over the slabs.
 */
ac_status ac_alpha_complex_partitioned(const double *d_xyz, const double *d_radii, int64_t n, double alpha,
                                       int32_t parts, const ac_options *opt, void *stream, ac_complex **out);

/* ---- Partitioned build from host memory (out of core) ----
 *
 * As ac_alpha_complex_partitioned, with inputs and results in host memory:
 * only one slab (its core and halo) is on the device at a time. Each slab's
 * balls are copied to the device, built, and the rows it owns are copied
 * back; the slabs' row lists, each already in output order, are then merged
 * on the host. The device memory of a call is that of the largest slab's
 * build, so inputs whose build would not fit on the device at once can be
 * processed (the paper processes chunks of the sorted atom list, Sec. 4.6).
 * Runs on the current device's null stream and returns when done.
 *   xyz, radii  host arrays as in ac_alpha_complex (read during the call)
 *   parts       1 <= parts <= 1024
 * The result equals ac_alpha_complex's bit for bit; its arrays are host
 * memory (ac_simplices_device returns NULL); ac_candidate_count and
 * ac_work_count report -1. Errors as ac_alpha_complex_partitioned. */
ac_status ac_alpha_complex_partitioned_host(const double *xyz, const double *radii, int64_t n, double alpha,
                                            int32_t parts, const ac_options *opt, ac_complex **out);

/* ---- Alpha sweep ----
 *
 * The alpha complexes of one ball set for several alpha values from a single
 * candidate search at the largest of them. The candidates of a smaller alpha
 * are exactly the candidates of the larger that pass AC3 at the smaller
 * (OrthoSize is monotone over faces), and AC2 does not depend on alpha
 * (Sec. 2.4, 3.1), so each K_alpha is obtained by re-testing AC3 exactly at
 * that alpha and re-running the pruning (Steps 2-5) on the shared candidate
 * lists; the output order is sorted once. This is the reuse of a computed
 * complex for other alpha values that the paper names as future work
 * (Sec. 6).
 *   alphas   host, n_alpha values in square angstrom, any order, repeats
 *            allowed; 1 <= n_alpha <= AC_MAX_SWEEP
 *   out      host array of n_alpha handles: out[k] receives the complex of
 *            alphas[k], each to be released with ac_free (all NULL on error)
 * Other arguments as ac_alpha_complex_device. out[k] holds exactly what
 * ac_alpha_complex_device returns for alphas[k] (simplices and Sizes bit
 * for bit); ac_exact_fallbacks reports the whole call and ac_stage_ms of a
 * profiled call times the search stages and, as "emit", every alpha's
 * pruning and output together. Errors as ac_alpha_complex_device (the
 * range check uses the largest alpha).
 */
ac_status ac_alpha_sweep_device(const double *d_xyz, const double *d_radii, int64_t n, const double *alphas,
                                int64_t n_alpha, const ac_options *opt, void *stream, ac_complex **out);

/* ---- Batches of molecules ----
 *
 * Many independent molecules in one call: molecule m is the balls
 * [offsets[m], offsets[m+1]) of the concatenated arrays d_xyz / d_radii
 * (device, as in ac_alpha_complex_device). offsets is a host array of
 * n_mol + 1 int64 with offsets[0] = 0, strictly increasing (no empty
 * molecule), offsets[n_mol] < 2^26; 1 <= n_mol <= 2^20. Each molecule gets a
 * uniform grid of its own (Sec. 4.2) whose cells are numbered after those of
 * the molecules before it, so balls of different molecules never interact
 * (their coordinates may overlap). Every stage runs once over the whole
 * batch. The result is the union of the molecules' complexes, with ids into
 * the concatenated arrays: rows are sorted by least id, so molecule m's
 * d-simplices are rows [ac_molecule_rows(c, d)[m], ac_molecule_rows(c, d)[m+1]),
 * and subtracting offsets[m] from their ids gives exactly what
 * ac_alpha_complex_device returns for that molecule alone (simulation of
 * simplicity ranks by id, and the order of ids within a molecule is kept).
 * cell_mA: NULL, or a host array of n_mol positive cell sides in mA (e.g.
 * from ac_tune_cells); opt->cell_mA applies to every molecule otherwise.
 * Errors as ac_alpha_complex_device, plus AC_E_INVALID for bad offsets. */
ac_status ac_alpha_complex_batch(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol,
                                 double alpha, const ac_options *opt, const int32_t *cell_mA, void *stream,
                                 ac_complex **out);

/* ---- Recorded batch builds (graph replay) ----
 *
 * A batch build whose every size is fixed in advance, captured once in a HIP
 * graph and replayed: for a stream of inputs of one shape (the same molecules
 * with new coordinates, e.g. the frames of a trajectory), each replay is one
 * graph launch with no host synchronisation and no allocation.
 *
 * ac_plan_create runs one ordinary batch build of the given arrays to note
 * the sizes (grid cells per molecule, candidate edges, triangles and
 * tetrahedra), then fixes them with `headroom` (capacity = noted size x
 * headroom + 256; every molecule's grid gets at least one cell per ball),
 * takes the build's buffers and captures the whole pipeline on a stream of its
 * own. Arguments as ac_alpha_complex_batch; opt->profile must be 0;
 * 1 <= headroom <= 16. d_xyz / d_radii are recorded: every replay reads the
 * coordinates and radii found at those addresses when it runs, so they must
 * stay allocated until ac_plan_free. Synchronises `stream`. AC_E_CAPACITY if a
 * stage of the input needs the counted fill (rows longer than the single-pass
 * slots, e.g. solvent-accessible radii), which a recorded build does not have.
 *
 * ac_plan_launch enqueues one replay on `stream` (may be captured or ordered
 * like any kernel launch). ac_plan_result then synchronises `stream` and
 * returns the replay's complex as a new result (the same as
 * ac_alpha_complex_batch on the arrays as they were at the replay, bit for
 * bit, with ac_molecule_rows). If the input no longer fits what was recorded
 * (a radius above the largest recorded one, a grid or a candidate total above
 * its capacity, a row beyond its slot, duplicate or invalid values), the replay
 * stops early and ac_plan_result runs an ordinary batch build of the same
 * arrays instead (its errors are reported then); ac_plan_stopped gives the
 * reason bits of the last result (0: the replay itself produced it; 1 input,
 * 2 cells, 4 duplicates, 8 slot, 16 capacity) and ac_plan_ordinary_builds how
 * often that happened. One replay of a plan at a time: call ac_plan_result
 * before the next ac_plan_launch. The plan holds its buffers (about those of
 * one ordinary build, with headroom) until ac_plan_free. */
typedef struct ac_plan ac_plan;
ac_status ac_plan_create(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol, double alpha,
                         const ac_options *opt, const int32_t *cell_mA, double headroom, void *stream, ac_plan **out);
ac_status ac_plan_launch(ac_plan *p, void *stream);
ac_status ac_plan_result(ac_plan *p, void *stream, ac_complex **out);
int32_t ac_plan_stopped(const ac_plan *p);
int64_t ac_plan_ordinary_builds(const ac_plan *p);
void ac_plan_free(ac_plan *p);

/* Molecules of the call that made c (1 for the single-molecule calls). */
int64_t ac_molecule_count(const ac_complex *c);

/* Host array of n_mol + 1 row indices into the d-simplex array: molecule m
 * owns rows [rows[m], rows[m+1]). Valid until ac_free; NULL for a bad dim. */
const int64_t *ac_molecule_rows(const ac_complex *c, int dim);

/* Molecule of every d-simplex of a batch result: a host array of
 * ac_count(c, dim) int32 (row k belongs to molecule ac_molecule(c, dim)[k]),
 * built on first use from ac_molecule_rows and valid until ac_free. NULL for a
 * result not made by ac_alpha_complex_batch, or a bad dim. */
const int32_t *ac_molecule(ac_complex *c, int dim);

/* Cell-size autotuner for a batch (same arguments as ac_alpha_complex_batch).
 * The molecules are put in size buckets ([0, 2k), [2k, 8k), [8k, 32k) and
 * [32k, inf) balls); for each bucket its molecules are copied into one
 * sub-batch and built with cell sides of 0.5, 0.7, 1, 1.4 and 2 times the
 * grown radius s_g (default 1 s_g); each side is timed by two HIP events
 * around whole builds (the median of five, after a warm-up run), and the
 * fastest side, if it beats the default by more than 3 % (else the default),
 * is written to cell_mA_out[m] for every molecule m of the bucket (and the
 * bucket index to bucket_out[m] if not NULL). Both are host arrays of n_mol. The cell side never changes the
 * result, only the time. Synchronises `stream`. */
ac_status ac_tune_cells(const double *d_xyz, const double *d_radii, const int64_t *offsets, int64_t n_mol, double alpha,
                        const ac_options *opt, void *stream, int32_t *cell_mA_out, int32_t *bucket_out);

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

/* Sizes of internal structures of the call, for traffic accounting:
 * which = 0: cells of the uniform grid; 1: entries of the neighbour rows
 * (each ball's list of balls whose grown ball meets its own). -1 otherwise. */
int64_t ac_work_count(const ac_complex *c, int which);

/* Per-stage device time of a call made with opt->profile = 1 (every stage)
 * or 2 + i (stage i only), from HIP events recorded on the call's stream
 * between stages (milliseconds; -1 if the stage was not recorded or i is out
 * of range). Stage i is named by ac_stage_name(i), for
 * 0 <= i < ac_stage_count(). */
int ac_stage_count(void);
const char *ac_stage_name(int i);
double ac_stage_ms(const ac_complex *c, int i);

/* ---- Union of balls: volume and boundary area, and their gradients ----
 *
 * The alpha complex of a molecule is what its volume and surface area are
 * computed from (Sec. 1 of the paper). With c the complex at alpha = 0 of the
 * same n balls, V and A of the union of the balls are the alternating sums,
 * over the simplices of c, of the volume of the intersection of their balls
 * and of the area of each sphere's part inside the other balls (short
 * inclusion-exclusion over the dual complex, Edelsbrunner 1995).
 *
 * d_xyz (n x 3 row-major float64, angstrom) and d_radii (n float64) are device
 * arrays on the complex's device, read on `stream`; they are used as given
 * (not quantised), so finite differences over them see a smooth function of
 * the coordinates while the complex stays fixed. n must equal the number of
 * balls the complex was built on, and the complex must have been built at
 * alpha = 0, else AC_E_INVALID (for the union of balls grown to
 * sqrt(r^2 + alpha), build the complex of those grown radii at alpha = 0; it
 * is K_alpha of the original balls up to the rounding of the grown radii to
 * the milli-angstrom lattice).
 *
 * The work buffers are kept with the complex: after the first call on a
 * complex these calls allocate nothing and do not synchronise the host
 * (except ac_union_measure, which returns host values). Calls on one complex
 * must not overlap (same stream, or ordered by the caller). */

/* V (A^3) and A (A^2) into host doubles; synchronises `stream`. */
ac_status ac_union_measure(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n, double *V,
                           double *A, void *stream);

/* Same, written as d_out[0] = V, d_out[1] = A into device memory on `stream`. */
ac_status ac_union_measure_device(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                  double *d_out, void *stream);

/* Gradient of gV * V + gA * A with (gV, gA) = (d_grad[0], d_grad[1]) read from
 * device memory: d_dxyz (n x 3) and d_dradii (n) are overwritten on the device
 * (balls in no simplex get 0). The complex is held fixed. Deterministic: each
 * ball sums its simplices' terms in a fixed order. The first call on a complex
 * sorts its simplex corners by ball (kept until ac_free). */
ac_status ac_union_measure_backward(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                    const double *d_grad, double *d_dxyz, double *d_dradii, void *stream);

/* Forward and backward in one pass (each corner's terms evaluated once):
 * d_out[0] = V, d_out[1] = A as ac_union_measure_device writes them (equal up
 * to the rounding of a differently ordered evaluation), and the gradient as
 * ac_union_measure_backward writes it (bit for bit), for an optimisation
 * step that needs both. Arguments and rules as those two calls. */
ac_status ac_union_measure_fused(ac_complex *c, const double *d_xyz, const double *d_radii, int64_t n,
                                 const double *d_grad, double *d_out, double *d_dxyz, double *d_dradii, void *stream);

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
