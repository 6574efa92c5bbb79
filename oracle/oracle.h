/*
 * CPU oracle for the alpha complex of weighted points (test infrastructure).
 *
 * This is test infrastructure, not the product: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may call it. It shares no code
 * with the HIP path.
 *
 * It computes the plain definition: build the weighted Delaunay (regular)
 * triangulation D of the balls by incremental insertion, give every simplex
 * its Size (the smallest power distance over its witnesses) and keep the
 * simplices with Size <= alpha (Masood, Ray, Natarajan, "Parallel Computation
 * of Alpha Complexes for Biomolecules", Sec. 2.3 definitions of witness, Size
 * and OrthoSize; Sec. 2.4 definition of K_alpha). Degenerate inputs are
 * resolved by simulation of simplicity on the weights, ranked by input index
 * (the paper's Sec. 2 general-position remark).
 */
#ifndef ALPHACX_ORACLE_H
#define ALPHACX_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ORACLE_OK = 0,
    ORACLE_E_INVALID = 1,    /* n < 1, non-finite value, radius <= 0, non-finite alpha */
    ORACLE_E_DUPLICATE = 2,  /* two equal quantised centres */
    ORACLE_E_RANGE = 3,      /* |coordinate| >= 2^19 mA, or W_max + alpha_q >= 2^26 mA^2 */
    ORACLE_E_NOMEM = 4,
    ORACLE_E_DEGENERATE = 7  /* all centres coplanar and n too large for the subset search */
};

typedef struct {
    int64_t count[4];   /* simplices of K_alpha per dimension */
    int32_t *simp[4];   /* count[d] x (d+1) input ids, ascending in a row, rows sorted */
    double *size[4];    /* Size of each simplex, square angstrom */
    int64_t n_hidden;   /* balls that are not vertices of D */
    int64_t d_count[4]; /* finite simplices of D per dimension */
} oracle_result;

/*
 * xyz: n x 3 row-major angstrom; radii: n angstrom; alpha: square angstrom.
 * Coordinates and radii are quantised to integer milli-angstrom (round half
 * to even); alpha to integer milli-angstrom squared. order_seed picks the
 * insertion order (the result does not depend on it).
 */
int oracle_alpha_complex(int64_t n, const double *xyz, const double *radii, double alpha, uint64_t order_seed,
                         oracle_result *out);
void oracle_free(oracle_result *r);

#ifdef __cplusplus
}
#endif
#endif
