/*
 * btog.h -- C interface of the libraries the BTO compiler generates.
 *
 * For a program in the kernel language of Section II (Fig. 1), the
 * compiler (paper_1205_1098_amd/btoc_gen.py) emits one HIP source per
 * program: every sweep over a matrix that the schedule fuses (Section III:
 * the products of one matrix at one point of the schedule, the update that
 * forms or contracts the matrix) becomes one loop nest,
 *     for each row band p(i) across workgroups
 *       for each row i of the band, across the band's waves
 *         for each column j, across lanes:
 *           b = A_ij (+ u0_i v0_j + u1_i v1_j + ...)   stored as B_ij, or kept
 *                                                      in registers (contracted)
 *           col_q[j] += b * y_q[i]                      for every column sum q
 *           row_p[i] += b * x_p[j]                      for every row dot p
 * followed by a fixed-order reduction of the partial sums.  The partition
 * of the loop nest (the tile shape across and down a workgroup and the band
 * height, i.e. the thread count of Section III-C) is not fixed at
 * generation: every pass is compiled for each tile shape, and the search of
 * Section IV picks them at run time.  The source is compiled once with
 * hipcc into its own shared library, which exports the functions below.
 *
 * Conventions are those of bto.h: device pointers owned by the caller,
 * row-major matrices with a leading dimension, outputs overwritten, work
 * enqueued on `stream` without synchronizing, errors returned before
 * anything is enqueued.
 */
#ifndef BTOG_H
#define BTOG_H

#include <stddef.h>
#include <stdint.h>

#include "bto.h"

#ifdef __cplusplus
extern "C" {
#endif

#define BTOG_ABI_VERSION 1
#define BTOG_MAX_TERMS 8   /* rank-1 terms of one update */
#define BTOG_MAX_RED 8     /* row dots, and column sums, of one pass */

/* The operands of one pass.  A is m x n (lda); B (ldb) is written when the
 * pass stores its update (else NULL; B may be exactly A with ldb == lda).
 * u[r] (length m) and v[r] (length n) are the update's terms, in the order
 * of the statement.  Row dot p: row_out[p] (length m) = scale_p *
 * (M x[p]) + add_scale_p * row_add[p] (row_add[p] may be NULL), with M the
 * updated matrix; column sum q: col_out[q] (length n) = scale_q * (M' y[q])
 * + add_scale_q * col_add[q].  The scales are products of literals and the
 * program's scalar inputs, evaluated by the generated code from `scalars`
 * (host memory, the program's scalar inputs in declaration order).  Every
 * output is overwritten; an empty sum is 0. */
typedef struct {
    int64_t m, n, lda, ldb;
    const double *A;
    double *B;
    const double *u[BTOG_MAX_TERMS];
    const double *v[BTOG_MAX_TERMS];
    const double *x[BTOG_MAX_RED];
    double *row_out[BTOG_MAX_RED];
    const double *row_add[BTOG_MAX_RED];
    const double *y[BTOG_MAX_RED];
    double *col_out[BTOG_MAX_RED];
    const double *col_add[BTOG_MAX_RED];
    const double *scalars;
    int nscalars;
} btog_pass_args;

int btog_abi_version(void);
/* The program's name and a digest of the generated source. */
const char *btog_program(void);
const char *btog_source_digest(void);
int btog_pass_count(void);

/* A pass's structure: counts[0] update terms, counts[1] 1 if the update is
 * stored, counts[2] row dots, counts[3] column sums. */
bto_status btog_pass_layout(int pass, int counts[4]);

/* Tile shapes every pass is compiled for: waves_across x waves_down waves,
 * kv 16-byte pairs per lane (a block of 128 * kv * waves_across columns),
 * depth rows of loads in flight per wave. */
int btog_shape_count(void);
bto_status btog_shape(int shape, int *kv, int *depth, int *waves_across, int *waves_down);

/* Whether `pass` runs with tile shape `shape` and bands of rb rows: rb a
 * multiple of waves_down, at most 4096, and at most 64 rows per wave when
 * the pass has row dots.  1 if so, 0 if not. */
int btog_config_ok(int pass, int shape, int rb);

/* Bytes of scratch `pass` needs at m x n under (shape, rb); 0 for an
 * invalid configuration or negative sizes. */
size_t btog_pass_workspace_bytes(int pass, int64_t m, int64_t n, int shape, int rb);

/* Enqueue one pass.  Errors: BTO_ERR_INVALID_ARG (pass index, negative
 * size, leading dimension below n, a NULL operand with a nonzero extent, a
 * configuration btog_config_ok refuses, too few scalars), BTO_ERR_WORKSPACE
 * (ws_bytes below btog_pass_workspace_bytes), BTO_ERR_UNSUPPORTED (more row
 * bands than a launch grid holds: take taller bands), BTO_ERR_HIP. */
bto_status btog_run_pass(int pass, const btog_pass_args *args, int shape, int rb, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/* Text of the last error on the calling thread. */
const char *btog_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BTOG_H */
