/*
 * bto.h -- C interface of libbto.so: fused FP64 BLAS-1/2 sequences on AMD
 * MI355X (gfx950).
 *
 * The seven kernels are those of Table I (Section V-A) of Belter, Jessup,
 * Nelson, Norris and Siek, "Reliable Generation of High-Performance Matrix
 * Algebra".  Each entry point computes exactly the statements of its table
 * row, in the order listed there; the argument lists follow the paper's
 * kernel specifications: named inputs, then named outputs (Section II,
 * Fig. 1), row-major matrices (Section II) with the BLAS-style row count,
 * column count and leading dimension of the dgemv listing of Section V-A.
 *
 * Every entry point offers two forms:
 *   BTO_FUSED    -- loop fusion and array contraction applied as the
 *                   paper's search would pick them (Sections III-IV): every
 *                   statement sharing a matrix pass runs in one kernel, and
 *                   temporaries never reach memory;
 *   BTO_UNFUSED  -- one kernel per BLAS operation, each reading its inputs
 *                   and writing its output once, out of place (the plain
 *                   per-BLAS-call loops the paper measures against,
 *                   Section V-B).
 * Both forms give results within 1e-12 normwise relative error of the plain
 * definition; with integer-valued data both are exact.
 *
 * Conventions shared by all entry points
 *   - Matrices are m x n, row-major: element (i, j) at A[i*lda + j],
 *     lda >= max(1, n).
 *   - Every array pointer is a DEVICE pointer on the current HIP device,
 *     allocated and owned by the caller.  The kernel entry points never
 *     allocate or free device memory; plans (batch and tiled batch) own
 *     what their create calls allocate, and bto_gemver_noalloc uses a
 *     static array the library keeps per device.
 *   - Work is enqueued on `stream` (NULL = the default stream) and the call
 *     returns without synchronizing.  Inputs must stay valid, and outputs
 *     untouched by others, until the stream reaches the end of the call.
 *   - Outputs are overwritten (never accumulated into).  A zero extent is
 *     valid: an empty sum is 0, so e.g. BiCGK with m = 0 writes s = 0.
 *   - NaN and Inf propagate as IEEE arithmetic makes them; nothing checks.
 *   - Reductions use fixed summation trees that depend only on the sizes,
 *     so repeated calls give bitwise-identical results.
 *   - `ws` is caller-provided device scratch of at least
 *     bto_workspace_bytes(kernel, m, n, form) bytes, 256-byte aligned; its
 *     contents on entry are ignored.  It may be NULL when that size is 0.
 *   - Errors are returned synchronously before anything is enqueued:
 *       BTO_ERR_INVALID_ARG  negative size, lda/ldb too small, NULL pointer
 *                            with a nonzero extent, unknown form;
 *       BTO_ERR_ALIAS        an output overlaps another operand other than
 *                            in the exact aliases the entry point allows;
 *       BTO_ERR_WORKSPACE    ws_bytes below the required size;
 *       BTO_ERR_HIP          a launch failed (bto_last_error() tells why).
 *   - The library is thread-safe; calls on one stream execute in order.
 */
#ifndef BTO_H
#define BTO_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The input enumerations span the whole int range (the _RANGE_ members are
 * never valid arguments), so any int a caller passes is a value of the type
 * and is rejected with BTO_ERR_INVALID_ARG, rather than being a value the
 * implementation's language leaves undefined. */
typedef enum {
    BTO_FUSED = 0,
    BTO_UNFUSED = 1,
    BTO_FORM_RANGE_MIN_ = -2147483647 - 1,
    BTO_FORM_RANGE_MAX_ = 2147483647
} bto_form;

typedef enum {
    BTO_SUCCESS = 0,
    BTO_ERR_INVALID_ARG = 1,
    BTO_ERR_ALIAS = 2,
    BTO_ERR_WORKSPACE = 3,
    BTO_ERR_HIP = 4,
    BTO_ERR_UNSUPPORTED = 5
} bto_status;

typedef enum {
    BTO_K_BICGK = 0,
    BTO_K_GEMVER = 1,
    BTO_K_ATAX = 2,
    BTO_K_DGEMVT = 3,
    BTO_K_AXPYDOT = 4,
    BTO_K_WAXPBY = 5,
    BTO_K_VADD = 6,
    BTO_K_GEMVER_CONTRACTED = 7,   /* GEMVER without B (bto_gemver_contracted) */
    BTO_K_BATAX = 8,               /* y <- beta A^T A x (bto_batax) */
    BTO_K_DGEMV = 9,               /* z <- alpha A x + beta y (bto_dgemv) */
    BTO_K_GESUMMV = 10,            /* y <- alpha A x + beta B x (bto_gesummv) */
    BTO_KERNEL_RANGE_MIN_ = -2147483647 - 1,
    BTO_KERNEL_RANGE_MAX_ = 2147483647
} bto_kernel;

/* Library version, as 10000*major + 100*minor + patch. */
int bto_version(void);

/* Bytes of scratch that `kernel` needs at size (m, n) in form `form`.
 * Vector kernels take their length as n and ignore m.  Returns 0 on bad
 * arguments.  The value only depends on the arguments. */
size_t bto_workspace_bytes(bto_kernel kernel, int64_t m, int64_t n, bto_form form);

/* Static text for a status code. */
const char *bto_status_string(bto_status s);

/* Text of the last error raised on the calling thread ("" if none). */
const char *bto_last_error(void);

/* BICGK (Table I):  q <- A p ;  s <- A^T r.
 * A: m x n (lda); p: n; r: m; outputs q: m, s: n.
 * Fused: one pass over A computes both products (Section V-B notes this is
 * the fusion the best tools found).  Unfused: dgemv 'N' then dgemv 'T'. */
bto_status bto_bicgk(int64_t m, int64_t n, const double *A, int64_t lda,
                     const double *p, const double *r, double *q, double *s,
                     void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* GEMVER (Table I):
 *   B <- A + u1 v1^T + u2 v2^T ;  x <- beta B^T y + z ;  w <- alpha B x
 * in that order (w uses the new x).  A, B: m x n (lda, ldb); u1, u2, y, w:
 * m; v1, v2, z, x: n.  B may be exactly A (B == A and ldb == lda): an
 * in-place update.  Fused: pass 1 forms B and the x partial sums in one
 * sweep of A; pass 2 computes w from B.  Unfused: ger, ger, dgemv 'T',
 * dgemv 'N'. */
bto_status bto_gemver(int64_t m, int64_t n, double alpha, double beta,
                      const double *A, int64_t lda,
                      const double *u1, const double *v1,
                      const double *u2, const double *v2,
                      const double *y, const double *z,
                      double *B, int64_t ldb, double *x, double *w,
                      void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* GEMVER without a workspace argument and without allocating, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Arguments, results,
 * forms and errors are those of bto_gemver; the results are bitwise those
 * of bto_gemver with the same arguments.  The partial sums live in a device
 * array of bto_gemver_noalloc_max_scratch_bytes() bytes (80 MiB) that the
 * library owns: one per device, set up by the first call on that device
 * (the current device, which must be the one `stream` belongs to) and kept
 * until the process ends.  A call whose scratch need,
 * bto_workspace_bytes(BTO_K_GEMVER, m, n, form), exceeds it returns
 * BTO_ERR_WORKSPACE before enqueuing anything (n = m = 16384 fits exactly).
 * All calls on one device share that array: calls whose kernels overlap
 * on the device (other streams, other threads) race and give invalid
 * results; calls enqueued on one stream are ordered and safe.  Nothing in
 * the array needs clearing between calls.  No hipMalloc, hipFree or other
 * allocating routine is called. */
size_t bto_gemver_noalloc_max_scratch_bytes(void);
bto_status bto_gemver_noalloc(int64_t m, int64_t n, double alpha, double beta,
                              const double *A, int64_t lda,
                              const double *u1, const double *v1,
                              const double *u2, const double *v2,
                              const double *y, const double *z,
                              double *B, int64_t ldb, double *x, double *w,
                              bto_form form, hipStream_t stream);

/* GEMVER with its B contracted away: the same x and w as bto_gemver, for
 * a caller that does not need B.  Contracting a temporary that only feeds
 * the later statements is the heuristic of Section III-E; here it turns
 * B's store and re-read into two reads of A:
 *   x <- beta (A^T y + v1 (u1.y) + v2 (u2.y)) + z
 *   w <- alpha (A x + u1 (v1.x) + u2 (v2.x))              (new x)
 * which equal beta B^T y + z and alpha B x for B = A + u1 v1^T + u2 v2^T
 * (up to rounding order).  Shapes as bto_gemver; there is no unfused form
 * (the unfused GEMVER must materialize B).  Pass 1 forms A^T y's partial
 * sums and the two dots with y in one sweep of A, pass 2 A x's partial
 * sums and the dots with x; each finish adds its rank-2 correction. */
bto_status bto_gemver_contracted(int64_t m, int64_t n, double alpha, double beta,
                                 const double *A, int64_t lda,
                                 const double *u1, const double *v1,
                                 const double *u2, const double *v2,
                                 const double *y, const double *z, double *x, double *w,
                                 void *ws, size_t ws_bytes, hipStream_t stream);

/* BATAX:  y <- beta A^T A x, ATAX with its result scaled (the scale is
 * applied after the reduction).  Arguments and forms as bto_atax. */
bto_status bto_batax(int64_t m, int64_t n, double beta, const double *A, int64_t lda,
                     const double *x, double *y,
                     void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* ATAX (Table I):  y <- A^T A x.  A: m x n (lda); x, y: n.
 * Fused: each row of A is read once and kept on chip while its dot with x
 * is reduced and then used to update y (the partitioning p(i) of
 * Section III-D); the temporary A x never reaches memory.  For n above
 * 16384 the fused form falls back to two passes.  Unfused: dgemv 'N' into
 * a temporary, then dgemv 'T'. */
bto_status bto_atax(int64_t m, int64_t n, const double *A, int64_t lda,
                    const double *x, double *y,
                    void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* DGEMVT (Table I):  x <- beta A^T y + z ;  w <- alpha A x  (new x).
 * A: m x n (lda); y, w: m; z, x: n.  Two passes in both forms (w needs all
 * of x); the fused form folds the scaling and the +z into the reduction
 * epilogues and reads A in the order that reuses what the first pass left
 * in cache. */
bto_status bto_dgemvt(int64_t m, int64_t n, double alpha, double beta,
                      const double *A, int64_t lda, const double *y, const double *z,
                      double *x, double *w,
                      void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* DGEMV (Table I):  z <- alpha A x + beta y, each scale applied after its
 * reduction: z_i = alpha * (sum_j A_ij x_j) + beta * y_i.
 * A: m x n (lda); x: n; y, z: m.  z may be exactly y (the in-place BLAS
 * call); no other overlap with an operand is allowed.  A single BLAS
 * operation (Section V-A), so both forms run the same sweep: row dots of A
 * per column tile, then a fixed-order reduction whose epilogue adds beta y.
 * ws: bto_workspace_bytes(BTO_K_DGEMV, m, n, form) bytes of device scratch. */
bto_status bto_dgemv(int64_t m, int64_t n, double alpha, double beta,
                     const double *A, int64_t lda, const double *x, const double *y,
                     double *z, void *ws, size_t ws_bytes, bto_form form,
                     hipStream_t stream);

/* GESUMMV (Table I):  y <- alpha A x + beta B x, i.e.
 * y_i = alpha * (sum_j A_ij x_j) + beta * (sum_j B_ij x_j).
 * A (lda) and B (ldb) are both m x n; x: n; y: m.  B may be exactly A
 * (same pointer and leading dimension); y may not overlap any input.
 * Fused: the row dots of A, then of B, into separate partials, and one
 * reduction that forms y.  The two matrices share only x, so the fusion
 * saves the temporary and a reduction, not matrix traffic (a single launch
 * over both matrices measured slower than two).  Unfused: the BLAS form,
 * dgemv into a temporary t = alpha A x, then y = beta B x + t. */
bto_status bto_gesummv(int64_t m, int64_t n, double alpha, double beta,
                       const double *A, int64_t lda, const double *B, int64_t ldb,
                       const double *x, double *y, void *ws, size_t ws_bytes,
                       bto_form form, hipStream_t stream);

/* ---- one fused pass over a matrix ----------------------------------------
 * The building block that the spec compiler (paper_1205_1098_amd/btoc.py)
 * lowers a program to: one sweep of a row-major m x n matrix with the loop
 * bodies fused (Section III-C's {p(i){i{j ...}}} nest), then the fixed-order
 * reductions of its partial sums with their epilogues.  M below is A, or
 * A + u1 v1^T + u2 v2^T when STORE or CONTRACT is set (pass zero vectors
 * for a rank-1 update).
 *   ROWDOT    row_out = row_scale * (M x) + row_add_scale * row_add      (m)
 *   COLSUM    col_out = col_scale * (M^T y) + col_add_scale * col_add    (n)
 *   STORE     M is formed and written to B (B may be exactly A, ldb == lda)
 *   CONTRACT  M is never formed: M x = A x + u1 (v1.x) + u2 (v2.x) and
 *             M^T y = A^T y + v1 (u1.y) + v2 (u2.y)  (Section III-E); with
 *             ROWDOT or COLSUM (not both), and an add scale of 1
 *   CHAIN     with ROWDOT | COLSUM over A alone: the column sums are
 *             weighted by the row dots themselves, col_out = col_scale *
 *             A^T (A x), with the row held on chip (ATAX's one-pass form,
 *             Section IV-A); row_out, y and col_add must be NULL
 * A NULL row_add or col_add adds nothing.  row_out may be exactly row_add
 * and col_out exactly col_add; no other output may overlap an operand.
 * ws: bto_pass_workspace_bytes(ops, m, n) bytes. */
enum {
    BTO_PASS_ROWDOT = 1,
    BTO_PASS_COLSUM = 2,
    BTO_PASS_STORE = 4,
    BTO_PASS_CONTRACT = 8,
    BTO_PASS_CHAIN = 16
};
typedef struct {
    int ops;                      /* BTO_PASS_* flags */
    int64_t m, n;
    const double *A;
    int64_t lda;
    double *B;                    /* STORE only */
    int64_t ldb;
    const double *u1, *v1, *u2, *v2;   /* STORE, CONTRACT: u m, v n */
    const double *x;              /* ROWDOT weights, n */
    const double *y;              /* COLSUM weights, m */
    double *row_out;
    double row_scale;
    const double *row_add;
    double row_add_scale;
    double *col_out;
    double col_scale;
    const double *col_add;
    double col_add_scale;
} bto_pass_desc;

size_t bto_pass_workspace_bytes(int ops, int64_t m, int64_t n);
bto_status bto_pass(const bto_pass_desc *desc, void *ws, size_t ws_bytes, hipStream_t stream);

/* AXPYDOT (Table I, whose scalar result is named beta there):
 *   z <- w - alpha v ;  r <- z^T u.
 * Vectors of length n; r points to ONE double in device memory.  z may be
 * exactly w.  Fused: one sweep writes z and the dot partial sums. */
bto_status bto_axpydot(int64_t n, double alpha, const double *w, const double *v,
                       const double *u, double *z, double *r,
                       void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* r <- x^T y: the dot product of AXPYDOT's second statement on its own
 * (Table I), with the same pairwise-order partial sums and fixed-order
 * finish.  Length n; r points to ONE double in device memory.
 * ws: bto_dot_workspace_bytes(n) bytes. */
size_t bto_dot_workspace_bytes(int64_t n);
bto_status bto_dot(int64_t n, const double *x, const double *y, double *r,
                   void *ws, size_t ws_bytes, hipStream_t stream);

/* out <- coef[0] x[0] + coef[1] x[1] + ... + coef[count-1] x[count-1], added
 * left to right, in one pass: the scaled vector sums of a statement fused
 * (Section III-E), for the spec compiler.  count is 1 to 8; x and coef are
 * HOST arrays of count entries (device vector pointers, scalars); vectors
 * of length n.  out may be exactly one of the x[k]; no other overlap. */
bto_status bto_lincomb(int64_t n, int count, const double *const *x, const double *coef,
                       double *out, hipStream_t stream);

/* WAXPBY (Table I):  w <- alpha x + beta y.  Length n; w may be exactly x
 * or exactly y.  Unfused: scal into a temporary, then axpy. */
bto_status bto_waxpby(int64_t n, double alpha, const double *x, double beta,
                      const double *y, double *w,
                      void *ws, size_t ws_bytes, bto_form form, hipStream_t stream);

/* VADD (Table I):  x <- w + y + z, evaluated as (w + y) + z.  Length n; x
 * may be exactly w, y or z.  Unfused: two vector adds through a temporary. */
bto_status bto_vadd(int64_t n, const double *w, const double *y, const double *z,
                    double *x, void *ws, size_t ws_bytes, bto_form form,
                    hipStream_t stream);

/* ---- batched execution -----------------------------------------------------
 * Many independent GEMVER, BICGK and ATAX instances (square or not, of
 * uneven size, n <= 2048 columns each) run in one persistent launch.  Each
 * instance has the operands and semantics of its entry point above; `in`
 * and `out` list the vectors in the entry point's argument order:
 *   GEMVER  in = {u1, v1, u2, v2, y, z}, out = {x, w}, B (may be A)
 *   BICGK   in = {p, r},                 out = {q, s}
 *   ATAX    in = {x},                    out = {y}
 * Instances may share inputs (the same A for many requests); an output may
 * not overlap any operand of any instance, other than B == A of its own.
 * Matrices and vectors must be 16-byte aligned with even leading
 * dimensions.  One workgroup computes a whole instance, in an order fixed by
 * the instance and the workgroup size, so for a given workgroup size the
 * results do not depend on the grid, the graph, the other instances or
 * which workgroup takes the instance (another workgroup size or tile size
 * adds the same terms in another fixed order).  A fused instance larger
 * than config.split_bytes is cut into row tiles taken by several
 * workgroups: each tile writes its partial column sums to the plan's
 * scratch, the last tile to finish adds them in tile order, and GEMVER's
 * second-sweep tiles (queued after every first-sweep tile) start once that
 * instance's x is complete.
 *
 * bto_batch_plan_create validates every instance, orders the work by
 * decreasing size and copies the table to device memory (the plan owns that
 * memory, and a scratch area for unfused ATAX temporaries and tile
 * partials, until it is destroyed).
 * With use_graph set, the launch (a queue reset and the persistent kernel)
 * is captured once in a HIP graph.  bto_batch_plan_launch enqueues the
 * whole batch on `stream` and allocates nothing; successive launches of one
 * plan must not overlap (they share the plan's queue counter).  This is the
 * GPU counterpart of the paper's generated kernel partitioning its loops
 * over threads (Sections III-C, IV-D), applied across instances. */
typedef struct {
    bto_kernel kind;          /* BTO_K_GEMVER, BTO_K_BICGK or BTO_K_ATAX */
    bto_form form;
    int64_t m, n, lda, ldb;   /* ldb: GEMVER only */
    double alpha, beta;       /* GEMVER only */
    const double *A;
    double *B;                /* GEMVER only */
    const double *in[6];
    double *out[2];
} bto_batch_desc;

typedef struct {
    int threads;       /* workgroup size: 256 or 512 (0 = default 512) */
    int wgs_per_cu;    /* persistent workgroups per compute unit, 1..8 (0 = default 2;
                          more than can be resident at once only queue) */
    int use_graph;     /* capture the launch in a HIP graph */
    int64_t split_bytes;  /* fused instances whose matrix is larger are cut into
                             row tiles of about this many bytes, run by several
                             workgroups (0 = default 16 MiB; negative = never) */
} bto_batch_config;

typedef struct bto_batch_plan bto_batch_plan;

/* Largest column count a batched instance may have. */
int64_t bto_batch_max_n(void);

/* Doubles of plan scratch the instances need (unfused ATAX temporaries and
 * the column-sum partials of split instances) under `config` (may be NULL
 * for the defaults); only kind, form, m and n are read.  -1 for a negative
 * count or size. */
int64_t bto_batch_scratch_doubles(const bto_batch_desc *descs, int count,
                                  const bto_batch_config *config);
bto_status bto_batch_plan_create(const bto_batch_desc *descs, int count,
                                 const bto_batch_config *config, bto_batch_plan **plan);

/* A plan that is filled later, for loops that run a different set of
 * instances each step (continuous batching in a server).  `capacity` is the
 * most instances one refill may hold; `scratch_doubles` the scratch area
 * (bto_batch_scratch_doubles of the largest set of instances it will hold).
 * The plan starts with no instances. */
bto_status bto_batch_plan_create_empty(int capacity, int64_t scratch_doubles,
                                       const bto_batch_config *config, bto_batch_plan **plan);

/* Replace the plan's instances.  The instances are validated as in
 * bto_batch_plan_create (BTO_ERR_INVALID_ARG / BTO_ERR_ALIAS, and
 * BTO_ERR_INVALID_ARG for more than `capacity`, BTO_ERR_WORKSPACE for more
 * scratch than the plan has); on error the plan keeps its previous
 * instances.  The new table is copied to the device asynchronously on
 * `stream` through pinned memory the plan owns, so it takes effect for
 * launches enqueued on the same stream afterwards; the host call waits only
 * until the previous refill's copy has been read.  Refills and launches of
 * one plan must all be issued on one stream.  No device memory is
 * allocated. */
bto_status bto_batch_plan_reset(bto_batch_plan *plan, const bto_batch_desc *descs, int count,
                                hipStream_t stream);
bto_status bto_batch_plan_launch(bto_batch_plan *plan, hipStream_t stream);

/* Wait for `stream` and report whether the plan's last launch completed
 * its waits: a second-sweep tile waits a bounded time for its instance's
 * first sweep, and BTO_ERR_HIP here means one gave up (the launch's results
 * are then not valid).  Synchronizes; for tests and diagnostics. */
bto_status bto_batch_plan_check(bto_batch_plan *plan, hipStream_t stream);

/* The same check without waiting: enqueue on `stream` a copy of the plan's
 * error word (nonzero when a bounded wait of the launch before it gave up)
 * into `dst`, one int of caller-owned memory (pinned host memory from
 * hipHostMalloc, or device memory).  The value is there once the stream has
 * passed the copy, e.g. when an event recorded after it completes.  For
 * servers that check every launch without synchronizing. */
bto_status bto_batch_plan_error_async(bto_batch_plan *plan, int *dst, hipStream_t stream);
bto_status bto_batch_plan_destroy(bto_batch_plan *plan);

/* ---- tiled batches ---------------------------------------------------------
 * The same fused GEMVER and BiCGK instances (descriptors as above; ATAX and
 * the unfused form are refused with BTO_ERR_UNSUPPORTED) cut into
 * short-lived workgroup tiles instead of one workgroup per instance: a tile
 * is one sweep of one instance over a band of rows and a block of columns.
 * The tiles form five launches, each of a kernel specialised for its tile
 * shape: the first sweeps (GEMVER's B = A + u1 v1^T + u2 v2^T stored with
 * partial column sums of B^T y, and BiCGK's row dots and column sums in one
 * pass, each tile taking its instance's operations and band height), a
 * launch that adds each instance's partial sums in a fixed order (BiCGK's q
 * and s, GEMVER's x = beta B^T y + z), GEMVER's second sweeps (w = alpha B
 * x) of narrow and of wide matrices, and the sums of w.  The kernel boundaries
 * order the phases, so no tile waits for another.  Each result depends only
 * on its own instance and the plan's configuration (a fixed tile and
 * summation order), not on the other instances or the launch; it rounds
 * differently from the persistent plan's.  This is the loop partition of
 * Section III-C (row bands across workgroups, columns across lanes)
 * applied to many instances at once; the configuration holds the
 * partition's parameters that the search of Section IV tunes here. */
typedef struct {
    int store_shape;   /* tile shape (bto_tiled_shape) of GEMVER's first sweeps */
    int narrow_shape;  /* of the read-only sweeps of matrices at most narrow_n wide */
    int wide_shape;    /* of the read-only sweeps of wider matrices */
    int narrow_n;      /* column count up to which narrow_shape is used (>= 0) */
    int store_rb;      /* rows per band of GEMVER's first sweeps */
    int bicgk_rb;      /* rows per band of BiCGK's sweeps (in the first launch, with
                          store_shape; at most 64 rows per wave) */
    int read_rb;       /* rows per band of the read-only sweeps (at most 64 rows per
                          wave: read_rb / waves_down <= 64) */
    int wgs_per_cu;    /* 0: one workgroup per tile; 1..16: that many persistent
                          workgroups per compute unit in each launch, stepping
                          through the group's tiles */
    int use_graph;     /* capture the launches in a HIP graph (0 or 1) */
} bto_tiled_config;

typedef struct bto_tiled_batch bto_tiled_batch;

/* The default configuration (the tuned one), for callers to adjust. */
void bto_tiled_config_default(bto_tiled_config *config);
/* The tile shapes a configuration may name: a workgroup of waves_across x
 * waves_down waves, kv 16-byte pairs per lane (a block of
 * 128 * kv * waves_across columns), depth rows of loads in flight per wave.
 * Band heights must be multiples of waves_down. */
int bto_tiled_shape_count(void);
bto_status bto_tiled_shape(int shape, int *kv, int *depth, int *waves_across, int *waves_down);

/* bto_tiled_batch_create validates the instances as bto_batch_plan_create
 * does, then allocates and fills the plan's device tables and partial-sum
 * scratch (for the defaults: column sums 1/16 of each GEMVER matrix and
 * 1/64 of each BiCGK matrix, row dots 1/256 of each matrix), which the plan
 * owns until it is destroyed.
 * With use_graph set the launches are captured once in a HIP graph.
 * bto_tiled_batch_create_config does the same under `config` (NULL: the
 * defaults; an invalid configuration gives BTO_ERR_INVALID_ARG).
 * bto_tiled_batch_launch enqueues the batch on `stream` and allocates
 * nothing; launches of one plan must not overlap (they share its scratch). */
bto_status bto_tiled_batch_create(const bto_batch_desc *descs, int count, int use_graph,
                                  bto_tiled_batch **plan);
bto_status bto_tiled_batch_create_config(const bto_batch_desc *descs, int count,
                                         const bto_tiled_config *config,
                                         bto_tiled_batch **plan);

/* A tiled plan that is filled later, for loops that run a different set of
 * instances each step (continuous batching in a server).  It holds tables
 * and scratch for `capacity` instances of either kind of at most max_m rows
 * and max_n columns (max_n <= bto_batch_max_n()).  With use_graph the graph
 * is captured once and replayed after every refill: its launches have a
 * fixed number of persistent workgroups that read each group's tile count
 * from the device, so config->wgs_per_cu must then be 1..16 (0 is refused).
 * Without a graph, each launch is sized from the last refill's tiles and
 * launches of empty groups are skipped.  NULL takes the defaults, with 2
 * workgroups per compute unit if the defaults have one per tile.  The plan
 * starts with no instances. */
bto_status bto_tiled_batch_create_empty(int capacity, int64_t max_m, int64_t max_n,
                                        const bto_tiled_config *config,
                                        bto_tiled_batch **plan);

/* Replace a refillable plan's instances.  They are validated as in
 * bto_tiled_batch_create (BTO_ERR_INVALID_ARG / BTO_ERR_ALIAS /
 * BTO_ERR_UNSUPPORTED, BTO_ERR_INVALID_ARG for more than `capacity`
 * instances or a plan not made by _create_empty, BTO_ERR_WORKSPACE for more
 * tiles or scratch than the plan holds); on error the plan keeps its
 * previous instances.  The tables are copied to the device asynchronously
 * on `stream` through pinned memory the plan owns, so they take effect for
 * launches enqueued on the same stream afterwards; the host call waits only
 * until the previous refill's copy has been read.  Refills and launches of
 * one plan must all be issued on one stream.  No device memory is
 * allocated. */
bto_status bto_tiled_batch_reset(bto_tiled_batch *plan, const bto_batch_desc *descs, int count,
                                 hipStream_t stream);
bto_status bto_tiled_batch_launch(bto_tiled_batch *plan, hipStream_t stream);
bto_status bto_tiled_batch_destroy(bto_tiled_batch *plan);

/* ---- measurement support ------------------------------------------------
 * Per-kernel timing with HIP events recorded on the stream each kernel is
 * launched on.  While enabled, every kernel the library launches is
 * bracketed by a pair of events.  bto_timing_collect() waits for the
 * recorded events and folds them into per-kernel totals; bto_timing_get()
 * reads total milliseconds and launch count of the idx-th kernel name
 * (idx < bto_timing_count()).  Names stay valid until bto_timing_reset(). */
bto_status bto_timing_enable(int enable);
/* Time only the launches named `name` (NULL or "" = all): fewer events in
 * the stream when one kernel is the subject. */
bto_status bto_timing_only(const char *name);
bto_status bto_timing_collect(void);
int bto_timing_count(void);
bto_status bto_timing_get(int idx, const char **name, int64_t *launches,
                          double *total_ms);
void bto_timing_reset(void);

/* ---- tuning --------------------------------------------------------------
 * Every matrix sweep the entry points launch belongs to a slot (for example
 * pass 1 of fused GEMVER, or the unfused dgemv 'N').  A slot's tile
 * configuration is (shape, rb, rev): `shape` picks one of the compiled tile
 * shapes (bto_tune_shape describes it: 16-byte column pairs per lane, rows
 * of loads in flight per wave, waves across the columns and down the rows
 * of a workgroup), `rb` is the number of rows per workgroup band and `rev`
 * walks the bands in reverse.  These are the GPU counterparts of the
 * partitioning and thread-count choices of Sections III-C and IV-D: they
 * change speed, never results beyond summation order.  bto_tune_set
 * returns BTO_ERR_INVALID_ARG for a configuration the slot cannot run; the
 * table is process-wide and guarded by a lock.  The last two slots are not
 * tile sweeps: "atax_rowres" and "bicgk_rowres" pick the workgroup size
 * (shape 256, 512 or 1024; rb = rev = 0) of the row-resident fused ATAX and
 * BiCGK sweeps, which hold whole rows on chip; for "bicgk_rowres" shape 0
 * selects the tile sweep of slot "bicgk_fused" instead. */
int bto_tune_slot_count(void);
const char *bto_tune_slot_name(int slot);
int bto_tune_slot_ops(int slot);
bto_status bto_tune_get(int slot, int *shape, int *rb, int *rev);
bto_status bto_tune_set(int slot, int shape, int rb, int rev);

/* Configurations are kept per size bucket: problems are grouped by
 * max(m, n) into <= 256, <= 512, ..., <= 16384 and larger
 * (bto_tune_bucket_count() buckets; bto_tune_bucket(size) gives the index).
 * The _for calls address the bucket of a problem with max(m, n) = size; size
 * 0 addresses every bucket (set) or the 16384 bucket (get), which is what
 * bto_tune_set and bto_tune_get do. */
bto_status bto_tune_get_for(int slot, int64_t size, int *shape, int *rb, int *rev);
bto_status bto_tune_set_for(int slot, int64_t size, int shape, int rb, int rev);
int bto_tune_bucket_count(void);
int bto_tune_bucket(int64_t size);
bto_status bto_tune_shape(int shape, int *kv, int *depth, int *waves_across,
                          int *waves_down);

/* Bandwidth probes, used to calibrate hardware byte counters and to
 * measure the achievable HBM ceiling: dst <- src (copy), *out <- sum(src)
 * (read; out is one device double, the sum order is fixed), and
 * a <- b + s*c (triad).  n doubles each. */
bto_status bto_probe_copy(const double *src, double *dst, int64_t n, hipStream_t stream);
bto_status bto_probe_read(const double *src, int64_t n, double *out, void *ws,
                          size_t ws_bytes, hipStream_t stream);
bto_status bto_probe_triad(double *a, const double *b, const double *c, double s,
                           int64_t n, hipStream_t stream);
size_t bto_probe_read_workspace_bytes(int64_t n);

/* ---- synthetic inputs ------------------------------------------------------
 * Fill a rows x cols block (leading dimension ld, device memory) with element
 * (i, j) = element offset + i*cols + j of a SplitMix64 stream whose state
 * starts at `state` (Steele, Lea and Flood 2014): kind 0 gives doubles
 * uniform on [-1, 1), kind 1 integers uniform on [lo, hi].  Bit-identical to
 * the package's host generator; used to build large benchmark workloads in
 * place.  Returns BTO_ERR_INVALID_ARG for bad sizes or kinds. */
bto_status bto_synth_fill(double *out, int64_t rows, int64_t cols, int64_t ld, uint64_t state,
                          int64_t offset, int kind, int lo, int hi, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* BTO_H */
