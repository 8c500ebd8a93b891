/*
 * tqr -- tiled QR factorisation on one AMD MI355X (gfx950).
 *
 * The method is the tiled QR of Buttari, Langou, Kurzak and Dongarra,
 * "Parallel Tiled QR Factorization for Multicore Architectures":
 * the matrix is cut into b x b tiles (Sec. 3.1), factorised by four tile
 * kernels -- GEQRT (their DGEQT2), LARFB (DLARFB), TSQRT (DTSQT2) and
 * SSRFB (DSSRFB) -- in the order of Algorithm 1, and the tasks are run out of
 * order as their dependencies allow, highest priority first (Sec. 3.3).
 * Here one persistent GPU kernel runs that task graph: dependency counters
 * and priority-ordered ready queues live in device memory.
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Every matrix, T array and workspace pointer is DEVICE memory owned by
 *    the caller.  The library never allocates or frees device memory in a
 *    call; the workspace size comes from tqr_workspace_bytes().
 *  - Matrices are column-major with a leading dimension (lda >= max(1,m)).
 *  - Tile size b (tile_b) and inner block ib (inner_ib): supported pairs are
 *    b in {16, 32, 64, 128, 256} and ib in {16, 32, 64} with ib <= b,
 *    b % ib == 0 and ib * (b + ib) <= 9216 (the panel of a tile kernel is
 *    staged on chip).  ib == b is the paper's unblocked tile kernel with a
 *    b x b T (Sec. 3.1); ib < b applies each tile's reflectors in blocks of ib.
 *  - m >= n is required (the paper assumes q <= p, Sec. 3.2; least squares
 *    needs it).  m == 0 or n == 0 returns TQR_OK at once.
 *  - Sizes that are not multiples of b are handled by zero-padded edge tiles:
 *    padded rows give reflector entries that are exactly zero and padded
 *    columns give tau = 0, so the m x n result is unchanged.
 *  - Argument errors are reported synchronously, before anything is
 *    enqueued: the return value is -i when the i-th argument (1-based, in
 *    signature order) is illegal, as LAPACK's convention; nothing is printed.
 *    HIP errors return TQR_EDEVICE; tqr_last_error_string() describes the
 *    last error of the calling thread.
 *  - All work is enqueued on `stream`; calls return without synchronising.
 *    Calls on different streams with disjoint buffers are independent.
 *  - Arithmetic is IEEE FP64; NaN and Inf in the input propagate and are
 *    not detected.
 */
#ifndef TQR_H
#define TQR_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int tqr_status;
#define TQR_OK 0
#define TQR_EDEVICE (-1000)   /* a HIP call failed; see tqr_last_error_string() */
#define TQR_EABORTED (-1001)  /* device-side abort flag or wait time-out (tqr_factor_ex) */
#define TQR_ESCRATCH (-1002)  /* the problem needs more than the fixed scratch of tqr_factor_noalloc */

/* Number of doubles of the T array for an m x n factorisation: p*q slots of
 * ib x b, p = ceil(m/b), q = ceil(n/b).  Slot (i,k) (0-based tile indices)
 * starts at element ((k*p) + i) * ib * b and holds, column-major with
 * leading dimension ib, the ib x ib upper-triangular T of every inner block
 * s at columns s*ib .. s*ib+ib-1: the compact WY form
 * H_{s*ib} ... H_{s*ib+ib-1} = I - V_s T_s V_s^T of the block's reflectors
 * (Sec. 2.1).  Only slots with i >= k are written.  Returns -1 for illegal
 * sizes. */
int64_t tqr_t_elems(int64_t m, int64_t n, int tile_b, int inner_ib);

/* Bytes of device workspace needed by tqr_factor (nrhs = 0), tqr_apply_qt /
 * tqr_apply_q and tqr_solve_ls (nrhs right-hand sides).  Returns -1 for
 * illegal sizes. */
int64_t tqr_workspace_bytes(int64_t m, int64_t n, int64_t nrhs, int tile_b, int inner_ib);

/* QR factorisation A = QR by tiles (Sec. 3.1, Algorithm 1).
 *   m, n     : rows, columns, m >= n >= 0.
 *   A        : device, m x n column-major, leading dimension lda.  On exit the
 *              upper triangle of the leading n rows holds R; below it are the
 *              tiled Householder vectors: V_kk strictly below the diagonal of
 *              each diagonal tile (unit diagonal implicit) and the full V_ik
 *              in each tile below (the identity block on top of it is
 *              implicit, Sec. 3.1).  They are only meaningful together with
 *              T and the same tile_b / inner_ib; they are not LAPACK's V.
 *   T        : device, tqr_t_elems() doubles, written (see tqr_t_elems).
 *   work     : device workspace of at least tqr_workspace_bytes(m,n,0,..)
 *              bytes; contents on entry are ignored, on exit undefined.
 *   stream   : HIP stream the work is enqueued on.
 * Errors: -1 m<0 or m<n, -2 n<0, -3 A null, -4 lda, -5 tile_b, -6 inner_ib,
 * -7 T null, -8 work null, -9 work_bytes too small. */
tqr_status tqr_factor(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib,
                      double *T, void *work, int64_t work_bytes, hipStream_t stream);

/* Execution options for tqr_factor_ex. */
typedef struct tqr_options {
    int32_t struct_size;       /* sizeof(tqr_options) */
    int32_t workgroups;        /* persistent workers; 0 = one per resident slot */
    int32_t mode;              /* TQR_MODE_PERSISTENT or TQR_MODE_SERIAL */
    int32_t policy;            /* TQR_POLICY_PAPER, TQR_POLICY_LOOKAHEAD or TQR_POLICY_COLUMN (the
                                  policy of the calls that take no options) */
    int64_t *trace;            /* device, 8 int64 per task or NULL: taken, acquired,
                                  body done, released (device constant-rate clock
                                  ticks), workgroup, XCD, the wave's
                                  HW_ID register (CU/SE ids), and 1 if the
                                  task ran as the continuation of the worker's
                                  previous task (0 if taken from a queue) */
    const volatile int32_t *abort_flag; /* host-mapped or device int polled while
                                           waiting for work; nonzero aborts; or NULL */
    int32_t *status;           /* device int or NULL: 0 done, TQR_EABORTED */
    int64_t timeout_ticks;     /* per-wait bound in device clock ticks; 0 = 2 s */
    void *event_begin;         /* hipEvent_t recorded on `stream` right before the  */
    void *event_end;           /* scheduler launch and right after it, or NULL     */
    int32_t precision;         /* TQR_PRECISION_FP64 (0, default), TQR_PRECISION_FP32_UPDATES or
                                  TQR_PRECISION_BF16_UPDATES */
    int32_t reserved;          /* 0 */
} tqr_options;

#define TQR_MODE_PERSISTENT 0  /* one launch; tasks run out of order as the graph allows */
#define TQR_MODE_SERIAL 1      /* one launch per task, in Algorithm 1 order (reference order) */
#define TQR_POLICY_PAPER 0     /* ready tasks by kind: GEQRT > TSQRT > LARFB > SSRFB (Sec. 3.3) */
#define TQR_POLICY_LOOKAHEAD 1 /* as PAPER, but updates of the next panel's tile column first */
#define TQR_POLICY_COLUMN 2    /* GEQRT > TSQRT > LARFB/SSRFB ordered by the distance of their tile
                                  column from the next panel (the later of step k+1 and the GEQRT
                                  started last; nearer first, six levels); on grids at least as
                                  wide as tall, one worker in four takes the farthest first */
#define TQR_PRECISION_FP64 0         /* every kernel in FP64 */
#define TQR_PRECISION_FP32_UPDATES 1 /* LARFB and SSRFB (the trailing updates, nearly all the
                                        flops) on the FP32 matrix cores; GEQRT/TSQRT (norms,
                                        reflectors, T) in FP64; inner_ib must be 16.  The
                                        factor is then accurate to FP32 rounding: a starting
                                        point for FP64 refinement (tqr_solve_ls_mixed). */
#define TQR_PRECISION_BF16_UPDATES 2 /* as TQR_PRECISION_FP32_UPDATES, with the two large products of
                                        LARFB/SSRFB taking BF16 operands (V, the strip, and W after
                                        op(T)) and accumulating in FP32 on the BF16 matrix cores;
                                        inner_ib 16 and tile_b 64, 128 or 256.  The factor is
                                        accurate to BF16 rounding (about 4e-3 relative). */

/* tqr_factor with explicit execution options (argument errors as
 * tqr_factor; -11 for a bad options struct). */
tqr_status tqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib,
                         double *T, void *work, int64_t work_bytes, hipStream_t stream,
                         const tqr_options *options);

/* B <- Q^T B with Q from tqr_factor (the DORMQR analogue that the paper's
 * Sec. 5 names as future work): for k = 0..: LARFB with (V_kk, T_kk) on row
 * tile k of B, then for i > k the SSRFB form with (V_ik, T_ik) on row tiles
 * (k, i) -- the factorisation's own transformations in its own order.
 *   A, T : the output of tqr_factor with the same m, n, tile_b, inner_ib.
 *   B    : device, m x nrhs column-major, leading dimension ldb, in place.
 * Errors: -1 m, -2 n, -3 nrhs<0, -4 A null, -5 lda, -6 T null, -7 tile_b,
 * -8 inner_ib, -9 B null, -10 ldb, -11 work null, -12 work_bytes. */
tqr_status tqr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                        const double *T, int tile_b, int inner_ib, double *B, int64_t ldb,
                        void *work, int64_t work_bytes, hipStream_t stream);

/* B <- Q B: the transformations of tqr_apply_qt transposed, in reverse
 * order.  Q [I_n; 0] is the thin Q.  Arguments and errors as tqr_apply_qt. */
tqr_status tqr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                       const double *T, int tile_b, int inner_ib, double *B, int64_t ldb,
                       void *work, int64_t work_bytes, hipStream_t stream);

/* The thin Q of the factorisation, formed explicitly: Q[0:m, 0:n] <- Q [I_n; 0]
 * (what LAPACK's DORGQR returns; Sec. 5 lists the Q-forming and Q-applying
 * routines as the natural companions of the tiled factorisation).  Q is
 * filled with [I_n; 0] and the transformations of tqr_apply_q are applied.
 *   A, T : the output of tqr_factor with the same m, n, tile_b, inner_ib.
 *   Q    : device, m x n column-major, leading dimension ldq; written.
 *   work : at least tqr_workspace_bytes(m, n, n, tile_b, inner_ib) bytes.
 * Errors: -1 m, -2 n (also n > 65535), -3 A null, -4 lda, -5 T null,
 * -6 tile_b, -7 inner_ib, -8 Q null, -9 ldq, -10 work null, -11 work_bytes. */
tqr_status tqr_form_q(int64_t m, int64_t n, const double *A, int64_t lda, const double *T, int tile_b,
                      int inner_ib, double *Q, int64_t ldq, void *work, int64_t work_bytes, hipStream_t stream);

/* Least squares min ||A X - B||_F for m >= n (the problem of Sec. 2.1 solved
 * with the tiled factorisation, as LAPACK's dgels does with dgeqrf):
 * factor A (overwritten as by tqr_factor, T written), B <- Q^T B, then
 * X = R^{-1} (Q^T B)[0:n] by tiled back substitution; X overwrites
 * B[0:n, :] and B[n:m, :] holds the residual's coordinates in Q's complement.
 *   d_info : device int, written 0, or k > 0 when R(k,k) (1-based) is
 *            exactly zero (then B[0:n,:] is unspecified), as dgels.
 * Errors: -1 m, -2 n, -3 nrhs, -4 A null, -5 lda, -6 B null, -7 ldb,
 * -8 tile_b, -9 inner_ib, -10 T null, -11 work null, -12 work_bytes,
 * -13 d_info null. */
tqr_status tqr_solve_ls(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                        int tile_b, int inner_ib, double *T, void *work, int64_t work_bytes,
                        int32_t *d_info, hipStream_t stream);

/* tqr_solve_ls with execution options (a serving loop runs several solves
 * at once and sizes each one's worker count).  The options apply to all
 * three phases (factorisation, Q^T B, back substitution): workgroups,
 * policy, abort flag, wait bound, and status (set by the factorisation, then
 * overwritten only by a later phase's TQR_EABORTED); event_begin / event_end
 * bracket the whole solve; trace is ignored; mode must be
 * TQR_MODE_PERSISTENT.  Errors as tqr_solve_ls; -15 for bad options. */
tqr_status tqr_solve_ls_ex(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                           int tile_b, int inner_ib, double *T, void *work, int64_t work_bytes,
                           int32_t *d_info, hipStream_t stream, const tqr_options *options);

/* ---- Mixed-precision least squares with FP64 refinement ----
 * min ||A X - B||_F for m >= n (the least-squares problem that QR solves,
 * Sec. 2.1).  A copy of A is factorised with the trailing updates on the
 * FP32 matrix cores (TQR_PRECISION_FP32_UPDATES; options may ask for
 * TQR_PRECISION_BF16_UPDATES or TQR_PRECISION_FP64 instead); the norms,
 * reflectors and T stay FP64.  Then,
 * for each right-hand side, CGLS in FP64 on min ||(A R^{-1}) y - b||,
 * x = R^{-1} y, from x = 0, with R the factor's triangle as a right
 * preconditioner: every product with A and A^T uses the caller's FP64 A, and
 * A R^{-1} is orthogonal up to the factor's rounding, so each iteration cuts
 * the error by about cond(A) times the factor's relative accuracy, and the
 * iteration still converges (more slowly) where that product exceeds one.
 * The iteration of a column stops when its backward-error estimate
 *     eta = ||R^{-T} A^T r|| / (||A||_F ||x||)          (r = b - A x)
 * (Karlson and Walden's estimate with R in place of the triangle of
 * [A; mu I]) is at most TQR_REFINE_ETA_TOL, when three iterations in a row
 * have not halved ||R^{-T} A^T r|| (rounding limits it), or after
 * `iterations`.  The residual r is recomputed as b - A x in FP64 at every
 * iteration (the recurrence's r drifts from it by rounding).
 * Everything runs on the stream; the stopping test is evaluated on the
 * device.  A and B are not modified.
 *   X       : device, n x nrhs column-major (ldx >= max(1, n)), written.
 *   T       : device, tqr_t_elems(m, n, tile_b, 16) doubles, written.
 *   work    : tqr_ls_mixed_workspace_bytes(m, n, nrhs, tile_b) bytes.
 *   iterations: the most CGLS iterations per right-hand side (0..200; 0
 *             leaves X = 0).
 *   d_info  : device int: 0, or k > 0 when R(k,k) is exactly zero.
 *   d_stats : device array of nrhs tqr_refine_stats, written, or NULL.
 * inner_ib is 16.  Errors: -1 m, -2 n, -3 nrhs, -4 A null, -5 lda, -6 B null,
 * -7 ldb, -8 X null, -9 ldx, -10 tile_b (64, 128 or 256), -11 iterations,
 * -12 T null, -13 work null, -14 work_bytes, -15 d_info null, -17 options. */
#define TQR_REFINE_ETA_TOL 1e-15
#define TQR_REFINE_CONVERGED 1       /* eta <= TQR_REFINE_ETA_TOL (or a zero gradient) */
#define TQR_REFINE_STAGNATED 2       /* three iterations without halving ||R^{-T} A^T r|| */
#define TQR_REFINE_MAX_ITERATIONS 3  /* the iteration limit was reached */
#define TQR_REFINE_BREAKDOWN 4       /* A R^{-1} p == 0 (a singular R) */
typedef struct tqr_refine_stats {
    int32_t iterations;  /* CGLS iterations applied */
    int32_t stop;        /* TQR_REFINE_* */
    double eta;          /* the estimate at the last test, or -1 if none */
} tqr_refine_stats;
int64_t tqr_ls_mixed_workspace_bytes(int64_t m, int64_t n, int64_t nrhs, int tile_b);
tqr_status tqr_solve_ls_mixed(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                              int64_t ldb, double *X, int64_t ldx, int tile_b, int iterations, double *T, void *work,
                              int64_t work_bytes, int32_t *d_info, tqr_refine_stats *d_stats, hipStream_t stream,
                              const tqr_options *options);

/* ---- Batched factorisation: many independent problems in one launch ----
 * Each problem is factorised exactly as tqr_factor does it (the tiled
 * algorithm of Sec. 3.1, Algorithm 1) with its own tile size and inner block.
 * One persistent launch; a workgroup takes the next problem from a counter,
 * converts it to tiles, runs its tasks in the order of Algorithm 1 and
 * converts it back, so problems are independent of the schedule and of each
 * other (bitwise).  Problems are taken in array order: put the largest
 * first. */
typedef struct tqr_batch_problem {
    int64_t m, n, lda;   /* m >= n >= 0, lda >= max(1, m) */
    double *A;           /* device, column-major; overwritten as by tqr_factor */
    double *T;           /* device, tqr_t_elems(m, n, tile_b, inner_ib) doubles, written */
    int32_t tile_b;      /* with inner_ib one of 16/16, 32/16, 32/32, 64/16, 64/32, 64/64, 128/16, 128/32 */
    int32_t inner_ib;    /* 16, 32 or 64; 0 means 16 */
    int64_t work_offset; /* byte offset of the problem's tiles in work: set by tqr_batch_plan */
} tqr_batch_problem;

/* Host-side plan: checks every problem and sets its work_offset.  Returns
 * the workspace bytes that tqr_factor_batched needs, or -1 (count < 0),
 * -2 (problems null, or a problem with m < n, n < 0, lda < max(1, m), a
 * null A or T with m*n > 0, or an unsupported (tile_b, inner_ib): the
 * message names the index). */
int64_t tqr_batch_plan(int64_t count, tqr_batch_problem *problems);

/* Factorises the planned problems.  d_problems: device copy of the planned
 * array (count entries); work: tqr_batch_plan's bytes; precision:
 * TQR_PRECISION_FP64, or TQR_PRECISION_FP32_UPDATES (every problem's LARFB
 * and SSRFB on the FP32 matrix cores, as tqr_factor_ex does it; inner_ib 16
 * only); d_status (optional device int): 0, or i+1 when problem i's
 * (tile_b, inner_ib) is not supported for the precision (it is skipped).
 * workgroups: 0 for one per resident slot, else at most that many.
 * Enqueued on stream; no host synchronisation, no memset (the launch may be
 * captured in a graph).  Errors: -1 count, -2 d_problems null, -3 work null,
 * -4 work_bytes below 256, -6 workgroups < 0, -7 precision. */
tqr_status tqr_factor_batched(int64_t count, const tqr_batch_problem *d_problems, void *work, int64_t work_bytes,
                              int32_t *d_status, int32_t workgroups, int32_t precision, hipStream_t stream);

/* ---- Factorisation without a workspace argument ----
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Exactly
 * tqr_factor (same kernels, same result bit for bit), with the workspace
 * taken from a fixed device array inside the library instead of an argument:
 * TQR_NOALLOC_SCRATCH_BYTES per GPU, set up on the first call on each device
 * and held until the process ends.  Nothing is allocated or freed in a call
 * (no hipMalloc, no library allocation); the caller still owns A and T.
 * Problems whose tqr_workspace_bytes(m, n, 0, tile_b, inner_ib) exceeds the
 * scratch are rejected with TQR_ESCRATCH before anything is enqueued (for
 * example 3840 x 3840 at tile_b 256 fits, 4096 x 4096 does not).
 * Every call on one GPU uses that GPU's single array: calls that overlap in
 * time on one GPU (different streams, or different host threads without
 * ordering) race and give undefined results; calls on one stream are
 * ordered and safe.
 * Errors: -1 .. -7 as tqr_factor (m, n, A, lda, tile_b, inner_ib, T),
 * TQR_ESCRATCH, TQR_EDEVICE. */
#define TQR_NOALLOC_SCRATCH_BYTES (128ll << 20)
tqr_status tqr_factor_noalloc(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib, double *T,
                              hipStream_t stream);

/* Description of the last error returned to the calling host thread. */
const char *tqr_last_error_string(void);

/* ---- task-graph introspection (host only, no device work) --------------
 * The persistent scheduler runs a closed-form task graph; these expose it so
 * that it can be checked against a hazard analysis of Algorithm 1.
 * Tasks of the factorisation are numbered 0..tqr_graph_tasks()-1.  A task is
 * (kind, i, j, k, strip): kind 0 GEQRT(k), 1 TSQRT(i,k), 2 LARFB(k,j) on
 * column strip `strip` of tile (k,j), 3 SSRFB(i,j,k) on column strip
 * `strip` of tiles (k,j) and (i,j); tile indices 0-based.  Strips are
 * groups of 64 columns of a tile (one strip when b <= 64). */
int64_t tqr_graph_tasks(int64_t p, int64_t q, int tile_b);
int tqr_graph_task(int64_t p, int64_t q, int tile_b, int64_t task, int32_t out[5]);
int tqr_graph_indegree(int64_t p, int64_t q, int tile_b, int64_t task);
/* Writes up to max_out successor task ids; returns the successor count. */
int tqr_graph_successors(int64_t p, int64_t q, int tile_b, int64_t task, int64_t *out, int max_out);

#ifdef __cplusplus
}
#endif

#endif /* TQR_H */
