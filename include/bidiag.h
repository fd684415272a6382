/*
 * bidiag.h -- C ABI of libbidiag: tiled band bidiagonalization on AMD MI355X.
 *
 * Operation (Faverge, Langou, Robert, Dongarra, "Bidiagonalization with
 * Parallel Tiled Algorithms", Sections 3.4 and 3.5): for an m x n matrix A
 * with m >= n and a tile size nb, compute orthogonal Q and P with
 *
 *     B = Q^T A P,     B(i,j) = 0 unless 0 <= j - i <= nb,   rows >= n zero,
 *
 * For m < n the reduction is that of A^T (Section 3.6): A^T = Q' B' P'^T,
 * so A = Q B P^T with Q = P', P = Q' and the lower band form B = B'^T,
 * B(i,j) = 0 unless 0 <= i - j <= nb, columns >= m zero.  The graph is that
 * of A^T, run on A's own storage through transposed tile views.
 *
 * by alternating QR and LQ tile-panel eliminations along a reduction tree:
 *   BiDiag   : QR(1); LQ(1); QR(2); ...; QR(q-1); LQ(q-1); QR(q)   (Section 3.4)
 *   R-BiDiag : QR(p,q); LQ(1); QR(2); ...; LQ(q-1); QR(q)           (Section 3.5)
 * where p = ceil(m/nb), q = ceil(n/nb) and each step uses the tile kernels of
 * Table 1 (GEQRT/TSQRT/TTQRT and UNMQR/TSMQR/TTMQR, Algorithms 2 and 3; the LQ
 * steps use the same kernels on transposed tiles, Algorithm 4).  Trees:
 * FlatTS, FlatTT and Greedy (Section 3.3) and Auto (Section 5).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major FP64 in device memory, leading dimension
 *     lda >= max(1, m).  m and n need not be multiples of nb: the last tile
 *     row/column is handled as if zero-padded (padding is never read or
 *     written in memory).
 *   - All device memory is owned by the caller: matrices, V/T records and
 *     the workspace.  The library allocates no device memory, never frees or
 *     retains a caller's pointer past the call, and keeps no device state
 *     between calls.  A plan owns host memory only: its task graph and a copy
 *     of what the device reads of it (page-locked when a device is present),
 *     which every execution copies into the workspace with an asynchronous
 *     copy on the caller's stream.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL means
 *     the default stream) and is asynchronous: results are valid once the
 *     stream has reached the enqueued work.  No entry point that enqueues
 *     work waits for the device, except the bb_*poll_error and
 *     bb_*last_kernel_ms queries, which say so.
 *   - Return codes: BB_OK (0); -i when argument i (1-based) is invalid, in the
 *     LAPACK convention; a positive BB_E* code for runtime errors.  No C++
 *     exception crosses the ABI.
 *   - Reentrancy: calls with distinct buffers may run concurrently from
 *     several host threads, also with the same plan (an execution only reads
 *     its plan); executions that overlap on one workspace race.  Destroying a
 *     plan waits for the devices it uploaded on (its host copy may still be
 *     the source of an enqueued copy), so it must not race with executions
 *     of that plan.
 */
#ifndef BIDIAG_H
#define BIDIAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define BB_OK        0
#define BB_ENOTSUP   1   /* valid but unsupported request (e.g. nb not in {32,64,128,256}) */
#define BB_EHIP      2   /* a HIP runtime call failed */
#define BB_ETIMEOUT  3   /* the device scheduler's watchdog fired (no progress) */
#define BB_EDAG      4   /* the task graph failed validation on the host */
#define BB_ENOMEM    5   /* host or device allocation for the plan failed */
#define BB_EWORKSPACE 6  /* workspace or V/T buffer smaller than bb_plan_workspace reports */

/* ---- enumerations ------------------------------------------------------ */
/* Reduction trees: Section 3.3 (FlatTS, FlatTT, Greedy) and Section 5 (Auto). */
enum { BB_FLATTS = 0, BB_FLATTT = 1, BB_GREEDY = 2, BB_AUTO = 3 };
/* Algorithms: Section 3.4 (BiDiag), Section 3.5 (R-BiDiag).  BB_QRONLY runs
 * only the tiled QR factorization QR(p,q) of Algorithm 1 (A is overwritten by
 * R, rows >= n zero).  BB_THREESTEP is the three-step reduction of Section
 * 4.5: BiDiag steps QR(k); LQ(k) for k < s, then R-BiDiag on the trailing
 * (p-s) x (q-s) tiles; s is bb_opts.switch_step when positive, else the
 * first k whose trailing tiles satisfy p - k >= delta (q - k) (the
 * BiDiag/R-BiDiag switching point of Section 4.3.4), q if none. */
enum { BB_BIDIAG = 0, BB_RBIDIAG = 1, BB_QRONLY = 2, BB_THREESTEP = 3 };
/* Arithmetic.  BB_F64 computes everything in FP64.  The two other modes keep
 * the matrix, the panels (reflector generation, V and T) in FP64 and run the
 * trailing updates (UNMQR/TSMQR/TTMQR and their LQ twins) on FP32 matrix
 * cores: BB_F64_UPD_F32 rounds the operands to FP32 (RNE), accumulates each
 * product in FP32 and adds it into the FP64 tiles; BB_F64_UPD_SPLIT32 also
 * carries the FP32 rounding error of every operand (x = x_hi + x_lo), forms
 * A_hi B_hi + A_hi B_lo + A_lo B_hi, and accumulates 16-row chunks in FP64.
 * Accuracy: both modes reduce A + dA exactly with ||dA|| of order
 * n eps_32 ||A||.  The split mode is NOT more accurate than BB_F64_UPD_F32:
 * the FP32 matrix-core instruction rounds every product and its 4-term sum
 * to FP32 before the FP64 chunk sum, so the hi x hi term alone carries FP32
 * rounding; the split mode only lowers the Frobenius-norm (orthogonality)
 * drift.  Neither mode is faster than BB_F64 at the measured sizes: panels,
 * which bound the runtime, stay FP64.  All-FP32 data (FP32 matrices and
 * panels) is not provided.  (Section 3.6 notes the tile codes exist in
 * single and double precision; the mixed forms are an extension.) */
enum { BB_F64 = 0, BB_F64_UPD_F32 = 2, BB_F64_UPD_SPLIT32 = 3 };
/* Execution of the task graph: one persistent launch whose workgroups take
 * work units in a precomputed priority order (a list-scheduling simulation
 * on the GPU's workgroups, by bottom level in the task graph) and wait on
 * dependency counters (default), or one
 * launch per topological level of the graph. */
enum { BB_SCHED_PERSISTENT = 0, BB_SCHED_LEVELS = 1 };

typedef struct {
    int    workgroups;   /* workers assumed by Auto and used by the persistent
                            launch; 0 = number of compute units */
    double gamma;        /* Auto parallelism factor (Section 5); 0 = 2.0 */
    int    auto_a;       /* > 0 forces Auto's FlatTS domain size; 0 = per step */
    int    sched;        /* BB_SCHED_* */
    double watchdog_s;   /* persistent scheduler: seconds without progress before
                            BB_ETIMEOUT; 0 = 30 s */
    int    flags;        /* BB_FLAG_* */
    int    switch_step;  /* BB_THREESTEP: > 0 forces the switch step s; 0 = from delta */
    double delta;        /* BB_THREESTEP: switch ratio; 0 = 5 (Section 4.3.4 puts
                            the switching point at 5 to 8) */
} bb_opts;

#define BB_FLAG_TIMING 1  /* record HIP events around the main kernel(s) */
#define BB_FLAG_TRACE  2  /* persistent scheduler: record per-unit timestamps in the
                             workspace (bb_plan_trace); the workspace grows by
                             32 bytes per work unit */

typedef struct bb_plan bb_plan;

typedef struct {
    int32_t p, q, nb;
    int64_t ntasks;          /* kernel invocations in the graph */
    int64_t nunits;          /* scheduled work units (updates split in column strips) */
    int64_t nslots;          /* V/T records (one per panel task) */
    int64_t nlevels;         /* topological levels */
    int64_t count_by_kind[6];/* GEQRT, TSQRT, TTQRT, UNMQR, TSMQR, TTMQR (QR and LQ) */
    double  critical_path;   /* longest path with Table 1 weights, units of nb^3/3 */
    double  total_weight;    /* sum of Table 1 weights over all tasks */
} bb_plan_stats;

/*
 * bb_plan_create -- build the task graph of one reduction (host work only: no
 * device memory and no device work; the host copy of the graph is
 * page-locked when a device is present).  Arguments: out plan (1), m (2),
 * n (3) >= 1 (m < n: the graph of A^T, see above), nb (4) in
 * {32, 64, 128, 256}, tree (5)
 * BB_FLATTS..BB_AUTO, variant (6), prec (7) BB_F64*,
 * opts (8, may be NULL for defaults).  The plan is independent of the data and
 * of lda; it can be executed any number of times.
 */
int bb_plan_create(bb_plan** plan, int64_t m, int64_t n, int nb, int tree, int variant,
                   int prec, const bb_opts* opts);

/* Release a plan (after synchronizing the devices it uploaded its graph on).
 * NULL is ignored. */
void bb_plan_destroy(bb_plan* plan);

/*
 * Bytes of device memory the caller must provide to bb_execute:
 *   vt_bytes : reflector records, one per panel task, FP64 column-major:
 *              V (nb x nb), then nb/16 blocks T_b^T (16 x 16),
 *              where the panel's transformation is Q = Q_0 Q_1 ... with
 *              Q_b = I - V_b T_b V_b^T, V_b = columns 16b..16b+15 of V and T_b
 *              upper triangular (compact WY form blocked by 16 columns).
 *              Kept after the call (Q and P are the products of these records
 *              in task order).
 *   ws_bytes : scheduler state (error flag, ticket and done counters, one
 *              dependency counter per task, the optional trace) followed by
 *              the copy of the task graph that each execution uploads
 *              (tasks, successor lists, unit order) and, for nb = 256, the
 *              panels' scratch (512 KiB per workgroup of a persistent launch,
 *              or per panel of the widest level).  Contents are not kept
 *              between executions.
 */
int bb_plan_workspace(const bb_plan* plan, size_t* vt_bytes, size_t* ws_bytes);

int bb_plan_get_stats(const bb_plan* plan, bb_plan_stats* stats);

/*
 * Export the task graph in program order, for inspection and static checks.
 * tasks: ntasks x 8 int32 {kind, trans, r1, c1, r2, c2, slot, step} with
 * physical tile coordinates (see plan.hpp); pred_off: ntasks+1 offsets into
 * pred_idx.  Pass NULL arrays to query *npred only.
 */
int bb_plan_export(const bb_plan* plan, int32_t* tasks, int32_t* pred_off, int32_t* pred_idx,
                   int64_t* npred);

/*
 * bb_execute -- reduce A in place to its band form B (Sections 3.4/3.5).
 * A (2): device, column-major, lda (3) >= m.  On completion A holds B with
 * exact zeros outside the band.  vt (4) / ws (6): device buffers of at least
 * the sizes from bb_plan_workspace (5, 7).  stream (8): hipStream_t or NULL.
 * Returns after enqueueing; device-side scheduler failures (watchdog) are
 * reported by bb_poll_error after the stream has completed.
 */
int bb_execute(bb_plan* plan, void* A, int64_t lda, void* vt, size_t vt_bytes, void* ws,
               size_t ws_bytes, void* stream);

/*
 * bb_execute_noalloc -- bb_execute without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The scheduler state and
 * the task graph go to a workspace the library holds in a file-scope device
 * array of BB_NOALLOC_WS_MAX bytes, one per device, kept until the process
 * ends; the call itself allocates nothing (no hipMalloc, hipFree or
 * allocating library routine) and records no timing events.  A plan whose
 * bb_plan_workspace ws_bytes exceeds BB_NOALLOC_WS_MAX is rejected with
 * BB_EWORKSPACE (every nb = 256 plan: its panel scratch alone exceeds it).
 * Every call on a device shares that device's array, so
 * calls whose executions overlap on one device (other streams, other
 * threads) race; calls in one stream order do not.  Arguments as
 * bb_execute: plan (1), A (2), lda (3), vt (4), vt_bytes (5), stream (6).
 * Scheduler errors: bb_poll_error with ws = NULL.
 */
#define BB_NOALLOC_WS_MAX (32u << 20)
int bb_execute_noalloc(bb_plan* plan, void* A, int64_t lda, void* vt, size_t vt_bytes, void* stream);

/*
 * bidiag_band -- one-shot form of bb_plan_create + bb_execute with a plan
 * cached inside the library by (m, n, nb, tree, variant, prec, opts).  The
 * cache holds at most 16 plans (least recently used out first; bb_query
 * fills it too) and bb_cache_clear empties it; a plan in use by another
 * thread's call is released when that call returns.
 * Argument numbering: A (1), m (2), n (3), lda (4), nb (5), tree (6),
 * variant (7), prec (8), vt (9), vt_bytes (10), ws (11), ws_bytes (12),
 * opts (13), stream (14).
 */
int bidiag_band(void* A, int64_t m, int64_t n, int64_t lda, int nb, int tree, int variant,
                int prec, void* vt, size_t vt_bytes, void* ws, size_t ws_bytes,
                const bb_opts* opts, void* stream);

/* Workspace sizes for bidiag_band with the same arguments (caches the plan). */
int bb_query(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts* opts,
             size_t* vt_bytes, size_t* ws_bytes);

/*
 * bb_plan_trace -- where a BB_FLAG_TRACE plan's execution trace lives in its
 * workspace: *offset (bytes from ws) of nunits records of 4 int64
 * {ready-wait start, run start, run end, workgroup}, wall-clock ticks of
 * *tick_hz, in ticket order; units[2k], units[2k+1] (optional, host, 2 *
 * nunits int32) receive the (task, column strip) of record k.  Valid after a
 * bb_execute of the plan with BB_SCHED_PERSISTENT has completed.
 */
int bb_plan_trace(bb_plan* plan, size_t* offset, int64_t* nunits, double* tick_hz, int32_t* units);

/*
 * bb_apply_q / bb_apply_p -- apply the orthogonal factors of a finished
 * reduction, read from its V/T records (Sections 3.4 and 3.5: B = Q^T A P,
 * Q the product of the QR-step panel reflectors in task order, P that of the
 * LQ-step ones, so A = Q B P^T).
 *   bb_apply_q: C (m x ncols) <- Q C       (transpose = 0) or Q^T C (1);
 *   bb_apply_p: C (n x ncols) <- P C       (transpose = 0) or P^T C (1).
 * (C P is (P^T C^T)^T.)  Arguments: plan (1) of the reduction that wrote vt;
 * transpose (2); vt (3) with vt_bytes (4) as from bb_plan_workspace, device,
 * read only; C (5) device, column-major, ldc (6) >= rows of C, modified in
 * place; ncols (7) >= 0 (0: nothing is done); ws (8) with ws_bytes (9) >=
 * bb_apply_workspace's size (scheduler state, contents not kept); stream
 * (10).  Runs on FP64 matrix cores whatever the plan's prec.  The plan keeps
 * one host task graph per (side, transpose, ceil(ncols/nb)), built on first
 * use (normally by bb_apply_workspace) under a lock; that graph is uploaded
 * into ws like the reduction's.
 */
int bb_apply_q(bb_plan* plan, int transpose, const void* vt, size_t vt_bytes, void* C,
               int64_t ldc, int64_t ncols, void* ws, size_t ws_bytes, void* stream);
int bb_apply_p(bb_plan* plan, int transpose, const void* vt, size_t vt_bytes, void* C,
               int64_t ldc, int64_t ncols, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for bb_apply_q (side 0) or bb_apply_p (side 1) with the
 * given transpose and column count (host only). */
int bb_apply_workspace(bb_plan* plan, int side, int transpose, int64_t ncols, size_t* ws_bytes);

/*
 * bidiag_band_adjoint -- gradient of L = sum_ij W(i,j) B(i,j) over the band of
 * a finished reduction with respect to its input A (the sensitivity of
 * B = Q^T A P, Sections 3.4 and 3.5): Abar = Q_thin G P^T, where G (n x n)
 * solves the transposed band-constraint system of the perturbations
 * Q^T dQ and P^T dP (block sweep over the nb-blocks of B in reverse order),
 * and Q, P are applied from the V/T records as in bb_apply_q/p.
 * Arguments: plan (1) of the reduction; B (2) its output (m x n, device,
 * column-major) with ldb (3) >= m; W (4) n x n device weights, column-major,
 * ldw (5) >= n (entries outside the band 0 <= j - i <= nb are ignored); vt (6)
 * with vt_bytes (7): that reduction's records; Abar (8) m x n device output,
 * ldabar (9) >= m; ws (10) / ws_bytes (11) >= bb_adjoint_workspace; stream
 * (12).  FP64.  The gradient exists where every diagonal and super-diagonal
 * block of B is nonsingular (true almost surely); BB_QRONLY plans, plans
 * with nb = 256 and plans of m < n (reduced as A^T) return BB_ENOTSUP.
 */
int bidiag_band_adjoint(bb_plan* plan, const void* B, int64_t ldb, const void* W, int64_t ldw,
                        const void* vt, size_t vt_bytes, void* Abar, int64_t ldabar, void* ws,
                        size_t ws_bytes, void* stream);
int bb_adjoint_workspace(bb_plan* plan, size_t* ws_bytes);

/* Scheduler status of the last bidiag_band_adjoint on workspace ws (its
 * applications of P and Q run the persistent scheduler): synchronizes
 * `stream`, then *device_status = 0 or a BB_E* code, as bb_poll_error.
 * Arguments: plan (1), ws (2), stream (3), device_status (4). */
int bb_adjoint_poll_error(bb_plan* plan, const void* ws, void* stream, int* device_status);

/* ---- batches of independent reductions ------------------------------- */
/*
 * A batch reduces `count` independent matrices, each by its own task graph
 * (the graphs of Sections 3.4/3.5 for its own p x q tile grid, nb, tree and
 * variant).  The graphs are joined, without edges between matrices, into one
 * graph that one persistent launch executes; its tasks carry their own tile
 * size (32, 64 or 128).  Matrices with nb = 256 form a second graph, launched
 * after the first on the same stream.  Sizes may differ freely (ragged
 * tiles as in the single form).
 */
typedef struct bb_batch bb_batch;

/*
 * bb_tuned_config -- the (nb, tree, variant) that the offline tuner measured
 * as fastest (batch throughput) for the size class of an m x n matrix.
 * Arguments: m (1) >= n (2) >= 1, prec (3), out nb/tree/variant (4-6).
 */
int bb_tuned_config(int64_t m, int64_t n, int prec, int* nb, int* tree, int* variant);

/*
 * bb_batch_create -- plan a batch (host only).  Arguments: out batch (1);
 * count (2) >= 0; m (3), n (4): host arrays of count sizes, m[i] >= n[i] >= 1;
 * nb (5), tree (6), variant (7): host arrays or NULL.  nb == NULL or
 * nb[i] == 0 selects bb_tuned_config's choice for matrix i (tree and variant
 * entries are then ignored); otherwise tree == NULL means BB_GREEDY and
 * variant == NULL BB_BIDIAG.  prec (8), opts (9) as in bb_plan_create.
 */
int bb_batch_create(bb_batch** batch, int64_t count, const int64_t* m, const int64_t* n,
                    const int* nb, const int* tree, const int* variant, int prec,
                    const bb_opts* opts);
void bb_batch_destroy(bb_batch* batch);

/* Device bytes for the records of all matrices and the scheduler state. */
int bb_batch_workspace(const bb_batch* batch, size_t* vt_bytes, size_t* ws_bytes);

/*
 * Per-matrix facts of a batch: the nb/tree/variant used, the byte offset of
 * matrix i's first V/T record in vt and its number of records (records of one
 * matrix are contiguous, in the order of its task graph, in the format of
 * bb_plan_workspace for that nb).
 */
int bb_batch_info(const bb_batch* batch, int64_t i, int* nb, int* tree, int* variant,
                  int64_t* rec_offset, int64_t* nrec);

/*
 * bb_batch_execute -- reduce every matrix of the batch in place.  A (2):
 * DEVICE array of count device pointers (matrix i column-major, m[i] x n[i]);
 * lda (3): DEVICE array of count leading dimensions, lda[i] >= m[i] (read by
 * the device, not validated on the host); vt (4)/vt_bytes (5), ws (6)/
 * ws_bytes (7) >= bb_batch_workspace's sizes; stream (8).  Device-side errors
 * are read with bb_batch_poll_error.
 */
int bb_batch_execute(bb_batch* batch, double* const* A, const int64_t* lda, void* vt,
                     size_t vt_bytes, void* ws, size_t ws_bytes, void* stream);

/* Milliseconds between HIP events recorded before the first and after the
 * last launch of the last bb_batch_execute (requires BB_FLAG_TIMING). */
int bb_batch_last_kernel_ms(bb_batch* batch, double* ms);

/* bb_poll_error over every launch of a batch's last execution. */
int bb_batch_poll_error(const bb_batch* batch, const void* ws, void* stream, int* device_status);

/* Workspace sizes of a batch (arguments as bb_batch_create from count on). */
int bb_query_batched(int64_t count, const int64_t* m, const int64_t* n, const int* nb,
                     const int* tree, const int* variant, int prec, const bb_opts* opts,
                     size_t* vt_bytes, size_t* ws_bytes);

/*
 * bidiag_band_batched -- one-shot bb_batch_create + bb_batch_execute with the
 * batch plan cached inside the library by its arguments (at most 4 batch
 * plans, least recently used out first; bb_cache_clear empties the cache).  Numbering: A (1),
 * lda (2) (device arrays), count (3), m (4), n (5), nb (6), tree (7),
 * variant (8) (host arrays), prec (9), vt (10), vt_bytes (11), ws (12),
 * ws_bytes (13), opts (14), stream (15).
 */
int bidiag_band_batched(double* const* A, const int64_t* lda, int64_t count, const int64_t* m,
                        const int64_t* n, const int* nb, const int* tree, const int* variant,
                        int prec, void* vt, size_t vt_bytes, void* ws, size_t ws_bytes,
                        const bb_opts* opts, void* stream);

/*
 * bb_poll_error -- synchronize `stream` and read the scheduler's error word
 * from ws: *device_status = 0 if the last execution completed, else a BB_E*
 * code.  ws = NULL reads the word of the last bb_execute_noalloc on the
 * current device.  The word is written by bb_execute; on a workspace that no
 * execution has used yet its value is undefined.  Returns BB_OK or BB_EHIP.
 */
int bb_poll_error(const void* ws, void* stream, int* device_status);

/*
 * Milliseconds between the HIP events recorded around the main kernel(s) of
 * the last bb_execute of this plan (requires BB_FLAG_TIMING; synchronizes on
 * the end event).  For BB_SCHED_PERSISTENT this is the one persistent launch.
 */
int bb_plan_last_kernel_ms(bb_plan* plan, double* ms);

/*
 * bb_graph_check -- static race check of a task graph in the bb_plan_export
 * format (host only): predecessors precede their task, every two consecutive
 * tasks touching the same tile are joined by an edge (tile accesses are
 * read-modify-write, Algorithms 2 and 3), and each update depends on the
 * panel that wrote its V/T slot.  Arguments: tile grid p (1) >= q (2) >= 1,
 * ntasks (3), tasks/pred_off/pred_idx (4-6).  Returns BB_OK or BB_EDAG.
 * bb_plan_create runs the same check on every graph it builds.
 */
int bb_graph_check(int p, int q, int64_t ntasks, const int32_t* tasks, const int32_t* pred_off,
                   const int32_t* pred_idx);

/*
 * FlatTS domain size Auto chose for each QR/LQ step of the plan (Section 5:
 * the largest a with ceil(u/a) * v >= gamma * workgroups for a step with u
 * panel tiles and v trailing tiles, else 1); 0 for steps of other trees.
 * Pass a = NULL to query *nsteps only.
 */
int bb_plan_auto_domains(const bb_plan* plan, int32_t* a, int64_t* nsteps);

/*
 * Critical path (Section 4) of the task graph for a p x q tile matrix, with
 * the Table 1 weights, host only.  Returns a negative value on bad input.
 */
double bb_critical_path(int p, int q, int tree, int variant, int auto_a, int workgroups,
                        double gamma);

/*
 * bb_choose -- the (tree, variant) with the shortest estimated run time for
 * an m x n matrix at tile size nb, among BiDiag, R-BiDiag and the three-step
 * reduction (switch step from delta) with the Greedy and Auto trees
 * (Sections 4.3.4 and 4.5 compare these by critical path; here the
 * estimate is the list schedule of each task graph on opts->workgroups
 * workers under the execution-cost model the device scheduler orders work
 * with, which accounts for both the critical path and the total work).
 * Host only.  Arguments: m (1), n (2), nb (3), opts (4, may be NULL),
 * out tree (5), out variant (6), out estimate (7, may be NULL: the
 * schedule length in cost-model units, for comparisons only).
 */
int bb_choose(int64_t m, int64_t n, int nb, const bb_opts* opts, int* tree, int* variant, double* estimate);

/* ---- band to singular values (the GE2VAL pipeline, Sections 2 and 6.2) ----
 * After the band reduction, the singular values of A are those of the n x n
 * upper band B (m >= n; for m < n, of B^T).  The paper leaves the two
 * remaining steps to any published method; here both run on the device.
 *
 * bb_bnd2bd -- BND2BD: reduce the upper band of bandwidth nb held in the
 * leading n x n part of the column-major B (device, leading dimension ldb;
 * only entries with 0 <= j - i <= nb are read, B is not written) to upper
 * bidiagonal form U^T B V (U, V orthogonal, V e1 = e1, neither formed) by
 * two-sided Householder bulge chasing, one row per sweep, the sweeps
 * pipelined over the GPU in one persistent launch (for nb > 64 each sweep
 * is run by a group of workgroups).  Writes the diagonal
 * d[0..n-1] and the superdiagonal e[0..n-2] (device).  The diagonal and
 * superdiagonal are those of the Golub-Kahan bidiagonalization of B started
 * at e1, so they are unique up to signs.
 * ws: device workspace of bb_bnd2bd_workspace bytes (control words, the band
 * with room for the fill, 24 nb n bytes, and a progress counter and a
 * group-barrier counter per sweep), overwritten.  watchdog_s: seconds a sweep may wait for the one
 * before it (0 = 30); when it fires the launch stops and bb_poll_error(ws)
 * reports BB_ETIMEOUT.  Arguments: B (1), ldb >= max(1, n) (2), n >= 0 (3),
 * 1 <= nb <= 256 (4), d (5), e (6), ws (7), ws_bytes (8, BB_EWORKSPACE when
 * too small), watchdog_s (9), stream (10).  Asynchronous.
 */
int bb_bnd2bd_workspace(int64_t n, int nb, size_t* ws_bytes);
int bb_bnd2bd(const double* B, int64_t ldb, int64_t n, int nb, double* d, double* e, void* ws,
              size_t ws_bytes, double watchdog_s, void* stream);
/* bb_bnd2bd_group -- bb_bnd2bd with the number of workgroups that run each
 * sweep for nb > 64 given: group (10) in 1..16, 0 = ceil(nb / 16) as
 * bb_bnd2bd uses (ignored for nb <= 64, where one workgroup runs a sweep).
 * The result does not depend on it.  -10 for group out of range. */
int bb_bnd2bd_group(const double* B, int64_t ldb, int64_t n, int nb, double* d, double* e, void* ws,
                    size_t ws_bytes, double watchdog_s, int group, void* stream);

/*
 * bb_bd2val -- BD2VAL: the singular values of the upper bidiagonal with
 * diagonal d[0..n-1] and superdiagonal e[0..n-2] (device), in decreasing
 * order, into sigma[0..n-1] (device).  Bisection (multisection, 4 to 32
 * lanes per singular value) on the Sturm counts of the 2n x 2n Golub-Kahan
 * tridiagonal, all values at once, to an absolute accuracy of a few
 * eps * ||B||.  Arguments: d (1), e (2), n >= 0
 * (3), sigma (4), stream (5).  Asynchronous; no workspace.
 */
int bb_bd2val(const double* d, const double* e, int64_t n, double* sigma, void* stream);

/*
 * bb_ge2val -- singular values of the m x n matrix A by the whole GE2VAL
 * pipeline of Sections 2 and 6.2 in stream order: bidiag_band (GE2BND, plan
 * cached as there; A is overwritten by its band form B and vt holds the
 * reflectors), bb_bnd2bd on B (for m < n on the transpose of the lower
 * band) and bb_bd2val into sigma[0..min(m,n)-1] (device), in decreasing
 * order.  ws: one workspace of bb_ge2val_workspace bytes, used by each step
 * in turn; the band reduction's status word is kept through the chase, so
 * bb_poll_error(ws) after the call reports the first error of the pipeline
 * (a failed reduction stops the chase at its first wait; sigma is then
 * undefined).  opts->watchdog_s bounds the chase's waits too.  Arguments as
 * bidiag_band: A (1), m (2), n (3), lda (4), nb (5, at most 256), tree (6),
 * variant (7), prec (8); sigma (9); vt (10), vt_bytes (11), ws (12),
 * ws_bytes (13), opts (14), stream (15).  -9: sigma NULL; BB_EWORKSPACE:
 * vt or ws too small; bidiag_band's codes otherwise.
 */
int bb_ge2val_workspace(int64_t m, int64_t n, int nb, int tree, int variant, int prec, const bb_opts* opts,
                        size_t* vt_bytes, size_t* ws_bytes);
int bb_ge2val(void* A, int64_t m, int64_t n, int64_t lda, int nb, int tree, int variant, int prec, double* sigma,
              void* vt, size_t vt_bytes, void* ws, size_t ws_bytes, const bb_opts* opts, void* stream);

/* Drop every plan the one-shot entry points cache (bidiag_band, bb_query,
 * bidiag_band_batched).  Plans in use by a running call are released when
 * that call returns. */
void bb_cache_clear(void);

const char* bb_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* BIDIAG_H */
