/*
 * bcgs.h -- C ABI of the MI355X (gfx950) block classical Gram-Schmidt QR
 * library.
 *
 * Computes the economic QR factorization X = Q R of a tall-skinny matrix
 * (section 1 of Carson & Ma, "The Performance of Low-Synchronization
 * Variants of Reorthogonalized Block Classical Gram-Schmidt", arXiv
 * 2507.21791): X is m x n with m >= n, Q is m x n with orthonormal columns,
 * R is n x n upper triangular with a positive diagonal.  The n columns are
 * split into q = n / s block columns of width s (section 1), which are
 * orthogonalized one after another by one of the variants of section 2.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major.  X, Q are addressed by (pointer, leading
 *     dimension); block column k (0-based) starts at column k*s.
 *   - Pointers are DEVICE pointers unless the parameter says "host".
 *   - All work is enqueued on the given HIP stream; calls return after
 *     enqueueing (asynchronous), except argument errors, which are reported
 *     synchronously before anything is enqueued.
 *   - Numerical breakdown (a non-positive or non-finite pivot in one of the
 *     Cholesky factorizations of Alg. 1 / Alg. 2) is not an error return:
 *     the device writes it to a bcgs_info record, lets NaN propagate into
 *     Q and R, and keeps going; read the record after the stream has
 *     synchronized (bcgs_get_info, or the caller's own d_info).
 *   - No call throws, exits or aborts.  The library is thread-safe for
 *     calls on different streams.
 */
#ifndef BCGS_H
#define BCGS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The variants compared in the paper (section 2; Table 1 lists their
 * synchronization counts and stability assumptions). */
typedef enum {
    /* BCGSI+: BCGS applied twice per block column, TSQR for both
     * intra-orthogonalizations; 4 synchronizations per block column
     * (section 1; Table 1). */
    BCGS_I_PLUS = 0,
    /* BCGSI+P-2S: Alg. 2 with TSQR as the first intra-orthogonalization;
     * 2 synchronizations per block column (section 2.3). */
    BCGS_P_2S = 1,
    /* BCGSI+P-1S: Alg. 2, one synchronization per block column, Pythagorean
     * Cholesky for both intra-orthogonalizations and delayed normalization
     * through eq. (1) (section 2.2). */
    BCGS_P_1S = 2,
    /* BCGS-PIPI+: Alg. 1, Pythagorean Cholesky for both
     * intra-orthogonalizations, 2 synchronizations per block column
     * (section 2.1; 2q - 1 in all with TSQR(X_1)). */
    BCGS_PIPI_PLUS = 3,
    /* BCGSI+1s: Alg. 2 without the first intra-orthogonalization
     * (S_{k,k} = I: U_k = X_k - Q S is not scaled), one synchronization per
     * block column; LOO O(u) kappa^2 (section 2.2; Table 1). */
    BCGS_I_PLUS_1S = 4
} bcgs_variant;

/* Arithmetic of the streamed m-row data.  BCGS_FP64: everything in binary64.
 * BCGS_FP32_BULK: X and Q are binary32 in memory and the per-row products are
 * accumulated in binary32; the cross-row reductions, the s x s Gram and
 * Cholesky work, the Pythagorean subtraction and R stay binary64. */
typedef enum { BCGS_FP64 = 0, BCGS_FP32_BULK = 1 } bcgs_precision;

typedef enum {
    BCGS_OK = 0,
    BCGS_ERR_ARG = 1,          /* invalid argument; nothing was enqueued */
    BCGS_ERR_BREAKDOWN = 2,    /* Cholesky breakdown (only in bcgs_info) */
    BCGS_ERR_NOMEM = 3,        /* device allocation failed */
    BCGS_ERR_HIP = 4,          /* a HIP runtime call failed */
    BCGS_ERR_QUEUE_FULL = 5,   /* request queue cannot admit more work */
    BCGS_PENDING = 6,          /* request not finished yet */
    BCGS_ERR_UNSUPPORTED = 7   /* valid but not supported in this build */
} bcgs_status;

/* Device-resident outcome of one factorization.
 *   status  BCGS_OK or BCGS_ERR_BREAKDOWN
 *   block   0-based block column whose Cholesky factor broke down (first one)
 *   pivot   0-based pivot index inside that s x s factorization
 *   stage   0: the first intra-orthogonalization (S_{k,k}),
 *           1: the second one (Y_{k,k}), of Alg. 2
 *   syncs   synchronization points (section 1) the factorization ran,
 *           counted on the device: each fixed-order reduction of the
 *           per-workgroup Gram partials and each TSQR tree root adds one
 *           as it completes (a breakdown does not stop the count)
 *   value   the offending pivot value */
typedef struct {
    int32_t status;
    int32_t block;
    int32_t pivot;
    int32_t stage;
    int32_t syncs;
    int32_t reserved;
    double value;
} bcgs_info;

/* X = Q R with library-owned workspace and info (section 1).
 *   X  m x n, leading dimension m, binary64, read only (never written)
 *   Q  m x n output, leading dimension m; must not overlap X
 *   R  n x n output, leading dimension n; the strictly lower part is set to 0
 *   s  block width: 1 <= s <= 64 and s divides n; m >= n
 * The library keeps one workspace per stream (grown on demand, freed by
 * bcgs_release) and one info record per stream (bcgs_get_info).  Returns
 * BCGS_ERR_ARG on invalid arguments, BCGS_ERR_NOMEM / BCGS_ERR_HIP when the
 * workspace cannot be set up, BCGS_OK otherwise. */
bcgs_status bcgs_qr(const double* X, int64_t m, int64_t n, int64_t s,
                    bcgs_variant variant, double* Q, double* R,
                    hipStream_t stream);

/* General form of bcgs_qr: leading dimensions, precision, caller-provided
 * workspace and info.
 *   X, Q     binary64 (BCGS_FP64) or binary32 (BCGS_FP32_BULK) elements
 *   ldx, ldq >= m
 *   R        always binary64, ldr >= n
 *   workspace, ws_bytes  device buffer of at least bcgs_workspace_size()
 *            bytes, 256-byte aligned, used exclusively by this call until
 *            the stream reaches its end
 *   d_info   device pointer to one bcgs_info, written by the call */
bcgs_status bcgs_qr_ex(const void* X, int64_t ldx, int64_t m, int64_t n,
                       int64_t s, bcgs_variant variant,
                       bcgs_precision precision, void* Q, int64_t ldq,
                       double* R, int64_t ldr, void* workspace,
                       size_t ws_bytes, bcgs_info* d_info,
                       hipStream_t stream);

/* Size of the fixed per-device scratch array of bcgs_qr_noalloc. */
#define BCGS_NOALLOC_SCRATCH_BYTES (64ull << 20)

/* bcgs_qr_ex without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments and results as bcgs_qr_ex (same
 * kernels, so the same bits for the same problem), except that the
 * workspace is a fixed device array of BCGS_NOALLOC_SCRATCH_BYTES inside
 * the library, one per GPU, held from the first call on that GPU until the
 * process ends.  The call makes no hipMalloc / hipFree and no allocating
 * library call (launch profiling through bcgs_profile_start must be off on
 * the stream).
 *   - BCGS_ERR_NOMEM, nothing enqueued, when bcgs_workspace_size() of the
 *     problem exceeds BCGS_NOALLOC_SCRATCH_BYTES (about m n <= 2^28 at
 *     s = 16 fits, e.g. m = 2^20, n = 256).
 *   - Every call on one GPU uses that GPU's one array: calls that overlap
 *     in time on the same GPU (other streams, other threads) race and
 *     corrupt each other's results; serialize them (one stream, or events).
 *     A call does not depend on what an earlier call left in the array:
 *     every value the factorization uses is written by the same call
 *     first.
 *   - The first call on a device resolves the array's address with that
 *     device current (hipGetSymbolAddress); BCGS_ERR_HIP if that fails. */
bcgs_status bcgs_qr_noalloc(const void* X, int64_t ldx, int64_t m, int64_t n,
                            int64_t s, bcgs_variant variant,
                            bcgs_precision precision, void* Q, int64_t ldq,
                            double* R, int64_t ldr, bcgs_info* d_info,
                            hipStream_t stream);

/* Bytes of device workspace bcgs_qr_ex needs for this problem (0 on invalid
 * arguments).  No device call is made. */
size_t bcgs_workspace_size(int64_t m, int64_t n, int64_t s,
                           bcgs_variant variant, bcgs_precision precision);

/* Number of device-wide reductions ("synchronization points", section 1)
 * the factorization of an m x n matrix with block width s is scheduled to
 * perform (a completed run reports what ran in bcgs_info.syncs): q + 1 for BCGSI+P-1S and BCGSI+1s, 2q for BCGSI+P-2S, 2q - 1 for
 * BCGS-PIPI+, 4q - 3 for BCGSI+ (Table 1 gives the per-block-column rates
 * q, q, 2q, 2q, 4q).  -1 on invalid arguments. */
int32_t bcgs_sync_count(int64_t m, int64_t n, int64_t s,
                        bcgs_variant variant);

/* Waits for `stream` and copies the info record of the last bcgs_qr call on
 * that stream into *host_out (host pointer).  BCGS_ERR_ARG if no bcgs_qr
 * ran on the stream. */
bcgs_status bcgs_get_info(hipStream_t stream, bcgs_info* host_out);

/* Frees the library-owned workspaces of every stream, the batch arenas,
 * cached graphs and library streams (waits for them). */
void bcgs_release(void);

/* ---- many problems in one launch -----------------------------------------
 * Independent factorizations (each exactly the computation bcgs_qr_ex does
 * for it: same variant, same kernels, same bits) enqueued together. */
typedef struct {
    const void* X;       /* m x n, ld ldx; binary64 or binary32 (precision) */
    void* Q;             /* m x n output, ld ldq, same element type as X */
    double* R;           /* n x n output, ld ldr */
    int64_t m, n, s, ldx, ldq, ldr;
    int32_t variant;     /* bcgs_variant */
    int32_t precision;   /* bcgs_precision */
    bcgs_info* d_info;   /* device, one record per problem */
} bcgs_problem;

/* Enqueue `count` problems (host array) on `stream` as one launch of a HIP
 * graph: every problem's schedule runs on one of a fixed set of library
 * streams forked from `stream` (largest modelled work first, each to the
 * least loaded branch) and joined back, so independent problems overlap on
 * the device.  The instantiated graph is cached per stream and replayed
 * while the problem array (pointers, shapes, tuned choices) is unchanged.
 * Workspace is library-owned (one arena per stream, grown on demand; freed
 * by bcgs_release).  Problems must not share Q, R or d_info.
 * Returns BCGS_ERR_ARG (nothing enqueued) if any problem fails the checks
 * of bcgs_qr_ex, BCGS_ERR_NOMEM if the arena cannot grow, BCGS_ERR_HIP on a
 * runtime failure, BCGS_OK otherwise (count == 0 enqueues nothing).
 * Environment BCGS_BATCH_MODE=streams enqueues the same branches directly,
 * without the graph (for comparison); BCGS_BATCH_BRANCHES (1..16, default
 * 8) sets the number of branch streams.  BCGS_BATCH_MODE=persistent runs
 * the whole batch as one persistent kernel whose workgroups claim
 * (problem, step, row range) work items, with per-problem device-side
 * barriers between dependent steps (same bits as the lone runs); it
 * supports binary64 problems with s in {4, 8, 16} and returns
 * BCGS_ERR_UNSUPPORTED (nothing enqueued) for any other batch. */
bcgs_status bcgs_qr_batched(const bcgs_problem* probs, int32_t count,
                            hipStream_t stream);

/* Launch choices of one problem class.  Problem classes are keyed by
 * (floor(log2 m), n, s, variant, precision); every entry point reads the
 * same process-wide table, so a problem alone, batched or queued runs the
 * same kernels and gives the same bits.
 *   max_wg  upper bound on the workgroups (row ranges) of a streaming pass,
 *           1..512; fewer cut the partial-sum traffic of short matrices
 *   shape   tile shape index of the s <= 16 FP64 pass, -1 = automatic */
typedef struct {
    int32_t max_wg;
    int32_t shape;
} bcgs_tuning;

/* Autotuner: for every problem whose class has no entry yet, time each
 * candidate choice on that problem (HIP events on `stream`, best of two
 * runs after a warm-up; first max_wg in 512, 256, ..., 16, then shape) and
 * store the fastest.  Writes the problems' Q, R and d_info as a side effect
 * and synchronizes `stream`.  BCGS_ERR_ARG as bcgs_qr_batched. */
bcgs_status bcgs_autotune(const bcgs_problem* probs, int32_t count,
                          hipStream_t stream);

/* Read the entry of a class: BCGS_OK (filled), BCGS_PENDING (no entry; the
 * defaults max_wg = 512, shape = -1 are filled), BCGS_ERR_ARG. */
bcgs_status bcgs_tuning_get(int64_t m, int64_t n, int64_t s,
                            bcgs_variant variant, bcgs_precision precision,
                            bcgs_tuning* out);

/* Set (choice != NULL) or erase (choice == NULL) the entry of a class. */
bcgs_status bcgs_tuning_set(int64_t m, int64_t n, int64_t s,
                            bcgs_variant variant, bcgs_precision precision,
                            const bcgs_tuning* choice);

/* Erase every entry. */
void bcgs_tuning_clear(void);

/* ---- request queue with continuous batching -------------------------------
 * For serving: callers on any thread submit requests without blocking; one
 * scheduler thread per queue admits them onto up to max_inflight library
 * streams whenever a stream is free and the next request's HBM footprint
 * (X + Q + R + its workspace) fits in the budget left by the running
 * requests (a request is always admitted when nothing runs, so one larger
 * than the budget still completes).  The next request is the oldest
 * (BCGS_ADMIT_ARRIVAL) or the one whose estimated device time minus the
 * time it has waited is least (BCGS_ADMIT_SHORTEST: the estimate is the
 * streamed bytes at 3 TB/s plus 25 us per synchronization point, so small
 * requests pass large ones, and a large one is passed for at most about
 * its own estimate); a retry always goes first.  Requests admitted while others
 * run overlap with them on the device.  Each request runs exactly the
 * computation bcgs_qr_ex would run for it (same kernels, same tuned
 * choices), so its results are bitwise the same alone and in the mix. */
typedef struct bcgs_queue* bcgs_queue_t;

typedef enum { BCGS_ADMIT_ARRIVAL = 0, BCGS_ADMIT_SHORTEST = 1 } bcgs_admission;

typedef struct {
    size_t hbm_budget_bytes;    /* > 0 */
    int32_t max_inflight;       /* 1..16 concurrently running requests */
    int32_t device;             /* HIP device ordinal */
    size_t output_arena_bytes;  /* device memory for queue-allocated Q and
                                   R (0: every request brings its own) */
    int32_t retry_on_breakdown; /* nonzero: a request that breaks down runs
                                   once more, first in line, with
                                   retry_variant (same outputs) */
    int32_t retry_variant;      /* bcgs_variant, e.g. BCGS_P_2S */
    int32_t admission;          /* bcgs_admission */
    int32_t reserved;           /* 0 */
} bcgs_queue_config;

/* Outcome of one request; times are seconds on the host's steady clock
 * since the queue was created: submitted, first admitted (work enqueued),
 * and found complete by the scheduler (which polls every ~20 us).  Q and R
 * are the queue-allocated outputs (ld = m and n), else NULL. */
typedef struct {
    bcgs_status status;       /* BCGS_PENDING, BCGS_OK, BCGS_ERR_BREAKDOWN,
                                 or the error that stopped the request */
    bcgs_info info;           /* copy of the request's device record */
    double t_submit, t_start, t_done;
    void* Q;
    double* R;
    int32_t variant;          /* variant of the run that produced the result */
    int32_t attempts;         /* 1, or 2 after a retry on breakdown */
} bcgs_request_stats;

/* Create a queue (library streams, pinned info buffers, the output arena,
 * scheduler thread).  BCGS_ERR_ARG on a bad configuration, BCGS_ERR_NOMEM
 * if the arena cannot be allocated, BCGS_ERR_HIP on runtime failure. */
bcgs_status bcgs_queue_create(const bcgs_queue_config* cfg,
                              bcgs_queue_t* out);

/* Submit one problem (host struct; device buffers stay owned by the caller
 * and must stay valid until the request completes).  With p->Q and p->R
 * both NULL the queue carves them out of its output arena at admission
 * (ld = m and n; admission waits, in arrival order, until the arena has
 * room) and returns them in the stats; the caller returns them with
 * bcgs_queue_free_output.  Never waits for the device.
 * Ordering: `stream` is the caller's stream that produced X (and, if the
 * caller owns them, last used Q, R and the info record).  The call records
 * an event on it, and the request's kernels (on a queue stream) start only
 * after everything enqueued on `stream` before the call has completed; so
 * X may be written asynchronously right before submitting.  The caller
 * must not touch X, Q, R or the info record again before poll or wait
 * reports the request finished.
 * BCGS_ERR_ARG (the checks of bcgs_qr_ex, queue-allocated outputs without
 * an arena, or the queue is being destroyed), BCGS_ERR_NOMEM (the outputs
 * can never fit the arena), BCGS_ERR_QUEUE_FULL (2^20 requests waiting),
 * BCGS_ERR_HIP (an earlier request hit a runtime failure), else BCGS_OK
 * and *ticket. */
bcgs_status bcgs_queue_submit(bcgs_queue_t q, const bcgs_problem* p,
                              hipStream_t stream, uint64_t* ticket);

/* Non-blocking: BCGS_PENDING (stats so far), or the final status with the
 * final stats, after which the ticket is forgotten (BCGS_ERR_ARG on an
 * unknown or already collected ticket). */
bcgs_status bcgs_queue_poll(bcgs_queue_t q, uint64_t ticket,
                            bcgs_request_stats* out);

/* Block until the request has finished; then as bcgs_queue_poll. */
bcgs_status bcgs_queue_wait(bcgs_queue_t q, uint64_t ticket,
                            bcgs_request_stats* out);

/* Return a queue-allocated Q or R to the arena once the work enqueued on
 * `stream` so far has finished (an event recorded there).  NULL is a
 * no-op; BCGS_ERR_ARG for a pointer the arena did not hand out. */
bcgs_status bcgs_queue_free_output(bcgs_queue_t q, void* ptr,
                                   hipStream_t stream);

/* Run every submitted request to completion (a request still waiting for
 * arena space that nothing will free finishes with BCGS_ERR_NOMEM), then
 * free the queue and its arena.  No other call on the queue may be in
 * progress or follow. */
bcgs_status bcgs_queue_destroy(bcgs_queue_t q);

/* ---- accuracy check ------------------------------------------------------
 * The loss of orthogonality ||Q^T Q - I||_2 and the relative residual
 * ||X - Q R||_2 / ||X||_2 of a computed factorization (section 1's two
 * accuracy measures) are 2-norms of n x n symmetric matrices built from
 * three Gram matrices.  bcgs_check forms them on the device:
 *   GQ = Q^T Q,  GE = E^T E with E = X - Q R,  GX = X^T X
 * each summed over chunks of 4096 rows with a compensated (two-sum)
 * addition of the chunk products, so the check's own error does not grow
 * with m; the caller takes the largest absolute eigenvalues (of GQ - I, GE,
 * GX) on the host.  Only the upper triangle of R is read.
 *   X, Q      m x n, binary64 (BCGS_FP64) or binary32 (BCGS_FP32_BULK, read
 *             and widened to binary64), ldx, ldq >= m
 *   R         n x n binary64, ldr >= n
 *   GQ, GE, GX  n x n binary64 outputs, both triangles, ldg >= n
 *   workspace device buffer of bcgs_check_workspace_size(m, n) bytes,
 *             256-byte aligned, used until the stream reaches its end
 * Everything is enqueued on `stream`; nothing is allocated.  BCGS_ERR_ARG
 * (nothing enqueued) for NULL pointers, m < n, n < 1, short leading
 * dimensions or a small/misaligned workspace; BCGS_ERR_HIP if a launch
 * fails. */
size_t bcgs_check_workspace_size(int64_t m, int64_t n);

bcgs_status bcgs_check(const void* X, int64_t ldx, const void* Q,
                       int64_t ldq, const double* R, int64_t ldr, int64_t m,
                       int64_t n, bcgs_precision precision, double* GQ,
                       double* GE, double* GX, int64_t ldg, void* workspace,
                       size_t ws_bytes, hipStream_t stream);

/* ---- launch profiling ----------------------------------------------------
 * Between bcgs_profile_start(stream) and bcgs_profile_stop(stream, ...), every
 * kernel the library enqueues on `stream` is bracketed by HIP events and
 * tagged with its ALGORITHMIC HBM bytes and flops: the data the method must
 * read and write and the arithmetic it must do for that step (per-row cost
 * times rows), not what the kernel actually moves.  Timing the events adds
 * a few microseconds per launch. */
enum {
    BCGS_KERNEL_PASS = 0,        /* streaming pass: block updates + Gram */
    BCGS_KERNEL_REDUCE = 1,      /* fixed-order sum of partial Grams */
    BCGS_KERNEL_EPILOGUE = 2,    /* s x s Cholesky, eq. (1), R assembly */
    BCGS_KERNEL_TSQR_LEAF = 3,   /* TSQR: per-chunk Householder R factors */
    BCGS_KERNEL_TSQR_NODE = 4,   /* TSQR: one level of the reduction tree */
    BCGS_KERNEL_TSQR_DOWN = 5,   /* TSQR: downward coefficients */
    BCGS_KERNEL_TSQR_APPLY = 6,  /* TSQR: explicit Q rows */
    BCGS_KERNEL_OTHER = 7
};

/* One profiled launch.  tag identifies the kernel instantiation.  For
 * BCGS_KERNEL_PASS, tags >= 10^9 are the s <= 16 pass, decimal digits
 * 1 W P B S TT PP N (waves, workgroups per CU, tile buffers, second partial
 * area, tile rows, Gram pairs per wave (+50 with a compile-time update step
 * count), Gram B blocks); smaller tags are the general pass,
 * 1000*(binary32) + 100*gram + 10*B blocks + A blocks per wave.
 * name: the kernel as profiler summaries print it (kernel name and
 * template arguments, no namespace or parameter list), NUL-terminated. */
typedef struct {
    int32_t kind;
    int32_t tag;
    double ms;
    double bytes;
    double flops;
    char name[112];
} bcgs_launch_record;

/* Start recording launches on `stream` (host-side; no device call). */
bcgs_status bcgs_profile_start(hipStream_t stream);

/* Wait for `stream`, write up to `capacity` records (host array, may be
 * NULL) in launch order, stop recording, and return the number of launches
 * recorded (-1 if profiling was not started on the stream). */
int32_t bcgs_profile_stop(hipStream_t stream, bcgs_launch_record* out,
                          int32_t capacity);

/* Human-readable name of a status code (static string). */
const char* bcgs_status_string(bcgs_status status);

#ifdef __cplusplus
}
#endif

#endif /* BCGS_H */
