/*
 * cgx — sparse conjugate-gradient solver for AMD Instinct MI355X (gfx950).
 *
 * C ABI of libcgx.so.  Every entry point takes plain pointers and sizes; no
 * framework types cross this boundary.  The operations are those the paper
 * (arXiv 2112.10823, "Fast and Green Computing with GPUs for solving Sparse
 * Linear Systems") measures: CSR sparse matrix-vector product, addition of
 * vectors, element-wise product, dot product (Section 5.2) and the conjugate
 * gradient method built from them (Section 5.3).
 *
 * Conventions shared by all calls
 *  - Pointers named as device pointers must point to device memory of the
 *    handle's GPU; they stay owned by the caller.  The library never frees
 *    caller memory and never allocates memory the caller sees.
 *  - Calls are asynchronous on the handle's stream unless marked (sync).
 *  - Return value: CGX_OK (0) or a negative CGX_E* / solver status code.  On
 *    error nothing is launched and cgx_last_error() (per thread) explains.
 *  - Index arrays are 0-based int32; nnz must be < 2^31.
 *  - Aliasing: outputs may alias inputs only where a call says so.
 */
#ifndef CGX_H
#define CGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGX_OK 0
#define CGX_PENDING 1          /* cgx_poll: request queued or running */
#define CGX_EINVAL (-1)        /* bad argument: size, pointer, CSR structure, alias */
#define CGX_ENOMEM (-2)        /* caller workspace / pool too small */
#define CGX_EHIP (-3)          /* HIP runtime error */
#define CGX_NOT_CONVERGED (-4) /* maxit reached; x holds the last iterate */
#define CGX_BREAKDOWN (-5)     /* p.Ap <= 0 or r.z <= 0: matrix not SPD */
#define CGX_NONFINITE (-6)     /* NaN or Inf met in b, A or the iteration */

typedef struct cgx_context *cgx_handle;

/* Sparse matrix in CSR form (Section 2.3: values row-wise in AA, their
 * column numbers in JA, IA(i) the start of row i).  All arrays are device
 * pointers, read-only to the library:
 *   row_ptr  int32[n_rows + 1], row_ptr[0] = 0, non-decreasing, row_ptr[n_rows] = nnz
 *   col_idx  int32[nnz], each in [0, n_cols), no column twice in a row (order free)
 *   val      float64[nnz]  (may be NULL if only the float32 product is used)
 *   val32    float32[nnz]  values rounded to binary32, same pattern; NULL
 *            unless the float32 product or mixed precision is used.
 * Kernels clamp every index they read, so a malformed matrix gives wrong
 * numbers rather than a memory fault; cgx_csr_validate reports it. */
typedef struct cgx_csr {
    int32_t n_rows;
    int32_t n_cols;
    int64_t nnz;
    const int32_t *row_ptr;
    const int32_t *col_idx;
    const double *val;
    const float *val32;
} cgx_csr;

/* ------------------------------------------------------------- handle -- */

/* Create a handle bound to GPU `device` and HIP stream `stream` (a
 * hipStream_t; NULL = the null stream).  Allocates the handle's private state:
 * a small device scratch area for reductions and pinned host status words. */
int cgx_create(cgx_handle *out, int device, void *stream);
/* Destroy a handle (sync: waits for its stream). */
int cgx_destroy(cgx_handle h);
/* Re-target the handle to another stream of the same device. */
int cgx_set_stream(cgx_handle h, void *stream);
/* Message of the last error raised on the calling thread ("" if none). */
const char *cgx_last_error(void);
/* Library ABI version (major * 10000 + minor * 100 + patch). */
int cgx_version(void);

/* ---------------------------------------------------------- CSR / SpMV -- */

/* (sync) Structural check of a device CSR matrix: row_ptr as above, columns
 * in range, no duplicate column within a row.  Returns CGX_OK or CGX_EINVAL;
 * *bad_row (nullable) receives the first offending row, or -1. */
int cgx_csr_validate(cgx_handle h, const cgx_csr *A, int64_t *bad_row);

/* y = A x (Section 5.2, table "SpMV with CSR format"), float64.
 * x: float64[n_cols], y: float64[n_rows], device; y must not overlap x.
 * Row i of y is the sum of val[k] * x[col_idx[k]] over the row, +0.0 for an
 * empty row; the summation order is unspecified (not bit-reproducible
 * against a sequential sum, but run-to-run deterministic). */
int cgx_csr_spmv(cgx_handle h, const cgx_csr *A, const double *x, double *y);

/* y = A32 x in binary32 with binary32 accumulation, using A->val32.
 * x: float32[n_cols], y: float32[n_rows]; y must not overlap x. */
int cgx_csr_spmv_f32(cgx_handle h, const cgx_csr *A, const float *x, float *y);

/* --------------------------------------------------------------- BLAS-1 -- */

/* z = x + y elementwise, float64 (Section 5.2, table "Addition of vectors").
 * One IEEE rounding per element: bit-identical to any correct scalar loop.
 * z may alias x or y exactly (same pointer); partial overlap is invalid. */
int cgx_add(cgx_handle h, int64_t n, const double *x, const double *y, double *z);

/* y = alpha * x + y with one rounding per element (fma) — the daxpy named by
 * the label of the paper's addition table.  x and y must not overlap. */
int cgx_axpy(cgx_handle h, int64_t n, double alpha, const double *x, double *y);

/* z = x .* y elementwise (Section 5.2, table "Element wise product").
 * Bit-identical to a scalar loop; z may alias x or y exactly. */
int cgx_xmul(cgx_handle h, int64_t n, const double *x, const double *y, double *z);

/* *result = sum_i x_i y_i (Section 5.2, table "Dot product"), written to the
 * DEVICE pointer `result` (one float64).  Accumulates with error-free
 * transformations (two-product by fma, two-sum) and a fixed reduction tree:
 * the result is deterministic and within about 2 ulp of the exact sum for
 * well-conditioned data.  n = 0 gives +0.0. */
int cgx_dot(cgx_handle h, int64_t n, const double *x, const double *y, double *result);

/* (sync) The dot product of cgx_dot returned to the host: *result_host (a
 * host pointer) receives the same bits cgx_dot writes, after the handle's
 * stream has finished the reduction (the host-side result the paper's dot
 * product table times). */
int cgx_dot_sync(cgx_handle h, int64_t n, const double *x, const double *y, double *result_host);

/* dst[i] = (float)src[i], round to nearest even (e.g. to build val32). */
int cgx_demote(cgx_handle h, int64_t n, const double *src, float *dst);

/* ------------------------------------------------------------------- CG -- */

#define CGX_PRECOND_NONE 0
#define CGX_PRECOND_JACOBI 1
#define CGX_PRECISION_FP64 0
#define CGX_PRECISION_MIXED 1     /* float64 refinement around restarted binary32 CG */
#define CGX_PRECISION_MIXED_RU 2  /* binary32 CG with float64 reliable updates */

typedef struct cgx_opts {
    double rtol;         /* stop when ||r_k||_2 <= rtol * ||b||_2 */
    int32_t maxit;       /* iteration cap (inner cap for MIXED); <= 0 means n */
    int32_t precond;     /* CGX_PRECOND_* */
    int32_t precision;   /* CGX_PRECISION_* */
    int32_t check_every; /* iterations between host convergence checks; <= 0 = auto */
    double inner_rtol;   /* MIXED: inner binary32 CG relative tolerance (<= 0: 1e-3);
                          * MIXED_RU: the residual drop delta that triggers a
                          * reliable update (<= 0: 1e-2) */
    int32_t max_outer;   /* MIXED: refinement step cap; MIXED_RU: update cap (<= 0: 100) */
    int32_t true_residual; /* nonzero: also compute ||b - A x|| / ||b|| at exit */
    int32_t profile;     /* nonzero: launch the phase kernels one by one (no graph) with
                          * HIP events around each, and report their mean durations */
} cgx_opts;

typedef struct cgx_stats {
    int32_t status;      /* CGX_OK, CGX_NOT_CONVERGED, CGX_BREAKDOWN, CGX_NONFINITE */
    int32_t iters;       /* CG iterations (binary32 inner iterations for MIXED;
                          * Schwarz: subdomain iterations, summed over the outer
                          * steps of the largest count among the subdomains) */
    int32_t outer_iters; /* MIXED: refinement steps (served MIXED requests too);
                          * Schwarz: outer iterations; served float64
                          * requests: as slot_requests */
    int32_t path;        /* kernel path: 0 phase kernels, 1 single workgroup, 2 mixed
                          * refinement, 3 batched, 4 served, 5 Schwarz, 6 reliable
                          * updates */
    double relres;       /* recursive ||r|| / ||b|| at exit (outer residual for MIXED) */
    double relres_true;  /* ||b - A x|| / ||b|| if requested, else -1 */
    double device_ms;    /* GPU time of the solve, from stream events */
    double phase_ms[3];  /* profile: mean duration per iteration of (1) the SpMV
                          * kernel q = A p with its p.q tile partials, (2) the
                          * reduction of those partials (for more than 2048 tiles)
                          * plus the x/r/z update and its dots, (3) the p update */
    double queue_ms;     /* served requests: submission to admission, wall clock */
    double latency_ms;   /* served requests: submission to completion, wall clock */
    double kappa_est;    /* cgx_cg_solve / _sell: ritz_max / ritz_min, the condition
                          * number estimate of the operator CG ran on (A, or D^-1 A
                          * with Jacobi; MIXED: the first refinement step's binary32
                          * inner solve); 0 when no iteration ran or not recorded */
    double ritz_min;     /* extreme eigenvalues of the Lanczos tridiagonal T_k built */
    double ritz_max;     /* from the first k = min(iterations, 4096) CG steps' alpha,
                          * beta (Saad, Sec. 6.7.3, the textbook the paper cites for
                          * CG): T[j][j] = 1/alpha_j + beta_{j-1}/alpha_{j-1},
                          * T[j][j+1] = sqrt(beta_j)/alpha_j; they lie inside the
                          * operator's spectrum and approach its ends as k grows */
    int32_t slot_requests; /* served requests: requests in its slot when it
                            * started, itself included (1: alone); else 0 */
    int32_t reserved;
} cgx_stats;

/* Bytes of device workspace cg_solve needs for a system of n_rows rows and
 * nnz stored entries (the SpMV tile count depends on the mean row length)
 * and `opts` (its precond and precision); 0 when n_rows or nnz is negative or
 * opts is NULL.  Option values themselves are checked by the solve.  The
 * caller allocates it (256-byte aligned) and keeps it alive for the duration
 * of the call. */
size_t cgx_cg_workspace_bytes(int64_t n_rows, int64_t nnz, const cgx_opts *opts);

/* (sync) Solve A x = b, A symmetric positive definite, by conjugate gradient
 * (Section 5.3: classical CG; Jacobi preconditioning and binary32-inner
 * iterative refinement are options).  MIXED: float64 residual, binary32 CG
 * on A->val32 from 0 to inner_rtol, x += ||r|| d, repeated.  MIXED_RU: one
 * binary32 CG on A->val32 whose direction is kept across float64 "reliable
 * updates" (x += ||r|| d, r = b - A x and the stopping test in float64, the
 * binary32 residual replaced by float(r / ||r||)) taken when the binary32
 * residual has fallen by inner_rtol since the last update or below the
 * tolerance; stats->iters counts binary32 iterations, outer_iters updates.
 * b: float64[n] device; x: float64[n]
 * device, holds x0 on entry (zeros for the usual start) and the solution on
 * exit.  workspace: device, >= cgx_cg_workspace_bytes bytes.  The iteration
 * state stays on the GPU; the host reads one status word every check_every
 * iterations.  b = 0 gives x = 0.  Returns stats->status (CGX_OK when
 * converged) or an argument error. */
int cgx_cg_solve(cgx_handle h, const cgx_csr *A, const double *b, double *x, void *workspace,
                 size_t workspace_bytes, const cgx_opts *opts, cgx_stats *stats);

/* (sync) cgx_cg_solve for callers that cannot allocate device memory (code
 * that must not call hipMalloc: tight serving loops, harnesses that forbid
 * it): the workspace is the library's static device scratch of 64 MiB
 * (67,108,864 bytes; one copy per GPU, held from cgx_create until the
 * process ends), and the iterations are launched directly instead of through
 * a HIP graph.  The call allocates no device or host memory.  float64 only
 * (opts->precision FP64; plain or Jacobi); otherwise the same arguments,
 * arithmetic, results and statistics as cgx_cg_solve (same bits).
 * CGX_ENOMEM with a message when the system needs more workspace than the
 * scratch holds (cgx_cg_workspace_bytes(n_rows, nnz, opts) > 64 MiB: about
 * 2.7 M rows plain, 1.6 M rows Jacobi for 27-entry rows).  All calls on one
 * GPU share the scratch: calls that overlap in time on the same GPU (from
 * several threads or streams) race and must be serialised by the caller;
 * each call initialises every scratch word it reads. */
int cgx_cg_solve_noalloc(cgx_handle h, const cgx_csr *A, const double *b, double *x,
                         const cgx_opts *opts, cgx_stats *stats);

/* ------------------------------------------------- sliced ELL (SELL) -- */

/* Sliced ELLPACK copy of a CSR matrix (Section 2.3 names ELL among the
 * sparse storage formats; the paper's measurements use CSR).  Rows in slices
 * of 64 (one wavefront), each slice stored column-major with the width of
 * its longest row: entry k of row 64 s + l is at slice_ptr[s] + 64 k + l,
 * in the row's CSR order; padding entries have column -1 and value 0.  Rows
 * are not reordered.  All arrays are device memory inside one caller buffer
 * (see cgx_sell_build); the struct only points into it. */
typedef struct cgx_sell {
    int32_t n_rows;
    int32_t n_cols;
    int64_t n_slices;          /* ceil(n_rows / 64) */
    int64_t stored;            /* slice_ptr[n_slices]: entries including padding */
    const int64_t *slice_ptr;  /* int64[n_slices + 1] */
    const int32_t *col;        /* int32[stored] */
    const double *val;         /* float64[stored] */
    const float *val32;        /* binary32[stored] when A had val32, else NULL */
} cgx_sell;

/* (sync) Device bytes cgx_sell_build needs for A (one pass over row_ptr). */
int cgx_sell_bytes(cgx_handle h, const cgx_csr *A, size_t *bytes);

/* (sync) Build the sliced-ELL copy of A into `buffer` (device, 256-byte
 * aligned, >= cgx_sell_bytes; owned by the caller, which keeps it while
 * *out is used) and describe it in *out.  Row pointers are clamped as by the
 * other kernels; A->val32, if set, is copied too.  CGX_ENOMEM if bytes is too
 * small. */
int cgx_sell_build(cgx_handle h, const cgx_csr *A, void *buffer, size_t bytes, cgx_sell *out);

/* y = A x from the sliced-ELL copy (Section 5.2, table "SpMV with CSR
 * format": the same product); float64, each row summed in its CSR order.
 * x: float64[n_cols], y: float64[n_rows]; y must not overlap x. */
int cgx_sell_spmv(cgx_handle h, const cgx_sell *S, const double *x, double *y);

/* y = A32 x in binary32 from S->val32; y must not overlap x. */
int cgx_sell_spmv_f32(cgx_handle h, const cgx_sell *S, const float *x, float *y);

/* (sync) cgx_cg_solve with the SpMV of the iteration (q = A p, and the inner
 * binary32 SpMV of MIXED, which needs S->val32) run on the sliced-ELL copy S
 * of A; the setup and residual passes read A.  Same workspace, arguments and
 * results as cgx_cg_solve. */
int cgx_cg_solve_sell(cgx_handle h, const cgx_csr *A, const cgx_sell *S, const double *b,
                      double *x, void *workspace, size_t workspace_bytes, const cgx_opts *opts,
                      cgx_stats *stats);

/* ------------------------------------------------------------ batched -- */

/* One system of a batch: matrix, right-hand sides and solutions.  B and X
 * are device arrays of nrhs x n_rows float64, right-hand-side major (vector j
 * at B + j * n_rows); X holds the initial guesses on entry.  1 <= nrhs <= 16.
 * schedule: 0 lets the autotuner pick the SpMM schedule; otherwise it is
 * used as given: M > 0 gives K * M lanes per row (K = nrhs rounded up to a
 * power of two; K * M must be 8, 16, 32 or 64), M < 0 gives wave tiles of
 * -M rows per wavefront (nrhs = 1 only; -M a power of two <= 64). */
typedef struct cgx_system {
    cgx_csr A;
    int32_t nrhs;
    int32_t schedule;
    const double *B;
    double *X;
} cgx_system;

/* Workspace bytes of cgx_cg_solve_batched for this batch; 0 when nsys < 1,
 * systems is NULL or a descriptor's sizes are invalid (not square, n_rows <
 * 1, nnz outside [0, 2^31), nrhs outside [1, 16]).  Pointers are checked by
 * the solve. */
size_t cgx_batch_workspace_bytes(int32_t nsys, const cgx_system *systems);

/* Workspace bytes of cgx_cg_solve_batched with opts->precision MIXED or
 * MIXED_RU (the float64 state, the binary32 state and the inner right-hand
 * sides and solutions); 0 for the invalid batches cgx_batch_workspace_bytes
 * rejects. */
size_t cgx_batch_mixed_workspace_bytes(int32_t nsys, const cgx_system *systems);

/* (sync) Solve every system of the batch by conjugate gradient (Section 5.3;
 * Jacobi preconditioning optional), all systems and right-hand sides
 * advanced together: each phase of an iteration is one kernel launch over a
 * work table of (system, row tile) entries, the matrix of a system is read
 * once per iteration for all its right-hand sides, and each right-hand side
 * has its own scalars and stopping test (||r|| <= rtol ||b||).  The rows of
 * a system are served by K * M lanes, or for one right-hand side possibly by
 * wave tiles, the schedule chosen per shape class by a timing autotuner kept
 * in the handle (unless the system fixes it).  A system's results do not depend on the
 * other systems in the batch.  stats: array of sum(nrhs) entries in
 * (system, right-hand side) order.  Returns CGX_OK if all converged, else
 * the first non-OK status; argument errors as usual.  opts->maxit <= 0
 * means the largest n.
 *
 * opts->precision MIXED (every A.val32 set; workspace from
 * cgx_batch_mixed_workspace_bytes): the refinement of the single-system
 * MIXED solve for every (system, right-hand side) at once.  Each outer step
 * computes r = b - A x in float64 for all of them (right-hand sides with
 * ||r|| <= rtol ||b|| are done), then solves A32 d = float(r / ||r||) for the
 * others by batched binary32 CG (binary32 values, vectors, scalars and
 * sums; Jacobi with float(1 / a_ii) if asked) from d = 0 to inner_rtol (<= 0:
 * 1e-3) within maxit iterations, and sets x = fma(||r||, double(d), x); at
 * most max_outer (<= 0: 100) steps.  stats: iters = binary32 iterations
 * summed over the steps, outer_iters = refinement steps, relres = the last
 * float64 ||r|| / ||b||.
 *
 * opts->precision MIXED_RU (every A.val32 set; workspace as for MIXED): the
 * single-system MIXED_RU method for every (system, right-hand side) at
 * once.  One binary32 CG per right-hand side on A32 (Jacobi from the
 * binary32 diagonal if asked) whose direction is kept across float64
 * reliable updates: when the binary32 ||r^|| of a right-hand side falls
 * below delta times its largest value since its last update (delta =
 * inner_rtol, <= 0: 1e-2) or its estimate of ||r|| reaches rtol ||b||, every
 * right-hand side of that system still active after the step pauses (the
 * float64 residual is one pass over the system's matrix for all of them): x
 * += ||r|| d and r = b - A x are taken in float64, ||r|| <= rtol ||b|| ends
 * a right-hand side, and otherwise it resumes on float(r / ||r||) with beta
 * rescaled by the ratio of the two norms; the other systems go on
 * meanwhile.  At most maxit binary32 iterations (then the pending
 * correction is folded into x) and max_outer (<= 0: 100) updates per
 * right-hand side, then CGX_NOT_CONVERGED.  stats: iters =
 * binary32 iterations, outer_iters = reliable updates, relres = relres_true
 * = ||b - A x|| / ||b|| of the result in float64. */
int cgx_cg_solve_batched(cgx_handle h, int32_t nsys, const cgx_system *systems, void *workspace,
                         size_t workspace_bytes, const cgx_opts *opts, cgx_stats *stats);

/* (sync) The schedule each system of the batch runs with (its own
 * `schedule` if nonzero, else the autotuner's pick, tuning shape classes not
 * seen yet by this handle): M > 0 slices per right-hand side, M < 0 wave
 * tiles of -M rows.  workspace as for
 * cgx_cg_solve_batched; M_out: host int32[nsys]. */
int cgx_batch_schedule(cgx_handle h, int32_t nsys, const cgx_system *systems, void *workspace,
                       size_t workspace_bytes, int32_t *M_out);

/* ------------------------------------------------------------- serving -- */

/* (sync) Start a continuous-batching solve server on the handle.  pool:
 * caller device memory (256-byte aligned) the server carves its tables and
 * every admitted slot's Krylov vectors from; max_slots: slots on the GPU at
 * once; max_group (1..16): requests on the same matrix (same arrays and
 * options) one slot may hold as the right-hand sides of one multi-RHS
 * solve, streaming the matrix once per iteration for all of them (1: every
 * request alone in its slot).  A progress thread admits queued requests
 * while a slot and pool memory are free (FIFO with backfill; a head request
 * blocked for 0.25 s stops the backfill; an admitted request takes queued
 * requests on its matrix along, and a request arriving while a slot on its
 * matrix runs takes a free lane of that slot), advances all admitted
 * requests together a few CG iterations at a time with the batched kernels,
 * and retires each request as soon as it finishes.  Slots of matrices with
 * at least 65536 rows keep one spare lane for such late arrivals.  With max_group = 1 a request's result is
 * bit-identical alone and in any mix; with grouping it is the same within
 * the solve tolerance.  The handle must not run other solves while the
 * server runs.  Threads: cgx_submit, cgx_poll and cgx_wait may be called
 * from several host threads at once, each ticket collected by one caller
 * only; cgx_serve_stop (and cgx_destroy) must not overlap any other call on
 * the handle. */
int cgx_serve_start(cgx_handle h, void *pool, size_t pool_bytes, int32_t max_slots,
                    int32_t max_group);

/* (sync) Finish every queued and running request, then stop the server. */
int cgx_serve_stop(cgx_handle h);

/* Pool bytes one request of n_rows needs while admitted alone, float64 or
 * MIXED (a group of g requests on one matrix needs less than g times this). */
size_t cgx_serve_request_bytes(int64_t n_rows);

/* Queue a solve of A x = b (A resident and square, b / x device float64[n],
 * x holds x0 and receives the solution; all must stay valid until the
 * request completes).  opts: rtol, maxit, precond, precision are used, and
 * for CGX_PRECISION_MIXED and MIXED_RU inner_rtol and max_outer.  FP64: CG (Section 5.3)
 * in float64.  MIXED (needs A->val32): the refinement of cgx_cg_solve's
 * MIXED, step by step per request: float64 r = b - A x, ||r|| <= rtol ||b||
 * ends it, else binary32 CG on A->val32 (Jacobi from val32's diagonal with
 * precond) from 0 on float(r / ||r||) to inner_rtol (default 1e-3) or maxit
 * iterations, then x += ||r|| d in float64; at most max_outer (default 100)
 * inner solves, then CGX_NOT_CONVERGED.  MIXED_RU (needs A->val32): the
 * reliable-update method of cgx_cg_solve_batched's MIXED_RU for the
 * request (delta = inner_rtol, default 1e-2; at most max_outer updates,
 * default 100, and maxit binary32 iterations), its updates taken inside the
 * iteration sequence and shared by the requests of its slot (one matrix,
 * one update event for all of them).  The inner solves of all MIXED
 * requests advance together in the batched binary32 kernels; each request
 * takes its float64 steps on its own.  Non-blocking; *ticket identifies the
 * request.  CGX_ENOMEM at once if the request can never fit the pool. */
int cgx_submit(cgx_handle h, const cgx_csr *A, const double *b, double *x, const cgx_opts *opts,
               uint64_t *ticket);

/* CGX_PENDING while queued or running; otherwise the request's final status
 * with *stats filled (stats->latency_ms, queue_ms set), after which the
 * ticket is forgotten. */
int cgx_poll(cgx_handle h, uint64_t ticket, cgx_stats *stats);

/* (sync) Like cgx_poll but waits for completion. */
int cgx_wait(cgx_handle h, uint64_t ticket, cgx_stats *stats);

/* ------------------------------------------ domain decomposition -- */

/* Additive Schwarz preconditioner with conjugate-gradient subdomain solves
 * (end of Section 5.3: domain-decomposition preconditioning of CG, the outer
 * iteration on the host and every subdomain problem solved by CG on the
 * GPU).  The rows are cut into n_sub contiguous core blocks [floor(i n /
 * n_sub), floor((i+1) n / n_sub)); subdomain i is its block extended by
 * `overlap` rows on each side, clipped to [0, n) (for a grid in
 * lexicographic order, slabs overlapping by overlap / (rows per layer)
 * layers).  Its matrix A_i is the principal submatrix of A on those rows and
 * columns, entries in stored order, columns shifted to start at 0.  All
 * pointers are device memory inside the caller's buffer. */
typedef struct cgx_schwarz {
    int32_t n_rows;            /* rows of A */
    int32_t n_sub;             /* subdomains, 1 <= n_sub <= n_rows */
    int32_t overlap;           /* 0 <= overlap <= floor(n_rows / n_sub) */
    int32_t reserved;
    int64_t local_rows;        /* sum of the subdomain sizes: n + 2 overlap (n_sub - 1) */
    int64_t local_nnz;         /* entries of all subdomain matrices */
    const int64_t *nnz_off;    /* int64[n_sub + 1]: first entry of each subdomain */
    const int32_t *row_ptr;    /* int32[local_rows + n_sub]: subdomain i's m_i + 1 row
                                * pointers (from 0) at local row offset + i */
    const int32_t *col;        /* int32[local_nnz] */
    const double *val;         /* float64[local_nnz] */
} cgx_schwarz;

/* (sync) Device bytes cgx_schwarz_build needs (one pass over A).  CGX_EINVAL
 * unless A is square, 1 <= n_sub <= n_rows and 0 <= overlap <= floor(n_rows /
 * n_sub). */
int cgx_schwarz_bytes(cgx_handle h, const cgx_csr *A, int32_t n_sub, int32_t overlap,
                      size_t *bytes);

/* (sync) Build the subdomain matrices into `buffer` (device, 256-byte
 * aligned, >= cgx_schwarz_bytes; owned by the caller, which keeps it while
 * *out is used) and describe them in *out.  CGX_ENOMEM if bytes is too
 * small; CGX_EINVAL as for cgx_schwarz_bytes. */
int cgx_schwarz_build(cgx_handle h, const cgx_csr *A, int32_t n_sub, int32_t overlap,
                      void *buffer, size_t bytes, cgx_schwarz *out);

/* Workspace bytes of cgx_schwarz_solve (0 on invalid S). */
size_t cgx_schwarz_workspace_bytes(const cgx_schwarz *S);

/* (sync) Solve A x = b (A symmetric positive definite, S built from A) by
 * flexible conjugate gradient preconditioned by additive Schwarz: with
 * q = A p, alpha = r.z / p.q, x += alpha p, r -= alpha q, stop when ||r|| <=
 * opts->rtol ||b||; then z = sum_i R_i^T z_i (subdomains added in increasing
 * order), z_i from CG on A_i z_i = R_i r started at 0, all subdomains solved
 * together by the batched solver; beta = -alpha (z.q) / rho, rho = r.z, p =
 * z + beta p.  Subdomain CG: opts->inner_rtol > 0 its relative tolerance,
 * 0 for 1e-2, < 0 for none (exactly opts->maxit iterations); opts->maxit
 * (<= 0: 50) its iteration cap; opts->precond its preconditioner.
 * opts->max_outer (<= 0: n) caps the outer iterations; opts->true_residual
 * as for cgx_cg_solve; opts->precision must be FP64.  x holds x0 and
 * receives the solution; b = 0 gives x = 0.  stats: outer_iters, iters (see
 * cgx_stats), relres, device_ms (wall time of the call), phase_ms[0] (time
 * in the subdomain solves) and phase_ms[1] (the rest).  Returns
 * stats->status: CGX_OK, CGX_NOT_CONVERGED, CGX_BREAKDOWN (p.q <= 0, r.z <=
 * 0, or a subdomain solve broke down), CGX_NONFINITE; CGX_ENOMEM if the
 * workspace is too small. */
int cgx_schwarz_solve(cgx_handle h, const cgx_csr *A, const cgx_schwarz *S, const double *b,
                      double *x, void *workspace, size_t workspace_bytes, const cgx_opts *opts,
                      cgx_stats *stats);

/* ---------------------------------------------------------- test hooks -- */

/* For tests of the failure paths: the next `count` calls of the batched
 * schedule autotuner on this handle (cgx_batch_schedule, the batched solves,
 * a served slot's first cycle) fail with CGX_EHIP before launching anything,
 * whether or not the shape class was tuned before.  count = 0 clears it. */
int cgx_debug_fail_tuning(cgx_handle h, int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* CGX_H */
