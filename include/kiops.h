/*
 * kiops.h - C ABI of the MI355X (gfx950) KIOPS phi-combination library.
 *
 * Computes, on one GPU,
 *
 *     w = phi_0(tau A) b_0 + tau phi_1(tau A) b_1 + ... + tau^p phi_p(tau A) b_p
 *
 * (Eq. (4)/(12) of Gaudreault, Rainwater & Tokman, "KIOPS: A fast adaptive
 * Krylov subspace solver for exponential integrators", J. Comput. Phys. 372
 * (2018)) as the first N entries of exp(tau A~) [b_0; e_p], A~ the augmented
 * matrix of Theorem 1 (Section 3.1, Eq. (13), column order of B as in the
 * corrigendum), by the adaptive Krylov method of Algorithm 1 with the
 * incomplete orthogonalization procedure of Algorithm 2 (Section 3.3), the
 * a-posteriori estimate of Eq. (36), the acceptance test of Eq. (39) and the
 * step-size / dimension control of Algorithm 4 (Section 3.6).  The whole
 * adaptive loop runs on the device in one persistent launch per solve.
 *
 * Conventions shared by every entry point:
 *   - Data pointers named "device" are HIP device memory owned by the caller;
 *     the library never allocates or frees device memory.
 *   - Every function returns a kiops_status; nothing is thrown across the ABI
 *     and the process is never terminated.
 *   - On KIOPS_ERR_INVALID_ARG no output is modified.
 *   - Vectors are float64, contiguous, length N (N = nx*ny*nz or nrows).
 */
#ifndef KIOPS_H
#define KIOPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KIOPS_OK = 0,
  KIOPS_ERR_INVALID_ARG = 1,     /* bad argument; outputs untouched */
  KIOPS_ERR_OUT_OF_MEMORY = 2,   /* no workspace set, or it is too small */
  KIOPS_ERR_DEVICE = 3,          /* a HIP call failed, or the launch could not be made co-resident */
  KIOPS_ERR_NONFINITE = 4,       /* NaN/Inf met in a norm, an inner product or the estimate */
  KIOPS_ERR_NOT_CONVERGED = 5,   /* substep limit reached; w holds the state at stats.t_reached */
  KIOPS_ERR_BUDGET = 6,          /* request larger than the caller's memory budget (serving) */
  KIOPS_ERR_UNSUPPORTED = 7      /* valid request the library does not handle */
} kiops_status;

typedef enum {
  KIOPS_FP64 = 0,   /* basis, matrix-vector products and coefficients in float64 */
  KIOPS_MIXED = 1   /* basis, products and coefficients in float32; inner products, norms,
                       H, the small exponential, the error estimate, control and w in float64 */
} kiops_precision;

typedef enum {
  KIOPS_OP_STENCIL2D_5PT = 0,   /* nz must be 1 */
  KIOPS_OP_STENCIL3D_7PT = 1,
  KIOPS_OP_CSR = 2
} kiops_op_kind;

/*
 * Operator description.  A is only applied, never assembled (Section 3.3,
 * remark after Algorithm 2).  Stencils act on a periodic nx*ny*nz box with x
 * the fastest index (i = x + nx (y + ny z)) and spacing h:
 *
 *   (A u)_i = sum_d [ (kf_{i,d+} (u_{i+e_d} - u_i) - kf_{i,d-} (u_i - u_{i-e_d})) / h^2
 *                     - adv[d] (u_{i+e_d} - u_{i-e_d}) / (2 h) ] + r_i u_i
 *
 * kf = diff when kappa == NULL, else the mean of the two cells' kappa.
 * CSR: square nrows x nrows, 0-based int32 row pointers (nrows+1) and column
 * indices (nnz), float64 values; nnz * 8 and nrows * 8 must stay below 4 GiB.
 * A column index outside [0, nrows) or a row pointer outside [0, nnz] is read
 * as a zero entry (the kernels bounds-check every access).
 * Stencils: N * 8 must stay below 4 GiB.
 * All array pointers are device memory, borrowed: they must stay valid while
 * the operator exists and unchanged during any call that uses it; between
 * calls the caller may rewrite their contents (e.g. the reaction field of a
 * Jacobian updated every time step), and the next call reads the new values.
 */
typedef struct {
  kiops_op_kind kind;
  int64_t nx, ny, nz;
  double h;
  double diff;
  const double* kappa;      /* device, N entries, or NULL */
  double adv[3];
  const double* reaction;   /* device, N entries, or NULL (r = 0) */
  int64_t nrows, nnz;
  const int32_t* rowptr;    /* device */
  const int32_t* col;       /* device */
  const double* val;        /* device */
  kiops_precision precision;
  /* General stencil form: per-cell weights [5|7][N] (device, borrowed), the
   * points in the order centre, +x, -x, +y, -y (2-D), then +z, -z (3-D):
   *   (A u)_i = W_0[i] u_i + W_1[i] u_{i+e_x} + W_2[i] u_{i-e_x} + ...  (periodic).
   * With weights, kappa and reaction must be NULL and diff and adv zero. */
  const double* weights;
} kiops_operator_desc;

/* Bounds of the Krylov dimension (Algorithm 1 inputs m_min, m_max; defaults
 * 10 and 128, Section 3.6.2; m_max defaults to 32 for KIOPS_MIXED operators,
 * whose FP32 basis loses accuracy over longer recurrences) and a cap on
 * substeps (default 100000).  A zero field takes its default.  m_max must not
 * exceed KIOPS_M_MAX_LIMIT.
 * tile_rows: rows of the 64-column tiles of the 2-D 5-point tile pass in the
 * batched form (kiops_batch_plan, kiops_phi_batch, kiops_batch_tune): 16
 * (0 = default), 8 or 4; other values are INVALID_ARG there.  Shorter tiles
 * give small grids more work items per group, taller ones re-read fewer halo
 * rows; kiops_batch_tune_shape picks it.  Single solves and other operator
 * kinds do not use it. */
typedef struct {
  int32_t m_min;
  int32_t m_max;
  int32_t max_substeps;
  int32_t estimate;   /* KIOPS_ESTIMATE_*: the error estimate of an attempt (Section 3.4) */
  int32_t tile_rows;  /* batched 2-D tile pass: 16 (0), 8 or 4 */
} kiops_options;

/* kiops_options.estimate.  Every variant takes its terms from the expansion
 * of the error, Eq. (35), whose first term is Eq. (36):
 *   ONE_TERM  (0, default): eps = beta |h_{m+1,m}| |tau e_m^T phi_1(tau H_m) e_1|, Eq. (36);
 *   TWO_TERM  (1): the norm of the first two terms of Eq. (35),
 *       eps = beta |h_{m+1,m}| || a v_{m+1} + b A~ v_{m+1} ||,
 *       a = tau e_m^T phi_1(tau H_m) e_1,  b = tau^2 e_m^T phi_2(tau H_m) e_1,
 *     where <v_{m+1}, A~ v_{m+1}> and ||A~ v_{m+1}|| come from the pass that
 *     formed v_{m+1} (it computes A~ v_{m+1} anyway), so it costs no product;
 *   CORRECTED (2): the corrected scheme (remark after Eq. (30)): the result
 *       also takes the first term of Eq. (35), beta h_{m+1,m} a v_{m+1}, and
 *       eps is the norm of the second term, beta |h_{m+1,m}| |b| ||A~ v_{m+1}||.
 * a and b come from one exponential of the (m+2) x (m+2) matrix
 * [[H_m, e_1, 0], [0, 0, 1], [0, 0, 0]] (Theorem 1 applied to H_m).  The
 * batched and served forms take ONE_TERM only; CORRECTED is not combined with
 * several output times (UNSUPPORTED and INVALID_ARG respectively). */
#define KIOPS_ESTIMATE_ONE_TERM 0
#define KIOPS_ESTIMATE_TWO_TERM 1
#define KIOPS_ESTIMATE_CORRECTED 2

#define KIOPS_M_MAX_LIMIT 128
#define KIOPS_P_MAX 8
#define KIOPS_MAX_TIMES 32   /* output times of one kiops_phi_combination_times call */

/* Statistics of one solve.  m_last is the dimension to use as m_init of a
 * following, similar solve (Algorithm 1 returns it, Section 3.6). */
typedef struct {
  int32_t m_last;
  int32_t substeps;       /* accepted substeps */
  int32_t rejections;     /* rejected attempts */
  int32_t expms;          /* small exponentials computed */
  int32_t breakdowns;     /* happy breakdowns (Algorithm 2) */
  int32_t grid_blocks;    /* workgroups that ran the solve (the launch, or the batched group) */
  int64_t matvecs;        /* products with A~ */
  double last_omega;      /* scaled error of the last attempt, Eq. (39) */
  double t_reached;       /* T_now at exit (== tau on success) */
  double alg_bytes;       /* algorithmic HBM bytes of the solve (reads + writes the method needs) */
  double beta_last;       /* norm of the last substep's start vector */
  double time_work_s;     /* workgroup 0: time in its own share of the passes and gathers */
  double time_wait_s;     /* workgroup 0: time waiting for the other workgroups at barriers */
  double time_epilogue_s; /* serial epilogues: reductions, small exponential, controller */
  double time_expm_s;     /* part of time_epilogue_s spent in small exponentials */
  /* With the environment variable KIOPS_PROFILE=1: sums over barriers (the
   * first excepted) of the latest and of the mean workgroup arrival after the
   * previous release, and of the latest and mean delay until a workgroup saw
   * that release; barriers counts all barriers. */
  double arrive_max_s, arrive_mean_s;
  int64_t barriers;
  double release_max_s, release_mean_s;
  int32_t status;          /* the solve's own status (useful for batched problems) */
  int32_t m_max;           /* the largest basis size the solve allowed (the option, or the default) */
  /* With KIOPS_PROFILE=1 only (else 0): parts of time_epilogue_s after passes */
  double time_reduce_s;    /* reductions of the per-workgroup partial sums */
  double time_publish_s;   /* copies of the control block */
  double time_serial_s;    /* normalisation, H column and next coefficients (thread 0) */
  int32_t pass_kind;       /* the pass that ran: KIOPS_PASS_* */
  int32_t reserved3;
  /* device clock (constant rate, the same on every CU) at the start and at
   * the end of the solve, in seconds from an arbitrary origin: in a batch,
   * end - the batch's earliest start is the problem's completion time */
  double clock_start_s, clock_end_s;
} kiops_stats;

/* kiops_stats.pass_kind */
#define KIOPS_PASS_TILE2D 0    /* 5-point tile pass (64 x 16 tiles) */
#define KIOPS_PASS_WIDE2D 1    /* 5-point tile pass for IOP windows of 3 and 4 */
#define KIOPS_PASS_MARCH2D 2   /* 5-point row-marching pass (large 2-D grids, windows of 1 and 2) */
#define KIOPS_PASS_7PT 3       /* 7-point marching pass (3-D, and 2-D with a diffusivity field) */
#define KIOPS_PASS_CSR 4       /* general sparse matrix */
#define KIOPS_PASS_WEIGHTS 5   /* stencil given by per-cell weights (two phases per step) */

typedef struct kiops_operator kiops_operator;

/* Validate desc and build an operator bound to hip_stream (hipStream_t, NULL
 * = default stream).  *out is owned by the caller until kiops_destroy_operator. */
kiops_status kiops_create_operator(const kiops_operator_desc* desc, void* hip_stream,
                                   kiops_operator** out);
kiops_status kiops_destroy_operator(kiops_operator* op);

/* Workspace needed by kiops_phi_combination for p (0..KIOPS_P_MAX), window q
 * (0 = full orthogonalisation, else 1..8) and options (NULL = defaults). */
kiops_status kiops_workspace_bytes(const kiops_operator* op, int p, int q,
                                   const kiops_options* opts, size_t* bytes);

/* Attach caller-owned device memory (256-byte aligned) used by later solves.
 * The library keeps the pointer, never frees it. */
kiops_status kiops_set_workspace(kiops_operator* op, void* dev_ptr, size_t bytes);

/*
 * One phi-combination (the paper's Task II at a single tau):
 *   tau   >= 0; tau == 0 copies b_0 to w with no product.
 *   p     0..KIOPS_P_MAX; V is a host array of p+1 device pointers, V[k] = b_k.
 *   tol   > 0, absolute tolerance of Eq. (39) (the paper's default is 1e-7).
 *   m_init initial Krylov dimension, clamped into [m_min, m_max] (Algorithm 1).
 *   q     IOP window (Algorithm 2): each new basis vector is orthogonalised
 *         against the last q ones, 1..4 (the paper uses 2); 0 = against all
 *         of them (full Arnoldi), computed as classical Gram-Schmidt with a
 *         Gram-matrix correction, h = c + (c - G c), from the inner products
 *         of an extra phase per step.  5..8 return KIOPS_ERR_UNSUPPORTED.
 *   w     device, N entries, written with the result; may equal V[0], must not
 *         overlap any other V[k].
 *   stats may be NULL.
 * Blocks until the result and statistics are ready.  On NONFINITE or
 * NOT_CONVERGED, w holds the last accepted state (time stats->t_reached).
 */
kiops_status kiops_phi_combination(kiops_operator* op, double tau, int p, const double* const* V,
                                   double tol, int m_init, int q, const kiops_options* opts,
                                   double* w, kiops_stats* stats);

/*
 * kiops_phi_combination_noalloc: kiops_phi_combination with no allocation and
 * no attached workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, results and errors as kiops_phi_combination;
 * the solver's workspace is a fixed array inside the library, 128 MiB per
 * GPU (one copy on every GPU the library runs on, held until the process
 * ends).  A problem whose workspace (kiops_workspace_bytes) exceeds it
 * returns KIOPS_ERR_OUT_OF_MEMORY and launches nothing: at the default
 * m_max = 128 in FP64 that is N up to about 128000 (a 350^2 grid).  Calls no
 * hipMalloc/hipFree; the control words the solve needs cleared are reset by
 * a kernel at the start of every call.  Every call on one GPU uses the same
 * array: calls that overlap on one GPU (other streams, other threads) race
 * and must be serialised by the caller.
 */
kiops_status kiops_phi_combination_noalloc(kiops_operator* op, double tau, int p, const double* const* V,
                                           double tol, int m_init, int q, const kiops_options* opts,
                                           double* w, kiops_stats* stats);

/* kiops_apply: y = A x for the operator's A (Section 3.3: A is only applied),
 * in FP64 whatever the operator's precision, one plain kernel enqueued on the
 * operator's stream and not waited for.  x, y: device, N doubles each, 8-byte
 * aligned, not overlapping.  For callers that need A x outside a solve: the
 * right-hand side f(u) = A u + g(u) of an exponential integrator (Section 2),
 * a residual.  The operator's arrays are read as they are when the kernel runs
 * (a caller that rewrites, say, the reaction field between solves gets the
 * new field).  Errors: INVALID_ARG (null or overlapping vectors), DEVICE. */
kiops_status kiops_apply(kiops_operator* op, const double* x, double* y);

/* Several output times (Algorithm 1 with T = [T_1, ..., T_n] and Algorithm 3):
 * one adaptive integration from 0 to T_n = T_end that, at every accepted
 * substep containing output times T_k < T_now + tau, forms
 * w_k = beta V F2(:, 1) with F2 = exp((T_k - T_now) H_j) from the same basis,
 * then continues.  times: host array of n (1 <= n <= KIOPS_MAX_TIMES) strictly
 * increasing positive values.  task: 2 (Task II) returns
 * w_k = sum_i T_k^i phi_i(T_k A) b_i; 1 (Task I) returns the same scaled by
 * (1 / T_k)^p (Algorithm 1, line 33; with only b_p nonzero this is
 * phi_p(T_k A) b_p).  W: host array of n device pointers (N doubles each),
 * distinct; W[n-1] also holds the running state (it may be V[0], in place);
 * W[k], k < n-1, must not alias any V[i].  The small exponentials of the
 * intermediate outputs count in stats->expms.  Errors as kiops_phi_combination
 * (INVALID_ARG for bad times, task or outputs). */
kiops_status kiops_phi_combination_times(kiops_operator* op, int n, const double* times, int task, int p,
                                         const double* const* V, double tol, int m_init, int q,
                                         const kiops_options* opts, double* const* W, kiops_stats* stats);

/*
 * Batched form: many independent phi-combinations in one persistent launch.
 * The grid is split into groups of workgroups; each group runs its share of
 * the problems one after another (each problem is a full Algorithm 1 solve on
 * that group, with the group's own grid barrier), so problems of different
 * sizes proceed concurrently.  A problem with a large share of the estimated
 * work (N (1 + tau ||A||_1)) gets a group of its own of group_size * 2^k
 * workgroups (such groups take at most half of the launch); the others share
 * groups of group_size, assigned by longest-estimated-work first.  All operators of a batch must have the same
 * kind and precision; p may differ (0..KIOPS_P_MAX), q in 0..4.
 */
typedef struct {
  kiops_operator* op;
  double tau;                 /* >= 0 */
  int32_t p;
  int32_t q;
  const double* const* V;     /* host array of p+1 device pointers */
  double tol;                 /* > 0 */
  int32_t m_init;
  int32_t reserved;
  double* w;                  /* device, N entries; may equal V[0] */
} kiops_problem;

/* Plan of a batch: workspace bytes and the number of groups.  group_size = 0
 * picks a size from the problem sizes; otherwise it is used as given (at most
 * the co-resident workgroups of the device). */
kiops_status kiops_batch_plan(int count, const kiops_problem* probs, const kiops_options* opts,
                              int group_size, size_t* workspace_bytes, int* groups, int* group_size_used);

/* Run a batch.  workspace: caller-owned device memory of at least the planned
 * bytes, 256-byte aligned.  stats: host array of count entries, or NULL.
 * Blocks until every problem is done; returns the first non-OK status of a
 * problem (each problem's own status is in stats[i] via its fields) or OK. */
kiops_status kiops_phi_batch(int count, const kiops_problem* probs, const kiops_options* opts,
                             int group_size, void* workspace, size_t workspace_bytes, void* hip_stream,
                             kiops_stats* stats);

/* Autotuner of the batched form: times the batch for each candidate group
 * size (the better of two runs; candidates: host array, n entries; each the
 * group_size of kiops_phi_batch) and returns the fastest in *best and its time
 * in *best_ms.  The workspace
 * must hold the largest plan among the candidates.  Outputs w are written. */
kiops_status kiops_batch_tune(int count, const kiops_problem* probs, const kiops_options* opts,
                              const int* candidates, int n, void* workspace, size_t workspace_bytes,
                              void* hip_stream, int* best, double* best_ms);

/* Autotuner over batch shapes: times the batch (the better of two runs) for
 * each pair (group_sizes[i], tile_rows[j]) (host arrays of ng and nt entries;
 * each tile_rows 16, 8 or 4, used as kiops_options.tile_rows, the other
 * fields from opts) and returns the fastest pair in *best_group_size, *best_tile_rows and its time in
 * *best_ms.  Operator kinds other than the 2-D 5-point stencil have one tile
 * shape: their candidates differ in group size only.  The workspace must hold
 * the largest plan among the candidates (kiops_batch_plan for each).  Outputs
 * w are written.  Errors as kiops_phi_batch; INVALID_ARG for empty or
 * invalid candidate lists. */
kiops_status kiops_batch_tune_shape(int count, const kiops_problem* probs, const kiops_options* opts,
                                    const int* group_sizes, int ng, const int* tile_rows, int nt,
                                    void* workspace, size_t workspace_bytes, void* hip_stream,
                                    int* best_group_size, int* best_tile_rows, double* best_ms);

/*
 * Served form (continuous batching): one long-lived launch whose workgroups
 * are split into groups of group_size; each admitted request runs on a gang,
 * an aligned run of 2^j groups sized so that each workgroup gets at most
 * points_per_workgroup grid points (capped at the largest power of two of
 * groups the launch holds).  Requests (2-D 5-point or 3-D 7-point stencil
 * operators, FP64 or mixed, p <= 4, q in 1..4) are queued by
 * kiops_server_submit and admitted in arrival order when a gang is free and
 * their workspace fits the memory pool (the HBM budget); when the oldest
 * waiting request finds no free gang, the gang with the fewest busy groups is
 * reserved for it and at most eight later requests may start elsewhere in the
 * meantime.  kiops_server_progress retires finished requests and admits
 * waiting ones.  The launch holds one workgroup fewer per CU than fit there
 * (one, for the current served kernel), so the device keeps room for the
 * copies and small kernels of other streams.  Memory: the caller's workspace holds the
 * per-group state and the pool; the group queues and parameter blocks, which
 * the host writes while the launch runs, are a small mailbox of fine-grained
 * device memory (about 6.3 KB per group) that the library allocates on the
 * first server of a device and reuses for later ones (it is never freed).  Not
 * thread-safe: one host thread drives a server.  A bounded wait that expires
 * inside the launch (a minute without progress) fails the request with
 * KIOPS_ERR_DEVICE and the server with it: every later call returns
 * KIOPS_ERR_DEVICE.
 */
typedef struct kiops_server kiops_server;

/* Bytes of the fixed part of a server workspace for groups of group_size
 * workgroups (0 = 16; a multiple of 8), and the number of groups; the pool is
 * what the caller adds on top. */
kiops_status kiops_server_fixed_bytes(int group_size, size_t* bytes, int* groups);

/* Launch the server on run_stream (hipStream_t); io_stream (another stream)
 * carries the uploads and polls.  points_per_workgroup: gang sizing (0 =
 * 8192).  workspace: device, 256-byte aligned, at least the fixed bytes; the
 * remainder is the request pool (the whole workspace is cleared here).
 * OUT_OF_MEMORY if the mailbox cannot be allocated. */
kiops_status kiops_server_create(int group_size, int64_t points_per_workgroup, void* workspace,
                                 size_t workspace_bytes, void* run_stream, void* io_stream, kiops_server** out);

/* Queue a request; *ticket identifies it.  The problem's arrays must stay
 * valid until the request is done.  BUDGET if it can never fit the pool. */
kiops_status kiops_server_submit(kiops_server* s, const kiops_problem* pr, int64_t* ticket);

/* Retire finished requests and admit waiting ones; *running and *waiting
 * report the counts afterwards (either may be NULL). */
kiops_status kiops_server_progress(kiops_server* s, int* running, int* waiting);

/* *done = 1 once the request has finished; then *stats holds its statistics
 * (stats->status is its status). */
kiops_status kiops_server_result(kiops_server* s, int64_t ticket, int* done, kiops_stats* stats);

/* Close the queues, wait for the launch to end and free the host object. */
kiops_status kiops_server_destroy(kiops_server* s);

/* Human-readable name of a status code (static storage). */
const char* kiops_status_string(kiops_status s);

/* Number of compute units and the persistent grid the library would use for
 * this operator (diagnostics). */
kiops_status kiops_device_info(const kiops_operator* op, int* compute_units, int* grid_blocks);

/*
 * Diagnostics that run the same device code as kiops_phi_combination:
 *
 * kiops_iop_basis: the first substep's basis after m steps of Algorithm 2
 *   from the start vector [b_0; mu e_p] (B scaled by nu, Eqs. (48)-(49)).
 *   basis (device, (m+1) x (N+p) row-major, row i = v_{i+1}), H (device,
 *   (m+1) x m row-major), *j_done = steps made (< m after a breakdown),
 *   *beta = norm of the start vector, *nu_out = nu.
 *
 *   Needs the workspace of kiops_workspace_bytes(op, p, q, {m_max = m}) plus
 *   8*N + 256 bytes (b_0 is staged there).
 *
 * kiops_small_expm: F = exp(tau Hs) for a device n x n row-major matrix Hs
 *   (n <= KIOPS_M_MAX_LIMIT + 1), F device n x n, by the device's scaling-and-squaring
 *   routine (Section 3.3.1; truncated Taylor series, degree <= 16).  scratch: device,
 *   KIOPS_EXPM_SCRATCH_DOUBLES doubles, caller-owned.
 */
kiops_status kiops_iop_basis(kiops_operator* op, int p, const double* const* V, int m, int q,
                             double* basis, double* H, int* j_done, double* beta, double* nu_out);
#define KIOPS_EXPM_SCRATCH_DOUBLES (9 * 144 * 144)
kiops_status kiops_small_expm(int n, const double* Hs, double tau, double* F, double* scratch,
                              void* hip_stream);

/*
 * kiops_stream_probe: dst[i] = src[0][i] + ... + src[nsrc-1][i], i < n, one
 *   plain unit-stride streaming kernel (16-byte loads, several in flight per
 *   thread) on `blocks` workgroups of 256 threads, enqueued on hip_stream and
 *   not waited for.  Diagnostics: it measures the HBM bandwidth a streaming
 *   kernel reaches on this device (nsrc reads + 1 write per element), the
 *   ceiling the solver's passes are compared with, and is a kernel of known
 *   traffic for scaling hardware byte counters.  src[s] and dst are device
 *   arrays of n doubles, 16-byte aligned, caller-owned, dst not overlapping
 *   any src; 1 <= nsrc <= 8; n even.  Errors: INVALID_ARG (nothing launched),
 *   DEVICE (the launch failed).
 */
kiops_status kiops_stream_probe(const double* const* src, int nsrc, double* dst, int64_t n, int blocks,
                                void* hip_stream);

/* Host-side copy of the device step controller (Algorithm 4), for tests. */
typedef struct {
  double T_end, tol, T_now, tau;
  int32_t m_min, m_max, m, have_old;
  double tau_old, eps_old, omega_old;
  int32_t m_old, reserved;
} kiops_ctrl_in;
typedef struct {
  int32_t accept, m_new, branch, reserved;   /* branch: 0 breakdown, 1 tau_reject, 2 tau_accept, 3 m_reject, 4 m_accept, -1 non-finite */
  double tau_new, omega;
} kiops_ctrl_out;
kiops_status kiops_controller_decide(const kiops_ctrl_in* in, int j, double eps, int breakdown,
                                     kiops_ctrl_out* out);

#ifdef __cplusplus
}
#endif
#endif /* KIOPS_H */
