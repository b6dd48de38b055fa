/*
 * psdproj -- randomized approximate projection onto the PSD cone on AMD MI355X (gfx950).
 *
 * C ABI, version 1.  Implements the two randomized projections of Jones & Anderson,
 * "Approximate Projection onto the Positive Semidefinite Cone Using Randomization":
 *
 *   plain  (Alg. 2): Q = range_finder(X, k, p, q)         (Alg. 1)
 *                    Q^T X Q = V D V^T
 *                    P = Q V max(D, 0) V^T Q^T
 *   scaled (Alg. 3): B = (X + alpha I) / alpha, Q = range_finder(B, k, p, q)
 *                    Q^T B Q = V D V^T
 *                    P = alpha Q V (max(D, 1) - I) V^T Q^T
 *                    alpha is given, or estimated by Alg. 5 (two runs of the power
 *                    iteration of Alg. 4, N steps each).  For N <= 32 both runs share
 *                    each read of X: the first run as written, and beside it a Krylov
 *                    basis of the second run's start vector whose shifts follow the first
 *                    run's sigma_1 estimate (tr(X)/n for the first two), from which the
 *                    second run's last two iterates are formed once sigma_1 is known
 *                    (N + 1 products of two vectors instead of 2 (N + 1) of one; alpha
 *                    equal to the literal iteration's to near FP64 rounding).  For N > 32
 *                    the runs are made one after the other.
 *
 * The oversampling parameter l of the paper is called p here; the sketch width is r = k + p.
 * The range finder orthonormalises after every product with X (subspace iteration), which
 * spans the same range as the printed (X X^T)^q X Omega (Alg. 1) in exact arithmetic.
 * All r eigenpairs of the r x r compressed matrix are kept; the clamp decides which
 * contribute.
 *
 * Memory and ownership
 *   X ("A" below), P, the workspace and result_dev are caller-owned DEVICE memory on the
 *   current HIP device.  Plans and servers are library-owned opaque handles.  A must stay
 *   valid and unchanged until the stream has passed the call (or the ticket completed).
 *   A must be exactly symmetric (the method projects a symmetric matrix, Sec. 2).  The passes
 *   of Alg. 1-3 read it in full (the BF16X3 pass reads A's rows as the columns of A^T = A);
 *   the power iterations of Alg. 4/5 read only its upper triangle and diagonal.  Row- and
 *   column-major are the same for a symmetric matrix; element (i, j) is at A[i * lda + j].
 *   Precision FP64: A and P hold double.  FP32 and BF16X3: A and P hold float.
 *   Requirements: lda >= n, ldp >= n, A and P 16-byte aligned.  When lda * sizeof(element)
 *   and n * sizeof(element) are multiples of 16 the passes over A use vector loads;
 *   otherwise they fall back to element loads (correct, slower).  P may alias A exactly (same pointer and ld): the
 *   rebuild runs after the last read of A.  Any other overlap is E_INVALID.
 *
 * Errors
 *   Argument errors are returned synchronously and nothing is enqueued.  Errors found on
 *   the device (non-finite input, estimated alpha <= 0) are written to
 *   result_dev->status after the stream completes; P is then unspecified.  No exception
 *   or abort crosses the ABI.
 *
 * Determinism
 *   No floating-point atomics are used: a fixed (desc, A) gives bitwise identical P
 *   whether run alone, in a batch, or through the server.
 *
 * Random numbers (Alg. 1 test matrix, Alg. 4 start vectors): Philox4x32-10 with
 *   key = (seed mod 2^32, seed div 2^32), counter = (c mod 2^32, c div 2^32, stream, 0).
 *   Element g of a stream uses counter g/2; words (x0,x1) and (x2,x3) give
 *   u = (((x_hi << 32) | x_lo) >> 11) * 2^-53 + 2^-54, and Box-Muller gives
 *   sqrt(-2 ln u1) cos(2 pi u2) (even g) or sqrt(-2 ln u1) sin(2 pi u2) (odd g).
 *   Test-matrix entry (i, j) is element j * n + i of stream 0; the start vectors of the
 *   first and second power iteration are streams 1 and 2.
 */
#ifndef PSDPROJ_H
#define PSDPROJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PSDPROJ_ABI_VERSION 1
#define PSDPROJ_MAX_RANK 256   /* k + p limit of this build */
#define PSDPROJ_STATIC_SCRATCH_BYTES (64u << 20)   /* workspace of psdproj_run_static, per device */

typedef enum {
    PSDPROJ_OK = 0,
    PSDPROJ_E_INVALID = 1,     /* bad argument (synchronous) */
    PSDPROJ_E_ALPHA = 2,       /* scaled: estimated alpha <= 0 or not finite (device) */
    PSDPROJ_E_NONFINITE = 3,   /* NaN/Inf met in a Gram or compressed matrix (device) */
    PSDPROJ_E_BREAKDOWN = 4,   /* reserved, never returned: a sketch column that the
                                  orthonormalisation finds dependent is dropped (a zero column
                                  of Q), which leaves range(Q) = range(Y) exact, and a sketch
                                  with no independent column is Y = 0, whose projection P = 0
                                  is the correct result (Alg. 1, Alg. 2) */
    PSDPROJ_E_NOMEM = 5,       /* workspace too small or host allocation failed */
    PSDPROJ_E_BUDGET = 6,      /* server: request larger than the HBM budget */
    PSDPROJ_E_DEVICE = 7,      /* a HIP runtime call failed */
    PSDPROJ_E_PENDING = 8,     /* server: ticket not finished yet */
    PSDPROJ_E_TIMEOUT = 9,     /* server: wait timed out */
    PSDPROJ_E_SCRATCH = 10     /* psdproj_run_static: the problem's workspace exceeds the static
                                  scratch array (synchronous) */
} psdproj_status;

typedef enum { PSDPROJ_PLAIN = 0 /* Alg. 2 */, PSDPROJ_SCALED = 1 /* Alg. 3 */ } psdproj_variant;

typedef enum {
    PSDPROJ_FP64 = 0,    /* A, P, panels in double; FP64 MFMA */
    PSDPROJ_FP32 = 1,    /* A, P, panels in float; FP32 MFMA, FP32 accumulation */
    PSDPROJ_BF16X3 = 2   /* A, P in float; products as hi*hi + hi*lo + lo*hi of BF16 splits
                            on MFMA with FP32 accumulation */
} psdproj_precision;

/* One projection problem.  Gram/Cholesky factors, the compressed matrix and its
 * eigensolve are FP64 in every precision. */
typedef struct {
    int64_t  n;           /* order of A, >= 1 */
    int32_t  k;           /* target rank, >= 1 */
    int32_t  p;           /* oversampling (the paper's l), >= 0; k + p <= min(n, 256) */
    int32_t  q;           /* power iterations, 0..16 */
    int32_t  variant;     /* psdproj_variant */
    int32_t  precision;   /* psdproj_precision */
    uint64_t seed;        /* Philox key for the test matrix and power-iteration starts */
    double   alpha;       /* scaled: > 0 use as given; <= 0 estimate with Alg. 5 */
    int32_t  alpha_iters; /* N of Alg. 4/5 when alpha is estimated, 1..1000 (paper: 10) */
    uint32_t flags;       /* PSDPROJ_FLAG_* (other bits must be 0) */
} psdproj_desc;

/* flags: the test matrix of Alg. 1 is the structured one of Sec. 3.1's footnote (a subsampled
 * randomized Hadamard transform, the real form of the SRFT) instead of Gaussian:
 *   Omega[i][j] = d_i (-1)^popcount(i & s_j), entries exactly +1 or -1 (the transform's
 *   normalisation is left out: only range(X Omega) is used), d_i = +-1 from the low bit of
 *   Philox word x0 of counter i in stream 3, and s_j = pi(j) for a permutation pi of [0, 2^m),
 *   2^m >= n (m >= 1): a four-round Feistel network on m + (m mod 2) bits (round t adds the low
 *   half-width bits of word x0 of counter t 2^(half width) + R, stream 4, to the left half),
 *   re-applied while the value is 2^m or more.  The matrix is formed on the device and applied
 *   by the same passes as a Gaussian one. */
#define PSDPROJ_FLAG_SRHT 1u
/* flags: the plan is for a sparse A given to psdproj_run_csr (and only there): A in CSR form with
 * both triangles of the symmetric matrix stored.  The passes of Alg. 1-3 then add a_ij Z[j, :]
 * over the stored nonzeros (FP64 for FP64 storage, FP32 for FP32 and BF16X3, whose split
 * products are not used) and the power iterations of Alg. 4 use the sparse product; every other
 * step, and P (dense n x n), are as for a dense A. */
#define PSDPROJ_FLAG_CSR 2u

/* Written by the device at the end of a run (read it after synchronising). */
typedef struct {
    int32_t status;       /* psdproj_status */
    int32_t r_plus;       /* number of eigenpairs with positive weight */
    double  alpha_used;   /* scaled: alpha applied (given or estimated); plain: 0 */
    double  sigma1;       /* scaled with estimation: Alg. 4 on X; else 0 */
    double  sigma2;       /* scaled with estimation: Alg. 4 on X - sigma1 I; else 0 */
} psdproj_result;

/* Where intermediate results live inside a run's workspace (byte offsets), for
 * inspection after the stream has passed the run.  Panels are column-major with
 * leading dimension panel_ld elements (column j of an n x r panel starts at j*panel_ld);
 * panel_ld is a multiple of 128 and at least n + 32, and rows n .. panel_ld-1 hold zeros. */
typedef struct {
    int32_t  r, r_pad, panel_ld, split_k;
    int32_t  panel_elem_bytes;  /* 8 (FP64) or 4 (FP32, BF16X3) */
    size_t   omega;      /* test matrix Omega, n x r, panel precision */
    size_t   q_panel;    /* final orthonormal basis Q, n x r, panel precision */
    size_t   compressed; /* C = Q^T M(Q) symmetrised, r x r double, ld r_pad, column-major */
    size_t   evals;      /* eigenvalues of C, ascending, r doubles */
    size_t   weights;    /* clamped weights of the kept eigenpairs (descending eigenvalue order), r_plus doubles */
    size_t   factor;     /* W = Q V_keep diag(sqrt(w)), n x r_plus, panel precision; P = W W^T */
    size_t   power_vec;  /* the two FP64 vectors (ping-pong) of the power iteration of Alg. 4 */
    size_t   y_panel;    /* output of the last pass over A, M(Q), n x r, panel precision */
    size_t   gram;       /* last CholeskyQR Gram matrix, r x r double, ld r_pad, column-major */
    size_t   total;      /* workspace bytes */
} psdproj_layout;

typedef struct psdproj_plan_s*   psdproj_plan_t;
typedef struct psdproj_server_s* psdproj_server_t;
typedef void*                    psdproj_stream_t;   /* a hipStream_t (NULL = default stream) */

/* Validate desc and fix the tiling and workspace size.  Host only: touches no device.
 * E_INVALID on a bad descriptor.  *out must be released with psdproj_plan_destroy. */
psdproj_status psdproj_plan(const psdproj_desc* desc, psdproj_plan_t* out, size_t* workspace_bytes);
void           psdproj_plan_destroy(psdproj_plan_t plan);
psdproj_status psdproj_plan_layout(psdproj_plan_t plan, psdproj_layout* out);

/* One projection, enqueued on stream (asynchronous).  workspace: at least the bytes that
 * psdproj_plan reported, 256-byte aligned, device memory.  result_dev: device memory. */
psdproj_status psdproj_run(psdproj_plan_t plan, const void* A, int64_t lda, void* P, int64_t ldp,
                           void* workspace, psdproj_result* result_dev, psdproj_stream_t stream);

/* One projection of a sparse symmetric A (plan created with PSDPROJ_FLAG_CSR): row_ptr (n + 1
 * int32, non-decreasing), col_idx (nnz int32 in [0, n)) and vals (nnz double for FP64, float
 * otherwise) in device memory, both triangles stored.  P is the dense n x n result (row stride
 * ldp, 16-byte aligned, not overlapping vals), workspace as for psdproj_run.  Column indices
 * outside [0, n) and row ranges outside [0, nnz) are skipped and reported as E_INVALID in
 * result_dev->status. */
psdproj_status psdproj_run_csr(psdproj_plan_t plan, const int32_t* row_ptr, const int32_t* col_idx, const void* vals,
                               int64_t nnz, void* P, int64_t ldp, void* workspace, psdproj_result* result_dev,
                               psdproj_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): psdproj_run without a workspace argument.  Its workspace is a
 * file-scope device array of PSDPROJ_STATIC_SCRATCH_BYTES (64 MiB) that each device the library
 * runs on holds until the process ends; its header is written by a kernel that carries it in its
 * arguments.  The call allocates nothing (no hipMalloc or hipFree, no pinned staging buffer, no
 * event) and times nothing while kernel timing is enabled.  A, P, ld's and result_dev as for
 * psdproj_run, and the same P bit for bit.  E_SCRATCH (synchronous, nothing enqueued) when the
 * plan's workspace exceeds the array; psdproj_static_scratch_bytes reports both sizes (for
 * example n = 4096, k + p = 110 needs about 31 MB in BF16X3).  Every call on a device uses that
 * device's one array: calls on one stream run one after the other, but calls whose runs overlap
 * on one device (other streams, other threads) race on the array and give undefined results. */
psdproj_status psdproj_run_static(psdproj_plan_t plan, const void* A, int64_t lda, void* P, int64_t ldp,
                                  psdproj_result* result_dev, psdproj_stream_t stream);
psdproj_status psdproj_static_scratch_bytes(psdproj_plan_t plan, size_t* needed, size_t* capacity);

/* count independent projections in one grouped launch sequence (each kernel's grid covers
 * the tiles of all problems).  Arrays have count entries.  workspace_bytes must be at least
 * what psdproj_batch_workspace reports for the same plans.  Problem i's result goes to
 * results_dev[i].  Every problem gets the tiling it would get alone, so its P is bitwise
 * identical to a psdproj_run of the same plan. */
psdproj_status psdproj_batch_workspace(int32_t count, const psdproj_plan_t* plans, size_t* bytes);
psdproj_status psdproj_batch(int32_t count, const psdproj_plan_t* plans, const void* const* A,
                             const int64_t* lda, void* const* P, const int64_t* ldp, void* workspace,
                             size_t workspace_bytes, psdproj_result* results_dev, psdproj_stream_t stream);

/* The launch sequence of a run or batch captured once as a HIP graph and replayed.  A grouped
 * sequence reaches its problems only through the descriptor header at the start of the
 * workspace, so psdproj_run, psdproj_batch and the server replay a captured sequence whenever a
 * run has the same schedule (plans, grouping) and the same workspace address as an earlier one;
 * the header is rewritten before each replay (a sequence is captured the second time it is
 * seen, at most 64 are kept; PSDPROJ_GRAPHS=0 in the environment launches every kernel
 * directly, and so does a run while kernel timing is enabled).  psdproj_graph_stats reports how
 * many sequences were captured and replayed that way.
 * psdproj_graph_create captures the batch given (arguments as psdproj_batch) into a graph that
 * owns nothing but its launches: it writes the header into the workspace now (synchronously) and
 * every psdproj_graph_launch replays the whole sequence on `stream` against the same A, P,
 * workspace and results, which must stay valid, and the workspace unused by anything else, until
 * psdproj_graph_destroy.  A may change between launches.  Each replay gives bitwise the P of
 * psdproj_batch on the same inputs. */
typedef struct psdproj_graph_s* psdproj_graph_t;
psdproj_status psdproj_graph_create(int32_t count, const psdproj_plan_t* plans, const void* const* A,
                                    const int64_t* lda, void* const* P, const int64_t* ldp, void* workspace,
                                    size_t workspace_bytes, psdproj_result* results_dev, psdproj_graph_t* out);
psdproj_status psdproj_graph_launch(psdproj_graph_t graph, psdproj_stream_t stream);
void           psdproj_graph_destroy(psdproj_graph_t graph);
psdproj_status psdproj_graph_stats(int64_t* captures, int64_t* replays);

/* The exact projection X_+ = U max(D, 0) U^T of Thm 1 (the scal = -1 branch of Alg. 6, and the
 * O(n^3) reference the randomized projections are measured against).  Computed without an
 * eigendecomposition, through the polar form X_+ = (X + |X|) / 2 with |X| = X sign(X) and sign(X)
 * by the scaled Newton-Schulz iteration started from X / ||X||_F, every product an n x n FP64
 * GEMM on the matrix cores.  Eigenvalues with |lambda| >= l0 ||X||_F converge to round-off (l0 =
 * 1e-13 for FP64 storage, 1e-9 for FP32 / BF16X3); each smaller one adds at most l0 ||X||_F / 2
 * to the error.  A, P: n x n symmetric, double (FP64) or float (FP32, BF16X3), row strides lda,
 * ldp; P may alias A exactly.  workspace: psdproj_exact_workspace bytes (4 n^2 doubles and a
 * little more), 256-byte aligned.  result_dev->r_plus receives the number of positive eigenvalues
 * (round(Tr(I + sign X) / 2)); status NONFINITE when ||X||_F is not finite.  n <= 65535. */
psdproj_status psdproj_exact_workspace(int64_t n, int32_t precision, size_t* bytes);
psdproj_status psdproj_exact(int64_t n, int32_t precision, const void* A, int64_t lda, void* P, int64_t ldp,
                             void* workspace, size_t workspace_bytes, psdproj_result* result_dev,
                             psdproj_stream_t stream);

/* Dual gradient descent for the semidefinite least-squares problem (Alg. 6, supplementary SDP
 * section):  min over PSD X of 1/2 ||X - C/rho||_F^2  subject to  Tr(A_i^T X) = b_i, i = 1..m.
 * Iteration it (1-based) forms X = C/rho + sum_i y_i A_i, projects it (scal = 0: Alg. 2;
 * scal = 1: Alg. 3 with alpha by Alg. 5, N = alpha_iters; scal = -1: the exact projection of
 * Thm 1), forms g_i = Tr(A_i^T Xhat_+) - b_i and updates y <- y - beta g.  The projection of
 * iteration it draws its random numbers from Philox key seed + it - 1.  The loop stops after the
 * first iteration whose ||g||_2 <= eps, or after max_iters iterations (at least one runs).
 * Storage: C, the A_i and X in double (precision FP64) or float (FP32, BF16X3); A_i at
 * A + i * a_stride elements with row stride lda; b (m doubles) and y (m doubles: the initial
 * iterate in, the final one out) in device memory; X (n x n, row stride ldx) receives the last
 * projection, the approximate primal solution.  The call runs the iterations on `stream` and
 * synchronises with it once per iteration to read ||g||; info (host memory) receives the status
 * (a device error of a projection stops the loop), the iterations run and the last ||g||. */
typedef struct {
    int64_t  n;           /* order, 1 .. 65535 */
    int32_t  m;           /* number of constraints, >= 1 */
    int32_t  k, p, q;     /* projection parameters as in psdproj_desc (unused for scal = -1) */
    int32_t  scal;        /* -1 exact (Thm 1), 0 Alg. 2, 1 Alg. 3 */
    int32_t  precision;   /* psdproj_precision */
    int32_t  alpha_iters; /* N of Alg. 5 (scal = 1) */
    int32_t  max_iters;   /* M, >= 1 */
    uint32_t flags;       /* reserved, must be 0 */
    double   rho;         /* > 0 */
    double   beta;        /* step size, > 0 */
    double   eps;         /* stopping tolerance on ||g||_2, >= 0 */
    uint64_t seed;
} psdproj_sdls_desc;
typedef struct { int32_t status; int32_t iters; double grad_norm; } psdproj_sdls_info;
psdproj_status psdproj_sdls_workspace(const psdproj_sdls_desc* desc, size_t* bytes);
psdproj_status psdproj_sdls_solve(const psdproj_sdls_desc* desc, const void* C, int64_t ldc, const void* A,
                                  int64_t lda, int64_t a_stride, const double* b_dev, double* y_dev, void* X,
                                  int64_t ldx, void* workspace, size_t workspace_bytes, psdproj_sdls_info* info,
                                  psdproj_stream_t stream);

/* Continuous-batching request server on the current device (the batching of many independent
 * projections, each one Alg. 1 + Alg. 2 or Alg. 3).  hbm_budget_bytes of device memory is
 * allocated at creation and holds the workspaces of the requests in flight.  Requests are
 * admitted in FIFO order while their workspaces fit in it and fewer than max_inflight are in
 * flight.  The budget covers only the memory the server itself allocates: A and P are
 * caller-owned buffers that exist before submit and stay allocated whether or not a request
 * is admitted, so admitting or deferring a request changes nothing in their footprint.  Each
 * admission round becomes one grouped launch sequence (as psdproj_batch) on a free one of four
 * server streams, and arrivals join at the next round.  A and P stay caller-owned and
 * must stay valid until the ticket completes.  Each request's P is bitwise identical to a
 * psdproj_run of the same desc.  submit validates synchronously (E_INVALID; E_BUDGET when the
 * request alone exceeds the budget); a device failure of a batch is reported in the status
 * of each of its requests.  All server functions are thread-safe. */
psdproj_status psdproj_server_create(size_t hbm_budget_bytes, int32_t max_inflight, psdproj_server_t* out);
psdproj_status psdproj_submit(psdproj_server_t server, const psdproj_desc* desc, const void* A, int64_t lda,
                              void* P, int64_t ldp, uint64_t* ticket);
/* E_PENDING while in flight; otherwise copies the result to *out (host memory), returns
 * PSDPROJ_OK, and forgets the ticket. */
psdproj_status psdproj_poll(psdproj_server_t server, uint64_t ticket, psdproj_result* out);
/* Blocks until the ticket completes (timeout_s < 0: no limit); E_TIMEOUT keeps the ticket. */
psdproj_status psdproj_wait(psdproj_server_t server, uint64_t ticket, psdproj_result* out, double timeout_s);
/* Per-request timestamps in seconds since server creation: submit, admit, finish. */
psdproj_status psdproj_server_times(psdproj_server_t server, uint64_t ticket, double* t_submit,
                                    double* t_admit, double* t_finish);
void           psdproj_server_destroy(psdproj_server_t server);

/* Utilities (asynchronous on stream, device output). */
/* Philox4x32-10 words for counters c0 .. c0+count-1 of (seed, stream): out[4*i + w]. */
psdproj_status psdproj_philox_words(uint64_t seed, uint32_t stream_id, uint64_t c0, int64_t count,
                                    uint32_t* out_dev, psdproj_stream_t stream);
/* The n x r structured test matrix of PSDPROJ_FLAG_SRHT for key seed, as double, column-major
 * (entry (i, j) at out_dev[j * n + i]); 1 <= r <= n <= 2^20. */
psdproj_status psdproj_srht_matrix(uint64_t seed, int64_t n, int32_t r, double* out_dev, psdproj_stream_t stream);
/* Elements start .. start+count-1 of a Gaussian stream, as double. */
psdproj_status psdproj_gaussian(uint64_t seed, uint32_t stream_id, uint64_t start, int64_t count,
                                double* out_dev, psdproj_stream_t stream);

/* Tile shapes.  The split-K factor of the passes over A (the number of K chunks whose partial
 * products are summed in a fixed order) comes from a table keyed by precision, n bucket
 * (2^b <= n < 2^(b+1), b clamped to 6..14) and padded width r_pad, written by the tuner that
 * times every candidate on the GPU (paper_2410_19208_amd/tune.py); outside the table a built-in
 * rule applies.  psdproj_tile_override(precision, split) makes plans created afterwards with that
 * precision use split (1..16; 0 restores the table), for the tuner's measurements.  A plan keeps
 * the factor it was created with, so a problem gets the same P alone, batched or served. */
psdproj_status psdproj_tile_override(int32_t precision, int32_t split);

/* Kernel timing (tracing aid, off by default).  While enabled, every launch of the library
 * is bracketed by HIP events recorded on the launch stream; psdproj_profile_read waits for
 * them and returns the accumulated device time and launch count of one kernel kind
 * (0 <= kind < psdproj_kernel_kinds(); psdproj_kernel_name gives the kernel's symbol stem).
 * psdproj_profile_select restricts the timing to the kinds whose bit is set in `kinds`
 * (bit k for kind k; all kinds until it is called; bits past the last kind are ignored).
 * Each timed launch adds two event records to its stream, which lengthen a step of many
 * short launches, so a throughput measurement times only the kinds it reports. */
psdproj_status psdproj_profile_enable(int32_t enable);
psdproj_status psdproj_profile_select(uint64_t kinds);
psdproj_status psdproj_profile_reset(void);
psdproj_status psdproj_profile_read(int32_t kind, double* total_ms, int64_t* launches);
int32_t        psdproj_kernel_kinds(void);
const char*    psdproj_kernel_name(int32_t kind);

const char* psdproj_status_str(psdproj_status status);
int32_t     psdproj_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PSDPROJ_H */
