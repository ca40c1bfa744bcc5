/*
 * svds.h -- C ABI of the MI355X (gfx950) two-stage hybrid partial SVD.
 *
 * The library computes the k largest or smallest singular triplets
 * (sigma_i, u_i, v_i) of a sparse m x n matrix A, A v_i = sigma_i u_i
 * (Section 1, eq. 1), to the residual of eq. (res):
 *     sqrt(||A v - sigma u||^2 + ||A^T u - sigma v||^2) < ||A||_2 * tol,
 * with the PHSVDS method (Algorithm 1, Section 3.1): a block GD+k eigensolver
 * on the normal equations C = A^T A (or A A^T when m < n, Section 2.1),
 * then, when stage 1 cannot reach the tolerance, the same eigensolver on the
 * augmented matrix B = [0 A^T; A 0] (eq. B_Augmented) seeded with the
 * stage-1 vectors [v; u]/sqrt(2) (eq. B_Initguess), using refined
 * projection at the stage-1 lower bounds for the smallest values
 * (Section 3.2).  The parameters mirror the paper's primme_svds_params
 * (Section 3.4) where they apply.
 *
 * Conventions for every entry point:
 *  - Matrix and vector pointers are DEVICE pointers unless marked "host".
 *    The caller owns all of them; the library never frees or keeps them
 *    past the call.
 *  - Dense matrices are column-major with the given leading dimension.
 *  - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL =
 *    default stream).  Calls that return results to host memory
 *    synchronise that stream before they return.
 *  - No C++ exception crosses the ABI; every entry point returns an int
 *    status code (below).  svds_error_string() names it.
 *  - Library state that outlives a call, all of it behind locks: per device,
 *    one stream-ordered memory pool; a cache of released device blocks keyed
 *    by (stream, size), at most 16 GiB for the process, reused by later calls
 *    on the same stream (svds_stream_release() frees the blocks of a stream
 *    before the caller destroys it); a table of SpMM launch shapes keyed by a
 *    matrix signature (autotuner); in each prepared matrix the launch
 *    shapes its solves use per block width; up to 4096 small pinned host
 *    records per (device, size) kept for reuse by later solves (control and
 *    status records); and the 64 MiB static scratch array of
 *    svds_matrix_normal_noalloc on every device the library runs on (part
 *    of the loaded code, held until the process ends).  Distinct streams may
 *    run distinct solves concurrently, also on one prepared matrix.
 *  - Environment: SVDS_DEBUG (any value) prints the autotuner's trial
 *    timings and the batched solve's phase times on stderr.
 */
#ifndef SVDS_H
#define SVDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define SVDS_OK 0
#define SVDS_NOT_CONVERGED 1   /* budget exhausted: the first stats.nconv   */
                               /* outputs are converged, the rest are the   */
                               /* best approximations (cf. initSize being   */
                               /* set to the converged count, Section 3.4)  */
#define SVDS_ERR_ARG (-1)      /* invalid argument (sizes, k, tol, ld, ...) */
#define SVDS_ERR_CSR (-2)      /* malformed CSR matrix                      */
#define SVDS_ERR_OOM (-3)      /* device allocation failed                  */
#define SVDS_ERR_HIP (-4)      /* HIP runtime error                         */
#define SVDS_ERR_BREAKDOWN (-5)/* NaN/Inf or repeated orthogonalisation     */
                               /* breakdown                                 */

/* ---- targets, precision, preconditioning --------------------------------- */
#define SVDS_LARGEST 0          /* largest singular values (Section 3.4)    */
#define SVDS_SMALLEST 1         /* smallest singular values                 */

#define SVDS_FP64 0             /* everything in FP64                       */
#define SVDS_MIXED 1            /* stage 1 stores the basis and does SpMM   */
                                /* in FP32 with BF16 MFMA projections; the  */
                                /* Rayleigh-Ritz eigenproblem, Gram matrix, */
                                /* reorthogonalisation and stage 2 are FP64, */
                                /* except that for the largest values the   */
                                /* JD correction equation's products with B */
                                /* use FP32 copies of A (the outer residuals */
                                /* and convergence tests stay FP64)         */

#define SVDS_PC_NONE 0          /* K = I                                     */
#define SVDS_PC_JACOBI 1        /* K = diag(A^T A)^-1 on C (diag(A A^T) when */
                                /* m < n); on B the composition              */
                                /* [K A^T y_u; A K y_v] (applyPreconditioner */
                                /* modes AtA / augmented, Section 3.4)       */
#define SVDS_PC_BLOCKJACOBI 3   /* K = inverses of the diagonal blocks of    */
                                /* A^T A over contiguous ranges of           */
                                /* opts.pc_block columns (Section 4's        */
                                /* generic preconditioner), same composition */
                                /* on B                                      */
#define SVDS_PC_LEARNED 2       /* K = the learned polynomial preconditioner */
                                /* of opts.pc_model (svds_lpc_* below), with */
                                /* the same composition on B                 */

#define SVDS_METHOD_HYBRID 0     /* the two-stage method (default)          */
#define SVDS_METHOD_NORMAL 1     /* stage 1 on A^T A alone, accepted as it  */
                                 /* ends (primme_svds_normalequations)      */
#define SVDS_METHOD_AUGMENTED 2  /* stage 2 on B alone from random vectors, */
                                 /* largest values only                     */
                                 /* (primme_svds_augmented; Section 3.4)    */

#define SVDS_STAGE2_GDK 0        /* second stage: GD+k with the stage-2      */
                                 /* preconditioner on the residuals         */
#define SVDS_STAGE2_JD 1         /* second stage (default): Jacobi-Davidson, */
                                 /* the correction equation                 */
                                 /* (I - QQ^T)(B - s I)(I - QQ^T) t = r     */
                                 /* (Q: locked and block Ritz vectors; s:   */
                                 /* the stage-1 bound for the smallest      */
                                 /* values, the Ritz value for the largest) */
                                 /* solved by symmetric QMR with the        */
                                 /* projected stage-2 preconditioner: the   */
                                 /* paper's default second stage (JDQMR,    */
                                 /* Section 3.4)                            */

/* ---- CSR matrix (device arrays, caller-owned, read-only) ----------------- */
typedef struct svds_csr {
  int64_t m, n, nnz;
  const int64_t* rowptr;  /* m+1 entries, rowptr[0] = 0, nondecreasing,    */
                          /* rowptr[m] = nnz                                */
  const int32_t* colind;  /* nnz entries, 0 <= col < n, strictly increasing */
                          /* within each row (duplicates are rejected)      */
  const double* values;   /* nnz entries                                    */
} svds_csr;

/* ---- options (host struct) ----------------------------------------------- */
typedef struct svds_opts {
  int max_basis_size;     /* g; 0 -> 15 when seeking < 10 largest, else 35  */
  int min_restart_size;   /* r; 0 -> 6 when seeking < 10 largest, else 14   */
                          /* (defaults of Section 3.4)                      */
  int block_size;         /* b, pairs corrected per iteration; 0 -> 1       */
  int max_prev_retain;    /* p, GD+k "+k" vectors kept at restart; -1 -> b  */
  int64_t max_matvecs;    /* budget in columns multiplied by A or A^T;      */
                          /* 0 -> 2,000,000                                 */
  double norm_A;          /* ||A||_2 if known; <= 0 -> 30-step Krylov       */
                          /* estimate on C                                  */
  double stage1_tol;      /* user tolerance of the stage-1 test; <= 0 ->    */
                          /* tol (per-stage settings, Section 3.4)          */
  uint64_t seed;          /* counter-based random vectors (initial block,   */
                          /* breakdown replacements)                        */
  int precision;          /* SVDS_FP64 or SVDS_MIXED                        */
  int precond;            /* SVDS_PC_NONE, SVDS_PC_JACOBI,                  */
                          /* SVDS_PC_BLOCKJACOBI or SVDS_PC_LEARNED         */
  int force_stage2;       /* 1: run stage 2 even when stage 1 met the       */
                          /* tolerance (testing)                            */
  int two_sided_cleanup;  /* 1 (default): final two-sided Rayleigh-Ritz     */
                          /* (SVD of U^T A V) of the returned vectors       */
  int print_level;        /* 0 silent; 2 a progress line every 2000 iterations;
                             3.. a trace line per iteration, on stderr       */
  int profile;            /* 1: time the sparse products, the basis         */
                          /* projections and the residual with HIP events  */
                          /* on `stream` and report them in svds_stats (one */
                          /* call in four, to keep the events' cost low)    */
  int autotune;           /* 1 (default): on the first solve of a prepared  */
                          /* matrix, time the SpMM launch shapes (row bins  */
                          /* or one launch with 1..64 lanes per row) for    */
                          /* the block width and keep the fastest; 0: use   */
                          /* the row-length rule of thumb                   */
  int method;             /* SVDS_METHOD_*                                  */
  int stage2_solver;      /* SVDS_STAGE2_JD (default) or SVDS_STAGE2_GDK    */
  int jd_max_inner;       /* JD: QMR steps per correction; 0 -> 20          */
  double jd_inner_tol;    /* JD: stop at this residual reduction; 0 -> 0.1  */
  int relative_tol;       /* 1: converged when ||r|| < tol * sigma (the     */
                          /* stopping rule of the condition estimate,       */
                          /* Section 4.4); needs SVDS_METHOD_NORMAL         */
  double max_seconds;     /* wall-clock budget of the solve (> 0), checked  */
                          /* once per iteration like max_matvecs; 0: none  */
  int pc_block;           /* SVDS_PC_BLOCKJACOBI: columns per block, 1..128;*/
                          /* 0 -> 64                                        */
  int pc_degree;          /* SVDS_PC_LEARNED: polynomial degree d, 1..15;   */
                          /* 0 -> 8                                         */
  const float* pc_model;  /* SVDS_PC_LEARNED: device array of               */
                          /* SVDS_LPC_NPARAMS FP32 parameters               */
  int fused_gram;         /* 1 (default): FP64 stage-1 products with C =    */
                          /* A^T A in one pass over A when the prepared     */
                          /* matrix has a plan for it (see                  */
                          /* svds_matrix_normal) and it moves fewer bytes   */
                          /* than the two products; 0: always A, then A^T   */
} svds_opts;

/* ---- statistics (host struct, filled by svds_solve) ---------------------- */
typedef struct svds_stats {
  int nconv;              /* triplets meeting eq. (res)                     */
  int stage_exit;         /* 1: returned after stage 1 (Algorithm 1)        */
  int stage1_status;      /* 0 converged, 1 attainable floor, 2 budget      */
  int pad_;
  int64_t matvecs[2];     /* columns multiplied by A or A^T per stage       */
  int64_t iters[2];       /* outer iterations per stage                     */
  int64_t restarts[2];    /* restarts per stage                             */
  int64_t resets;         /* restart-error resets (Section 3.2)             */
  int64_t breakdowns;     /* orthogonalisation breakdowns repaired          */
  double seconds[2];      /* wall time per stage                            */
  double setup_seconds;   /* CSR checks, transpose, binning, ||A||          */
  double norm_A_used;     /* ||A|| used by the convergence tests            */
  /* filled when opts.profile = 1 (zero otherwise): */
  int64_t spmm_calls;     /* sparse products timed (one call = all row bins) */
  double spmm_seconds;    /* their summed duration (HIP events)             */
  double spmm_bytes;      /* their algorithmic bytes: nnz*(8+4) + 4*(rows+1)*/
                          /* + 8*b*(rows + cols) per call                   */
  int64_t inner_iters;    /* JD second stage: symmetric-QMR steps (block    */
                          /* steps)                                         */
  /* filled when opts.profile = 1 (zero otherwise): */
  int64_t gram_calls;     /* one-pass A^T A products timed (the partial-sum */
                          /* kernel and the window combine together)        */
  double gram_seconds;    /* their summed duration (HIP events)             */
  double gram_bytes;      /* the method's bytes of those products: A read   */
                          /* once, X read and Z written once:               */
                          /* nnz*(8+4) + 4*(rows+1) + 16*b*cols per call    */
                          /* (the kernel reads a 16-bit window column and   */
                          /* rank per nonzero in place of the 4-byte column */
                          /* index; the plan's column pointers and window   */
                          /* partial sums are not counted)                  */
  /* filled when opts.profile = 1 (zero otherwise), FP64 iterations: */
  int64_t proj_calls;     /* basis projections timed (the first Gram-      */
                          /* Schmidt pass and the new H columns; the kernel */
                          /* without its partial-sum reduction)             */
  double proj_seconds;    /* their summed duration (HIP events)             */
  double proj_bytes;      /* their algorithmic bytes: 8*N*(columns read)    */
  int64_t resid_calls;    /* fused residual kernels timed (without their    */
                          /* partial-sum reduction)                         */
  double resid_seconds;   /* their summed duration (HIP events)             */
  double resid_bytes;     /* their algorithmic bytes: 8*N*(2*g + nc)        */
  double alg_bytes;       /* algorithmic bytes of every call of the         */
                          /* iterations' streaming kernels (sparse          */
                          /* products at the bytes above, projections,      */
                          /* updates, Cholesky QR passes, residuals,        */
                          /* restarts, corrections; a Gram-Schmidt second   */
                          /* pass that the device skips is not counted);    */
                          /* set-up, norm estimate, final Rayleigh-Ritz and */
                          /* clean-up are not counted (always filled)       */
} svds_stats;

/* Fill *opts with the defaults above.  Returns SVDS_OK or SVDS_ERR_ARG. */
int svds_opts_init(svds_opts* opts);

/* Name of a status code (static string). */
const char* svds_error_string(int code);

/* ---- prepared matrix ----------------------------------------------------- */
/* A prepared matrix holds the device-side copies the solver works from: the
 * validated CSR with 32-bit row offsets, the explicit transpose A^T (so that
 * both products of Section 3.3 are atomic-free row-parallel SpMMs), the
 * row-length bins of both, and diag(A^T A) / diag(A A^T).  When the work
 * matrix A_w (A if m >= n, else A^T) qualifies, it also holds the plan of a
 * one-pass product with A_w^T A_w (svds_matrix_normal).  Preparing reads the
 * caller's CSR arrays on `stream`; afterwards they are no longer needed. */
typedef struct svds_matrix svds_matrix;

/* Validate and prepare.  Returns SVDS_ERR_CSR for a malformed matrix. */
int svds_matrix_create(const svds_csr* A, svds_matrix** out, void* stream);
int svds_matrix_destroy(svds_matrix* h);

/* Block sparse product (row-major blocks, b columns, 1 <= b <= 8):
 *   trans = 0: Y (m x b) = A X (n x b);  trans = 1: Y (n x b) = A^T X (m x b).
 * X and Y are contiguous row-major (entry (i, c) at i*b + c).  This is the
 * matrixMatvec callback of Section 3.4 with blockSize = b, run on the device. */
int svds_matrix_spmm(const svds_matrix* h, int trans, int b, const double* X, double* Y,
                     void* stream);

/* Product with the first stage's operator C = A_w^T A_w (Section 3.3; A_w is
 * the work matrix above, p = min(m, n) its column count):
 *   Z (p x b) = C X (p x b), row-major blocks as for svds_matrix_spmm.
 * The prepared matrix has a one-pass plan when, for some R in 16..128, every
 * block of R consecutive rows of A_w holds at most 2048 nonzeros and touches
 * a window of at most 512 columns, the windows' first columns never
 * decrease, and the windows' summed widths stay within 4 p (banded matrices
 * and other locally coupled ones).  With fused != 0, a plan, and fewer
 * algorithmic bytes than two SpMMs for this b, C X is formed in one read of
 * A_w: each workgroup multiplies its row block by X and then by the block's
 * transpose from LDS, and a second kernel adds the windows' partial sums per
 * column in block order.  Otherwise it is A_w^T (A_w X) by two SpMMs.  Both
 * ways are deterministic.  *used (may be NULL) receives 1 for the one-pass
 * product, 0 otherwise.  Workspace (p x b, or the windows' partial sums) is
 * stream-ordered on `stream`. */
int svds_matrix_normal(const svds_matrix* h, int b, const double* X, double* Z, int fused,
                       int* used, void* stream);

/* The product of svds_matrix_normal without any allocation, for callers that
 * cannot allocate device memory (code under stream capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, result and
 * choice between the one-pass product and the two SpMMs, bit for bit; the
 * scratch (the windows' partial sums, wsum x b doubles, or A_w X, rows x b
 * doubles) lives in one static device array of 64 MiB per GPU that the
 * process holds until it ends.  SVDS_ERR_ARG when the scratch would exceed
 * 64 MiB.  Every call on a GPU shares that array: calls that overlap on one
 * GPU (different streams, or host threads without ordering) race. */
int svds_matrix_normal_noalloc(const svds_matrix* h, int b, const double* X, double* Z, int fused,
                               int* used, void* stream);

/* ---- solve ---------------------------------------------------------------- */
/* k triplets of A (1 <= k <= min(m, n)), target SVDS_LARGEST/SVDS_SMALLEST,
 * 0 < tol < 1.  Outputs (device): sigma (k), U (m x k, ld ldu >= m),
 * V (n x k, ld ldv >= n), rnorm (k, eq. (res) residuals), all in target
 * order (descending for largest, ascending for smallest), each pair (u, v)
 * signed so that the largest-magnitude entry of v is positive.
 * opts may be NULL (defaults); stats may be NULL.  Returns SVDS_OK,
 * SVDS_NOT_CONVERGED (partial results as described above) or an error;
 * on error the outputs are unspecified.  Device workspace (the prepared
 * matrix of the call and the solver's arrays) is stream-ordered on `stream`;
 * blocks released at the end of a call are kept by the library (at most
 * 16 GiB per process) and reused by later calls on the same stream that ask
 * for the same sizes.  A caller that supplies the workspace itself prepares
 * the matrix (svds_matrix_create) and calls svds_solve_prepared. */
int svds_solve(const svds_csr* A, int k, int target, double tol, const svds_opts* opts,
               double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
               svds_stats* stats, void* stream);

/* Bytes of device workspace that svds_solve_prepared needs on h for these
 * k, target and options (the workspace that Section 3.3 lets the library
 * allocate or the user supply): the search space V, W = Op V and their
 * restart copies, the refined factor's Q for the smallest values, the
 * locked and stage-1 vectors, the compact blocks, partial sums, the small
 * FP64 state, and what the chosen precision, preconditioner, second stage and
 * one-pass product add.  *bytes: host.  Launches nothing.  SVDS_ERR_ARG for
 * options out of range (as the solve would return). */
int svds_workspace_size(const svds_matrix* h, int k, int target, const svds_opts* opts,
                        size_t* bytes);

/* Same as svds_solve on a prepared matrix (setup excluded from the call).
 * workspace: NULL, or a device array of workspace_bytes >= the value of
 * svds_workspace_size for the same h, k, target and options (any alignment);
 * the solver's arrays are then carved from it and no device memory is
 * allocated for them.  Still allocated by the library: the autotuner's probe
 * blocks on the first solve of a block width (none with opts.autotune = 0),
 * the learned preconditioner's set-up temporaries (SVDS_PC_LEARNED), and
 * three small pinned host records of the control step.  The workspace must
 * not be used by anything else until the stream has passed the call.
 * SVDS_ERR_ARG if it is too small. */
int svds_solve_prepared(const svds_matrix* h, int k, int target, double tol,
                        const svds_opts* opts, double* sigma, double* U, int64_t ldu,
                        double* V, int64_t ldv, double* rnorm, void* workspace,
                        size_t workspace_bytes, svds_stats* stats, void* stream);

/* Free the device blocks the library keeps for reuse on `stream` (released
 * by earlier calls on it).  Call before destroying a stream that ran solves;
 * blocks kept for a destroyed stream would otherwise stay reserved until the
 * 16 GiB cap stops the caching.  Enqueues stream-ordered frees on `stream`. */
int svds_stream_release(void* stream);

/* ---- batched solve --------------------------------------------------------- */
/* nprob independent problems A[i] with the same k, target, tol and options;
 * outputs per problem as for svds_solve (sigma[i], U[i] with ldu[i], V[i] with
 * ldv[i], rnorm[i]; stats may be NULL or an array of nprob).
 * nworkers <= 0: the problems run in step on `stream`, in groups of up to
 * 256: every step of a first-stage iteration (residual, control step,
 * restart, correction, both Gram-Schmidt passes, Cholesky QR, the products
 * with A and A^T, the new columns of H, the Rayleigh-Ritz extraction) is one
 * launch for all problems of the group, each problem computing exactly what
 * its own svds_solve computes (the same bits), and the host reads all control
 * records of a round together.  The set-up before it (checks, transpose,
 * ||A|| estimate, first block) and the second stage and clean-up after it run
 * per problem on -nworkers host threads (0: 16), each with a stream of its
 * own that waits for `stream` first; the call returns after all of it has
 * finished.  This needs FP64, no preconditioner or point Jacobi, and
 * opts.profile = 0; problems whose matrix has a one-pass plan
 * (svds_matrix_normal) run their own first stage.  Otherwise, or with
 * nworkers > 0, the problems are distributed over that many (0 or negative:
 * |nworkers| or 16) host workers, each driving its own HIP stream at default
 * priority, and the caller's stream is made to wait for them.  Returns the
 * worst status over the problems (an error code if any failed, else
 * SVDS_NOT_CONVERGED if any ran out of budget, else SVDS_OK). */
int svds_solve_batched(int nprob, const svds_csr* A, int k, int target, double tol,
                       const svds_opts* opts, double* const* sigma, double* const* U,
                       const int64_t* ldu, double* const* V, const int64_t* ldv,
                       double* const* rnorm, svds_stats* stats, int nworkers, void* stream);

/* ---- condition-number estimate (Section 4.4) ------------------------------- */
/* One largest and one smallest singular value with block size 1 and stage 1
 * on A^T A stopped when the residual is below rtol * sigma (rtol <= 0 or
 * >= 1 -> 0.1, which the paper found to give about 10 % relative error);
 * opts supplies the rest (basis sizes, preconditioner, budget, seed).
 * sigma_max, sigma_min, kappa: host; stats: NULL or an array of 2 (largest,
 * smallest).  Returns the worse of the two solves' status codes. */
int svds_condest(const svds_matrix* A, double rtol, const svds_opts* opts, double* sigma_max,
                 double* sigma_min, double* kappa, svds_stats* stats, void* stream);

/* ---- learned preconditioner ----------------------------------------------- */
/* A preconditioner for the correction equation (the applyPreconditioner hook
 * of Section 3.4) whose per-row coefficients come from a small network over
 * local features of the operator.  For the work matrix A_w (the tall one of A
 * and A^T, N = its column count = min(m, n)) and C = A_w^T A_w:
 *
 *   K(r) = D^-1/2 sum_{l=0..d} c_l (.) T_l(2M - I) D^-1/2 r,
 *   M = D^-1/2 C D^-1/2 / rho,   D = diag(C) (zeros -> 1),
 *   rho = max_i (D^-1/2 |A_w|^T |A_w| D^-1/2 1)_i,
 *
 * T_l the Chebyshev polynomials, c_l (length N) the coefficients, (.) the
 * row-wise product.  Row i's polynomial is sum_m exp(o_{m,i}) times the
 * Jackson-damped Chebyshev series of 1/(x + delta_m), delta_m =
 * 10^(-5 + 5m/7), m = 0..7, hence positive on [0, 1] for any output o.  The
 * network (parameters: W1 16x32, b1 32, W2 64x32, b2 32, W3 32x8, b3 8,
 * row-major [in][out], in this order) reads 8 features per row:
 *   f = [1, log d_i - mean log d, (M 1)_i, (D^-1/2|A_w|^T|A_w|D^-1/2 1)_i/rho,
 *        column count / mean, (M^2 1)_i, 0, 0]
 * and computes x1 = [f, agg f], h1 = gelu(x1 W1 + b1), x2 = [h1, agg h1],
 * h2 = gelu(x2 W2 + b2), o = clip(h2 W3 + b3, -30, 30), with
 * agg(h) = S^-1 |A_w|^T |A_w| h, S = diag(|A_w|^T |A_w| 1) (zeros -> 1),
 * gelu(x) = x Phi(x).  The dense layers use BF16 matrix-core products with
 * FP32 accumulation; the polynomial is applied in FP64.
 * Training pairs come from the solver: residuals r of its stage-1 iterations
 * (svds_collect_residuals); with e = r/|r| the pair is (C e, e) and its loss
 * 1 - (t.e)^2/(|t|^2 |e|^2), t = K(C e).  Arrays of length N, N x 8, N x 16
 * are row-major FP32 unless stated. */
#define SVDS_LPC_NPARAMS 2888
#define SVDS_LPC_MAX_DEGREE 15
#define SVDS_LPC_CACHE_PER_ROW 192  /* floats of forward cache per row      */

/* Deterministic parameters: hidden weights uniform with variance 1/fan_in
 * from the counter generator at `seed`, biases and W3 zero, b3 = out_bias
 * (host, 8 values; NULL -> zeros).  params: device, SVDS_LPC_NPARAMS. */
int svds_lpc_init(float* params, uint64_t seed, const float* out_bias, void* stream);
/* The 8 features of every row (feat: N x 8). */
int svds_lpc_features(const svds_matrix* A, float* feat, void* stream);
/* Forward pass: coef (N x 16; entries beyond `degree` are zero) and, if
 * cache is not NULL, the activations the backward pass needs
 * (SVDS_LPC_CACHE_PER_ROW * N floats). */
int svds_lpc_forward(const svds_matrix* A, const float* params, const float* feat, int degree,
                     float* coef, float* cache, void* stream);
/* Backward pass: grad (SVDS_LPC_NPARAMS, overwritten) = d loss / d params for
 * dcoef = d loss / d coef (N x 16) and the cache of the forward pass. */
int svds_lpc_backward(const svds_matrix* A, const float* params, const float* cache, int degree,
                      const float* dcoef, float* grad, void* stream);
/* Mean pair loss of np pairs built from residuals R (N x np, column-major
 * FP64, ld ldr) for the coefficients coef, and dcoef = d loss / d coef
 * (N x 16).  loss: host. */
int svds_lpc_loss(const svds_matrix* A, int np, const double* R, int64_t ldr, const float* coef,
                  int degree, float* dcoef, double* loss, void* stream);
/* T = K(R) for nb <= 8 columns (N rows, column-major FP64; T may equal R). */
int svds_lpc_apply(const svds_matrix* A, const float* coef, int degree, int nb, const double* R,
                   int64_t ldr, double* T, int64_t ldt, void* stream);
/* One Adam step (Kingma and Ba 2015) on n FP32 parameters; step counts from 1. */
int svds_lpc_adam(int n, float* params, const float* grad, float* m, float* v, int step, float lr,
                  float beta1, float beta2, float eps, void* stream);

typedef struct svds_lpc_set {
  const svds_matrix* A;   /* training operator                              */
  int npairs;             /* residuals captured from its solve              */
  const double* R;        /* N x npairs, column-major FP64                  */
  int64_t ldr;
} svds_lpc_set;
/* Full-batch Adam (beta 0.9/0.999, eps 1e-8, learning rate lr) on the mean
 * over sets of each set's mean pair loss, `steps` steps, updating params in
 * place; loss_history (host, may be NULL) receives the loss of every step. */
int svds_lpc_train(int nsets, const svds_lpc_set* sets, int degree, int steps, float lr,
                   float* params, double* loss_history, void* stream);

/* Solve with A (as svds_solve_prepared, FP64 precision) and keep the stage-1
 * residual of the block's first target at every `every`-th iteration, at most
 * max_pairs of them, in R (N x max_pairs, column-major, ld ldr >= N);
 * *npairs (host) receives the count.  The triplets are not returned. */
int svds_collect_residuals(const svds_matrix* A, int k, int target, double tol,
                           const svds_opts* opts, int every, int max_pairs, double* R,
                           int64_t ldr, int* npairs, svds_stats* stats, void* stream);

/* ---- single steps of the iteration (used by parity tests) ----------------- */
/* T = K R with the block-Jacobi preconditioner of blocks of nb (1..128)
 * columns (SVDS_PC_BLOCKJACOBI), for b <= 8 vectors of length N = min(m, n)
 * (column-major FP64; T may equal R).  Builds the block inverses each call. */
int svds_blockjacobi_apply(const svds_matrix* A, int nb, int b, const double* R, int64_t ldr,
                           double* T, int64_t ldt, void* stream);

/* Symmetric eigenproblem of the g x g projected matrix (Section 3.3: the
 * small replicated problem), 1 <= g <= 64, on the device: H (ld ldh >= g),
 * theta (g) and Y (g x g, ld ldy >= g) in ascending (descending != 0:
 * descending) eigenvalue order.  One workgroup, cyclic Jacobi. */
int svds_small_eig(int g, const double* H, int64_t ldh, int descending, double* theta,
                   double* Y, int64_t ldy, void* stream);

/* Singular values (ascending) and right singular vectors of a g x g matrix
 * R (1 <= g <= 64), one-sided Jacobi; used by the refined projection. */
int svds_small_svd(int g, const double* R, int64_t ldr, double* s, double* Y, int64_t ldy,
                   void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SVDS_H */
