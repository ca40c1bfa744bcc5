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
 *  - The library keeps no global state between calls; distinct streams may
 *    run distinct solves concurrently.
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
                                /* reorthogonalisation and stage 2 are FP64 */

#define SVDS_PC_NONE 0          /* K = I                                     */
#define SVDS_PC_JACOBI 1        /* K = diag(A^T A)^-1 on C (diag(A A^T) when */
                                /* m < n); on B the composition              */
                                /* [K A^T y_u; A K y_v] (applyPreconditioner */
                                /* modes AtA / augmented, Section 3.4)       */

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
  int precond;            /* SVDS_PC_NONE or SVDS_PC_JACOBI                 */
  int force_stage2;       /* 1: run stage 2 even when stage 1 met the       */
                          /* tolerance (testing)                            */
  int two_sided_cleanup;  /* 1 (default): final two-sided Rayleigh-Ritz     */
                          /* (SVD of U^T A V) of the returned vectors       */
  int print_level;        /* 0 silent .. 5 per-iteration trace on stderr    */
  int profile;            /* 1: time the sparse products with HIP events on */
                          /* `stream` and report them in svds_stats         */
  int autotune;           /* 1 (default): on the first solve of a prepared  */
                          /* matrix, time the SpMM launch shapes (row bins  */
                          /* or one launch with 1..64 lanes per row) for    */
                          /* the block width and keep the fastest; 0: use   */
                          /* the row-length rule of thumb                   */
} svds_opts;

/* ---- statistics (host struct, filled by svds_solve) ---------------------- */
typedef struct svds_stats {
  int nconv;              /* triplets meeting eq. (res)                     */
  int stage_exit;         /* 1: returned after stage 1 (Algorithm 1 step 7) */
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
} svds_stats;

/* Fill *opts with the defaults above.  Returns SVDS_OK or SVDS_ERR_ARG. */
int svds_opts_init(svds_opts* opts);

/* Name of a status code (static string). */
const char* svds_error_string(int code);

/* ---- prepared matrix ----------------------------------------------------- */
/* A prepared matrix holds the device-side copies the solver works from: the
 * validated CSR with 32-bit row offsets, the explicit transpose A^T (so that
 * both products of Section 3.3 are atomic-free row-parallel SpMMs), the
 * row-length bins of both, and diag(A^T A) / diag(A A^T).  Preparing reads the
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

/* ---- solve ---------------------------------------------------------------- */
/* k triplets of A (1 <= k <= min(m, n)), target SVDS_LARGEST/SVDS_SMALLEST,
 * 0 < tol < 1.  Outputs (device): sigma (k), U (m x k, ld ldu >= m),
 * V (n x k, ld ldv >= n), rnorm (k, eq. (res) residuals), all in target
 * order (descending for largest, ascending for smallest), each pair (u, v)
 * signed so that the largest-magnitude entry of v is positive.
 * opts may be NULL (defaults); stats may be NULL.  Returns SVDS_OK,
 * SVDS_NOT_CONVERGED (partial results as described above) or an error;
 * on error the outputs are unspecified.  Device workspace is allocated and
 * freed inside the call. */
int svds_solve(const svds_csr* A, int k, int target, double tol, const svds_opts* opts,
               double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
               svds_stats* stats, void* stream);

/* Same on a prepared matrix (setup excluded from the call). */
int svds_solve_prepared(const svds_matrix* h, int k, int target, double tol,
                        const svds_opts* opts, double* sigma, double* U, int64_t ldu,
                        double* V, int64_t ldv, double* rnorm, svds_stats* stats, void* stream);

/* ---- batched solve --------------------------------------------------------- */
/* nprob independent problems A[i] with the same k, target, tol and options;
 * outputs per problem as for svds_solve (sigma[i], U[i] with ldu[i], V[i] with
 * ldv[i], rnorm[i]; stats may be NULL or an array of nprob).  The problems are
 * distributed over `nworkers` (0 -> min(nprob, 16)) host workers, each driving
 * its own HIP stream at default priority, so that the small per-problem
 * kernels of different problems overlap on the GPU; the caller's stream is
 * made to wait for all of them before the call returns.  Returns the worst
 * status over the problems (an error code if any failed, else
 * SVDS_NOT_CONVERGED if any ran out of budget, else SVDS_OK). */
int svds_solve_batched(int nprob, const svds_csr* A, int k, int target, double tol,
                       const svds_opts* opts, double* const* sigma, double* const* U,
                       const int64_t* ldu, double* const* V, const int64_t* ldv,
                       double* const* rnorm, svds_stats* stats, int nworkers, void* stream);

/* ---- single steps of the iteration (used by parity tests) ----------------- */
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
