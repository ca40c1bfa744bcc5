// Learned preconditioner for the correction step: internal declarations.
//
// The preconditioner plugs into the user-preconditioner hook of the solver
// (Section 3.4 of the paper, applyPreconditioner for A^T A, A A^T or the
// augmented matrix).  For the work matrix A (rows >= cols = N) and
// C = A^T A it is
//
//   K(r) = D^-1/2 sum_{l=0..d} c_l (.) T_l(2M - I) D^-1/2 r,
//   M = D^-1/2 C D^-1/2 / rho,  D = diag(C) (zeros -> 1),
//   rho = max_i (D^-1/2 |A|^T |A| D^-1/2 1)_i  (Gershgorin: spec(M) in [0, 1]),
//
// with T_l the Chebyshev polynomials and c_l (N-vectors, (.) row-wise
// product) the per-row coefficients.  Each row's polynomial is a positive
// mixture c_{l,i} = sum_m exp(o_{m,i}) Psi[l][m] of Jackson-damped Chebyshev
// series of 1/(x + delta_m), delta_m = 10^(-5 + 5m/7), so it is positive on
// [0, 1] whatever the mixture weights; the 8 log-weights o come from a small
// network over local features of the operator:
//
//   f (8)            features of each row (lpc_features)
//   x1 = [f, agg f]            z1 = x1 W1 + b1 (32)  h1 = gelu(z1)
//   x2 = [h1, agg h1]          z2 = x2 W2 + b2 (32)  h2 = gelu(z2)
//   o  = clip(h2 W3 + b3, -30, 30) (8)
//   agg(h) = S^-1 |A|^T |A| h,  S = diag(|A|^T |A| 1) (zeros -> 1)
//
// The dense layers run on the matrix cores (BF16 operands, FP32
// accumulation); aggregation and GELU in FP32; the polynomial applied inside
// the solver in FP64 with the library's sparse products.
#pragma once

#include "common.h"

namespace svds {

constexpr int kLpcNF = 8;           // features per row
constexpr int kLpcHid = 32;         // hidden width
constexpr int kLpcOut = 8;          // mixture log-weights per row
constexpr int kLpcCoef = 16;        // stored coefficients per row (degree <= 15)
constexpr int kLpcMaxDegree = 15;
constexpr int kLpcDefaultDegree = 8;
constexpr float kLpcClip = 30.0f;

// flat FP32 parameters, weights row-major [in][out]
constexpr int kW1 = 0;
constexpr int kB1 = kW1 + 2 * kLpcNF * kLpcHid;
constexpr int kW2 = kB1 + kLpcHid;
constexpr int kB2 = kW2 + 2 * kLpcHid * kLpcHid;
constexpr int kW3 = kB2 + kLpcHid;
constexpr int kB3 = kW3 + kLpcHid * kLpcOut;
constexpr int kLpcNParams = kB3 + kLpcOut;  // 2888

// forward cache: row-major arrays of N rows, offsets in units of N floats
constexpr int kCx1 = 0;                          // [f, agg f]      16
constexpr int kCz1 = kCx1 + 2 * kLpcNF;          // z1              32
constexpr int kCx2 = kCz1 + kLpcHid;             // [h1, agg h1]    64
constexpr int kCz2 = kCx2 + 2 * kLpcHid;         // z2              32
constexpr int kCh2 = kCz2 + kLpcHid;             // h2              32
constexpr int kCo = kCh2 + kLpcHid;              // o (unclipped)   8
constexpr int kCw = kCo + kLpcOut;               // exp(clip(o))    8
constexpr int kLpcCacheRow = kCw + kLpcOut;      // 192 floats per row

// Psi[l][m] = g_l a_l(delta_m): Jackson factor times Chebyshev coefficient
// of 1/(x + delta_m); rows l > degree are zero
struct LpcPsi {
  float v[kLpcCoef * kLpcOut];
};
LpcPsi lpc_psi(int degree);

// per-matrix quantities
struct LpcOp {
  const Csr32* A = nullptr;   // work matrix, rows >= cols
  const Csr32* At = nullptr;  // its transpose
  const double* diag = nullptr;  // diag(C) (device, length N)
  int64_t N = 0, mw = 0;
  double* dh = nullptr;       // D^-1/2
  float* sinv = nullptr;      // S^-1
  double rho = 1.0;
};
void lpc_prepare(const svds_matrix* M, LpcOp& op, DeviceBuffers& buf, hipStream_t s);
// the same in two parts: the operator's arrays (no launch), then their values
void lpc_alloc(const svds_matrix* M, LpcOp& op, DeviceBuffers& buf);
void lpc_compute(LpcOp& op, hipStream_t s);
// features (N x 8, row-major)
void lpc_features(const LpcOp& op, float* feat, hipStream_t s);
// coefficients (N x 16, row-major) and the cache of the backward pass
// (kLpcCacheRow * N floats); gbuf: mw x 32 floats of scratch
void lpc_forward(const LpcOp& op, const float* params, const float* feat, int degree, float* coef,
                 float* cache, float* gbuf, hipStream_t s);
// gradient of the loss with respect to the parameters given dloss/dcoef;
// accumulate: grad += instead of grad =.  work: N x 104 floats, gbuf: mw x 32,
// part: lpc_partial_floats(N) floats
void lpc_backward(const LpcOp& op, const float* params, const float* cache, int degree,
                  const float* dcoef, float* grad, bool accumulate, float* work, float* gbuf,
                  float* part, hipStream_t s);
int64_t lpc_partial_floats(int64_t N);

// Chebyshev sequence of the Jacobi-scaled operator on a row-major block
// X (N x nb): z_0 = D^-1/2 X, z_1 = (2M - I) z_0, z_{l+1} = 2(2M - I) z_l - z_{l-1}.
// With coef: acc = sum_l coef_l (.) z_l and Out = D^-1/2 acc (column-major,
// ld ldo).  With Z: z_l stored as FP32 at Z + (l * ldl) + j * N (column j of
// the block at Z's column col0 + j, layout [l][pair][row]).
struct LpcScratch {
  double *z[3] = {nullptr, nullptr, nullptr};
  double *w = nullptr, *y = nullptr, *q = nullptr, *acc = nullptr;
  int nbmax = 0;
};
void lpc_scratch(const LpcOp& op, int nbmax, LpcScratch& sc, DeviceBuffers& buf);
void lpc_cheb(const LpcOp& op, int nb, const double* X, int degree, const float* coef,
              double* Out, int64_t ldo, float* Z, int64_t ldl, int64_t col0, LpcScratch& sc,
              hipStream_t s);
// T = K(R) for nb columns (column-major; T may alias R)
void lpc_apply(const LpcOp& op, const float* coef, int degree, int nb, const double* R,
               int64_t ldr, double* T, int64_t ldt, LpcScratch& sc, hipStream_t s);


// ---- training -------------------------------------------------------------
// pairs from captured residuals R (N x np, column-major): E = R / |R| per
// column, Q = C E (both N x np, ld ldp, FP64)
void lpc_make_pairs(const LpcOp& op, int np, const double* R, int64_t ldr, double* Q, double* E,
                    int64_t ldp, hipStream_t s);

// one training matrix: operator data, features, the Chebyshev basis of its
// pairs' inputs (FP32, [l][pair][row]), labels and the work arrays of a step
struct LpcSet {
  DeviceBuffers buf;
  LpcOp op;
  int npairs = 0;
  float *feat = nullptr, *coef = nullptr, *dcoef = nullptr, *cache = nullptr, *work = nullptr;
  float *gbuf = nullptr, *part = nullptr, *Z = nullptr, *E = nullptr, *T = nullptr;
  int64_t ldl = 0;
  int nbx = 1;
  double *lpart = nullptr, *ab = nullptr;
  LpcSet(const svds_matrix* M, int np, const double* R, int64_t ldr, int degree, hipStream_t s);
};
// loss of the set's pairs for its current coef; loss_out[0] += weight * mean
// loss; st.dcoef = weight * dloss/dcoef
void lpc_loss(LpcSet& st, int degree, double weight, double* loss_out, hipStream_t s);
void lpc_adam(int n, float* p, const float* g, float* m, float* v, int step, float lr, float b1,
              float b2, float eps, hipStream_t s);
void lpc_fill(float* x, int64_t n, float v, hipStream_t s);
// full-batch Adam over all sets (the mean over sets of each set's mean pair
// loss); loss_hist_host[step] (host, may be null)
void lpc_train(std::vector<LpcSet*>& sets, int degree, int steps, float lr, float* params,
               double* loss_hist_host, hipStream_t s);

}  // namespace svds
