// Small kernels of the stage-1 finalisation and the stage-2 hand-over
// (Algorithm 1) and of the final two-sided clean-up.
#include "small.h"

namespace svds {

// sigma = |lambda|^(1/2), inv = 1/sigma (0 when sigma = 0)
__global__ void k_sigma(int k, const double* lam, double* sig, double* inv) {
  const int i = threadIdx.x;
  if (i >= k) return;
  const double s = sqrt(fabs(lam[i]));
  sig[i] = s;
  inv[i] = s > 0.0 ? 1.0 / s : 0.0;
}

void sigma_from_lambda(int k, const double* lam, double* sig, double* inv, hipStream_t s) {
  k_sigma<<<1, 64, 0, s>>>(k, lam, sig, inv);
  SVDS_LAUNCH_CHECK();
}

// eq. (res) from the two squared halves; all-below-tolerance flag; stage-2
// shifts max(sigma - sqrt(2)||r||, ||A|| eps) (||r^C|| = sigma ||r||)
__global__ void k_stage1_check(int k, const double* rl2, const double* rr2, const double* sig,
                               double normA, double tol, int rel, double* rn, double* taus,
                               int* ok) {
  if (threadIdx.x != 0) return;
  int good = 1;
  for (int i = 0; i < k; ++i) {
    double r = sqrt(fmax(rl2[i], 0.0) + fmax(rr2[i], 0.0));
    if (!(sig[i] > 0.0)) r = INFINITY;
    rn[i] = r;
    good = good && (r < (rel ? sig[i] : normA) * tol);
    const double rr = isfinite(r) ? r : sig[i];
    taus[i] = fmax(sig[i] - 1.4142135623730951 * rr, normA * kEps);
  }
  *ok = good;
}

void stage1_check(int k, const double* rl2, const double* rr2, const double* sig, double normA,
                  double tol, int rel, double* rn, double* taus, int* ok, hipStream_t s) {
  k_stage1_check<<<1, 64, 0, s>>>(k, rl2, rr2, sig, normA, tol, rel, rn, taus, ok);
  SVDS_LAUNCH_CHECK();
}

// rn = sqrt(a + b) elementwise
__global__ void k_sqrt_sum(int k, const double* a, const double* b, double* out) {
  const int i = threadIdx.x;
  if (i < k) out[i] = sqrt(fmax(a[i], 0.0) + fmax(b[i], 0.0));
}

void sqrt_sum(int k, const double* a, const double* b, double* out, hipStream_t s) {
  k_sqrt_sum<<<1, 64, 0, s>>>(k, a, b, out);
  SVDS_LAUNCH_CHECK();
}

// f = 1/sqrt(x) (0 when x = 0)
__global__ void k_rsqrt(int k, const double* x, double* f) {
  const int i = threadIdx.x;
  if (i < k) f[i] = x[i] > 0.0 ? 1.0 / sqrt(x[i]) : 0.0;
}

void inv_sqrt(int k, const double* x, double* f, hipStream_t s) {
  k_rsqrt<<<1, 64, 0, s>>>(k, x, f);
  SVDS_LAUNCH_CHECK();
}

// sigma_j = |locked value j|
__global__ void k_abs(int k, const double* x, double* y) {
  const int i = threadIdx.x;
  if (i < k) y[i] = fabs(x[i]);
}

void abs_vec(int k, const double* x, double* y, hipStream_t s) {
  k_abs<<<1, 64, 0, s>>>(k, x, y);
  SVDS_LAUNCH_CHECK();
}

// clean-up: from s (ascending), right vectors Yq and H2 Yq = P diag(s), build
// P and Q in target order and sigma
__global__ void k_cleanup_finish(int k, const double* s, const double* Yq, int ldy,
                                 const double* AVq, int ldav, int descending, double* sig,
                                 double* P, double* Q, int ldk) {
  for (int a = threadIdx.x; a < k * k; a += blockDim.x) {
    const int i = a % k, j = a / k;
    const int src = descending ? (k - 1 - j) : j;
    const double sj = s[src];
    Q[j * ldk + i] = Yq[src * ldy + i];
    P[j * ldk + i] = sj > 0.0 ? AVq[src * ldav + i] / sj : (i == j ? 1.0 : 0.0);
    if (i == 0) sig[j] = sj;
  }
}

void cleanup_finish(int k, const double* s, const double* Yq, int ldy, const double* AVq,
                    int ldav, int descending, double* sig, double* P, double* Q, int ldk,
                    hipStream_t st) {
  k_cleanup_finish<<<1, 256, 0, st>>>(k, s, Yq, ldy, AVq, ldav, descending, sig, P, Q, ldk);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
