// Jacobi-Davidson correction for the second stage (the paper's default
// second-stage solver, Section 3.4): for each of the nb block columns,
//   (I - QQ^T)(B - s_j I)(I - QQ^T) t_j = r_j
// solved approximately by MINRES (Paige and Saunders) from t_j = 0.  The nb
// columns run side by side: the Lanczos vectors are column-major N x nb
// blocks, the products with B are the library's block SpMMs, and the scalar
// recurrences (Givens rotations of the tridiagonal projection) run in a
// one-wavefront kernel on per-column state in device memory, so the inner
// loop needs no host synchronisation.  A column that has met its residual
// reduction (or lost its Lanczos vector) stops updating its solution.
#include "common.h"

namespace svds {

namespace {

constexpr int kJT = 256;

inline int blocks_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kJT - 1) / kJT, 2048));
}

// per-block partial sums of x_j . y_j (y null: x_j . x_j), partial[j * nblk + block]
__global__ __launch_bounds__(kJT) void k_jd_dots(const double* __restrict__ X,
                                                 const double* __restrict__ Yv, int64_t ld,
                                                 int64_t N, int nb, double* __restrict__ partial) {
  __shared__ double sh[kJT / kWave][kMaxBlock];
  double acc[kMaxBlock];
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) acc[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kJT) {
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) {
      if (j < nb) {
        const double x = X[i + j * ld];
        acc[j] = fma(x, Yv ? Yv[i + j * ld] : x, acc[j]);
      }
    }
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) sh[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < nb) {
    double v = 0.0;
    for (int ww = 0; ww < kJT / kWave; ++ww) v += sh[ww][threadIdx.x];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// start: beta1 = ||b_j||, q = b / beta1, the other vectors zero
__global__ void k_jd_start(int nb, const double* __restrict__ n2, JdCol* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nb) return;
  JdCol c{};
  c.beta1 = sqrt(fmax(n2[j], 0.0));
  c.phi = c.beta1;
  c.c1 = c.c2 = 1.0;
  c.s1 = c.s2 = 0.0;
  c.beta = 0.0;
  c.done = c.beta1 > 0.0 ? 0 : 1;
  st[j] = c;
}

__global__ void k_jd_init_vecs(int64_t N, int nb, int64_t ld, const double* __restrict__ b,
                               const JdCol* __restrict__ st, double* __restrict__ q,
                               double* __restrict__ qp, double* __restrict__ d1,
                               double* __restrict__ d2, double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t % N;
  const int j = (int)(t / N);
  if (j >= nb) return;
  const int64_t e = i + j * ld;
  const double b1 = st[j].beta1;
  q[e] = b1 > 0.0 ? b[e] / b1 : 0.0;
  qp[e] = 0.0;
  d1[e] = 0.0;
  d2[e] = 0.0;
  x[e] = 0.0;
}

// z = (B q)_compact - s_j q   (the product arrives as a row-major N x nb block)
__global__ void k_jd_shift(int64_t N, int nb, const double* __restrict__ Wc,
                           const double* __restrict__ q, int64_t ld,
                           const double* __restrict__ shift, double* __restrict__ z) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int j = (int)(t % nb);
  if (i >= N) return;
  z[i + j * ld] = Wc[t] - shift[j] * q[i + j * ld];
}

// z -= alpha_j q + beta_j q_prev, and partial sums of ||z_j||^2
__global__ __launch_bounds__(kJT) void k_jd_lanczos(int64_t N, int nb, int64_t ld,
                                                    double* __restrict__ z,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ qp,
                                                    const double* __restrict__ alpha,
                                                    const JdCol* __restrict__ st,
                                                    double* __restrict__ partial) {
  __shared__ double sh[kJT / kWave][kMaxBlock];
  double a[kMaxBlock], bt[kMaxBlock], acc[kMaxBlock];
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) {
    a[j] = j < nb ? alpha[j] : 0.0;
    bt[j] = j < nb ? st[j].beta : 0.0;
    acc[j] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kJT) {
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) {
      if (j < nb) {
        const int64_t e = i + j * ld;
        const double v = z[e] - a[j] * q[e] - bt[j] * qp[e];
        z[e] = v;
        acc[j] = fma(v, v, acc[j]);
      }
    }
  }
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) {
    const double v = wave_sum(acc[j]);
    if (lane == 0) sh[w][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < nb) {
    double v = 0.0;
    for (int ww = 0; ww < kJT / kWave; ++ww) v += sh[ww][threadIdx.x];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// the scalar step of MINRES for every column: the new column
// [beta_k, alpha_k, beta_{k+1}] of the tridiagonal matrix through the two
// previous rotations, the new rotation, the solution coefficient tau_k and
// the residual norm |phi|
__global__ void k_jd_scalar(int nb, const double* __restrict__ alpha,
                            const double* __restrict__ bnext2, double tol,
                            JdCol* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nb) return;
  JdCol c = st[j];
  c.apply = 0;
  if (!c.done) {
    const double al = alpha[j];
    const double bn = sqrt(fmax(bnext2[j], 0.0));
    const double eps = c.s2 * c.beta;
    const double dlt = c.c2 * c.beta;
    const double delta = c.c1 * dlt + c.s1 * al;
    const double gbar = -c.s1 * dlt + c.c1 * al;
    const double gamma = hypot(gbar, bn);
    if (gamma > 0.0) {
      const double cn = gbar / gamma, sn = bn / gamma;
      c.tk = cn * c.phi;
      c.phi = -sn * c.phi;
      c.delta = delta;
      c.eps = eps;
      c.invg = 1.0 / gamma;
      c.c2 = c.c1;
      c.s2 = c.s1;
      c.c1 = cn;
      c.s1 = sn;
      c.beta = bn;
      c.apply = 1;
      if (fabs(c.phi) <= tol * c.beta1 || bn == 0.0) c.done = 1;
    } else {
      c.done = 1;
    }
  }
  st[j] = c;
}

// d_new = (q - delta d1 - eps d2) / gamma;  x += tau d_new;  d2 <- d1, d1 <- d_new;
// q_prev <- q;  q <- z / beta_{k+1}
__global__ void k_jd_vec(int64_t N, int nb, int64_t ld, double* __restrict__ q,
                         double* __restrict__ qp, const double* __restrict__ z,
                         double* __restrict__ d1, double* __restrict__ d2,
                         double* __restrict__ x, const JdCol* __restrict__ st) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t % N;
  const int j = (int)(t / N);
  if (j >= nb) return;
  const JdCol& c = st[j];
  if (!c.apply) return;
  const int64_t e = i + j * ld;
  const double qv = q[e];
  const double d1v = d1[e];
  const double dn = (qv - c.delta * d1v - c.eps * d2[e]) * c.invg;
  x[e] += c.tk * dn;
  d2[e] = d1v;
  d1[e] = dn;
  qp[e] = qv;
  q[e] = c.beta > 0.0 ? z[e] / c.beta : 0.0;
}

}  // namespace

void jd_col_dots(const double* X, const double* Y, int64_t ld, int64_t N, int nb, double* partial,
                 double* out, hipStream_t s) {
  const int nblk = blocks_for(N);
  k_jd_dots<<<nblk, kJT, 0, s>>>(X, Y, ld, N, nb, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nblk, nb, out, s);
}

void jd_start(int64_t N, int nb, int64_t ld, const double* b, const double* n2, JdCol* st,
              double* q, double* qp, double* d1, double* d2, double* x, hipStream_t s) {
  k_jd_start<<<1, 64, 0, s>>>(nb, n2, st);
  const int64_t tot = N * nb;
  k_jd_init_vecs<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(N, nb, ld, b, st, q, qp, d1, d2, x);
  SVDS_LAUNCH_CHECK();
}

void jd_shift(int64_t N, int nb, const double* Wc, const double* q, int64_t ld,
              const double* shift, double* z, hipStream_t s) {
  const int64_t tot = N * nb;
  k_jd_shift<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(N, nb, Wc, q, ld, shift, z);
  SVDS_LAUNCH_CHECK();
}

void jd_step(int64_t N, int nb, int64_t ld, double* z, double* q, double* qp, double* d1,
             double* d2, double* x, const double* alpha, double* bnext2, double tol, JdCol* st,
             double* partial, hipStream_t s) {
  const int nblk = blocks_for(N);
  k_jd_lanczos<<<nblk, kJT, 0, s>>>(N, nb, ld, z, q, qp, alpha, st, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nblk, nb, bnext2, s);
  k_jd_scalar<<<1, 64, 0, s>>>(nb, alpha, bnext2, tol, st);
  const int64_t tot = N * nb;
  k_jd_vec<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(N, nb, ld, q, qp, z, d1, d2, x, st);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
