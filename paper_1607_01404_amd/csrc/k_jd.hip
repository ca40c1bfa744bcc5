// Jacobi-Davidson correction for the second stage (the paper's default
// second-stage solver, JDQMR, Section 3.4): for each of the nb block columns,
//   (I - QQ^T)(B - s_j I)(I - QQ^T) t_j = r_j
// solved approximately from t_j = 0 by symmetric QMR (Freund and Nachtigal)
// with the stage-2 preconditioner projected the same way.  The nb columns run
// side by side: the vectors are column-major N x nb blocks, the products with
// B and the preconditioner are the library's block kernels, and the scalar
// recurrences run in a one-wavefront kernel on per-column state in device
// memory, so the inner loop needs no host synchronisation.  A column that has
// met its residual reduction (or broken down) stops updating its solution.
//
// One inner step of column j, from the residual r, direction q, increment d:
//   w = M q,  sigma = q.w,  alpha = rho / sigma,  r -= alpha w,
//   theta' = ||r|| / tau,  c2 = 1 / (1 + theta'^2),  tau = tau theta' sqrt(c2),
//   d = c2 theta^2 d + c2 alpha q,  x += d,  theta = theta',
//   t = P r,  rho' = r.t,  q = t + (rho' / rho) q,  rho = rho'
// (P = I: t = r and rho' = ||r||^2, and the iterates are those of MINRES).
#include "common.h"

namespace svds {

namespace {

constexpr int kJT = 256;

inline int blocks_for(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kJT - 1) / kJT, 2048));
}

inline unsigned elem_blocks(int64_t tot) { return (unsigned)((tot + 255) / 256); }

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
  wave_sums_to<kMaxBlock>(acc, sh[threadIdx.x / kWave]);
  __syncthreads();
  if (threadIdx.x < nb) {
    double v = 0.0;
    for (int ww = 0; ww < kJT / kWave; ++ww) v += sh[ww][threadIdx.x];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// start: tau = tau0 = ||r_0||, rho = r_0 . t_0 (no preconditioner: ||r_0||^2)
__global__ void k_jd_start(int nb, const double* __restrict__ n2, const double* __restrict__ rho0,
                           JdCol* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nb) return;
  JdCol c{};
  c.tau0 = sqrt(fmax(n2[j], 0.0));
  c.tau = c.tau0;
  c.theta = 0.0;
  c.rho = rho0 ? rho0[j] : n2[j];
  c.done = (c.tau0 > 0.0 && c.rho != 0.0) ? 0 : 1;
  c.apply = 0;
  st[j] = c;
}

// q = t_0, d = 0, x = 0
__global__ void k_jd_init_vecs(int64_t N, int nb, int64_t ld, const double* __restrict__ t,
                               double* __restrict__ q, double* __restrict__ d,
                               double* __restrict__ x) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = e0 % N;
  const int j = (int)(e0 / N);
  if (j >= nb) return;
  const int64_t e = i + j * ld;
  q[e] = t[e];
  d[e] = 0.0;
  x[e] = 0.0;
}

// w = (B q)_compact - s_j q   (the product arrives as a row-major N x nb block)
template <typename TW>
__global__ void k_jd_shift(int64_t N, int nb, const TW* __restrict__ Wc,
                           const double* __restrict__ q, int64_t ld,
                           const double* __restrict__ shift, double* __restrict__ w) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int j = (int)(t % nb);
  if (i >= N) return;
  w[i + j * ld] = (double)Wc[t] - shift[j] * q[i + j * ld];
}

// the direction block for the FP32 operator: row-major, rounded to FP32
__global__ void k_jd_pack_f32(const double* __restrict__ q, int64_t ld, int64_t N, int nb,
                              float* __restrict__ c) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int j = (int)(t % nb);
  if (i >= N) return;
  c[t] = (float)q[i + j * ld];
}

__device__ inline double step_alpha(const JdCol& c, double sigma) {
  return (!c.done && sigma != 0.0) ? c.rho / sigma : 0.0;
}

// r -= alpha_j w (alpha_j = rho_j / sigma_j of an active column, else 0) and
// partial sums of ||r_j||^2
__global__ __launch_bounds__(kJT) void k_jd_resid(int64_t N, int nb, int64_t ld,
                                                  double* __restrict__ r,
                                                  const double* __restrict__ w,
                                                  const double* __restrict__ sigma,
                                                  const JdCol* __restrict__ st,
                                                  double* __restrict__ partial) {
  __shared__ double sh[kJT / kWave][kMaxBlock];
  double a[kMaxBlock], acc[kMaxBlock];
#pragma unroll
  for (int j = 0; j < kMaxBlock; ++j) {
    a[j] = j < nb ? step_alpha(st[j], sigma[j]) : 0.0;
    acc[j] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * kJT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kJT) {
#pragma unroll
    for (int j = 0; j < kMaxBlock; ++j) {
      if (j < nb) {
        const int64_t e = i + j * ld;
        const double v = fma(-a[j], w[e], r[e]);
        r[e] = v;
        acc[j] = fma(v, v, acc[j]);
      }
    }
  }
  wave_sums_to<kMaxBlock>(acc, sh[threadIdx.x / kWave]);
  __syncthreads();
  if (threadIdx.x < nb) {
    double v = 0.0;
    for (int ww = 0; ww < kJT / kWave; ++ww) v += sh[ww][threadIdx.x];
    partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = v;
  }
}

// the scalar QMR step of every column: the smoothing parameters, the new
// quasi-residual norm tau, the increment coefficients, the stopping test;
// without a preconditioner also rho' = ||r||^2 and beta
__global__ void k_jd_scalar(int nb, const double* __restrict__ sigma,
                            const double* __restrict__ rn2, double tol, int precond,
                            JdCol* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nb) return;
  JdCol c = st[j];
  c.apply = 0;
  if (!c.done) {
    const double sg = sigma[j];
    if (sg == 0.0) {
      c.done = 1;  // breakdown: keep the current solution
    } else {
      const double alpha = c.rho / sg;
      const double th = sqrt(fmax(rn2[j], 0.0)) / c.tau;
      const double c2 = 1.0 / (1.0 + th * th);
      c.tau = c.tau * th * sqrt(c2);
      c.dcoef = c2 * c.theta * c.theta;
      c.acoef = c2 * alpha;
      c.theta = th;
      c.apply = 1;
      if (c.tau <= tol * c.tau0) c.done = 1;
      if (!precond && !c.done) {
        const double rho_next = rn2[j];
        c.beta = rho_next / c.rho;
        c.rho = rho_next;
        if (rho_next == 0.0) c.done = 1;
      }
    }
  }
  st[j] = c;
}

// d = dcoef d + acoef q;  x += d;  then, without a preconditioner, q = r + beta q,
// with one, t = r (the input of the preconditioner)
__global__ void k_jd_vec(int64_t N, int nb, int64_t ld, double* __restrict__ q,
                         double* __restrict__ d, double* __restrict__ x,
                         const double* __restrict__ r, double* __restrict__ t,
                         const JdCol* __restrict__ st) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = e0 % N;
  const int j = (int)(e0 / N);
  if (j >= nb) return;
  const JdCol& c = st[j];
  if (!c.apply) return;
  const int64_t e = i + j * ld;
  const double qv = q[e];
  const double dn = c.dcoef * d[e] + c.acoef * qv;
  d[e] = dn;
  x[e] += dn;
  if (t) {
    t[e] = r[e];
  } else if (!c.done) {
    q[e] = r[e] + c.beta * qv;
  }
}

// preconditioned: rho' = r . t, beta = rho' / rho, rho = rho'
__global__ void k_jd_beta(int nb, const double* __restrict__ rho_next, JdCol* __restrict__ st) {
  const int j = threadIdx.x;
  if (j >= nb) return;
  JdCol c = st[j];
  if (c.apply && !c.done) {
    c.beta = rho_next[j] / c.rho;
    c.rho = rho_next[j];
    if (c.rho == 0.0) c.done = 1;
  }
  st[j] = c;
}

// q = t + beta q for the columns that go on
__global__ void k_jd_qupd(int64_t N, int nb, int64_t ld, const double* __restrict__ t,
                          double* __restrict__ q, const JdCol* __restrict__ st) {
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = e0 % N;
  const int j = (int)(e0 / N);
  if (j >= nb) return;
  const JdCol& c = st[j];
  if (!c.apply || c.done) return;
  const int64_t e = i + j * ld;
  q[e] = t[e] + c.beta * q[e];
}

}  // namespace

void jd_col_dots(const double* X, const double* Y, int64_t ld, int64_t N, int nb, double* partial,
                 double* out, hipStream_t s) {
  const int nblk = blocks_for(N);
  k_jd_dots<<<nblk, kJT, 0, s>>>(X, Y, ld, N, nb, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nblk, nb, out, s);
}

void jd_start(int64_t N, int nb, int64_t ld, const double* t, const double* n2,
              const double* rho0, JdCol* st, double* q, double* d, double* x, hipStream_t s) {
  k_jd_start<<<1, 64, 0, s>>>(nb, n2, rho0, st);
  k_jd_init_vecs<<<elem_blocks(N * nb), 256, 0, s>>>(N, nb, ld, t, q, d, x);
  SVDS_LAUNCH_CHECK();
}

void jd_shift(int64_t N, int nb, const double* Wc, const double* q, int64_t ld,
              const double* shift, double* w, hipStream_t s) {
  k_jd_shift<double><<<elem_blocks(N * nb), 256, 0, s>>>(N, nb, Wc, q, ld, shift, w);
  SVDS_LAUNCH_CHECK();
}

void jd_shift(int64_t N, int nb, const float* Wc, const double* q, int64_t ld,
              const double* shift, double* w, hipStream_t s) {
  k_jd_shift<float><<<elem_blocks(N * nb), 256, 0, s>>>(N, nb, Wc, q, ld, shift, w);
  SVDS_LAUNCH_CHECK();
}

void jd_pack_f32(const double* q, int64_t ld, int64_t N, int nb, float* c, hipStream_t s) {
  if (N <= 0 || nb <= 0) return;
  k_jd_pack_f32<<<elem_blocks(N * nb), 256, 0, s>>>(q, ld, N, nb, c);
  SVDS_LAUNCH_CHECK();
}

void jd_step(int64_t N, int nb, int64_t ld, double* r, const double* w, double* q, double* d,
             double* x, double* t, const double* sigma, double* rn2, double tol, JdCol* st,
             double* partial, hipStream_t s) {
  const int nblk = blocks_for(N);
  k_jd_resid<<<nblk, kJT, 0, s>>>(N, nb, ld, r, w, sigma, st, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nblk, nb, rn2, s);
  k_jd_scalar<<<1, 64, 0, s>>>(nb, sigma, rn2, tol, t != nullptr, st);
  k_jd_vec<<<elem_blocks(N * nb), 256, 0, s>>>(N, nb, ld, q, d, x, r, t, st);
  SVDS_LAUNCH_CHECK();
}

void jd_precond_step(int64_t N, int nb, int64_t ld, const double* rho_next, const double* t,
                     double* q, JdCol* st, hipStream_t s) {
  k_jd_beta<<<1, 64, 0, s>>>(nb, rho_next, st);
  k_jd_qupd<<<elem_blocks(N * nb), 256, 0, s>>>(N, nb, ld, t, q, st);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
