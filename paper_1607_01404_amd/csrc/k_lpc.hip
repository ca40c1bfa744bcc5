// Learned preconditioner: kernels and their launchers (definitions in lpc.h).
#include <cmath>

#include "lpc.h"

namespace svds {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;

inline int blocks_for(int64_t n, int per = kT) {
  return (int)std::max<int64_t>(1, (n + per - 1) / per);
}

__device__ __forceinline__ float gelu(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// operator quantities and features (one thread per row; done once per matrix)
// ---------------------------------------------------------------------------
// y[row] = sum_k |a_k| x[col_k]   (x null: all ones)
__global__ void k_abs_spmv(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                           const double* __restrict__ val, int64_t rows,
                           const double* __restrict__ x, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double acc = 0.0;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) acc += fabs(val[k]) * (x ? x[ci[k]] : 1.0);
  y[r] = acc;
}

__global__ void k_dh(const double* __restrict__ diag, int64_t N, double* __restrict__ dh) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double d = diag[i];
  dh[i] = 1.0 / sqrt(d > 0.0 ? d : 1.0);
}

__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b, int64_t N,
                      double* __restrict__ c) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) c[i] = a[i] * b[i];
}

__global__ void k_sinv(const double* __restrict__ S, int64_t N, float* __restrict__ sinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) sinv[i] = (float)(1.0 / (S[i] > 0.0 ? S[i] : 1.0));
}

// per-block partials of (sum log d, sum column count, max dh*v)
__global__ void k_feat_stats(const double* __restrict__ diag, const int32_t* __restrict__ rpt,
                             const double* __restrict__ dh, const double* __restrict__ v,
                             int64_t N, double* __restrict__ part) {
  __shared__ double s0[kT], s1[kT], s2[kT];
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
    const double d = diag[i];
    a += log(d > 0.0 ? d : 1.0);
    b += (double)(rpt[i + 1] - rpt[i]);
    c = fmax(c, dh[i] * v[i]);
  }
  s0[threadIdx.x] = a;
  s1[threadIdx.x] = b;
  s2[threadIdx.x] = c;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + off]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x * 3 + 0] = s0[0];
    part[blockIdx.x * 3 + 1] = s1[0];
    part[blockIdx.x * 3 + 2] = s2[0];
  }
}

__global__ void k_feat_stats_final(const double* __restrict__ part, int nblk, int64_t N,
                                   double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int k = 0; k < nblk; ++k) {
    a += part[k * 3 + 0];
    b += part[k * 3 + 1];
    c = fmax(c, part[k * 3 + 2]);
  }
  out[0] = a / (double)N;  // mean log d
  out[1] = b / (double)N;  // mean column count
  out[2] = c > 0.0 ? c : 1.0;
}

// f0..f4 and f6, f7; f2 = dh*q/rho with q = C dh; f3 = dh*v/rho
__global__ void k_feat_assemble(const double* __restrict__ diag, const int32_t* __restrict__ rpt,
                                const double* __restrict__ dh, const double* __restrict__ q,
                                const double* __restrict__ v, const double* __restrict__ stats,
                                int64_t N, float* __restrict__ f, double* __restrict__ x2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const double rho = stats[2];
  const double d = diag[i];
  const double f2 = dh[i] * q[i] / rho;
  float* fi = f + i * kLpcNF;
  fi[0] = 1.0f;
  fi[1] = (float)(log(d > 0.0 ? d : 1.0) - stats[0]);
  fi[2] = (float)f2;
  fi[3] = (float)(dh[i] * v[i] / rho);
  fi[4] = (float)((double)(rpt[i + 1] - rpt[i]) / fmax(stats[1], 1e-300));
  fi[6] = 0.0f;
  fi[7] = 0.0f;
  x2[i] = dh[i] * f2;  // input of the product for f5 = M f2
}

__global__ void k_feat_f5(const double* __restrict__ dh, const double* __restrict__ q,
                          const double* __restrict__ stats, int64_t N, float* __restrict__ f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) f[i * kLpcNF + 5] = (float)(dh[i] * q[i] / stats[2]);
}

// ---------------------------------------------------------------------------
// aggregation: out[r, :] (+)= oscale[r] * sum_k |a_k| iscale[c_k] in[c_k, :]
// F lanes per row (one per feature), 64/F rows per wavefront
// ---------------------------------------------------------------------------
template <int F, bool ACCUM>
__global__ __launch_bounds__(kT) void k_agg(const int32_t* __restrict__ rp,
                                            const int32_t* __restrict__ ci,
                                            const float* __restrict__ val, int64_t rows,
                                            const float* __restrict__ in, int64_t ldi,
                                            const float* __restrict__ iscale,
                                            float* __restrict__ out, int64_t ldo,
                                            const float* __restrict__ oscale) {
  const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
  const int64_t r = t / F;
  const int f = (int)(t % F);
  if (r >= rows) return;
  float acc = 0.0f;
  for (int32_t k = rp[r]; k < rp[r + 1]; ++k) {
    const int32_t c = ci[k];
    float x = in[(int64_t)c * ldi + f];
    if (iscale) x *= iscale[c];
    acc += fabsf(val[k]) * x;
  }
  if (oscale) acc *= oscale[r];
  float* o = out + r * ldo + f;
  *o = ACCUM ? *o + acc : acc;
}

// ---------------------------------------------------------------------------
// dense layers on the matrix cores (v_mfma_f32_16x16x32_bf16)
// Operand layout: lane l supplies A[m = l%16][k = 8(l/16)+i] and
// B[k = 8(l/16)+i][n = l%16], i = 0..7, and receives D[m = 4(l/16)+i][n = l%16].
// ---------------------------------------------------------------------------
// Z = X W + b (N x FOUT); X row-major (ld ldx), W row-major [KIN][FOUT].
// ACT: also H = gelu(Z) at H (ld ldh).  Each wavefront takes 16 rows.
template <int KIN, int FOUT, bool ACT>
__global__ __launch_bounds__(kT) void k_layer_fwd(const float* __restrict__ X, int64_t ldx,
                                                  int64_t N, const float* __restrict__ W,
                                                  const float* __restrict__ bias,
                                                  float* __restrict__ Z, int64_t ldz,
                                                  float* __restrict__ H, int64_t ldh) {
  constexpr int KS = (KIN + 31) / 32;  // MFMA steps along K
  constexpr int KP = KS * 32;
  constexpr int NT = (FOUT + 15) / 16;  // output tiles
  __shared__ __bf16 wl[NT * 16 * KP];   // W^T as [n][k], zero padded
  for (int e = threadIdx.x; e < NT * 16 * KP; e += kT) {
    const int n = e / KP, k = e % KP;
    wl[e] = (__bf16)((n < FOUT && k < KIN) ? W[k * FOUT + n] : 0.0f);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
  if (r0 >= N) return;
  const int64_t ra = r0 + (lane & 15);
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k0 = ks * 32 + 8 * (lane >> 4);
    bf16x8 a;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      a[i] = (__bf16)((ra < N && k0 + i < KIN) ? X[ra * ldx + k0 + i] : 0.0f);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 b;
      const __bf16* wp = wl + (t * 16 + (lane & 15)) * KP + k0;
#pragma unroll
      for (int i = 0; i < 8; ++i) b[i] = wp[i];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = t * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + 4 * (lane >> 4) + i;
      if (r < N && n < FOUT) {
        const float z = acc[t][i] + bias[n];
        Z[r * ldz + n] = z;
        if (ACT) H[r * ldh + n] = gelu(z);
      }
    }
  }
}

// dX = dZ W^T (N x KOUT); dZ row-major (ld ldz) with FIN columns, W row-major
// [KOUT][FIN].  EPI: dX *= gelu'(Zc) (ld ldc).
template <int FIN, int KOUT, bool EPI>
__global__ __launch_bounds__(kT) void k_layer_dx(const float* __restrict__ dZ, int64_t ldz,
                                                 int64_t N, const float* __restrict__ W,
                                                 const float* __restrict__ Zc, int64_t ldc,
                                                 float* __restrict__ dX, int64_t ldo) {
  constexpr int KS = (FIN + 31) / 32;
  constexpr int KP = KS * 32;
  constexpr int NT = KOUT / 16;
  __shared__ __bf16 wl[NT * 16 * KP];  // W as [n][k] (n < KOUT, k < FIN)
  for (int e = threadIdx.x; e < NT * 16 * KP; e += kT) {
    const int n = e / KP, k = e % KP;
    wl[e] = (__bf16)(k < FIN ? W[n * FIN + k] : 0.0f);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * 16;
  if (r0 >= N) return;
  const int64_t ra = r0 + (lane & 15);
  floatx4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int k0 = ks * 32 + 8 * (lane >> 4);
    bf16x8 a;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      a[i] = (__bf16)((ra < N && k0 + i < FIN) ? dZ[ra * ldz + k0 + i] : 0.0f);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      bf16x8 b;
      const __bf16* wp = wl + (t * 16 + (lane & 15)) * KP + k0;
#pragma unroll
      for (int i = 0; i < 8; ++i) b[i] = wp[i];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int n = t * 16 + (lane & 15);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = r0 + 4 * (lane >> 4) + i;
      if (r < N) {
        float v = acc[t][i];
        if (EPI) v *= gelu_grad(Zc[r * ldc + n]);
        dX[r * ldo + n] = v;
      }
    }
  }
}

// partial weight and bias gradients of one row chunk per workgroup:
// part[blk][k * FOUT + n] = sum_r X[r][k] dZ[r][n],  part[blk][KIN*FOUT + n] = sum_r dZ[r][n]
template <int KIN, int FOUT>
__global__ __launch_bounds__(kT) void k_layer_dw(const float* __restrict__ X, int64_t ldx,
                                                 const float* __restrict__ dZ, int64_t ldz,
                                                 int64_t N, int64_t chunk,
                                                 float* __restrict__ part) {
  constexpr int MT = KIN / 16;
  constexpr int NT = (FOUT + 15) / 16;
  constexpr int STRIDE = KIN * FOUT + FOUT;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t rbeg = (int64_t)blockIdx.x * chunk;
  const int64_t rend = (rbeg + chunk < N) ? rbeg + chunk : N;
  float* out = part + (int64_t)blockIdx.x * STRIDE;
  for (int tile = wv; tile < MT * NT; tile += 4) {
    const int mt = tile / NT, nt = tile % NT;
    const int kcol = mt * 16 + (lane & 15);
    const int ncol = nt * 16 + (lane & 15);
    const bool nok = ncol < FOUT;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    for (int64_t rb = rbeg; rb < rend; rb += 32) {
      bf16x8 a, b;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int64_t r = rb + 8 * (lane >> 4) + i;
        const bool rok = r < rend;
        a[i] = (__bf16)(rok ? X[r * ldx + kcol] : 0.0f);
        const float zv = (rok && nok) ? dZ[r * ldz + ncol] : 0.0f;
        b[i] = (__bf16)zv;
        bsum += zv;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = mt * 16 + 4 * (lane >> 4) + i;
      if (nok) out[k * FOUT + ncol] = acc[i];
    }
    if (mt == 0) {
      bsum += __shfl_xor(bsum, 16, 64);
      bsum += __shfl_xor(bsum, 32, 64);
      if (lane < 16 && nok) out[KIN * FOUT + ncol] = bsum;
    }
  }
}

// out[e] (+)= sum over blocks of part[blk][e], fixed order
__global__ void k_reduce_part(const float* __restrict__ part, int nblk, int stride,
                              float* __restrict__ out, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= stride) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += (double)part[(int64_t)b * stride + e];
  out[e] = accumulate ? out[e] + (float)s : (float)s;
}

// w = exp(clip(o)), coef[l] = sum_m Psi[l][m] w[m]
__global__ void k_coef(const float* __restrict__ o, int64_t N, LpcPsi psi, int degree,
                       float* __restrict__ w, float* __restrict__ coef) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  float wm[kLpcOut];
#pragma unroll
  for (int m = 0; m < kLpcOut; ++m) {
    const float x = fminf(fmaxf(o[i * kLpcOut + m], -kLpcClip), kLpcClip);
    wm[m] = expf(x);
    w[i * kLpcOut + m] = wm[m];
  }
#pragma unroll
  for (int l = 0; l < kLpcCoef; ++l) {
    float c = 0.0f;
    if (l <= degree) {
#pragma unroll
      for (int m = 0; m < kLpcOut; ++m) c += psi.v[l * kLpcOut + m] * wm[m];
    }
    coef[i * kLpcCoef + l] = c;
  }
}

// dO[m] = w[m] [|o[m]| < clip] sum_{l <= degree} dc[l] Psi[l][m]
__global__ void k_coef_bwd(const float* __restrict__ o, const float* __restrict__ w,
                           const float* __restrict__ dc, int64_t N, LpcPsi psi, int degree,
                           float* __restrict__ dO) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
#pragma unroll
  for (int m = 0; m < kLpcOut; ++m) {
    float s = 0.0f;
    for (int l = 0; l <= degree; ++l) s += dc[i * kLpcCoef + l] * psi.v[l * kLpcOut + m];
    const bool in = fabsf(o[i * kLpcOut + m]) < kLpcClip;
    dO[i * kLpcOut + m] = in ? s * w[i * kLpcOut + m] : 0.0f;
  }
}

// dz = dh * gelu'(z) in place on dh (N x 32, ld ldd; z ld ldz)
__global__ void k_gelu_bwd(float* __restrict__ d, int64_t ldd, const float* __restrict__ z,
                           int64_t ldz, int64_t N) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t / kLpcHid;
  const int c = (int)(t % kLpcHid);
  if (r >= N) return;
  d[r * ldd + c] *= gelu_grad(z[r * ldz + c]);
}

__global__ void k_copy_f32(const float* __restrict__ in, int64_t ldi, int64_t N, int ncols,
                           float* __restrict__ out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = t / ncols;
  const int c = (int)(t % ncols);
  if (r < N) out[r * ldo + c] = in[r * ldi + c];
}

// ---------------------------------------------------------------------------
// Chebyshev sequence (FP64, row-major blocks N x nb)
// ---------------------------------------------------------------------------
// z0 = dh * X, w = dh * z0, acc = coef_0 z0, Z[0] = z0
__global__ void k_cheb_init(const double* __restrict__ X, const double* __restrict__ dh, int64_t N,
                            int nb, const float* __restrict__ coef, double* __restrict__ z0,
                            double* __restrict__ w, double* __restrict__ acc,
                            float* __restrict__ Z, int64_t col0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int c = (int)(t % nb);
  if (i >= N) return;
  const double z = dh[i] * X[t];
  z0[t] = z;
  w[t] = dh[i] * z;
  if (coef) acc[t] = (double)coef[i * kLpcCoef] * z;
  if (Z) Z[(col0 + c) * N + i] = (float)z;
}

// mz = dh q / rho; zn = first ? 2 mz - zc : 2 (2 mz - zc) - zp; acc += coef_l zn;
// w = dh zn; Z[l] = zn
__global__ void k_cheb_step(const double* __restrict__ q, const double* __restrict__ dh,
                            double inv_rho, int64_t N, int nb, int l,
                            const double* __restrict__ zp, const double* __restrict__ zc,
                            double* __restrict__ zn, double* __restrict__ w,
                            const float* __restrict__ coef, double* __restrict__ acc,
                            float* __restrict__ Z, int64_t ldl, int64_t col0) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int c = (int)(t % nb);
  if (i >= N) return;
  const double mz = dh[i] * q[t] * inv_rho;
  const double z = (l == 1) ? 2.0 * mz - zc[t] : 2.0 * (2.0 * mz - zc[t]) - zp[t];
  zn[t] = z;
  w[t] = dh[i] * z;
  if (coef) acc[t] += (double)coef[i * kLpcCoef + l] * z;
  if (Z) Z[(int64_t)l * ldl + (col0 + c) * N + i] = (float)z;
}

// Out (column-major) = dh * acc
__global__ void k_cheb_out(const double* __restrict__ acc, const double* __restrict__ dh,
                           int64_t N, int nb, double* __restrict__ Out, int64_t ldo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / nb;
  const int c = (int)(t % nb);
  if (i < N) Out[i + c * ldo] = dh[i] * acc[t];
}

// ---------------------------------------------------------------------------
// pair loss: t_j = dh (.) sum_l coef_l (.) Z[l][j];  L_j = 1 - (t.e)^2 / (|t|^2 |e|^2)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kT) void k_loss_partial(const float* __restrict__ Z, int64_t ldl,
                                                     const float* __restrict__ E,
                                                     const float* __restrict__ coef,
                                                     const double* __restrict__ dh, int64_t N,
                                                     int degree, float* __restrict__ T,
                                                     double* __restrict__ part) {
  __shared__ double s0[kT], s1[kT], s2[kT];
  const int j = blockIdx.y;
  double te = 0.0, tt = 0.0, ee = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kT) {
    float acc = 0.0f;
    for (int l = 0; l <= degree; ++l) acc += coef[i * kLpcCoef + l] * Z[l * ldl + j * N + i];
    const float t = (float)(dh[i] * (double)acc);
    const float e = E[j * N + i];
    T[j * N + i] = t;
    te += (double)t * e;
    tt += (double)t * t;
    ee += (double)e * e;
  }
  s0[threadIdx.x] = te;
  s1[threadIdx.x] = tt;
  s2[threadIdx.x] = ee;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      s0[threadIdx.x] += s0[threadIdx.x + off];
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* p = part + ((int64_t)j * gridDim.x + blockIdx.x) * 3;
    p[0] = s0[0];
    p[1] = s1[0];
    p[2] = s2[0];
  }
}

// per pair: sums in fixed order, loss and the factors of dL/dt = a t - b e
// (already divided by the number of valid pairs and multiplied by weight);
// loss_out[0] += weight * mean loss
__global__ void k_loss_pairs(const double* __restrict__ part, int nbx, int npairs, double weight,
                             double* __restrict__ ab, double* __restrict__ loss_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int nv = 0;
  for (int j = 0; j < npairs; ++j) {
    double te = 0.0, tt = 0.0, ee = 0.0;
    for (int b = 0; b < nbx; ++b) {
      const double* p = part + ((int64_t)j * nbx + b) * 3;
      te += p[0];
      tt += p[1];
      ee += p[2];
    }
    ab[3 * j + 0] = te;
    ab[3 * j + 1] = tt;
    ab[3 * j + 2] = ee;
    if (ee > 0.0 && tt > 0.0) ++nv;
  }
  const double inv = 1.0 / (double)(nv > 0 ? nv : 1);
  double L = 0.0;
  for (int j = 0; j < npairs; ++j) {
    const double te = ab[3 * j + 0], tt = ab[3 * j + 1], ee = ab[3 * j + 2];
    double a = 0.0, b = 0.0;
    if (ee > 0.0 && tt > 0.0) {
      L += 1.0 - te * te / (tt * ee);
      a = 2.0 * te * te / (tt * tt * ee) * inv * weight;
      b = 2.0 * te / (tt * ee) * inv * weight;
    }
    ab[3 * j + 0] = a;
    ab[3 * j + 1] = b;
  }
  loss_out[0] += weight * L * inv;
}

// dcoef[i][l] = dh_i sum_j (a_j t_ij - b_j e_ij) Z[l][j][i]
__global__ void k_loss_dcoef(const float* __restrict__ Z, int64_t ldl, const float* __restrict__ E,
                             const float* __restrict__ T, const double* __restrict__ ab,
                             const double* __restrict__ dh, int64_t N, int npairs, int degree,
                             float* __restrict__ dc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s[kLpcCoef];
#pragma unroll
  for (int l = 0; l < kLpcCoef; ++l) s[l] = 0.0;
  for (int j = 0; j < npairs; ++j) {
    const double g = ab[3 * j] * T[j * N + i] - ab[3 * j + 1] * E[j * N + i];
    if (g == 0.0) continue;
#pragma unroll
    for (int l = 0; l < kLpcCoef; ++l)
      if (l <= degree) s[l] += g * Z[l * ldl + j * N + i];
  }
#pragma unroll
  for (int l = 0; l < kLpcCoef; ++l) dc[i * kLpcCoef + l] = (float)(l <= degree ? dh[i] * s[l] : 0.0);
}

// training pairs: E = R / |R| (column-wise, zero columns stay zero), FP64
__global__ __launch_bounds__(kT) void k_colnorm(const double* __restrict__ R, int64_t ldr,
                                                int64_t N, double* __restrict__ nrm) {
  __shared__ double sh[kT];
  const int j = blockIdx.x;
  double a = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += kT) {
    const double x = R[i + j * ldr];
    a += x * x;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = kT / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm[j] = sqrt(sh[0]);
}

__global__ void k_colscale(const double* __restrict__ R, int64_t ldr, int64_t N, int np,
                           const double* __restrict__ nrm, double* __restrict__ E, int64_t lde) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t % N;
  const int j = (int)(t / N);
  if (j >= np) return;
  const double n = nrm[j];
  E[i + j * lde] = n > 0.0 ? R[i + j * ldr] / n : 0.0;
}

__global__ void k_to_f32_cols(const double* __restrict__ X, int64_t ldx, int64_t N, int np,
                              float* __restrict__ Y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t % N;
  const int j = (int)(t / N);
  if (j < np) Y[j * N + i] = (float)X[i + j * ldx];
}

// Adam (Kingma and Ba 2015) with bias corrections bc1 = 1 - beta1^t, bc2 = 1 - beta2^t
__global__ void k_adam(int n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_fill_f32(float* __restrict__ x, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
LpcPsi lpc_psi(int degree) {
  LpcPsi p;
  for (float& x : p.v) x = 0.0f;
  const int n = degree + 1;
  const double th = M_PI / (n + 1);
  for (int l = 0; l <= degree; ++l) {
    const double g = ((n - l + 1) * std::cos(l * th) + std::sin(l * th) / std::tan(th)) / (n + 1);
    for (int m = 0; m < kLpcOut; ++m) {
      const double delta = std::pow(10.0, -5.0 + 5.0 * m / (kLpcOut - 1));
      const double a = 1.0 + 2.0 * delta;
      const double sq = std::sqrt(a * a - 1.0);
      const double q = a - sq;
      const double al = l == 0 ? 2.0 / sq : 4.0 / sq * std::pow(-q, l);
      p.v[l * kLpcOut + m] = (float)(g * al);
    }
  }
  return p;
}

void lpc_alloc(const svds_matrix* M, LpcOp& op, DeviceBuffers& buf) {
  op.A = &M->A;
  op.At = &M->At;
  op.diag = M->diagC;
  op.N = M->A.cols;
  op.mw = M->A.rows;
  op.dh = buf.get<double>(op.N);
  op.sinv = buf.get<float>(op.N);
}

void lpc_prepare(const svds_matrix* M, LpcOp& op, DeviceBuffers& buf, hipStream_t s) {
  lpc_alloc(M, op, buf);
  lpc_compute(op, s);
}

void lpc_compute(LpcOp& op, hipStream_t s) {
  const int64_t N = op.N, mw = op.mw;
  DeviceBuffers tmp(s);
  double* u = tmp.get<double>(mw);
  double* v = tmp.get<double>(N);
  k_dh<<<blocks_for(N), kT, 0, s>>>(op.diag, N, op.dh);
  // S = |A|^T |A| 1
  k_abs_spmv<<<blocks_for(mw), kT, 0, s>>>(op.A->rp, op.A->ci, op.A->val, mw, nullptr, u);
  k_abs_spmv<<<blocks_for(N), kT, 0, s>>>(op.At->rp, op.At->ci, op.At->val, N, u, v);
  k_sinv<<<blocks_for(N), kT, 0, s>>>(v, N, op.sinv);
  // rho = max dh * (|A|^T |A| dh)
  k_abs_spmv<<<blocks_for(mw), kT, 0, s>>>(op.A->rp, op.A->ci, op.A->val, mw, op.dh, u);
  k_abs_spmv<<<blocks_for(N), kT, 0, s>>>(op.At->rp, op.At->ci, op.At->val, N, u, v);
  const int nblk = std::min(1024, blocks_for(N));
  double* part = tmp.get<double>(3 * nblk);
  double* stats = tmp.get<double>(3);
  k_feat_stats<<<nblk, kT, 0, s>>>(op.diag, op.At->rp, op.dh, v, N, part);
  k_feat_stats_final<<<1, 64, 0, s>>>(part, nblk, N, stats);
  SVDS_LAUNCH_CHECK();
  double h[3];
  SVDS_HIP(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, s));
  SVDS_HIP(hipStreamSynchronize(s));
  op.rho = h[2];
}

void lpc_features(const LpcOp& op, float* feat, hipStream_t s) {
  const int64_t N = op.N, mw = op.mw;
  DeviceBuffers tmp(s);
  double* u = tmp.get<double>(mw);
  double* v = tmp.get<double>(N);
  double* q = tmp.get<double>(N);
  double* x2 = tmp.get<double>(N);
  const int nblk = std::min(1024, blocks_for(N));
  double* part = tmp.get<double>(3 * nblk);
  double* stats = tmp.get<double>(3);
  // v = |A|^T |A| dh and the global statistics
  k_abs_spmv<<<blocks_for(mw), kT, 0, s>>>(op.A->rp, op.A->ci, op.A->val, mw, op.dh, u);
  k_abs_spmv<<<blocks_for(N), kT, 0, s>>>(op.At->rp, op.At->ci, op.At->val, N, u, v);
  k_feat_stats<<<nblk, kT, 0, s>>>(op.diag, op.At->rp, op.dh, v, N, part);
  k_feat_stats_final<<<1, 64, 0, s>>>(part, nblk, N, stats);
  // q = C dh (signed products)
  spmm(*op.A, 1, op.dh, u, s);
  spmm(*op.At, 1, u, q, s);
  k_feat_assemble<<<blocks_for(N), kT, 0, s>>>(op.diag, op.At->rp, op.dh, q, v, stats, N, feat,
                                                x2);
  // f5 = M f2 = dh * C (dh * f2) / rho
  spmm(*op.A, 1, x2, u, s);
  spmm(*op.At, 1, u, q, s);
  k_feat_f5<<<blocks_for(N), kT, 0, s>>>(op.dh, q, stats, N, feat);
  SVDS_LAUNCH_CHECK();
}

namespace {

// out (+)= S^-1 |A|^T |A| in  (F columns), or with transposed weights
// (TRANS: |A|^T |A| S^-1 in)
template <int F, bool ACCUM>
void aggregate(const LpcOp& op, const float* in, int64_t ldi, float* out, int64_t ldo,
               float* gbuf, bool trans, hipStream_t s) {
  k_agg<F, false><<<blocks_for(op.mw * F), kT, 0, s>>>(op.A->rp, op.A->ci, op.A->val32, op.mw,
                                                        in, ldi, trans ? op.sinv : nullptr, gbuf,
                                                        F, nullptr);
  k_agg<F, ACCUM><<<blocks_for(op.N * F), kT, 0, s>>>(op.At->rp, op.At->ci, op.At->val32, op.N,
                                                      gbuf, F, nullptr, out, ldo,
                                                      trans ? nullptr : op.sinv);
}

int dw_blocks(int64_t N, int64_t* chunk) {
  const int nblk = (int)std::min<int64_t>(512, std::max<int64_t>(1, (N + 255) / 256));
  int64_t c = (N + nblk - 1) / nblk;
  c = (c + 31) / 32 * 32;
  *chunk = c;
  return (int)std::max<int64_t>(1, (N + c - 1) / c);
}

template <int KIN, int FOUT>
void weight_grad(const float* X, int64_t ldx, const float* dZ, int64_t ldz, int64_t N,
                 float* part, float* grad_w, bool accumulate, hipStream_t s) {
  int64_t chunk;
  const int nblk = dw_blocks(N, &chunk);
  k_layer_dw<KIN, FOUT><<<nblk, kT, 0, s>>>(X, ldx, dZ, ldz, N, chunk, part);
  constexpr int stride = KIN * FOUT + FOUT;
  k_reduce_part<<<blocks_for(stride), kT, 0, s>>>(part, nblk, stride, grad_w, accumulate ? 1 : 0);
}

}  // namespace

int64_t lpc_partial_floats(int64_t N) {
  int64_t chunk;
  const int nblk = dw_blocks(N, &chunk);
  return (int64_t)nblk * (2 * kLpcHid * kLpcHid + kLpcHid);
}

void lpc_forward(const LpcOp& op, const float* params, const float* feat, int degree, float* coef,
                 float* cache, float* gbuf, hipStream_t s) {
  const int64_t N = op.N;
  float* x1 = cache + kCx1 * N;
  float* z1 = cache + kCz1 * N;
  float* x2 = cache + kCx2 * N;
  float* z2 = cache + kCz2 * N;
  float* h2 = cache + kCh2 * N;
  float* o = cache + kCo * N;
  float* w = cache + kCw * N;
  const int rows_blocks = blocks_for(N, 64);
  // x1 = [f, agg f]
  k_copy_f32<<<blocks_for(N * kLpcNF), kT, 0, s>>>(feat, kLpcNF, N, kLpcNF, x1, 2 * kLpcNF);
  aggregate<kLpcNF, false>(op, feat, kLpcNF, x1 + kLpcNF, 2 * kLpcNF, gbuf, false, s);
  // layer 1 -> z1, h1 (into x2[:, :32])
  k_layer_fwd<2 * kLpcNF, kLpcHid, true><<<rows_blocks, kT, 0, s>>>(
      x1, 2 * kLpcNF, N, params + kW1, params + kB1, z1, kLpcHid, x2, 2 * kLpcHid);
  aggregate<kLpcHid, false>(op, x2, 2 * kLpcHid, x2 + kLpcHid, 2 * kLpcHid, gbuf, false, s);
  // layer 2 -> z2, h2
  k_layer_fwd<2 * kLpcHid, kLpcHid, true><<<rows_blocks, kT, 0, s>>>(
      x2, 2 * kLpcHid, N, params + kW2, params + kB2, z2, kLpcHid, h2, kLpcHid);
  // output layer -> o
  k_layer_fwd<kLpcHid, kLpcOut, false><<<rows_blocks, kT, 0, s>>>(
      h2, kLpcHid, N, params + kW3, params + kB3, o, kLpcOut, nullptr, 0);
  k_coef<<<blocks_for(N), kT, 0, s>>>(o, N, lpc_psi(degree), degree, w, coef);
  SVDS_LAUNCH_CHECK();
}

void lpc_backward(const LpcOp& op, const float* params, const float* cache, int degree,
                  const float* dcoef, float* grad, bool accumulate, float* work, float* gbuf,
                  float* part, hipStream_t s) {
  const int64_t N = op.N;
  const float* x1 = cache + kCx1 * N;
  const float* z1 = cache + kCz1 * N;
  const float* x2 = cache + kCx2 * N;
  const float* z2 = cache + kCz2 * N;
  const float* h2 = cache + kCh2 * N;
  const float* o = cache + kCo * N;
  const float* w = cache + kCw * N;
  float* dO = work;                       // N x 8
  float* dz2 = work + kLpcOut * N;        // N x 32
  float* dx2 = dz2 + kLpcHid * N;         // N x 64
  const int rows_blocks = blocks_for(N, 64);
  k_coef_bwd<<<blocks_for(N), kT, 0, s>>>(o, w, dcoef, N, lpc_psi(degree), degree, dO);
  weight_grad<kLpcHid, kLpcOut>(h2, kLpcHid, dO, kLpcOut, N, part, grad + kW3, accumulate, s);
  // dz2 = (dO W3^T) * gelu'(z2)
  k_layer_dx<kLpcOut, kLpcHid, true><<<rows_blocks, kT, 0, s>>>(dO, kLpcOut, N, params + kW3, z2,
                                                                 kLpcHid, dz2, kLpcHid);
  weight_grad<2 * kLpcHid, kLpcHid>(x2, 2 * kLpcHid, dz2, kLpcHid, N, part, grad + kW2,
                                    accumulate, s);
  // dx2 = dz2 W2^T; dh1 = dx2[:, :32] + agg^T(dx2[:, 32:]); dz1 = dh1 * gelu'(z1)
  k_layer_dx<kLpcHid, 2 * kLpcHid, false><<<rows_blocks, kT, 0, s>>>(
      dz2, kLpcHid, N, params + kW2, nullptr, 0, dx2, 2 * kLpcHid);
  aggregate<kLpcHid, true>(op, dx2 + kLpcHid, 2 * kLpcHid, dx2, 2 * kLpcHid, gbuf, true, s);
  k_gelu_bwd<<<blocks_for(N * kLpcHid), kT, 0, s>>>(dx2, 2 * kLpcHid, z1, kLpcHid, N);
  weight_grad<2 * kLpcNF, kLpcHid>(x1, 2 * kLpcNF, dx2, 2 * kLpcHid, N, part, grad + kW1,
                                   accumulate, s);
  SVDS_LAUNCH_CHECK();
}

void lpc_scratch(const LpcOp& op, int nbmax, LpcScratch& sc, DeviceBuffers& buf) {
  const size_t nN = (size_t)op.N * nbmax;
  for (auto& z : sc.z) z = buf.get<double>(nN);
  sc.w = buf.get<double>(nN);
  sc.q = buf.get<double>(nN);
  sc.acc = buf.get<double>(nN);
  sc.y = buf.get<double>((size_t)op.mw * nbmax);
  sc.nbmax = nbmax;
}

void lpc_cheb(const LpcOp& op, int nb, const double* X, int degree, const float* coef,
              double* Out, int64_t ldo, float* Z, int64_t ldl, int64_t col0, LpcScratch& sc,
              hipStream_t s) {
  if (nb < 1 || nb > sc.nbmax || nb > kMaxBlock) throw Error(SVDS_ERR_ARG, "lpc_cheb: block");
  if (degree < 0 || degree > kLpcMaxDegree) throw Error(SVDS_ERR_ARG, "lpc_cheb: degree");
  const int64_t N = op.N;
  const int grid = blocks_for(N * nb);
  double* zp = sc.z[0];
  double* zc = sc.z[1];
  double* zn = sc.z[2];
  k_cheb_init<<<grid, kT, 0, s>>>(X, op.dh, N, nb, coef, zc, sc.w, sc.acc, Z, col0);
  const double inv_rho = 1.0 / op.rho;
  for (int l = 1; l <= degree; ++l) {
    spmm(*op.A, nb, sc.w, sc.y, s);
    spmm(*op.At, nb, sc.y, sc.q, s);
    k_cheb_step<<<grid, kT, 0, s>>>(sc.q, op.dh, inv_rho, N, nb, l, zp, zc, zn, sc.w, coef,
                                    sc.acc, Z, ldl, col0);
    double* t = zp;
    zp = zc;
    zc = zn;
    zn = t;
  }
  if (coef && Out) k_cheb_out<<<grid, kT, 0, s>>>(sc.acc, op.dh, N, nb, Out, ldo);
  SVDS_LAUNCH_CHECK();
}

void lpc_apply(const LpcOp& op, const float* coef, int degree, int nb, const double* R,
               int64_t ldr, double* T, int64_t ldt, LpcScratch& sc, hipStream_t s) {
  // the row-major input block goes through sc.q (free until the first product)
  pack_rows(R, ldr, nullptr, 0.0, op.N, nb, sc.q, s);
  lpc_cheb(op, nb, sc.q, degree, coef, T, ldt, nullptr, 0, 0, sc, s);
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
void lpc_make_pairs(const LpcOp& op, int np, const double* R, int64_t ldr, double* Q, double* E,
                    int64_t ldp, hipStream_t s) {
  if (np <= 0) return;
  const int64_t N = op.N;
  DeviceBuffers tmp(s);
  double* nrm = tmp.get<double>(np);
  double* xc = tmp.get<double>((size_t)N * kMaxBlock);
  double* yc = tmp.get<double>((size_t)op.mw * kMaxBlock);
  double* qc = tmp.get<double>((size_t)N * kMaxBlock);
  k_colnorm<<<np, kT, 0, s>>>(R, ldr, N, nrm);
  k_colscale<<<blocks_for(N * np), kT, 0, s>>>(R, ldr, N, np, nrm, E, ldp);
  for (int j0 = 0; j0 < np; j0 += kMaxBlock) {
    const int nb = std::min(kMaxBlock, np - j0);
    pack_rows(E + j0 * ldp, ldp, nullptr, 0.0, N, nb, xc, s);
    spmm(*op.A, nb, xc, yc, s);
    spmm(*op.At, nb, yc, qc, s);
    unpack_rows(qc, N, nb, Q + j0 * ldp, ldp, s);
  }
  SVDS_LAUNCH_CHECK();
}

LpcSet::LpcSet(const svds_matrix* M, int np, const double* R, int64_t ldr, int degree,
               hipStream_t s)
    : buf(s), npairs(np) {
  lpc_prepare(M, op, buf, s);
  const int64_t N = op.N;
  feat = buf.get<float>((size_t)N * kLpcNF);
  lpc_features(op, feat, s);
  coef = buf.get<float>((size_t)N * kLpcCoef);
  dcoef = buf.get<float>((size_t)N * kLpcCoef);
  cache = buf.get<float>((size_t)N * kLpcCacheRow);
  work = buf.get<float>((size_t)N * (kLpcOut + 3 * kLpcHid));
  gbuf = buf.get<float>((size_t)op.mw * kLpcHid);
  part = buf.get<float>((size_t)lpc_partial_floats(N));
  ldl = (int64_t)np * N;
  Z = buf.get<float>((size_t)(degree + 1) * ldl);
  E = buf.get<float>((size_t)ldl);
  T = buf.get<float>((size_t)ldl);
  nbx = std::min(64, blocks_for(N));
  lpart = buf.get<double>((size_t)np * nbx * 3);
  ab = buf.get<double>((size_t)np * 3);
  if (np > 0) {
    DeviceBuffers tmp(s);
    double* Q = tmp.get<double>((size_t)N * np);
    double* E64 = tmp.get<double>((size_t)N * np);
    lpc_make_pairs(op, np, R, ldr, Q, E64, N, s);
    k_to_f32_cols<<<blocks_for(N * np), kT, 0, s>>>(E64, N, N, np, E);
    LpcScratch sc;
    lpc_scratch(op, kMaxBlock, sc, tmp);
    double* xc = tmp.get<double>((size_t)N * kMaxBlock);
    for (int j0 = 0; j0 < np; j0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, np - j0);
      pack_rows(Q + j0 * N, N, nullptr, 0.0, N, nb, xc, s);
      lpc_cheb(op, nb, xc, degree, nullptr, nullptr, 0, Z, ldl, j0, sc, s);
    }
    SVDS_HIP(hipStreamSynchronize(s));
  }
}

void lpc_loss(LpcSet& st, int degree, double weight, double* loss_out, hipStream_t s) {
  const int64_t N = st.op.N;
  if (st.npairs <= 0) {
    k_fill_f32<<<blocks_for(N * kLpcCoef), kT, 0, s>>>(st.dcoef, N * kLpcCoef, 0.0f);
    return;
  }
  dim3 grid(st.nbx, st.npairs);
  k_loss_partial<<<grid, kT, 0, s>>>(st.Z, st.ldl, st.E, st.coef, st.op.dh, N, degree, st.T,
                                     st.lpart);
  k_loss_pairs<<<1, 64, 0, s>>>(st.lpart, st.nbx, st.npairs, weight, st.ab, loss_out);
  k_loss_dcoef<<<blocks_for(N), kT, 0, s>>>(st.Z, st.ldl, st.E, st.T, st.ab, st.op.dh, N,
                                            st.npairs, degree, st.dcoef);
  SVDS_LAUNCH_CHECK();
}

void lpc_adam(int n, float* p, const float* g, float* m, float* v, int step, float lr, float b1,
              float b2, float eps, hipStream_t s) {
  const float bc1 = (float)(1.0 - std::pow((double)b1, step));
  const float bc2 = (float)(1.0 - std::pow((double)b2, step));
  k_adam<<<blocks_for(n), kT, 0, s>>>(n, p, g, m, v, lr, b1, b2, eps, bc1, bc2);
  SVDS_LAUNCH_CHECK();
}

void lpc_fill(float* x, int64_t n, float v, hipStream_t s) {
  k_fill_f32<<<blocks_for(n), kT, 0, s>>>(x, n, v);
}

void lpc_train(std::vector<LpcSet*>& sets, int degree, int steps, float lr, float* params,
               double* loss_hist_host, hipStream_t s) {
  DeviceBuffers tmp(s);
  float* grad = tmp.get<float>(kLpcNParams);
  float* m = tmp.get<float>(kLpcNParams);
  float* v = tmp.get<float>(kLpcNParams);
  double* lh = tmp.get<double>(std::max(steps, 1));
  lpc_fill(m, kLpcNParams, 0.0f, s);
  lpc_fill(v, kLpcNParams, 0.0f, s);
  SVDS_HIP(hipMemsetAsync(lh, 0, sizeof(double) * std::max(steps, 1), s));
  int nonempty = 0;
  for (auto* st : sets) nonempty += st->npairs > 0 ? 1 : 0;
  const double weight = 1.0 / std::max(nonempty, 1);
  for (int step = 1; step <= steps; ++step) {
    bool first = true;
    for (auto* st : sets) {
      if (st->npairs <= 0) continue;
      lpc_forward(st->op, params, st->feat, degree, st->coef, st->cache, st->gbuf, s);
      lpc_loss(*st, degree, weight, lh + (step - 1), s);
      lpc_backward(st->op, params, st->cache, degree, st->dcoef, grad, !first, st->work,
                   st->gbuf, st->part, s);
      first = false;
    }
    if (first) break;  // no pairs at all
    lpc_adam(kLpcNParams, params, grad, m, v, step, lr, 0.9f, 0.999f, 1e-8f, s);
  }
  if (loss_hist_host && steps > 0)
    SVDS_HIP(hipMemcpyAsync(loss_hist_host, lh, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
  SVDS_HIP(hipStreamSynchronize(s));
}

}  // namespace svds
