// Tall-skinny dense kernels of one GD+k iteration (Section 3.3, Table 3:
// O((m+n) g) work per iteration, all of it HBM-bound).  Vectors are stored
// column-major (column j of an N x g basis at p + j*ld), so that every load of
// a wavefront is 64 consecutive doubles.  Reductions over the N rows are done
// in two fixed-order phases (per-workgroup partials, then a column reduction)
// so that results do not depend on scheduling.
#include "common.h"

namespace svds {

constexpr int kThreads = 256;
constexpr int kMaxSegCols = 256;  // columns of [X_lock V T] in one projection

// workgroups of the streaming kernels: about one 256-row chunk per workgroup,
// at most 2048 (8 per CU on 256 CUs), whole rounds of the 8 XCDs
int reduce_blocks(int64_t N) {
  int64_t nb = (N + kThreads - 1) / kThreads;
  nb = std::max<int64_t>(1, std::min<int64_t>(nb, 2048));
  if (nb >= 64) nb = (nb / 8) * 8;
  return (int)nb;
}

template <typename TB>
struct Segs3T {
  const TB* p[3];
  int64_t ld[3];
  int n0, n1, n2;  // columns per segment
};
using Segs3 = Segs3T<double>;

template <typename TB>
__device__ __forceinline__ const TB* seg_col(const Segs3T<TB>& s, int v) {
  if (v < s.n0) return s.p[0] + (int64_t)v * s.ld[0];
  v -= s.n0;
  if (v < s.n1) return s.p[1] + (int64_t)v * s.ld[1];
  v -= s.n1;
  return s.p[2] + (int64_t)v * s.ld[2];
}

// sum over the block of acc[] (NA values per thread) -> out[0..NA) (thread 0..NA-1)
template <int NA>
__device__ __forceinline__ void block_reduce_store(double (&acc)[NA], double* sh, double* out,
                                                   int64_t stride_out, int nvalid) {
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    double v = wave_sum(acc[a]);
    if (lane == 0) sh[w * NA + a] = v;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < NA; a += kThreads) {
    if (a < nvalid) {
      double v = ((sh[a] + sh[NA + a]) + sh[2 * NA + a]) + sh[3 * NA + a];
      out[a * stride_out] = v;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// C = [segs]^T T  (partials per workgroup)
// Workgroup (x, y) takes a contiguous row range and the column groups
// 4y .. 4y+3 of kCPW basis columns, one group per wavefront; each lane covers
// rows lane, lane + 64, ... with kTU row groups' loads issued together.  When
// fewer than four groups remain for the workgroup, its spare wavefronts split
// the row range of a group, and the pieces are added in row order before the
// partial is written, so every partial has the same layout.
// ---------------------------------------------------------------------------
constexpr int kCPW = 4;   // basis columns per wavefront (16 per workgroup column)
constexpr int kTU = 8;    // 64-row groups per step: all their loads are issued first

template <int B, typename TB>
__global__ __launch_bounds__(kThreads) void k_tsgemm_tn(Segs3T<TB> segs, int total, int64_t N,
                                                        const double* __restrict__ T,
                                                        int64_t ldt, int64_t chunk,
                                                        double* __restrict__ partial,
                                                        const int* __restrict__ skip) {
  if (skip && *skip) return;  // device-side decision: this pass is not needed (uniform)
  __shared__ double red[4][kCPW * B];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int g0 = blockIdx.y * 4;
  const int ncg = min(4, (total + kCPW - 1) / kCPW - g0);  // column groups here, 1..4
  const int spl = 4 / ncg;                                  // wavefronts per group
  const int grp = w % ncg, sub = w / ncg;
  const bool active = sub < spl;
  const int c0 = (g0 + grp) * kCPW;
  const TB* qp[kCPW];
  bool ok[kCPW];
#pragma unroll
  for (int jj = 0; jj < kCPW; ++jj) {
    const int col = c0 + jj;
    ok[jj] = col < total;
    qp[jj] = seg_col(segs, min(col, total - 1));
  }
  double acc[kCPW * B];
#pragma unroll
  for (int a = 0; a < kCPW * B; ++a) acc[a] = 0.0;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int64_t rb = (int64_t)bid * chunk;
  const int64_t re = (rb + chunk < N) ? rb + chunk : N;
  constexpr int64_t kStep = kWave * kTU;
  const int64_t nsteps = (re > rb) ? (re - rb + kStep - 1) / kStep : 0;
  const int64_t r0 = rb + (active ? nsteps * sub / spl : nsteps) * kStep;
  const int64_t r1e = rb + (active ? nsteps * (sub + 1) / spl : nsteps) * kStep;
  const int64_t r1 = (r1e < re) ? r1e : re;
  for (int64_t base = r0; base < r1; base += kStep) {
    double tv[kTU][B], q[kTU][kCPW];
#pragma unroll
    for (int u = 0; u < kTU; ++u) {
      const int64_t row = base + u * kWave + lane;
      const bool in = row < r1;
#pragma unroll
      for (int c = 0; c < B; ++c) tv[u][c] = in ? T[row + c * ldt] : 0.0;
#pragma unroll
      for (int jj = 0; jj < kCPW; ++jj) q[u][jj] = (in && ok[jj]) ? (double)qp[jj][row] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kTU; ++u)
#pragma unroll
      for (int jj = 0; jj < kCPW; ++jj)
#pragma unroll
        for (int c = 0; c < B; ++c) acc[jj * B + c] = fma(q[u][jj], tv[u][c], acc[jj * B + c]);
  }
#pragma unroll
  for (int a = 0; a < kCPW * B; ++a) {
    const double v = wave_sum(acc[a]);
    if (lane == 0) red[w][a] = v;
  }
  __syncthreads();
  // partial layout: [c * total + col][block]
  if (active && sub == 0 && lane < kCPW * B) {
    const int jj = lane / B, c = lane % B;
    double v = red[w][lane];
    for (int q = 1; q < spl; ++q) v += red[grp + q * ncg][lane];
    if (c0 + jj < total)
      partial[((int64_t)c * total + c0 + jj) * gridDim.x + blockIdx.x] = v;
  }
}

// one wavefront per output: out[o] = sum over blocks of P[o * nblk + block]
__global__ __launch_bounds__(64) void k_reduce_partials(const double* __restrict__ P, int nblk,
                                                        double* __restrict__ out,
                                                        const int* __restrict__ skip) {
  const int o = blockIdx.x;
  if (skip && *skip) {  // the producing pass was skipped: its result is zero
    if (threadIdx.x == 0) out[o] = 0.0;
    return;
  }
  const double* p = P + (int64_t)o * nblk;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += p[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[o] = s;
}

void reduce_partials(const double* P, int nblk, int nout, double* out, hipStream_t s,
                     const int* skip) {
  if (nout <= 0) return;
  k_reduce_partials<<<nout, 64, 0, s>>>(P, nblk, out, skip);
  SVDS_LAUNCH_CHECK();
}

template <typename TB>
static Segs3T<TB> make_segs(const SegT<TB>* segs, int nseg, int& total) {
  if (nseg > 3) throw Error(SVDS_ERR_ARG, "at most 3 segments");
  Segs3T<TB> s{};
  int n[3] = {0, 0, 0};
  for (int i = 0; i < 3; ++i) {
    s.p[i] = i < nseg ? segs[i].p : nullptr;
    s.ld[i] = i < nseg ? segs[i].ld : 0;
    n[i] = i < nseg ? segs[i].ncols : 0;
  }
  s.n0 = n[0];
  s.n1 = n[1];
  s.n2 = n[2];
  total = n[0] + n[1] + n[2];
  // the last segment must be non-empty for the clamped column pointer
  return s;
}

template <int B, typename TB>
static int tsgemm_b(const Segs3T<TB>& sg, int total, int64_t N, const double* T, int64_t ldt,
                    double* partial, double* C, hipStream_t s, const int* skip) {
  // one contiguous row range per workgroup column (several 256-row steps
  // amortise the final wave reductions)
  int nb = std::min(reduce_blocks(N), 256);
  int64_t chunk = (N + nb - 1) / nb;
  chunk = (chunk + kWave * kTU - 1) / (kWave * kTU) * (kWave * kTU);
  nb = (int)((N + chunk - 1) / chunk);
  if (nb >= 64 && nb % 8) {  // whole XCD rounds for the remap
    nb = (nb + 7) / 8 * 8;
  }
  dim3 grid(nb, (total + 4 * kCPW - 1) / (4 * kCPW));
  k_tsgemm_tn<B, TB><<<grid, kThreads, 0, s>>>(sg, total, N, T, ldt, chunk, partial, skip);
  SVDS_LAUNCH_CHECK();
  if (C) reduce_partials(partial, nb, total * B, C, s, skip);
  return nb;
}

template <typename TB>
static int tsgemm_any(const SegT<TB>* segs, int nseg, int64_t N, const double* T, int64_t ldt,
                      int b, double* partial, double* C, hipStream_t s, const int* skip) {
  int total = 0;
  Segs3T<TB> sg = make_segs(segs, nseg, total);
  if (total == 0) return 0;
  if (total > kMaxSegCols) throw Error(SVDS_ERR_ARG, "projection too wide");
  switch (b) {
    case 1: return tsgemm_b<1>(sg, total, N, T, ldt, partial, C, s, skip);
    case 2: return tsgemm_b<2>(sg, total, N, T, ldt, partial, C, s, skip);
    case 3: return tsgemm_b<3>(sg, total, N, T, ldt, partial, C, s, skip);
    case 4: return tsgemm_b<4>(sg, total, N, T, ldt, partial, C, s, skip);
    case 5: return tsgemm_b<5>(sg, total, N, T, ldt, partial, C, s, skip);
    case 6: return tsgemm_b<6>(sg, total, N, T, ldt, partial, C, s, skip);
    case 7: return tsgemm_b<7>(sg, total, N, T, ldt, partial, C, s, skip);
    case 8: return tsgemm_b<8>(sg, total, N, T, ldt, partial, C, s, skip);
    default: throw Error(SVDS_ERR_ARG, "tsgemm: b must be 1..8");
  }
}

template <typename TB>
void tsgemm_tn(const SegT<TB>* segs, int nseg, int64_t N, const double* T, int64_t ldt, int b,
               double* partial, double* C, hipStream_t s, const int* skip) {
  tsgemm_any(segs, nseg, N, T, ldt, b, partial, C, s, skip);
}

int tsgemm_tn_partial(const Seg* segs, int nseg, int64_t N, const double* T, int64_t ldt, int b,
                      double* partial, hipStream_t s) {
  return tsgemm_any(segs, nseg, N, T, ldt, b, partial, nullptr, s, nullptr);
}

template void tsgemm_tn<double>(const SegT<double>*, int, int64_t, const double*, int64_t, int,
                                double*, double*, hipStream_t, const int*);
template void tsgemm_tn<float>(const SegT<float>*, int, int64_t, const double*, int64_t, int,
                               double*, double*, hipStream_t, const int*);

// ---------------------------------------------------------------------------
// T -= [segs] C      (C: total x b, column-major)
// ---------------------------------------------------------------------------
template <int B, typename TB>
__global__ __launch_bounds__(kThreads) void k_ts_update(Segs3T<TB> segs, int total, int64_t N,
                                                        const double* __restrict__ C, int ldc,
                                                        double* __restrict__ T, int64_t ldt,
                                                        const int* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ double cs[kMaxSegCols * B];
  for (int a = threadIdx.x; a < total * B; a += kThreads) {
    int j = a / B, c = a % B;
    cs[a] = C[(int64_t)c * ldc + j];
  }
  __syncthreads();
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    double t[B];
#pragma unroll
    for (int c = 0; c < B; ++c) t[c] = T[i + c * ldt];
    for (int j = 0; j < total; ++j) {
      const double q = (double)seg_col(segs, j)[i];
#pragma unroll
      for (int c = 0; c < B; ++c) t[c] = fma(-q, cs[j * B + c], t[c]);
    }
#pragma unroll
    for (int c = 0; c < B; ++c) T[i + c * ldt] = t[c];
  }
}

template <typename TB>
void ts_update(const SegT<TB>* segs, int nseg, int64_t N, const double* C, int ldc, double* T,
               int64_t ldt, int b, hipStream_t s, const int* skip) {
  int total = 0;
  Segs3T<TB> sg = make_segs(segs, nseg, total);
  if (total == 0) return;
  if (total > kMaxSegCols) throw Error(SVDS_ERR_ARG, "update too wide");
  int nb = reduce_blocks(N);
  switch (b) {
#define CASE(BB) \
  case BB: k_ts_update<BB, TB><<<nb, kThreads, 0, s>>>(sg, total, N, C, ldc, T, ldt, skip); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw Error(SVDS_ERR_ARG, "ts_update: b must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}
template void ts_update<double>(const SegT<double>*, int, int64_t, const double*, int, double*,
                                int64_t, int, hipStream_t, const int*);
template void ts_update<float>(const SegT<float>*, int, int64_t, const double*, int, double*,
                               int64_t, int, hipStream_t, const int*);

// ---------------------------------------------------------------------------
// Out = Q Y   (restart V <- V Y, W <- W Y, Q <- Q Q~, locking x = V y)
// ---------------------------------------------------------------------------
constexpr int kOC = 24;

template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void k_gemm_nn(const TI* __restrict__ Q, int64_t ldq,
                                                      int nq, int64_t N,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      int nout, TO* __restrict__ Out,
                                                      int64_t ldo) {
  __shared__ double ys[kMaxBasis * kOC];
  const int o0 = blockIdx.y * kOC;
  const int no = min(kOC, nout - o0);
  for (int a = threadIdx.x; a < nq * kOC; a += kThreads) {
    int j = a / kOC, o = a % kOC;
    ys[a] = (o < no) ? Y[(int64_t)(o0 + o) * ldy + j] : 0.0;
  }
  __syncthreads();
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    double acc[kOC];
#pragma unroll
    for (int o = 0; o < kOC; ++o) acc[o] = 0.0;
    int j = 0;
    for (; j + 4 <= nq; j += 4) {  // four loads in flight, same summation order
      double q[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] = (double)Q[i + (int64_t)(j + u) * ldq];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int o = 0; o < kOC; ++o) acc[o] = fma(q[u], ys[(j + u) * kOC + o], acc[o]);
    }
    for (; j < nq; ++j) {
      const double q = (double)Q[i + (int64_t)j * ldq];
#pragma unroll
      for (int o = 0; o < kOC; ++o) acc[o] = fma(q, ys[j * kOC + o], acc[o]);
    }
#pragma unroll
    for (int o = 0; o < kOC; ++o)
      if (o < no) Out[i + (int64_t)(o0 + o) * ldo] = (TO)acc[o];
  }
}

template <typename TI, typename TO>
void ts_gemm_nn(const TI* Q, int64_t ldq, int nq, int64_t N, const double* Y, int64_t ldy,
                int nout, TO* Out, int64_t ldo, hipStream_t s) {
  if (nout <= 0 || N == 0) return;
  if (nq > kMaxBasis) throw Error(SVDS_ERR_ARG, "gemm: inner dimension too large");
  dim3 grid(reduce_blocks(N), (nout + kOC - 1) / kOC);
  k_gemm_nn<TI, TO><<<grid, kThreads, 0, s>>>(Q, ldq, nq, N, Y, ldy, nout, Out, ldo);
  SVDS_LAUNCH_CHECK();
}
template void ts_gemm_nn<double, double>(const double*, int64_t, int, int64_t, const double*,
                                         int64_t, int, double*, int64_t, hipStream_t);
template void ts_gemm_nn<float, float>(const float*, int64_t, int, int64_t, const double*,
                                       int64_t, int, float*, int64_t, hipStream_t);
template void ts_gemm_nn<float, double>(const float*, int64_t, int, int64_t, const double*,
                                        int64_t, int, double*, int64_t, hipStream_t);

// ---------------------------------------------------------------------------
// T <- T Rinv (upper triangular b x b, column-major), optional row-major copy
// ---------------------------------------------------------------------------
template <int B>
__global__ __launch_bounds__(kThreads) void k_ts_scale(double* __restrict__ T, int64_t ldt,
                                                       int64_t N, const double* __restrict__ Rinv,
                                                       double* __restrict__ compact) {
  __shared__ double r[B * B];
  for (int a = threadIdx.x; a < B * B; a += kThreads) r[a] = Rinv[a];
  __syncthreads();
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    double t[B], o[B];
#pragma unroll
    for (int c = 0; c < B; ++c) t[c] = T[i + c * ldt];
#pragma unroll
    for (int c = 0; c < B; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j <= c; ++j) acc = fma(t[j], r[c * B + j], acc);
      o[c] = acc;
    }
#pragma unroll
    for (int c = 0; c < B; ++c) T[i + c * ldt] = o[c];
    if (compact) {
#pragma unroll
      for (int c = 0; c < B; ++c) compact[i * B + c] = o[c];
    }
  }
}

void ts_scale(double* T, int64_t ldt, int64_t N, int b, const double* Rinv, double* compact,
              hipStream_t s) {
  int nb = reduce_blocks(N);
  switch (b) {
#define CASE(BB) \
  case BB: k_ts_scale<BB><<<nb, kThreads, 0, s>>>(T, ldt, N, Rinv, compact); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw Error(SVDS_ERR_ARG, "ts_scale: b must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// fused residual: x = V y_c, r_c = W y_c - theta_c x  and the six sums per
// candidate  [||r_lo||^2, x_lo.r_lo, ||x_lo||^2, ||r_hi||^2, x_hi.r_hi, ||x_hi||^2]
// with lo = rows < nsplit (the v-half on B), hi = the rest (the u-half).
// One pass over V and W (the "special kernels" of Section 3.3).
// ---------------------------------------------------------------------------
template <int NCC, int NS, typename TB>
__global__ __launch_bounds__(kThreads) void k_residual(
    const TB* __restrict__ V, const TB* __restrict__ W, int64_t ld, int64_t N,
    int64_t nsplit, int g, const double* __restrict__ Y, int64_t ldy,
    const double* __restrict__ theta, int nc, double* __restrict__ R, int64_t ldr,
    double* __restrict__ partial) {
  __shared__ double ys[kMaxBasis * NCC];
  __shared__ double th[NCC];
  __shared__ double sh[4 * NS * NCC];
  const int c0 = blockIdx.y * NCC;
  const int ncc = min(NCC, nc - c0);
  for (int a = threadIdx.x; a < g * NCC; a += kThreads) {
    int j = a / NCC, c = a % NCC;
    ys[a] = (c < ncc) ? Y[(int64_t)(c0 + c) * ldy + j] : 0.0;
  }
  if (threadIdx.x < NCC) th[threadIdx.x] = (threadIdx.x < ncc) ? theta[c0 + threadIdx.x] : 0.0;
  __syncthreads();
  double acc[NS * NCC];
#pragma unroll
  for (int a = 0; a < NS * NCC; ++a) acc[a] = 0.0;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    double x[NCC], w[NCC];
#pragma unroll
    for (int c = 0; c < NCC; ++c) x[c] = w[c] = 0.0;
    // four basis columns per step, their loads issued together (the same
    // summation order as one column at a time)
    int j = 0;
    for (; j + 4 <= g; j += 4) {
      double v[4], ww[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        v[u] = (double)V[i + (int64_t)(j + u) * ld];
        ww[u] = (double)W[i + (int64_t)(j + u) * ld];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
#pragma unroll
        for (int c = 0; c < NCC; ++c) {
          x[c] = fma(v[u], ys[(j + u) * NCC + c], x[c]);
          w[c] = fma(ww[u], ys[(j + u) * NCC + c], w[c]);
        }
      }
    }
    for (; j < g; ++j) {
      const double v = (double)V[i + (int64_t)j * ld];
      const double ww = (double)W[i + (int64_t)j * ld];
#pragma unroll
      for (int c = 0; c < NCC; ++c) {
        x[c] = fma(v, ys[j * NCC + c], x[c]);
        w[c] = fma(ww, ys[j * NCC + c], w[c]);
      }
    }
    const bool lo = i < nsplit;
#pragma unroll
    for (int c = 0; c < NCC; ++c) {
      const double r = fma(-th[c], x[c], w[c]);
      if (c < ncc) R[i + (int64_t)(c0 + c) * ldr] = r;
      if constexpr (NS == 1) {
        acc[c] = fma(r, r, acc[c]);
      } else {
        double* a6 = acc + 6 * c;
        const double rr = r * r, xr = x[c] * r, xx = x[c] * x[c];
        if (lo) {
          a6[0] += rr; a6[1] += xr; a6[2] += xx;
        } else {
          a6[3] += rr; a6[4] += xr; a6[5] += xx;
        }
      }
    }
  }
  // partial layout: [q * nc + cand][block]
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int a = 0; a < NS * NCC; ++a) {
    double v = wave_sum(acc[a]);
    if (lane == 0) sh[w * NS * NCC + a] = v;
  }
  __syncthreads();
  for (int a = threadIdx.x; a < NS * NCC; a += kThreads) {
    const int c = a / NS, q = a % NS;
    if (c < ncc) {
      double v = ((sh[a] + sh[NS * NCC + a]) + sh[2 * NS * NCC + a]) + sh[3 * NS * NCC + a];
      partial[((int64_t)q * nc + c0 + c) * gridDim.x + blockIdx.x] = v;
    }
  }
}

// nsplit >= N: one sum per candidate (||r||^2 in sums[c]); otherwise the six
// sums of the two halves in sums[q*nc + c]
template <typename TB>
int ts_residual(const TB* V, const TB* W, int64_t ld, int64_t N, int64_t nsplit, int g,
                 const double* Y, int64_t ldy, const double* theta, int nc, double* R,
                 int64_t ldr, double* partial, double* sums, hipStream_t s) {
  if (g > kMaxBasis) throw Error(SVDS_ERR_ARG, "residual: basis too large");
  int nb = reduce_blocks(N);
  if (nsplit >= N) {
    constexpr int NCC = 16;
    dim3 grid(nb, (nc + NCC - 1) / NCC);
    k_residual<NCC, 1, TB><<<grid, kThreads, 0, s>>>(V, W, ld, N, nsplit, g, Y, ldy, theta, nc,
                                                      R, ldr, partial);
    SVDS_LAUNCH_CHECK();
    if (sums) reduce_partials(partial, nb, nc, sums, s);
  } else {
    constexpr int NCC = 8;
    dim3 grid(nb, (nc + NCC - 1) / NCC);
    k_residual<NCC, 6, TB><<<grid, kThreads, 0, s>>>(V, W, ld, N, nsplit, g, Y, ldy, theta, nc,
                                                      R, ldr, partial);
    SVDS_LAUNCH_CHECK();
    if (sums) reduce_partials(partial, nb, 6 * nc, sums, s);
  }
  return nb;
}
template int ts_residual<double>(const double*, const double*, int64_t, int64_t, int64_t, int,
                                  const double*, int64_t, const double*, int, double*, int64_t,
                                  double*, double*, hipStream_t);
template int ts_residual<float>(const float*, const float*, int64_t, int64_t, int64_t, int,
                                 const double*, int64_t, const double*, int, double*, int64_t,
                                 double*, double*, hipStream_t);

// ---------------------------------------------------------------------------
// small helpers: pack / unpack between column-major and row-major blocks,
// preconditioned gather, row scaling, column copies
// ---------------------------------------------------------------------------
// Conversions between column-major columns and row-major compact blocks (the
// operand layout of the sparse products).  The block width is a template
// argument so that each thread issues all of its row's loads before its
// stores, and a row's B values leave as one contiguous store sequence.
template <int B>
__global__ void k_pack(const double* __restrict__ A, int64_t lda, const double* __restrict__ Bm,
                       double beta, int64_t N, double* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride) {
    double v[B];
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = A[i + c * lda];
    if (Bm) {
#pragma unroll
      for (int c = 0; c < B; ++c) v[c] = fma(beta, Bm[i + c * lda], v[c]);
    }
#pragma unroll
    for (int c = 0; c < B; ++c) out[i * B + c] = v[c];
  }
}

template <int B>
__global__ void k_unpack(const double* __restrict__ in, int64_t N, double* __restrict__ A,
                         int64_t lda) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride) {
    double v[B];
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = in[i * B + c];
#pragma unroll
    for (int c = 0; c < B; ++c) A[i + c * lda] = v[c];
  }
}

#define SVDS_BLOCK_SWITCH(b, CALL)          \
  switch (b) {                              \
    case 1: CALL(1); break;                 \
    case 2: CALL(2); break;                 \
    case 3: CALL(3); break;                 \
    case 4: CALL(4); break;                 \
    case 5: CALL(5); break;                 \
    case 6: CALL(6); break;                 \
    case 7: CALL(7); break;                 \
    case 8: CALL(8); break;                 \
    default: throw Error(SVDS_ERR_ARG, "block width must be 1..8"); \
  }

void pack_rows(const double* A, int64_t lda, const double* B, double beta, int64_t N, int b,
               double* compact, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1) return;
#define SVDS_PACK(BB) k_pack<BB><<<blocks, 256, 0, s>>>(A, lda, B, beta, N, compact)
  SVDS_BLOCK_SWITCH(b, SVDS_PACK)
#undef SVDS_PACK
  SVDS_LAUNCH_CHECK();
}

void unpack_rows(const double* compact, int64_t N, int b, double* A, int64_t lda, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1) return;
#define SVDS_UNPACK(BB) k_unpack<BB><<<blocks, 256, 0, s>>>(compact, N, A, lda)
  SVDS_BLOCK_SWITCH(b, SVDS_UNPACK)
#undef SVDS_UNPACK
  SVDS_LAUNCH_CHECK();
}

// T[:, c] = R[:, blk[c]] * dinv for the block's nb columns (blk on the device,
// read once per workgroup into LDS)
template <int B>
__global__ void k_gather(const double* __restrict__ R, int64_t ldr, const int* __restrict__ blk,
                         const double* __restrict__ dinv, int64_t N, double* __restrict__ T,
                         int64_t ldt) {
  __shared__ int cols[B];
  if (threadIdx.x < B) cols[threadIdx.x] = blk[threadIdx.x];
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride) {
    const double d = dinv ? dinv[i] : 1.0;
    double v[B];
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = R[i + (int64_t)cols[c] * ldr];
#pragma unroll
    for (int c = 0; c < B; ++c) T[i + c * ldt] = v[c] * d;
  }
}

void gather_precond(const double* R, int64_t ldr, const int* d_blk, int nb, const double* dinv,
                    int64_t N, double* T, int64_t ldt, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1) return;
#define SVDS_GATHER(BB) k_gather<BB><<<blocks, 256, 0, s>>>(R, ldr, d_blk, dinv, N, T, ldt)
  SVDS_BLOCK_SWITCH(nb, SVDS_GATHER)
#undef SVDS_GATHER
  SVDS_LAUNCH_CHECK();
}

__global__ void k_scale_rows(double* __restrict__ T, int64_t ldt, int64_t N, int b,
                             const double* __restrict__ dinv) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride) {
    const double d = dinv[i];
    for (int c = 0; c < b; ++c) T[i + c * ldt] *= d;
  }
}

// out[i] = 1 / d[i], or 1 where d[i] is not positive (an empty column)
__global__ void k_invert_diag(const double* __restrict__ d, int64_t n, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double x = d[i];
    out[i] = x > 0.0 ? 1.0 / x : 1.0;
  }
}

void invert_diag(const double* d, int64_t n, double* out, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>(8192, (n + 255) / 256);
  if (blocks < 1) return;
  k_invert_diag<<<blocks, 256, 0, s>>>(d, n, out);
  SVDS_LAUNCH_CHECK();
}

void scale_rows(double* T, int64_t ldt, int64_t N, int b, const double* dinv, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1) return;
  k_scale_rows<<<blocks, 256, 0, s>>>(T, ldt, N, b, dinv);
  SVDS_LAUNCH_CHECK();
}

__global__ void k_copy_cols(const double* __restrict__ A, int64_t lda, int64_t N, int b,
                            double* __restrict__ Bm, int64_t ldb) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride)
    for (int c = 0; c < b; ++c) Bm[i + c * ldb] = A[i + c * lda];
}

template <typename TI, typename TO>
__global__ void k_copy_cols_cvt(const TI* __restrict__ A, int64_t lda, int64_t N, int b,
                                TO* __restrict__ Bm, int64_t ldb, TO* __restrict__ compact) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride)
    for (int c = 0; c < b; ++c) {
      const TO v = (TO)A[i + c * lda];
      if (Bm) Bm[i + c * ldb] = v;
      if (compact) compact[i * b + c] = v;
    }
}

template <typename TI, typename TO>
void copy_cols_cvt(const TI* A, int64_t lda, int64_t N, int b, TO* B, int64_t ldb, TO* compact,
                   hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1 || b < 1) return;
  k_copy_cols_cvt<TI, TO><<<blocks, 256, 0, s>>>(A, lda, N, b, B, ldb, compact);
  SVDS_LAUNCH_CHECK();
}
template void copy_cols_cvt<double, float>(const double*, int64_t, int64_t, int, float*, int64_t,
                                           float*, hipStream_t);
template void copy_cols_cvt<float, double>(const float*, int64_t, int64_t, int, double*, int64_t,
                                           double*, hipStream_t);
template void copy_cols_cvt<float, float>(const float*, int64_t, int64_t, int, float*, int64_t,
                                          float*, hipStream_t);

__global__ void k_unpack_f32(const float* __restrict__ in, int64_t N, int b, float* __restrict__ A,
                             int64_t lda) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride)
    for (int c = 0; c < b; ++c) A[i + c * lda] = in[i * b + c];
}

void unpack_rows_f32(const float* compact, int64_t N, int b, float* A, int64_t lda,
                     hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1) return;
  k_unpack_f32<<<blocks, 256, 0, s>>>(compact, N, b, A, lda);
  SVDS_LAUNCH_CHECK();
}

void copy_cols(const double* A, int64_t lda, int64_t N, int b, double* B, int64_t ldb,
               hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1 || b < 1) return;
  k_copy_cols<<<blocks, 256, 0, s>>>(A, lda, N, b, B, ldb);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds

namespace svds {

// ---------------------------------------------------------------------------
// per-column sums  out[c] = sum_i (A_ic - s_c B_ic)^2  (B may be null: norms)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_colres(const double* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ Bm, int64_t ldb,
                                                     const double* __restrict__ sc, int64_t N,
                                                     int k, double* __restrict__ partial) {
  __shared__ double sh[4];
  const int c = blockIdx.y;
  const double s = (Bm && sc) ? sc[c] : 0.0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    double v = A[i + c * lda];
    if (Bm) v = fma(-s, Bm[i + c * ldb], v);
    acc = fma(v, v, acc);
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[(int64_t)c * gridDim.x + blockIdx.x] = ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

void col_residual2(const double* A, int64_t lda, const double* B, int64_t ldb, const double* sc,
                   int64_t N, int k, double* partial, double* out, hipStream_t s) {
  if (k <= 0) return;
  int nb = reduce_blocks(N);
  dim3 grid(nb, k);
  k_colres<<<grid, kThreads, 0, s>>>(A, lda, B, ldb, sc, N, k, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nb, k, out, s);
}

__global__ void k_col_scale(double* __restrict__ X, int64_t ld, int64_t N, int k,
                            const double* __restrict__ f) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < N; i += stride)
    for (int c = 0; c < k; ++c) X[i + c * ld] *= f[c];
}

void col_scale(double* X, int64_t ld, int64_t N, int k, const double* f, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(8192, (N + 255) / 256);
  if (blocks < 1 || k < 1) return;
  k_col_scale<<<blocks, 256, 0, s>>>(X, ld, N, k, f);
  SVDS_LAUNCH_CHECK();
}

// per-column position of the largest |x| (first one on ties): partial pass
__global__ __launch_bounds__(kThreads) void k_colargmax(const double* __restrict__ X, int64_t ld,
                                                        int64_t N, int k,
                                                        double* __restrict__ pval,
                                                        int64_t* __restrict__ pidx) {
  __shared__ double sv[kThreads];
  __shared__ int64_t si[kThreads];
  const int c = blockIdx.y;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kThreads) {
    const double v = fabs(X[i + c * ld]);
    if (v > best) {  // rows visited in increasing order: keeps the first maximum
      best = v;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = kThreads / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      const double v2 = sv[threadIdx.x + off];
      const int64_t i2 = si[threadIdx.x + off];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    pval[(int64_t)blockIdx.x * k + c] = sv[0];
    pidx[(int64_t)blockIdx.x * k + c] = si[0];
  }
}

// flip (u_c, v_c) when the first largest-magnitude entry of v_c is negative;
// one wavefront per column c: lanes stride over the blocks' candidates, then
// the (largest value, smallest index) candidate wins across the lanes (a
// total order, so the winner does not depend on the reduction order)
__global__ __launch_bounds__(kWave) void k_sign_flip(const double* __restrict__ pval,
                                                     const int64_t* __restrict__ pidx, int nblk,
                                                     int k, const double* __restrict__ Vv,
                                                     int64_t ldv, double* __restrict__ f) {
  const int c = blockIdx.x;
  const int lane = threadIdx.x;
  double best = -1.0;
  int64_t bi = INT64_MAX;
  for (int b = lane; b < nblk; b += kWave) {
    const double v = pval[(int64_t)b * k + c];
    const int64_t i = pidx[(int64_t)b * k + c];
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    const double v = __shfl_xor(best, off, kWave);
    const int64_t i = __shfl_xor(bi, off, kWave);
    if (v > best || (v == best && i < bi)) {
      best = v;
      bi = i;
    }
  }
  if (lane == 0) f[c] = (bi != INT64_MAX && Vv[bi + c * ldv] < 0.0) ? -1.0 : 1.0;
}

void sign_factors(const double* V, int64_t ldv, int64_t N, int k, double* partial, double* f,
                  hipStream_t s) {
  int nb = reduce_blocks(N);
  double* pval = partial;
  int64_t* pidx = reinterpret_cast<int64_t*>(partial + (int64_t)nb * k);
  dim3 grid(nb, k);
  k_colargmax<<<grid, kThreads, 0, s>>>(V, ldv, N, k, pval, pidx);
  SVDS_LAUNCH_CHECK();
  k_sign_flip<<<k, kWave, 0, s>>>(pval, pidx, nb, k, V, ldv, f);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
