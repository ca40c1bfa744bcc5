// Tall-skinny dense kernels of one GD+k iteration (Section 3.3, Table 3:
// O((m+n) g) work per iteration, all of it HBM-bound).  Vectors are stored
// column-major (column j of an N x g basis at p + j*ld), so that every load of
// a wavefront is 64 consecutive doubles.  Reductions over the N rows are done
// in two fixed-order phases (per-workgroup partials, then a column reduction)
// so that results do not depend on scheduling.
#include <type_traits>

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
  const int w = threadIdx.x / kWave;
  wave_sums_to<NA>(acc, sh + w * NA);
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

template <typename TB>
struct TsgemmArgs {
  Segs3T<TB> segs;
  int total;
  int64_t N;
  const double* T;
  int64_t ldt, chunk;
  double* partial;
  const int* skip;
};

// workgroup (bx, by) of a launch with gx workgroup columns
template <int B, typename TB>
__device__ __forceinline__ void tsgemm_body(const TsgemmArgs<TB>& A, int bx, int by, int gx) {
  const Segs3T<TB>& segs = A.segs;
  const int total = A.total;
  const int64_t N = A.N, ldt = A.ldt, chunk = A.chunk;
  const double* __restrict__ T = A.T;
  double* __restrict__ partial = A.partial;
  if (A.skip && *A.skip) return;  // device-side decision: this pass is not needed (uniform)
  __shared__ double red[4][kCPW * B];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  const int g0 = by * 4;
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
  const int bid = xcd_block(bx, gx);
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
  wave_sums_to<kCPW * B>(acc, red[w]);
  __syncthreads();
  // partial layout: [c * total + col][block]
  if (active && sub == 0 && lane < kCPW * B) {
    const int jj = lane / B, c = lane % B;
    double v = red[w][lane];
    for (int q = 1; q < spl; ++q) v += red[grp + q * ncg][lane];
    if (c0 + jj < total)
      partial[((int64_t)c * total + c0 + jj) * gx + bx] = v;
  }
}

template <int B, typename TB>
__global__ __launch_bounds__(kThreads) void k_tsgemm_tn(TsgemmArgs<TB> a) {
  tsgemm_body<B, TB>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_tsgemm_tn_batch(const TsgemmArgs<double>* a,
                                                              BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  tsgemm_body<B, double>(a[q.p], q.x, q.y, q.gx);
}

// one wavefront per output: out[o] = sum over blocks of P[o * nblk + block]
struct ReduceArgs {
  const double* P;
  int nblk;
  double* out;
  const int* skip;
};

__device__ __forceinline__ void reduce_body(const ReduceArgs& A, int o) {
  if (A.skip && *A.skip) {  // the producing pass was skipped: its result is zero
    if (threadIdx.x == 0) A.out[o] = 0.0;
    return;
  }
  const double* p = A.P + (int64_t)o * A.nblk;
  double s = 0.0;
  for (int b = threadIdx.x; b < A.nblk; b += 64) s += p[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) A.out[o] = s;
}

__global__ __launch_bounds__(64) void k_reduce_partials(const double* __restrict__ P, int nblk,
                                                        double* __restrict__ out,
                                                        const int* __restrict__ skip) {
  reduce_body(ReduceArgs{P, nblk, out, skip}, blockIdx.x);
}

__global__ __launch_bounds__(64) void k_reduce_partials_batch(const ReduceArgs* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  reduce_body(a[q.p], q.x);
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

// launch geometry of the projection: one contiguous row range per workgroup
// column (several 256-row steps amortise the final wave reductions)
namespace {
// f(std::integral_constant<int, b>) for a block width b of 1..8
template <class F>
void block_switch(int b, F&& f) {
  switch (b) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    default: throw Error(SVDS_ERR_ARG, "block width must be 1..8");
  }
}
}  // namespace

static void tsgemm_geom(int64_t N, int total, int& nb, int64_t& chunk, int& gy) {
  nb = std::min(reduce_blocks(N), 256);
  chunk = (N + nb - 1) / nb;
  chunk = (chunk + kWave * kTU - 1) / (kWave * kTU) * (kWave * kTU);
  nb = (int)((N + chunk - 1) / chunk);
  if (nb >= 64 && nb % 8) {  // whole XCD rounds for the remap
    nb = (nb + 7) / 8 * 8;
  }
  gy = (total + 4 * kCPW - 1) / (4 * kCPW);
}

template <int B, typename TB>
static int tsgemm_b(const Segs3T<TB>& sg, int total, int64_t N, const double* T, int64_t ldt,
                    double* partial, double* C, hipStream_t s, const int* skip) {
  int nb = 0, gy = 0;
  int64_t chunk = 0;
  tsgemm_geom(N, total, nb, chunk, gy);
  dim3 grid(nb, gy);
  k_tsgemm_tn<B, TB><<<grid, kThreads, 0, s>>>(
      TsgemmArgs<TB>{sg, total, N, T, ldt, chunk, partial, skip});
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
template <typename TB>
struct UpdateArgs {
  Segs3T<TB> segs;
  int total;
  int64_t N;
  const double* C;
  int ldc;
  double* T;
  int64_t ldt;
  const int* skip;
  // optional: the second-pass test of classical Gram-Schmidt (Daniel, Gragg,
  // Kaufman and Stewart) on C, the first pass's coefficients with the
  // block's own Gram matrix in rows total..: after one pass against an
  // orthonormal basis a column whose norm fell by less than sqrt(2) is
  // orthogonal to working accuracy.  Workgroup 0 writes 1 when every column
  // passes (||c_j||^2 <= G_jj / 2), so that the second pass is skipped
  int* dgks_out;
};

template <int B, typename TB>
__device__ __forceinline__ void update_body(const UpdateArgs<TB>& A, int bx, int gx) {
  const Segs3T<TB>& segs = A.segs;
  const int total = A.total, ldc = A.ldc;
  const int64_t N = A.N, ldt = A.ldt;
  const double* __restrict__ C = A.C;
  double* __restrict__ T = A.T;
  if (A.skip && *A.skip) return;
  __shared__ double cs[kMaxSegCols * B];
  for (int a = threadIdx.x; a < total * B; a += kThreads) {
    int j = a / B, c = a % B;
    cs[a] = C[(int64_t)c * ldc + j];
  }
  __syncthreads();
  if (A.dgks_out && bx == 0 && threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    int need = 0;
    for (int c = 0; c < B; ++c) {
      double sq = 0.0;
      for (int j = lane; j < total; j += kWave) sq = fma(cs[j * B + c], cs[j * B + c], sq);
      sq = wave_sum(sq);
      const double g0 = C[(int64_t)c * ldc + total + c];
      if (!(sq <= 0.5 * g0)) need = 1;
    }
    if (lane == 0) *A.dgks_out = need ? 0 : 1;
  }
  const int bid = xcd_block(bx, gx);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gx * kThreads) {
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

template <int B, typename TB>
__global__ __launch_bounds__(kThreads) void k_ts_update(UpdateArgs<TB> a) {
  update_body<B, TB>(a, blockIdx.x, gridDim.x);
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_ts_update_batch(const UpdateArgs<double>* a,
                                                              BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  update_body<B, double>(a[q.p], q.x, q.gx);
}

template <typename TB>
void ts_update(const SegT<TB>* segs, int nseg, int64_t N, const double* C, int ldc, double* T,
               int64_t ldt, int b, hipStream_t s, const int* skip, int* dgks_out) {
  int total = 0;
  Segs3T<TB> sg = make_segs(segs, nseg, total);
  if (total == 0) return;
  if (total > kMaxSegCols) throw Error(SVDS_ERR_ARG, "update too wide");
  int nb = reduce_blocks(N);
  switch (b) {
#define CASE(BB) \
  case BB:                                                                           \
    k_ts_update<BB, TB><<<nb, kThreads, 0, s>>>(UpdateArgs<TB>{sg, total, N, C, ldc, T, ldt, skip, dgks_out}); \
    break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw Error(SVDS_ERR_ARG, "ts_update: b must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}
template void ts_update<double>(const SegT<double>*, int, int64_t, const double*, int, double*,
                                int64_t, int, hipStream_t, const int*, int*);
template void ts_update<float>(const SegT<float>*, int, int64_t, const double*, int, double*,
                               int64_t, int, hipStream_t, const int*, int*);

// ---------------------------------------------------------------------------
// Out = Q Y   (restart V <- V Y, W <- W Y, Q <- Q Q~, locking x = V y)
// ---------------------------------------------------------------------------
constexpr int kOC = 24;

template <typename TI, typename TO>
struct GemmArgs {
  const TI* Q;
  int64_t ldq;
  int nq;
  int64_t N;
  const double* Y;
  int64_t ldy;
  int nout;
  TO* Out;
  int64_t ldo;
};

template <typename TI, typename TO>
__device__ __forceinline__ void gemm_body(const GemmArgs<TI, TO>& A, int bx, int by, int gx) {
  const TI* __restrict__ Q = A.Q;
  const double* __restrict__ Y = A.Y;
  TO* __restrict__ Out = A.Out;
  const int64_t ldq = A.ldq, N = A.N, ldy = A.ldy, ldo = A.ldo;
  const int nq = A.nq, nout = A.nout;
  __shared__ double ys[kMaxBasis * kOC];
  const int o0 = by * kOC;
  const int no = min(kOC, nout - o0);
  for (int a = threadIdx.x; a < nq * kOC; a += kThreads) {
    int j = a / kOC, o = a % kOC;
    ys[a] = (o < no) ? Y[(int64_t)(o0 + o) * ldy + j] : 0.0;
  }
  __syncthreads();
  const int bid = xcd_block(bx, gx);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gx * kThreads) {
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
__global__ __launch_bounds__(kThreads) void k_gemm_nn(GemmArgs<TI, TO> a) {
  gemm_body<TI, TO>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

__global__ __launch_bounds__(kThreads) void k_gemm_nn_batch(const GemmArgs<double, double>* a,
                                                            BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  gemm_body<double, double>(a[q.p], q.x, q.y, q.gx);
}

template <typename TI, typename TO>
void ts_gemm_nn(const TI* Q, int64_t ldq, int nq, int64_t N, const double* Y, int64_t ldy,
                int nout, TO* Out, int64_t ldo, hipStream_t s) {
  if (nout <= 0 || N == 0) return;
  if (nq > kMaxBasis) throw Error(SVDS_ERR_ARG, "gemm: inner dimension too large");
  dim3 grid(reduce_blocks(N), (nout + kOC - 1) / kOC);
  k_gemm_nn<TI, TO><<<grid, kThreads, 0, s>>>(
      GemmArgs<TI, TO>{Q, ldq, nq, N, Y, ldy, nout, Out, ldo});
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
struct ScaleArgs {
  double* T;
  int64_t ldt, N;
  const double* Rinv;
  double* compact;
};

template <int B>
__device__ __forceinline__ void scale_body(const ScaleArgs& A, int bx, int gx) {
  double* __restrict__ T = A.T;
  const int64_t ldt = A.ldt, N = A.N;
  const double* __restrict__ Rinv = A.Rinv;
  double* __restrict__ compact = A.compact;
  __shared__ double r[B * B];
  for (int a = threadIdx.x; a < B * B; a += kThreads) r[a] = Rinv[a];
  __syncthreads();
  const int bid = xcd_block(bx, gx);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gx * kThreads) {
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

template <int B>
__global__ __launch_bounds__(kThreads) void k_ts_scale(ScaleArgs a) {
  scale_body<B>(a, blockIdx.x, gridDim.x);
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_ts_scale_batch(const ScaleArgs* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  scale_body<B>(a[q.p], q.x, q.gx);
}

void ts_scale(double* T, int64_t ldt, int64_t N, int b, const double* Rinv, double* compact,
              hipStream_t s) {
  int nb = reduce_blocks(N);
  switch (b) {
#define CASE(BB) \
  case BB: k_ts_scale<BB><<<nb, kThreads, 0, s>>>(ScaleArgs{T, ldt, N, Rinv, compact}); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw Error(SVDS_ERR_ARG, "ts_scale: b must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// One Cholesky QR step on a block T (N x b): the Gram matrix G = T^T T from
// the partial sums of the preceding pass, its Cholesky factor R and R^-1
// (with the breakdown tests of the orthogonalisation), then T <- T R^-1 and,
// for the next step, the partial sums of the new T's Gram matrix.  Every
// workgroup sums the partials and factors G itself, in the same order, so
// all of them scale with the same R^-1 and no workgroup waits for another;
// workgroup 0 stores R, R^-1 and the breakdown record.  The partial sums are
// few (one b x b matrix per row chunk of the producing pass), so the
// repeated reads stay in L2.
// ---------------------------------------------------------------------------
struct CholQRArgs {
  const double* P;   // Gram partial sums of T: P[o * nblk + k], o = c * b + c2
  int nblk;
  int which;         // 1: first factor (collapse test, starts the record); 2: second
  const double* G0;  // which == 1: squared pre-projection norms at G0[j * ldg0 + j]
  int ldg0;
  double* R;         // b x b factor and its inverse, column-major
  double* Rinv;
  int* bad;          // breakdown record: bit j set when column j broke down
  double* T;
  int64_t ldt, N, chunk;
  double* compact;   // optional row-major copy of the result
  double* Pout;      // optional: Gram partial sums of the result, Pout[o * gx + bx]
};

template <int B>
constexpr int cholqr_unroll() { return B <= 4 ? 8 : 4; }  // 64-row groups loaded together

template <int B>
__device__ __forceinline__ void cholqr_body(const CholQRArgs& A, int bx, int gx) {
  constexpr int NE = B * B;
  constexpr int TPE = (kThreads / NE) >= 64 ? 64 : (kThreads / NE) >= 16 ? 16
                    : (kThreads / NE) >= 4 ? 4 : 1;  // threads per Gram entry
  constexpr int U = cholqr_unroll<B>();
  constexpr int NG = B * (B + 1) / 2;
  __shared__ double part[NE * TPE];
  __shared__ double G[NE], R[NE], Ri[NE], g0[B];
  __shared__ double red[4][NG > 0 ? NG : 1];
  __shared__ int sbad;
  const int t = threadIdx.x;
  // this wavefront's first U row groups are loaded before anything else, so
  // that their latency passes while the factor is formed
  double* __restrict__ T = A.T;
  double* __restrict__ compact = A.compact;
  const int64_t ldt = A.ldt, N = A.N;
  const int lane = t % kWave, w = t / kWave;
  const int bid = xcd_block(bx, gx);
  const int64_t rb = (int64_t)bid * A.chunk;
  const int64_t re = (rb + A.chunk < N) ? rb + A.chunk : N;
  int64_t base = rb + (int64_t)w * kWave * U;
  double tv[U][B];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t row = base + u * kWave + lane;
#pragma unroll
    for (int c = 0; c < B; ++c) tv[u][c] = (row < re) ? T[row + c * ldt] : 0.0;
  }
  // the Gram matrix: TPE threads per entry, each a strided share of the
  // partials, then the shares added in order
  if (t < NE * TPE) {
    const int o = t / TPE, sub = t % TPE;
    const double* p = A.P + (int64_t)o * A.nblk;
    double acc = 0.0;
#pragma unroll 8
    for (int k = sub; k < A.nblk; k += TPE) acc += p[k];
    part[t] = acc;
  }
  if (t < B) g0[t] = (A.which == 1) ? A.G0[(int64_t)t * A.ldg0 + t] : 0.0;
  __syncthreads();
  if (t < NE) {
    double acc = 0.0;
    for (int q = 0; q < TPE; ++q) acc += part[t * TPE + q];
    G[t] = acc;
    R[t] = 0.0;
    Ri[t] = 0.0;
  }
  __syncthreads();
  if (t == 0) {
    int bad = 0;
    for (int j = 0; j < B; ++j) {
      const double gjj = G[j * B + j];
      const double dj = sqrt(fmax(gjj, 0.0));
      double sres = gjj;
      for (int i = 0; i < j; ++i) sres -= R[j * B + i] * R[j * B + i];
      bool ok = (sres > (kBreakRatio * dj) * (kBreakRatio * dj)) && dj > 0.0;
      if (A.which == 1 && ok) ok = (gjj > (kCollapse * kCollapse) * g0[j]) && g0[j] > 0.0;
      if (!ok) {
        bad |= 1 << j;
        R[j * B + j] = 1.0;  // keep the factor finite; the block is redone
        continue;
      }
      const double rjj = sqrt(sres);
      R[j * B + j] = rjj;
      for (int c = j + 1; c < B; ++c) {
        double v = 0.5 * (G[c * B + j] + G[j * B + c]);
        for (int i = 0; i < j; ++i) v -= R[j * B + i] * R[c * B + i];
        R[c * B + j] = v / rjj;  // column-major: R(j, c) at c*B + j
      }
    }
    for (int c = 0; c < B; ++c) {  // inverse of the upper triangular factor
      Ri[c * B + c] = 1.0 / R[c * B + c];
      for (int i = c - 1; i >= 0; --i) {
        double v = 0.0;
        for (int j = i + 1; j <= c; ++j) v += R[j * B + i] * Ri[c * B + j];
        Ri[c * B + i] = -v / R[i * B + i];
      }
    }
    sbad = bad;
  }
  __syncthreads();
  if (bx == 0) {
    if (t < NE) {
      A.R[t] = R[t];
      A.Rinv[t] = Ri[t];
    }
    // the first factor of a block starts the breakdown record, the second adds to it
    if (t == 0) {
      if (A.which == 1) *A.bad = sbad;
      else if (sbad) *A.bad |= sbad;
    }
  }
  // T <- T R^-1 over this workgroup's row chunk, U row groups per wavefront in flight
  double g[NG];
#pragma unroll
  for (int a = 0; a < NG; ++a) g[a] = 0.0;
  while (base < re) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = base + u * kWave + lane;
      double o[B];
#pragma unroll
      for (int c = 0; c < B; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j <= c; ++j) acc = fma(tv[u][j], Ri[c * B + j], acc);
        o[c] = acc;
      }
      if (row < re) {
#pragma unroll
        for (int c = 0; c < B; ++c) T[row + c * ldt] = o[c];
        if (compact) {
#pragma unroll
          for (int c = 0; c < B; ++c) compact[row * B + c] = o[c];
        }
      }
      if (A.Pout) {  // rows past the end hold zeros and add nothing
        int a = 0;
#pragma unroll
        for (int c = 0; c < B; ++c)
#pragma unroll
          for (int c2 = c; c2 < B; ++c2) {
            g[a] = fma(o[c], o[c2], g[a]);
            ++a;
          }
      }
    }
    base += (int64_t)4 * kWave * U;
    if (base >= re) break;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = base + u * kWave + lane;
#pragma unroll
      for (int c = 0; c < B; ++c) tv[u][c] = (row < re) ? T[row + c * ldt] : 0.0;
    }
  }
  if (!A.Pout) return;
  wave_sums_to<NG>(g, red[w]);
  __syncthreads();
  if (t < NG) {
    int c = 0, c2 = 0, a = 0;
    for (int i = 0; i < B; ++i)
      for (int j = i; j < B; ++j, ++a)
        if (a == t) {
          c = i;
          c2 = j;
        }
    const double v = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    A.Pout[(int64_t)(c * B + c2) * gx + bx] = v;
    A.Pout[(int64_t)(c2 * B + c) * gx + bx] = v;
  }
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_cholqr(CholQRArgs a) {
  cholqr_body<B>(a, blockIdx.x, gridDim.x);
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_cholqr_batch(const CholQRArgs* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  cholqr_body<B>(a[q.p], q.x, q.gx);
}

// the row chunks of a Cholesky QR step on N rows (also the number of partial
// sums it leaves for the next step)
static void cholqr_geom(int64_t N, int b, int& nb, int64_t& chunk) {
  int gy = 0;
  tsgemm_geom(N, b, nb, chunk, gy);
}

int cholqr_step(const double* P, int nblk, int which, const double* G0, int ldg0, double* R,
                double* Rinv, int* bad, double* T, int64_t ldt, int64_t N, int b,
                double* compact, double* Pout, hipStream_t s) {
  int nb = 0;
  int64_t chunk = 0;
  cholqr_geom(N, b, nb, chunk);
  const CholQRArgs a{P, nblk, which, G0, ldg0, R, Rinv, bad, T, ldt, N, chunk, compact, Pout};
  block_switch(b, [&](auto B) { k_cholqr<decltype(B)::value><<<nb, kThreads, 0, s>>>(a); });
  SVDS_LAUNCH_CHECK();
  return nb;
}

// ---------------------------------------------------------------------------
// fused residual: x = V y_c, r_c = W y_c - theta_c x  and the six sums per
// candidate  [||r_lo||^2, x_lo.r_lo, ||x_lo||^2, ||r_hi||^2, x_hi.r_hi, ||x_hi||^2]
// with lo = rows < nsplit (the v-half on B), hi = the rest (the u-half).
// One pass over V and W (the "special kernels" of Section 3.3).
// ---------------------------------------------------------------------------
template <typename TB>
struct ResidArgs {
  const TB* V;
  const TB* W;
  int64_t ld, N, nsplit;
  int g;
  const double* Y;
  int64_t ldy;
  const double* theta;
  int nc;
  double* R;
  int64_t ldr;
  double* partial;
};

template <int NCC, int NS, typename TB>
__device__ __forceinline__ void resid_body(const ResidArgs<TB>& A, int bx, int by, int gx) {
  const TB* __restrict__ V = A.V;
  const TB* __restrict__ W = A.W;
  const int64_t ld = A.ld, N = A.N, nsplit = A.nsplit, ldy = A.ldy, ldr = A.ldr;
  const int g = A.g, nc = A.nc;
  const double* __restrict__ Y = A.Y;
  const double* __restrict__ theta = A.theta;
  double* __restrict__ R = A.R;
  double* __restrict__ partial = A.partial;
  __shared__ double ys[kMaxBasis * NCC];
  __shared__ double th[NCC];
  __shared__ double sh[4 * NS * NCC];
  const int c0 = by * NCC;
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
  const int bid = xcd_block(bx, gx);
  for (int64_t i = (int64_t)bid * kThreads + threadIdx.x; i < N;
       i += (int64_t)gx * kThreads) {
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
  const int w = threadIdx.x / kWave;
  wave_sums_to<NS * NCC>(acc, sh + w * NS * NCC);
  __syncthreads();
  for (int a = threadIdx.x; a < NS * NCC; a += kThreads) {
    const int c = a / NS, q = a % NS;
    if (c < ncc) {
      double v = ((sh[a] + sh[NS * NCC + a]) + sh[2 * NS * NCC + a]) + sh[3 * NS * NCC + a];
      partial[((int64_t)q * nc + c0 + c) * gx + bx] = v;
    }
  }
}

template <int NCC, int NS, typename TB>
__global__ __launch_bounds__(kThreads) void k_residual(ResidArgs<TB> a) {
  resid_body<NCC, NS, TB>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

__global__ __launch_bounds__(kThreads) void k_residual_batch(const ResidArgs<double>* a,
                                                             BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  resid_body<16, 1, double>(a[q.p], q.x, q.y, q.gx);
}

// workgroups of a residual launch on N rows: at most 512 (each thread then
// takes several rows), so that the norm sums leave few partial sums
static int resid_blocks(int64_t N) { return std::min(reduce_blocks(N), 512); }

// nsplit >= N: one sum per candidate (||r||^2 in sums[c]); otherwise the six
// sums of the two halves in sums[q*nc + c]
template <typename TB>
int ts_residual(const TB* V, const TB* W, int64_t ld, int64_t N, int64_t nsplit, int g,
                 const double* Y, int64_t ldy, const double* theta, int nc, double* R,
                 int64_t ldr, double* partial, double* sums, hipStream_t s) {
  if (g > kMaxBasis) throw Error(SVDS_ERR_ARG, "residual: basis too large");
  const int nb = resid_blocks(N);
  if (nsplit >= N) {
    constexpr int NCC = 16;
    dim3 grid(nb, (nc + NCC - 1) / NCC);
    k_residual<NCC, 1, TB><<<grid, kThreads, 0, s>>>(
        ResidArgs<TB>{V, W, ld, N, nsplit, g, Y, ldy, theta, nc, R, ldr, partial});
    SVDS_LAUNCH_CHECK();
    if (sums) reduce_partials(partial, nb, nc, sums, s);
  } else {
    constexpr int NCC = 8;
    dim3 grid(nb, (nc + NCC - 1) / NCC);
    k_residual<NCC, 6, TB><<<grid, kThreads, 0, s>>>(
        ResidArgs<TB>{V, W, ld, N, nsplit, g, Y, ldy, theta, nc, R, ldr, partial});
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
// operand layout of the sparse products).  A workgroup moves tiles of 256
// rows through LDS, so that both the column-major side (one row per lane)
// and the row-major side (256 x B consecutive values, one per lane and
// step) are read and written in whole wavefront-wide runs.
constexpr int kPackRows = 256;  // rows per tile (the workgroup size)

template <int B>
__global__ __launch_bounds__(kPackRows) void k_pack(const double* __restrict__ A, int64_t lda,
                                                    const double* __restrict__ Bm, double beta,
                                                    int64_t N, double* __restrict__ out) {
  __shared__ double tile[kPackRows * (B + 1)];  // row stride B + 1 against bank conflicts
  const int t = threadIdx.x;
  for (int64_t r0 = (int64_t)blockIdx.x * kPackRows; r0 < N; r0 += (int64_t)gridDim.x * kPackRows) {
    const int nr = (int)((N - r0 < kPackRows) ? N - r0 : kPackRows);
    const int64_t i = r0 + t;
    if (t < nr) {
      double v[B];
#pragma unroll
      for (int c = 0; c < B; ++c) v[c] = A[i + c * lda];
      if (Bm) {
#pragma unroll
        for (int c = 0; c < B; ++c) v[c] = fma(beta, Bm[i + c * lda], v[c]);
      }
#pragma unroll
      for (int c = 0; c < B; ++c) tile[t * (B + 1) + c] = v[c];
    }
    __syncthreads();
    double* __restrict__ o = out + r0 * B;
    for (int k = t; k < nr * B; k += kPackRows) o[k] = tile[(k / B) * (B + 1) + k % B];
    __syncthreads();
  }
}

struct UnpackArgs {
  const double* in;
  int64_t N;
  double* A;
  int64_t lda;
};

template <int B>
__device__ __forceinline__ void unpack_body(const UnpackArgs& a, int bx, int gx) {
  const double* __restrict__ in = a.in;
  double* __restrict__ A = a.A;
  const int64_t N = a.N, lda = a.lda;
  __shared__ double tile[kPackRows * (B + 1)];  // row stride B + 1 against bank conflicts
  const int t = threadIdx.x;
  for (int64_t r0 = (int64_t)bx * kPackRows; r0 < N; r0 += (int64_t)gx * kPackRows) {
    const int nr = (int)((N - r0 < kPackRows) ? N - r0 : kPackRows);
    const double* __restrict__ src = in + r0 * B;
    for (int k = t; k < nr * B; k += kPackRows) tile[(k / B) * (B + 1) + k % B] = src[k];
    __syncthreads();
    if (t < nr) {
#pragma unroll
      for (int c = 0; c < B; ++c) A[r0 + t + c * lda] = tile[t * (B + 1) + c];
    }
    __syncthreads();
  }
}

template <int B>
__global__ __launch_bounds__(kPackRows) void k_unpack(const double* __restrict__ in, int64_t N,
                                                      double* __restrict__ A, int64_t lda) {
  unpack_body<B>(UnpackArgs{in, N, A, lda}, blockIdx.x, gridDim.x);
}

template <int B>
__global__ __launch_bounds__(kPackRows) void k_unpack_batch(const UnpackArgs* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  unpack_body<B>(a[q.p], q.x, q.gx);
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
struct GatherArgs {
  const double* R;
  int64_t ldr;
  const int* blk;
  const double* dinv;
  int64_t N;
  double* T;
  int64_t ldt;
};

template <int B>
__device__ __forceinline__ void gather_body(const GatherArgs& a, int bx, int gx) {
  const double* __restrict__ R = a.R;
  const double* __restrict__ dinv = a.dinv;
  double* __restrict__ T = a.T;
  const int64_t ldr = a.ldr, N = a.N, ldt = a.ldt;
  __shared__ int cols[B];
  if (threadIdx.x < B) cols[threadIdx.x] = a.blk[threadIdx.x];
  __syncthreads();
  int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gx * blockDim.x;
  for (; i < N; i += stride) {
    const double d = dinv ? dinv[i] : 1.0;
    double v[B];
#pragma unroll
    for (int c = 0; c < B; ++c) v[c] = R[i + (int64_t)cols[c] * ldr];
#pragma unroll
    for (int c = 0; c < B; ++c) T[i + c * ldt] = v[c] * d;
  }
}

template <int B>
__global__ void k_gather(const double* __restrict__ R, int64_t ldr, const int* __restrict__ blk,
                         const double* __restrict__ dinv, int64_t N, double* __restrict__ T,
                         int64_t ldt) {
  gather_body<B>(GatherArgs{R, ldr, blk, dinv, N, T, ldt}, blockIdx.x, gridDim.x);
}

template <int B>
__global__ void k_gather_batch(const GatherArgs* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  gather_body<B>(a[q.p], q.x, q.gx);
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

// ===========================================================================
// batched steps
// ===========================================================================
namespace svds {

void tsgemm_tn_batch(int b, const std::vector<BatchProj>& jobs, std::vector<int>& nblk,
                     BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  nblk.assign(np, 0);
  if (np == 0) return;
  std::vector<TsgemmArgs<double>> args(np);
  std::vector<int> gx(np), gy(np);
  std::vector<BatchReduce> red;
  for (int j = 0; j < np; ++j) {
    const BatchProj& q = jobs[j];
    int total = 0;
    Segs3T<double> sg = make_segs(q.segs, q.nseg, total);
    if (total > kMaxSegCols) throw Error(SVDS_ERR_ARG, "projection too wide");
    int nb = 0, g2 = 0;
    int64_t chunk = 0;
    if (total > 0) tsgemm_geom(q.N, total, nb, chunk, g2);
    args[j] = TsgemmArgs<double>{sg, total, q.N, q.T, q.ldt, chunk, q.partial, q.skip};
    gx[j] = nb;
    gy[j] = total > 0 ? g2 : 0;
    nblk[j] = nb;
    if (q.C && total > 0) red.push_back(BatchReduce{q.partial, nb, total * b, q.C, q.skip});
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const TsgemmArgs<double>* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(b, [&](auto B) {
      k_tsgemm_tn_batch<decltype(B)::value><<<tiles, kThreads, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
  if (!red.empty()) reduce_partials_batch(red, up, s);
}

void reduce_partials_batch(const std::vector<BatchReduce>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<ReduceArgs> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    args[j] = ReduceArgs{jobs[j].P, jobs[j].nblk, jobs[j].out, jobs[j].skip};
    gx[j] = jobs[j].nout;
    if (jobs[j].nout <= 0) gy[j] = 0;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const ReduceArgs* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0) k_reduce_partials_batch<<<tiles, 64, 0, s>>>(d, t);
  SVDS_LAUNCH_CHECK();
}

void ts_update_batch(int b, const std::vector<BatchUpdate>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<UpdateArgs<double>> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const BatchUpdate& q = jobs[j];
    int total = 0;
    Segs3T<double> sg = make_segs(q.segs, q.nseg, total);
    if (total > kMaxSegCols) throw Error(SVDS_ERR_ARG, "update too wide");
    args[j] = UpdateArgs<double>{sg, total, q.N, q.C, q.ldc, q.T, q.ldt, q.skip, q.dgks_out};
    gx[j] = reduce_blocks(q.N);
    if (total == 0) gy[j] = 0;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const UpdateArgs<double>* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(b, [&](auto B) {
      k_ts_update_batch<decltype(B)::value><<<tiles, kThreads, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
}

void ts_gemm_nn_batch(const std::vector<BatchGemm>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<GemmArgs<double, double>> args(np);
  std::vector<int> gx(np), gy(np);
  for (int j = 0; j < np; ++j) {
    const BatchGemm& q = jobs[j];
    if (q.nq > kMaxBasis) throw Error(SVDS_ERR_ARG, "gemm: inner dimension too large");
    args[j] = GemmArgs<double, double>{q.Q, q.ldq, q.nq, q.N, q.Y, q.ldy, q.nout, q.Out, q.ldo};
    gx[j] = reduce_blocks(q.N);
    gy[j] = (q.nout <= 0 || q.N == 0) ? 0 : (q.nout + kOC - 1) / kOC;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const GemmArgs<double, double>* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0) k_gemm_nn_batch<<<tiles, kThreads, 0, s>>>(d, t);
  SVDS_LAUNCH_CHECK();
}

void cholqr_batch(int b, const std::vector<BatchCholQR>& jobs, std::vector<int>& nblk,
                  BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  nblk.assign(np, 0);
  if (np == 0) return;
  std::vector<CholQRArgs> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const BatchCholQR& q = jobs[j];
    int nb = 0;
    int64_t chunk = 0;
    cholqr_geom(q.N, b, nb, chunk);
    args[j] = CholQRArgs{q.P, q.nblk, q.which, q.G0, q.ldg0, q.R, q.Rinv, q.bad,
                         q.T, q.ldt, q.N, chunk, q.compact, q.Pout};
    gx[j] = nb;
    nblk[j] = nb;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const CholQRArgs* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(b, [&](auto B) {
      k_cholqr_batch<decltype(B)::value><<<tiles, kThreads, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
}

void ts_scale_batch(int b, const std::vector<BatchScale>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<ScaleArgs> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const BatchScale& q = jobs[j];
    args[j] = ScaleArgs{q.T, q.ldt, q.N, q.Rinv, q.compact};
    gx[j] = reduce_blocks(q.N);
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const ScaleArgs* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(b, [&](auto B) {
      k_ts_scale_batch<decltype(B)::value><<<tiles, kThreads, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
}

void ts_residual_batch(const std::vector<BatchResid>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  constexpr int NCC = 16;
  std::vector<ResidArgs<double>> args(np);
  std::vector<int> gx(np), gy(np);
  std::vector<BatchReduce> red;
  for (int j = 0; j < np; ++j) {
    const BatchResid& q = jobs[j];
    if (q.g > kMaxBasis) throw Error(SVDS_ERR_ARG, "residual: basis too large");
    args[j] = ResidArgs<double>{q.V, q.W, q.ld, q.N, q.N, q.g, q.Y, q.ldy, q.theta, q.nc,
                                q.R, q.ldr, q.partial};
    gx[j] = resid_blocks(q.N);
    gy[j] = (q.nc + NCC - 1) / NCC;
    if (q.sums) red.push_back(BatchReduce{q.partial, gx[j], q.nc, q.sums, nullptr});
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const ResidArgs<double>* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0) k_residual_batch<<<tiles, kThreads, 0, s>>>(d, t);
  SVDS_LAUNCH_CHECK();
  if (!red.empty()) reduce_partials_batch(red, up, s);
}

void gather_batch(int nb, const std::vector<BatchGather>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<GatherArgs> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const BatchGather& q = jobs[j];
    args[j] = GatherArgs{q.R, q.ldr, q.blk, q.dinv, q.N, q.T, q.ldt};
    gx[j] = (int)std::min<int64_t>(8192, (q.N + 255) / 256);
    if (gx[j] < 1) gy[j] = 0;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const GatherArgs* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(nb, [&](auto B) {
      k_gather_batch<decltype(B)::value><<<tiles, 256, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
}

void unpack_batch(int nb, const std::vector<BatchUnpack>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  std::vector<UnpackArgs> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const BatchUnpack& q = jobs[j];
    args[j] = UnpackArgs{q.compact, q.N, q.A, q.lda};
    gx[j] = (int)std::min<int64_t>(8192, (q.N + 255) / 256);
    if (gx[j] < 1) gy[j] = 0;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const UnpackArgs* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0)
    block_switch(nb, [&](auto B) {
      k_unpack_batch<decltype(B)::value><<<tiles, 256, 0, s>>>(d, t);
    });
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
