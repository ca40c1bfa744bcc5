// Block CSR SpMM Y = A X for the products with A and A^T of Section 3.3
// (the user matrixMatvec of Section 3.4, here on the device).
//
// Rows are grouped into bins by length; each bin runs a kernel in which a
// group of L lanes (L = 1 ... 64, or a whole workgroup for very long rows)
// shares one row, each lane striding over the row's nonzeros (U at a time)
// and accumulating all b columns of the row-major block X (one contiguous
// b-wide gather per nonzero), followed by a shuffle reduction inside the
// group.  Alternatively one launch covers all rows in natural order with one
// lane shape (chosen by the autotuner or by the row-length rule).
// Every row is summed by one group in a fixed order: no atomics, results are
// bitwise reproducible.
#include "common.h"

namespace svds {

// sum over the L lanes of a group (L <= 64, a power of two); every lane of
// the group ends with the total
template <typename TV, int L>
__device__ __forceinline__ TV group_total(TV v) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// L lanes per row; each lane takes U of the row's nonzeros per step (lane
// offsets l, l+L, ..., l+(U-1)L).  The index and value loads of a step are
// issued together and without branches (positions past the row end read the
// row's last entry and are masked), then the U gathered rows of X, then the
// multiply-adds, so that U loads per lane are in flight.  The row bounds of
// the group's next row are loaded before the current row is processed.
// The summation order inside a lane is the same for every U, so the result
// depends on L only.  After the shuffle reduction lanes 0..B-1 of the group
// store the row's B outputs side by side (one coalesced store).
template <typename TV, int B, int L, int U>
__global__ __launch_bounds__(256) void k_spmm_group(const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const TV* __restrict__ val,
                                                    const int32_t* __restrict__ rows,
                                                    int64_t nrows, const TV* __restrict__ X,
                                                    TV* __restrict__ Y) {
  constexpr int RPB = 256 / L;
  const int grp = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  const int bid = xcd_block(blockIdx.x, gridDim.x);
  const int64_t stride = (int64_t)gridDim.x * RPB;
  int64_t slot = (int64_t)bid * RPB + grp;
  int32_t row = 0, a = 0, e = 0;
  if (slot < nrows) {
    row = rows ? rows[slot] : (int32_t)slot;
    a = rp[row];
    e = rp[row + 1];
  }
  while (slot < nrows) {
    // bounds of the next row first
    const int64_t nslot = slot + stride;
    int32_t nrow = 0, na = 0, ne = 0;
    if (nslot < nrows) {
      nrow = rows ? rows[nslot] : (int32_t)nslot;
      na = rp[nrow];
      ne = rp[nrow + 1];
    }
    TV acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = TV(0);
    for (int32_t k0 = a + lane; k0 < e; k0 += L * U) {
      int32_t c[U];
      TV v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * L;
        const int32_t kk = k < e ? k : e - 1;
        c[u] = ci[kk];
        v[u] = val[kk];
      }
      TV x[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const TV* __restrict__ xr = X + (int64_t)c[u] * B;
#pragma unroll
        for (int j = 0; j < B; ++j) x[u][j] = xr[j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = k0 + u * L < e;
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const TV t = fma(v[u], x[u][j], acc[j]);
          acc[j] = in ? t : acc[j];
        }
      }
    }
    if constexpr (L > 1) {
#pragma unroll
      for (int j = 0; j < B; ++j) acc[j] = group_total<TV, L>(acc[j]);
    }
    TV* __restrict__ y = Y + (int64_t)row * B;
    if constexpr (L >= B) {
      TV out = acc[0];
#pragma unroll
      for (int j = 1; j < B; ++j)
        if (lane == j) out = acc[j];
      if (lane < B) y[lane] = out;
    } else {
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) y[j] = acc[j];
      }
    }
    slot = nslot;
    row = nrow;
    a = na;
    e = ne;
  }
}

// Natural row order (one launch over all rows): the workgroup's RPB
// consecutive rows have consecutive row pointers, which it stages in LDS with
// one coalesced load per step; each group then starts on its row's nonzeros
// at once instead of waiting for its own row-pointer loads.  Same lane
// arithmetic and summation order as k_spmm_group.
template <typename TV>
struct NatArgs {
  const int32_t* rp;
  const int32_t* ci;
  const TV* val;
  int64_t nrows;
  const TV* X;
  TV* Y;
};

template <typename TV, int B, int L, int U>
__device__ __forceinline__ void nat_body(const NatArgs<TV>& A, int bx, int gx) {
  const int32_t* __restrict__ rp = A.rp;
  const int32_t* __restrict__ ci = A.ci;
  const TV* __restrict__ val = A.val;
  const TV* __restrict__ X = A.X;
  TV* __restrict__ Y = A.Y;
  const int64_t nrows = A.nrows;
  constexpr int RPB = 256 / L;
  __shared__ int32_t rps[RPB + 1];
  const int grp = threadIdx.x / L;
  const int lane = threadIdx.x % L;
  const int bid = xcd_block(bx, gx);
  const int64_t stride = (int64_t)gx * RPB;
  for (int64_t s0 = (int64_t)bid * RPB; s0 < nrows; s0 += stride) {
    __syncthreads();
    for (int t = threadIdx.x; t <= RPB; t += 256) {
      const int64_t r = s0 + t;
      rps[t] = rp[r < nrows ? r : nrows];
    }
    __syncthreads();
    const int64_t row = s0 + grp;
    if (row >= nrows) continue;
    const int32_t a = rps[grp], e = rps[grp + 1];
    TV acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = TV(0);
    for (int32_t k0 = a + lane; k0 < e; k0 += L * U) {
      int32_t c[U];
      TV v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * L;
        const int32_t kk = k < e ? k : e - 1;
        c[u] = ci[kk];
        v[u] = val[kk];
      }
      TV x[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const TV* __restrict__ xr = X + (int64_t)c[u] * B;
#pragma unroll
        for (int j = 0; j < B; ++j) x[u][j] = xr[j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = k0 + u * L < e;
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const TV t = fma(v[u], x[u][j], acc[j]);
          acc[j] = in ? t : acc[j];
        }
      }
    }
    if constexpr (L > 1) {
#pragma unroll
      for (int j = 0; j < B; ++j) acc[j] = group_total<TV, L>(acc[j]);
    }
    TV* __restrict__ y = Y + row * B;
    if constexpr (L >= B) {
      TV out = acc[0];
#pragma unroll
      for (int j = 1; j < B; ++j)
        if (lane == j) out = acc[j];
      if (lane < B) y[lane] = out;
    } else {
      if (lane == 0) {
#pragma unroll
        for (int j = 0; j < B; ++j) y[j] = acc[j];
      }
    }
  }
}

template <typename TV, int B, int L, int U>
__global__ __launch_bounds__(256) void k_spmm_nat(const int32_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const TV* __restrict__ val, int64_t nrows,
                                                  const TV* __restrict__ X,
                                                  TV* __restrict__ Y) {
  nat_body<TV, B, L, U>(NatArgs<TV>{rp, ci, val, nrows, X, Y}, blockIdx.x, gridDim.x);
}

template <int B, int L, int U>
__global__ __launch_bounds__(256) void k_spmm_nat_batch(const NatArgs<double>* a, BTiles t) {
  const BTile q = batch_tile(t, blockIdx.x);
  if (q.p < 0) return;  // an idle slot of the placement
  nat_body<double, B, L, U>(a[q.p], q.x, q.gx);
}

// one workgroup (256 lanes) per row, for rows longer than 4096
template <typename TV, int B>
__global__ __launch_bounds__(256) void k_spmm_wg(const int32_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const TV* __restrict__ val,
                                                 const int32_t* __restrict__ rows, int64_t nrows,
                                                 const TV* __restrict__ X, TV* __restrict__ Y) {
  __shared__ TV part[4][B];
  const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  for (int64_t slot = blockIdx.x; slot < nrows; slot += gridDim.x) {
    const int32_t row = rows[slot];
    const int32_t a = rp[row], e = rp[row + 1];
    TV acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = TV(0);
    for (int32_t k = a + threadIdx.x; k < e; k += 256) {
      const int32_t c = ci[k];
      const TV v = val[k];
#pragma unroll
      for (int j = 0; j < B; ++j) acc[j] = fma(v, X[(int64_t)c * B + j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc[j] += __shfl_xor(acc[j], off, kWave);
    }
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < B; ++j) part[w][j] = acc[j];
    }
    __syncthreads();
    if (threadIdx.x < B) {
      int j = threadIdx.x;
      Y[(int64_t)row * B + j] = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
    }
    __syncthreads();
  }
}

template <typename TV, int B, int L>
static void launch_group(int U, int blocks, const Csr32& A, const TV* val, const int32_t* rows,
                         int64_t nr, const TV* X, TV* Y, hipStream_t s) {
  if (!rows) {
    switch (U) {
      case 4: k_spmm_nat<TV, B, L, 4><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, nr, X, Y); break;
      case 2: k_spmm_nat<TV, B, L, 2><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, nr, X, Y); break;
      default: k_spmm_nat<TV, B, L, 1><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, nr, X, Y); break;
    }
    return;
  }
  switch (U) {
    case 4: k_spmm_group<TV, B, L, 4><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, rows, nr, X, Y); break;
    case 2: k_spmm_group<TV, B, L, 2><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, rows, nr, X, Y); break;
    default: k_spmm_group<TV, B, L, 1><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, rows, nr, X, Y); break;
  }
}

template <typename TV, int B>
static void spmm_b(const Csr32& A, const TV* val, const TV* X, TV* Y, hipStream_t s) {
  const bool merged = A.merged_bin >= 0;
  const int U = A.unroll;
  for (int bn = 0; bn < kNumBins; ++bn) {
    if (merged && bn != A.merged_bin) continue;
    int64_t r0 = merged ? 0 : A.bin_off[bn], r1 = merged ? A.rows : A.bin_off[bn + 1];
    int64_t nr = r1 - r0;
    if (nr <= 0) continue;
    const int32_t* rows = merged ? nullptr : A.binrows + r0;
    if (bn == kNumBins - 1) {
      int blocks = (int)std::min<int64_t>(nr, 8192);
      k_spmm_wg<TV, B><<<blocks, 256, 0, s>>>(A.rp, A.ci, val, rows, nr, X, Y);
    } else {
      const int L = 1 << bn;
      const int64_t rpb = 256 / L;
      int64_t need = (nr + rpb - 1) / rpb;
      int blocks = (int)std::min<int64_t>(need, 16384);
      if (blocks >= 64) blocks = (blocks / 8) * 8;  // whole XCD rounds for the remap
      switch (bn) {
        case 0: launch_group<TV, B, 1>(U, blocks, A, val, rows, nr, X, Y, s); break;
        case 1: launch_group<TV, B, 2>(U, blocks, A, val, rows, nr, X, Y, s); break;
        case 2: launch_group<TV, B, 4>(U, blocks, A, val, rows, nr, X, Y, s); break;
        case 3: launch_group<TV, B, 8>(U, blocks, A, val, rows, nr, X, Y, s); break;
        case 4: launch_group<TV, B, 16>(U, blocks, A, val, rows, nr, X, Y, s); break;
        case 5: launch_group<TV, B, 32>(U, blocks, A, val, rows, nr, X, Y, s); break;
        default: launch_group<TV, B, 64>(U, blocks, A, val, rows, nr, X, Y, s); break;
      }
    }
    SVDS_LAUNCH_CHECK();
  }
}

template <typename TV>
static void spmm_dispatch(const Csr32& A, int b, const TV* val, const TV* X, TV* Y,
                          hipStream_t s) {
  switch (b) {
    case 1: spmm_b<TV, 1>(A, val, X, Y, s); break;
    case 2: spmm_b<TV, 2>(A, val, X, Y, s); break;
    case 3: spmm_b<TV, 3>(A, val, X, Y, s); break;
    case 4: spmm_b<TV, 4>(A, val, X, Y, s); break;
    case 5: spmm_b<TV, 5>(A, val, X, Y, s); break;
    case 6: spmm_b<TV, 6>(A, val, X, Y, s); break;
    case 7: spmm_b<TV, 7>(A, val, X, Y, s); break;
    case 8: spmm_b<TV, 8>(A, val, X, Y, s); break;
    default: throw Error(SVDS_ERR_ARG, "spmm: block width must be 1..8");
  }
}

void spmm(const Csr32& A, int b, const double* X, double* Y, hipStream_t s) {
  spmm_dispatch<double>(A, b, A.val, X, Y, s);
}

void spmm_f32(const Csr32& A, int b, const float* X, float* Y, hipStream_t s) {
  if (!A.val32) throw Error(SVDS_ERR_ARG, "spmm_f32: no FP32 values");
  spmm_dispatch<float>(A, b, A.val32, X, Y, s);
}

// batched products of matrices that share one merged launch shape: each
// matrix runs the workgroups of its own natural-order launch
template <int B, int L>
static void nat_batch_launch(int U, int tiles, const NatArgs<double>* d, const BTiles& t,
                             hipStream_t s) {
  switch (U) {
    case 4: k_spmm_nat_batch<B, L, 4><<<tiles, 256, 0, s>>>(d, t); break;
    case 2: k_spmm_nat_batch<B, L, 2><<<tiles, 256, 0, s>>>(d, t); break;
    default: k_spmm_nat_batch<B, L, 1><<<tiles, 256, 0, s>>>(d, t); break;
  }
}

template <int B>
static void nat_batch_b(int bn, int U, int tiles, const NatArgs<double>* d, const BTiles& t,
                        hipStream_t s) {
  switch (bn) {
    case 0: nat_batch_launch<B, 1>(U, tiles, d, t, s); break;
    case 1: nat_batch_launch<B, 2>(U, tiles, d, t, s); break;
    case 2: nat_batch_launch<B, 4>(U, tiles, d, t, s); break;
    case 3: nat_batch_launch<B, 8>(U, tiles, d, t, s); break;
    case 4: nat_batch_launch<B, 16>(U, tiles, d, t, s); break;
    case 5: nat_batch_launch<B, 32>(U, tiles, d, t, s); break;
    default: nat_batch_launch<B, 64>(U, tiles, d, t, s); break;
  }
}

void spmm_batch(int b, const std::vector<BatchSpmm>& jobs, BatchUpload& up, hipStream_t s) {
  const int np = (int)jobs.size();
  if (np == 0) return;
  const int bn = jobs[0].A->merged_bin, U = jobs[0].A->unroll;
  if (bn < 0 || bn >= kNumBins - 1) throw Error(SVDS_ERR_ARG, "spmm_batch: needs a merged shape");
  std::vector<NatArgs<double>> args(np);
  std::vector<int> gx(np), gy(np, 1);
  for (int j = 0; j < np; ++j) {
    const Csr32& A = *jobs[j].A;
    if (A.merged_bin != bn || A.unroll != U)
      throw Error(SVDS_ERR_ARG, "spmm_batch: launch shapes differ");
    args[j] = NatArgs<double>{A.rp, A.ci, A.val, A.rows, jobs[j].X, jobs[j].Y};
    // the grid of the matrix's own merged launch (spmm_b)
    const int64_t rpb = 256 / (1 << bn);
    const int64_t need = (A.rows + rpb - 1) / rpb;
    int blocks = (int)std::min<int64_t>(need, 16384);
    if (blocks >= 64) blocks = (blocks / 8) * 8;
    gx[j] = blocks;
    if (A.rows <= 0 || blocks <= 0) gy[j] = 0;
  }
  BTiles t;
  const int tiles = up.tiles(gx, gy, t);
  const NatArgs<double>* d = up.put(args.data(), args.size());
  up.flush();  // this launch's arguments, one copy
  if (tiles > 0) {
    switch (b) {
      case 1: nat_batch_b<1>(bn, U, tiles, d, t, s); break;
      case 2: nat_batch_b<2>(bn, U, tiles, d, t, s); break;
      case 3: nat_batch_b<3>(bn, U, tiles, d, t, s); break;
      case 4: nat_batch_b<4>(bn, U, tiles, d, t, s); break;
      case 5: nat_batch_b<5>(bn, U, tiles, d, t, s); break;
      case 6: nat_batch_b<6>(bn, U, tiles, d, t, s); break;
      case 7: nat_batch_b<7>(bn, U, tiles, d, t, s); break;
      case 8: nat_batch_b<8>(bn, U, tiles, d, t, s); break;
      default: throw Error(SVDS_ERR_ARG, "spmm_batch: block width must be 1..8");
    }
  }
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
