// Setup kernels: CSR validation, 32-bit row offsets, explicit transpose,
// row-length binning, diag(A^T A), counter-based random blocks.
#include "common.h"

namespace svds {

// ---------------------------------------------------------------------------
// validation: monotone offsets, columns in range and strictly increasing
// ---------------------------------------------------------------------------
__global__ void k_check_csr(const int64_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            int64_t m, int64_t n, int64_t nnz, int* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    int64_t a = rp[i], e = rp[i + 1];
    if (a > e || a < 0 || e > nnz) {
      atomicOr(flag, 1);
      continue;
    }
    int32_t prev = -1;
    for (int64_t k = a; k < e; ++k) {
      int32_t c = ci[k];
      if (c < 0 || c >= n || c <= prev) {
        atomicOr(flag, 2);
        break;
      }
      prev = c;
    }
  }
}

void check_csr(const svds_csr& A, int* d_flag, hipStream_t s) {
  int blocks = (int)std::min<int64_t>(4096, (A.m + 255) / 256);
  if (blocks < 1) blocks = 1;
  k_check_csr<<<blocks, 256, 0, s>>>(A.rowptr, A.colind, A.m, A.n, A.nnz, d_flag);
  SVDS_LAUNCH_CHECK();
}

__global__ void k_rp32(const int64_t* __restrict__ rp, int32_t* __restrict__ out, int64_t n1) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n1) out[i] = (int32_t)rp[i];
}

void rowptr_to32(const int64_t* rp, int32_t* rp32, int64_t m, hipStream_t s) {
  int64_t n1 = m + 1;
  k_rp32<<<(unsigned)((n1 + 255) / 256), 256, 0, s>>>(rp, rp32, n1);
  SVDS_LAUNCH_CHECK();
}

void copy_csr_arrays(const svds_csr& A, Csr32& out, hipStream_t s) {
  rowptr_to32(A.rowptr, out.rp, A.m, s);
  SVDS_HIP(hipMemcpyAsync(out.ci, A.colind, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToDevice, s));
  SVDS_HIP(hipMemcpyAsync(out.val, A.values, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s));
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (three phases, 1024 elements per block)
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;

__device__ int block_exclusive_scan(int v, int* sh, int* total) {
  // Hillis-Steele on 1024 threads through shared memory
  int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int x = (t >= off) ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int incl = sh[t];
  if (total && t == kScanBlock - 1) *total = incl;
  return incl - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_local(const int32_t* in, int32_t* out,
                                                            int32_t* blocksum, int64_t n) {
  __shared__ int sh[kScanBlock];
  __shared__ int tot;
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int v = (i < n) ? in[i] : 0;
  int ex = block_exclusive_scan(v, sh, &tot);
  if (i < n) out[i] = ex;
  __syncthreads();
  if (threadIdx.x == 0) blocksum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(int32_t* out, const int32_t* off,
                                                          int64_t n) {
  int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  if (i < n) out[i] += off[blockIdx.x];
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  const StreamScratch sbs(sizeof(int32_t) * nb, s), sbso(sizeof(int32_t) * nb, s);
  int32_t* bs = sbs.as<int32_t>();
  int32_t* bso = sbso.as<int32_t>();
  k_scan_local<<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, bs, n);
  SVDS_LAUNCH_CHECK();
  if (nb > 1) {
    exclusive_scan_i32(bs, bso, nb, s);
    k_scan_add<<<(unsigned)nb, kScanBlock, 0, s>>>(out, bso, n);
    SVDS_LAUNCH_CHECK();
  }
}

// ---------------------------------------------------------------------------
// transpose: count per column, scan, scatter with atomic cursors, then sort
// each row of the transpose by its column (the original row) so the result
// is independent of the scatter order.
// ---------------------------------------------------------------------------
__global__ void k_count_cols(const int32_t* __restrict__ ci, int64_t nnz, int32_t* cnt) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; k < nnz; k += stride) atomicAdd(&cnt[ci[k]], 1);
}

__global__ void k_scatter_t(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                            const double* __restrict__ val, int64_t m, int32_t* cursor,
                            int32_t* __restrict__ ciT, double* __restrict__ valT) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < m; i += stride) {
    for (int32_t k = rp[i]; k < rp[i + 1]; ++k) {
      int32_t pos = atomicAdd(&cursor[ci[k]], 1);
      ciT[pos] = (int32_t)i;
      valT[pos] = val[k];
    }
  }
}

// one wavefront per row: rank of each entry = number of smaller keys
constexpr int kSortLds = 2048;
__global__ __launch_bounds__(64) void k_sort_rows(const int32_t* __restrict__ rp, int64_t rows,
                                                  int32_t* ci, double* val) {
  __shared__ int32_t key[kSortLds];
  __shared__ double vv[kSortLds];
  for (int64_t r = blockIdx.x; r < rows; r += gridDim.x) {
    int32_t a = rp[r], e = rp[r + 1];
    int len = e - a;
    if (len <= 1) continue;
    if (len <= kSortLds) {
      for (int t = threadIdx.x; t < len; t += 64) {
        key[t] = ci[a + t];
        vv[t] = val[a + t];
      }
      __syncthreads();
      for (int t = threadIdx.x; t < len; t += 64) {
        int32_t kt = key[t];
        int rank = 0;
        for (int u = 0; u < len; ++u) rank += key[u] < kt;
        ci[a + rank] = kt;
        val[a + rank] = vv[t];
      }
      __syncthreads();
    } else {
      // very long row: ranks from global memory into a second pass
      // (keys are distinct, so ranks form a permutation); stage through the
      // value array by cycles is avoided by sorting pairs with repeated
      // odd-even transposition, which needs no extra storage.
      for (int phase = 0; phase < len; ++phase) {
        for (int t = threadIdx.x; 2 * t + (phase & 1) + 1 < len; t += 64) {
          int p = a + 2 * t + (phase & 1);
          int32_t k0 = ci[p], k1 = ci[p + 1];
          if (k0 > k1) {
            double v0 = val[p], v1 = val[p + 1];
            ci[p] = k1;
            ci[p + 1] = k0;
            val[p] = v1;
            val[p + 1] = v0;
          }
        }
        __syncthreads();
      }
    }
  }
}

void transpose_csr(const Csr32& A, Csr32& T, int32_t* d_cursor, hipStream_t s) {
  // T.rp, T.ci, T.val allocated by the caller (cols+1, nnz, nnz); d_cursor: cols+1 ints
  int64_t nc = A.cols;
  SVDS_HIP(hipMemsetAsync(d_cursor, 0, sizeof(int32_t) * (nc + 1), s));
  int blocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (A.nnz + 255) / 256));
  if (A.nnz > 0) {
    k_count_cols<<<blocks, 256, 0, s>>>(A.ci, A.nnz, d_cursor);
    SVDS_LAUNCH_CHECK();
  }
  exclusive_scan_i32(d_cursor, T.rp, nc + 1, s);  // T.rp[nc] = nnz (count[nc] = 0)
  SVDS_HIP(hipMemcpyAsync(d_cursor, T.rp, sizeof(int32_t) * (nc + 1), hipMemcpyDeviceToDevice, s));
  int rblocks = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (A.rows + 255) / 256));
  k_scatter_t<<<rblocks, 256, 0, s>>>(A.rp, A.ci, A.val, A.rows, d_cursor, T.ci, T.val);
  SVDS_LAUNCH_CHECK();
  int sblocks = (int)std::min<int64_t>(65536, std::max<int64_t>(1, nc));
  k_sort_rows<<<sblocks, 64, 0, s>>>(T.rp, nc, T.ci, T.val);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// row-length bins (stable: row order is kept inside each bin)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int row_bin(int len) {
  // lanes per row chosen so that each lane handles about four nonzeros
  if (len <= 4) return 0;      // 1 lane
  if (len <= 8) return 1;      // 2
  if (len <= 16) return 2;     // 4
  if (len <= 32) return 3;     // 8
  if (len <= 64) return 4;     // 16
  if (len <= 128) return 5;    // 32
  if (len <= 4096) return 6;   // 64 (a wavefront)
  return 7;                    // 256 (a workgroup)
}

constexpr int kBinBlock = 1024;

__global__ __launch_bounds__(kBinBlock) void k_bin_hist(const int32_t* __restrict__ rp,
                                                        int64_t rows, int32_t* counts,
                                                        int64_t nblk) {
  __shared__ int c[kNumBins];
  if (threadIdx.x < kNumBins) c[threadIdx.x] = 0;
  __syncthreads();
  int64_t i = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
  if (i < rows) atomicAdd(&c[row_bin(rp[i + 1] - rp[i])], 1);
  __syncthreads();
  if (threadIdx.x < kNumBins) counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(kBinBlock) void k_bin_scatter(const int32_t* __restrict__ rp,
                                                           int64_t rows,
                                                           const int32_t* __restrict__ offs,
                                                           int64_t nblk, int32_t* binrows) {
  constexpr int nw = kBinBlock / kWave;
  __shared__ int wcount[nw][kNumBins];
  __shared__ int wbase[nw][kNumBins];
  int64_t i = (int64_t)blockIdx.x * kBinBlock + threadIdx.x;
  int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
  int my = (i < rows) ? row_bin(rp[i + 1] - rp[i]) : -1;
  int myrank = 0;
  for (int bn = 0; bn < kNumBins; ++bn) {
    uint64_t mask = __ballot(my == bn);
    if (my == bn) myrank = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wcount[w][bn] = __popcll(mask);
  }
  __syncthreads();
  if (threadIdx.x < kNumBins) {
    int bn = threadIdx.x, acc = 0;
    for (int ww = 0; ww < nw; ++ww) {
      wbase[ww][bn] = acc;
      acc += wcount[ww][bn];
    }
  }
  __syncthreads();
  if (my >= 0) binrows[offs[(int64_t)my * nblk + blockIdx.x] + wbase[w][my] + myrank] = (int32_t)i;
}

void build_bins(Csr32& A, hipStream_t s) {
  int64_t rows = A.rows;
  int64_t nblk = std::max<int64_t>(1, (rows + kBinBlock - 1) / kBinBlock);
  const StreamScratch sc(sizeof(int32_t) * (kNumBins * nblk + 1), s);
  const StreamScratch so(sizeof(int32_t) * (kNumBins * nblk + 1), s);
  int32_t* counts = sc.as<int32_t>();
  int32_t* offs = so.as<int32_t>();
  SVDS_HIP(hipMemsetAsync(counts, 0, sizeof(int32_t) * (kNumBins * nblk + 1), s));
  k_bin_hist<<<(unsigned)nblk, kBinBlock, 0, s>>>(A.rp, rows, counts, nblk);
  SVDS_LAUNCH_CHECK();
  exclusive_scan_i32(counts, offs, kNumBins * nblk + 1, s);
  k_bin_scatter<<<(unsigned)nblk, kBinBlock, 0, s>>>(A.rp, rows, offs, nblk, A.binrows);
  SVDS_LAUNCH_CHECK();
  // bin boundaries to the host (offs at bin starts)
  int32_t h[kNumBins + 1];
  for (int bn = 0; bn <= kNumBins; ++bn)
    SVDS_HIP(hipMemcpyAsync(&h[bn], offs + (int64_t)bn * nblk, sizeof(int32_t),
                            hipMemcpyDeviceToHost, s));
  SVDS_HIP(hipStreamSynchronize(s));
  for (int bn = 0; bn < kNumBins; ++bn) A.bin_off[bn] = h[bn];
  A.bin_off[kNumBins] = rows;
  // narrow spread (at most three adjacent lane shapes, no workgroup rows):
  // one launch over all rows in natural order, in the lane shape of the mean
  int lo = -1, hi = -1;
  for (int bn = 0; bn < kNumBins; ++bn)
    if (A.bin_off[bn + 1] > A.bin_off[bn]) {
      if (lo < 0) lo = bn;
      hi = bn;
    }
  A.merged_bin = -1;
  if (lo >= 0 && hi - lo <= 2 && hi < kNumBins - 1 && rows > 0) {
    const double mean = (double)A.nnz / (double)rows;
    int mb = 0;
    while (mb < kNumBins - 2 && mean > 4.0 * (double)(1 << mb)) ++mb;
    A.merged_bin = std::max(lo, std::min(mb, hi));
  }
  A.heuristic_bin = A.merged_bin;
}

// ---------------------------------------------------------------------------
// squared row norms (diag(A A^T) for rows of A; diag(A^T A) from rows of A^T)
// ---------------------------------------------------------------------------
__global__ void k_row_sq(const int32_t* __restrict__ rp, const double* __restrict__ val,
                         int64_t rows, double* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double s = 0.0;
  for (int32_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * val[k];
  out[i] = s;
}

void row_sqnorms(const Csr32& A, double* out, hipStream_t s) {
  if (A.rows == 0) return;
  k_row_sq<<<(unsigned)((A.rows + 255) / 256), 256, 0, s>>>(A.rp, A.val, A.rows, out);
  SVDS_LAUNCH_CHECK();
}

__global__ void k_to_f32(const double* in, float* out, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = (float)in[i];
}

void to_fp32(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>(8192, (n + 255) / 256);
  k_to_f32<<<blocks, 256, 0, s>>>(in, out, n);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// counter-based random block (column-major)
// ---------------------------------------------------------------------------
__global__ void k_fill_random(double* X, int64_t ld, int64_t N, int ncols, uint64_t seed,
                              uint64_t stream, int col0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  for (int c = 0; c < ncols; ++c)
    X[i + c * ld] = counter_uniform(seed, stream, (uint64_t)(col0 + c), (uint64_t)i);
}

void fill_random(double* X, int64_t ld, int64_t N, int ncols, uint64_t seed, uint64_t stream,
                 int col0, hipStream_t s) {
  if (N == 0 || ncols == 0) return;
  k_fill_random<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(X, ld, N, ncols, seed, stream, col0);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
