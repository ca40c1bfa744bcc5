// One-pass normal-equations product Z = A^T (A X) for the first stage, which
// works on C = A^T A through a product with A followed by one with A^T
// (Section 3.3).  For matrices whose blocks of R consecutive rows touch narrow
// column windows (banded matrices, discretised operators in a bandwidth-
// reducing order), a workgroup takes one block: it forms y = A_blk X in LDS
// from the block's CSR rows, storing each value it streams in LDS at its
// position in a block-local column ordering (built once per matrix: per
// nonzero, 16 bits holding its window column and its rank in that column,
// read in place of the 32-bit column index), and then A_blk^T y over its
// window from LDS.
// A is read from HBM once per product instead of A and its transpose.  The
// windows of neighbouring blocks overlap; a second kernel adds each column's
// partial sums in block order.  Every sum has a fixed order, so the results
// are bitwise reproducible.
#include "common.h"

namespace svds {

constexpr int kGramT = 256;  // threads per workgroup
constexpr int kGramL = 4;    // lanes per row in the product with A
constexpr int kGramU = 4;    // nonzeros in flight per lane

// ---------------------------------------------------------------------------
// set-up
// ---------------------------------------------------------------------------
// windows of blocks of kGramMinRows rows: first and last column touched and
// the number of nonzeros (column indices are increasing within a row)
__global__ void k_gram_windows(const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                               int64_t rows, int64_t nblk, int32_t* __restrict__ lo,
                               int32_t* __restrict__ hi, int32_t* __restrict__ nnzb) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nblk) return;
  const int64_t r0 = b * kGramMinRows, r1 = min(r0 + (int64_t)kGramMinRows, rows);
  int32_t mn = INT32_MAX, mx = -1;
  for (int64_t r = r0; r < r1; ++r) {
    const int32_t a = rp[r], e = rp[r + 1];
    if (e > a) {
      mn = min(mn, ci[a]);
      mx = max(mx, ci[e - 1]);
    }
  }
  lo[b] = mn;
  hi[b] = mx;
  nnzb[b] = rp[r1] - rp[r0];
}

void gram_windows(const Csr32& A, int64_t nblk, int32_t* lo, int32_t* hi, int32_t* nnzb,
                  hipStream_t s) {
  if (nblk <= 0) return;
  k_gram_windows<<<(unsigned)((nblk + 255) / 256), 256, 0, s>>>(A.rp, A.ci, A.rows, nblk, lo,
                                                                  hi, nnzb);
  SVDS_LAUNCH_CHECK();
}

// block-local column ordering: per block, the column pointers of its window
// and, for each nonzero in CSR order, its window column and its rank among
// the block's nonzeros of the same column (rows ascending), packed in 16
// bits, so that column-order position = column pointer + rank.  Each column
// of the window gets a bit mask of the block's rows that hold it (set with
// atomic ORs, whose result does not depend on their order); counts and ranks
// are population counts of these masks.
__global__ __launch_bounds__(kGramT) void k_gram_csc(const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ ci, int64_t rows,
                                                     int R, const int32_t* __restrict__ lo,
                                                     const int32_t* __restrict__ hi,
                                                     const int64_t* __restrict__ poff,
                                                     int32_t* __restrict__ colptr,
                                                     uint16_t* __restrict__ cidx) {
  constexpr int MW = kGramMaxRows / 64;  // mask words per column
  __shared__ unsigned long long mask[kGramMaxWidth * MW];
  __shared__ int32_t part[kGramT];
  const int t = threadIdx.x;
  const int64_t b = blockIdx.x;
  const int64_t r0 = b * R, r1 = min(r0 + (int64_t)R, rows);
  const int nr = (int)(r1 - r0);
  const int32_t c0 = lo[b];
  const int w = hi[b] - c0 + 1;
  int32_t* cp = colptr + poff[b] + b;
  for (int i = t; i < w * MW; i += kGramT) mask[i] = 0ull;
  __syncthreads();
  // one row per group of 4 lanes, its nonzeros strided over the lanes
  for (int r = t / 4; r < nr; r += kGramT / 4)
    for (int32_t k = rp[r0 + r] + (t % 4); k < rp[r0 + r + 1]; k += 4)
      atomicOr(&mask[(ci[k] - c0) * MW + r / 64], 1ull << (r % 64));
  __syncthreads();
  // exclusive scan of the column counts: one contiguous chunk per thread
  const int chunk = (w + kGramT - 1) / kGramT;
  const int ca = min(t * chunk, w), cb = min(ca + chunk, w);
  int sum = 0;
  for (int c = ca; c < cb; ++c)
    for (int q = 0; q < MW; ++q) sum += __popcll(mask[c * MW + q]);
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int i = 0; i < kGramT; ++i) {
      const int v = part[i];
      part[i] = run;
      run += v;
    }
  }
  __syncthreads();
  int run = part[t];
  for (int c = ca; c < cb; ++c) {
    cp[c] = run;
    for (int q = 0; q < MW; ++q) run += __popcll(mask[c * MW + q]);
  }
  if (t == 0) cp[w] = rp[r1] - rp[r0];
  // rank of (r, c): the rows above r holding column c
  for (int r = t / 4; r < nr; r += kGramT / 4)
    for (int32_t k = rp[r0 + r] + (t % 4); k < rp[r0 + r + 1]; k += 4) {
      const unsigned long long* m = mask + (ci[k] - c0) * MW;
      int below = 0;
      for (int q = 0; q < r / 64; ++q) below += __popcll(m[q]);
      below += __popcll(m[r / 64] & ((1ull << (r % 64)) - 1ull));
      cidx[k] = (uint16_t)((ci[k] - c0) | (below << kGramColBits));
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// cover[j] = the first block whose window holds column j (a minimum, so the
// result does not depend on the order of the atomics)
__global__ void k_gram_cover(const int32_t* __restrict__ lo, const int32_t* __restrict__ hi,
                             int32_t* __restrict__ cover) {
  const int b = blockIdx.x;
  for (int32_t j = lo[b] + (int32_t)threadIdx.x; j <= hi[b]; j += blockDim.x)
    atomicMin(&cover[j], b);
}

void gram_build(const Csr32& A, const GramPlan& G, hipStream_t s) {
  if (G.nblk <= 0) return;
  k_gram_csc<<<(unsigned)G.nblk, kGramT, 0, s>>>(A.rp, A.ci, A.rows, G.R, G.lo, G.hi, G.poff,
                                                 G.colptr, G.cidx);
  SVDS_LAUNCH_CHECK();
  k_fill_i32<<<(unsigned)((A.cols + 255) / 256), 256, 0, s>>>(G.cover, A.cols, (int32_t)G.nblk);
  SVDS_LAUNCH_CHECK();
  k_gram_cover<<<(unsigned)G.nblk, 256, 0, s>>>(G.lo, G.hi, G.cover);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// product
// ---------------------------------------------------------------------------
// one workgroup per block.  The window's column pointers are staged in LDS;
// then y = A_blk X (kGramL lanes per row, kGramU nonzeros in flight per lane),
// each value streamed being stored with its local row at its column-order
// position (column pointer + rank) in LDS; then the window's partial sums
// A_blk^T y with two lanes per column (alternate entries, then their sum),
// everything from LDS.
template <int B>
__global__ __launch_bounds__(kGramT) void k_gram_partial(
    const int32_t* __restrict__ rp, const double* __restrict__ val,
    const uint16_t* __restrict__ cidx, int64_t rows, int R,
    const double* __restrict__ X, const int32_t* __restrict__ lo,
    const int32_t* __restrict__ hi, const int64_t* __restrict__ poff,
    const int32_t* __restrict__ colptr, double* __restrict__ P) {
  constexpr int L = kGramL, U = kGramU, RPP = kGramT / kGramL;
  __shared__ double vs[kGramMaxNnz];         // values in column order
  __shared__ uint8_t rs[kGramMaxNnz];        // their local rows
  __shared__ int32_t cpl[kGramMaxWidth + 1];  // the window's column pointers
  __shared__ double ys[kGramMaxRows * B];
  const int t = threadIdx.x;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);
  const int64_t r0 = b * R, r1 = min(r0 + (int64_t)R, rows);
  const int32_t c0 = lo[b];
  const int w = hi[b] - c0 + 1;
  const int32_t* __restrict__ cp = colptr + poff[b] + b;
  for (int c = t; c <= w; c += kGramT) cpl[c] = cp[c];
  __syncthreads();
  const int grp = t / L, lane = t % L;
  for (int rr = grp; rr < (int)(r1 - r0); rr += RPP) {
    const int32_t a = rp[r0 + rr], e = rp[r0 + rr + 1];
    double acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = 0.0;
    for (int32_t k0 = a + lane; k0 < e; k0 += L * U) {
      int32_t c[U];
      double v[U];
      int rk[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t k = k0 + u * L;
        const int32_t kk = k < e ? k : e - 1;
        const int p = cidx[kk];
        c[u] = c0 + (p & ((1 << kGramColBits) - 1));
        v[u] = val[kk];
        rk[u] = p >> kGramColBits;
      }
      double x[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const double* __restrict__ xr = X + (int64_t)c[u] * B;
#pragma unroll
        for (int j = 0; j < B; ++j) x[u][j] = xr[j];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const bool in = k0 + u * L < e;
        if (in) {
          const int pos = cpl[c[u] - c0] + rk[u];
          vs[pos] = v[u];
          rs[pos] = (uint8_t)rr;
        }
#pragma unroll
        for (int j = 0; j < B; ++j) {
          const double q = fma(v[u], x[u][j], acc[j]);
          acc[j] = in ? q : acc[j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = lane_sum<double, L>(acc[j]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < B; ++j) ys[rr * B + j] = acc[j];
    }
  }
  __syncthreads();
  double* __restrict__ pb = P + poff[b] * B;
  const int half = t & 1;
  // whole pairs of lanes iterate together (w is the same for the block)
  for (int c = t >> 1; c < w; c += kGramT / 2) {
    double acc[B];
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = 0.0;
    const int qe = cpl[c + 1];
    for (int q = cpl[c] + half; q < qe; q += 2) {
      const double v = vs[q];
      const double* y = ys + (int)rs[q] * B;
#pragma unroll
      for (int j = 0; j < B; ++j) acc[j] = fma(v, y[j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < B; ++j) acc[j] = lane_sum<double, 2>(acc[j]);
    if (half == 0) {
#pragma unroll
      for (int j = 0; j < B; ++j) pb[(int64_t)c * B + j] = acc[j];
    }
  }
}

// Z[j] = the sum of column j's partial sums over the blocks whose windows
// hold it, in block order (the windows' first columns are nondecreasing, so
// these blocks lie between cover[j] and the first block starting past j).
// Z is row-major (ldz = 0: entry (j, q) at j*B + q) or column-major with
// leading dimension ldz (entry (j, q) at j + q*ldz).
template <int B>
__global__ void k_gram_combine(const int32_t* __restrict__ cover, const int32_t* __restrict__ lo,
                               const int32_t* __restrict__ hi, const int64_t* __restrict__ poff,
                               int64_t nblk, const double* __restrict__ P, int64_t cols,
                               double* __restrict__ Z, int64_t ldz) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= cols) return;
  double acc[B];
#pragma unroll
  for (int q = 0; q < B; ++q) acc[q] = 0.0;
  for (int64_t b = cover[j]; b < nblk && lo[b] <= j; ++b) {
    if (j > hi[b]) continue;
    const double* __restrict__ p = P + (poff[b] + (j - lo[b])) * B;
#pragma unroll
    for (int q = 0; q < B; ++q) acc[q] += p[q];
  }
  if (ldz > 0) {
#pragma unroll
    for (int q = 0; q < B; ++q) Z[j + q * ldz] = acc[q];
  } else {
#pragma unroll
    for (int q = 0; q < B; ++q) Z[j * B + q] = acc[q];
  }
}

template <int B>
static void partial_b(const Csr32& A, const GramPlan& G, const double* X, double* P,
                      hipStream_t s) {
  k_gram_partial<B><<<(unsigned)G.nblk, kGramT, 0, s>>>(A.rp, A.val, G.cidx, A.rows, G.R,
                                                       X, G.lo, G.hi, G.poff, G.colptr, P);
}

template <int B>
static void combine_b(const GramPlan& G, int64_t cols, const double* P, double* Z, int64_t ldz,
                      hipStream_t s) {
  k_gram_combine<B><<<(unsigned)((cols + 255) / 256), 256, 0, s>>>(G.cover, G.lo, G.hi, G.poff,
                                                                  G.nblk, P, cols, Z, ldz);
}

void gram_partial(const Csr32& A, const GramPlan& G, int b, const double* X, double* P,
                  hipStream_t s) {
  if (G.R <= 0 || G.nblk <= 0) throw Error(SVDS_ERR_ARG, "gram: no plan");
  switch (b) {
    case 1: partial_b<1>(A, G, X, P, s); break;
    case 2: partial_b<2>(A, G, X, P, s); break;
    case 3: partial_b<3>(A, G, X, P, s); break;
    case 4: partial_b<4>(A, G, X, P, s); break;
    case 5: partial_b<5>(A, G, X, P, s); break;
    case 6: partial_b<6>(A, G, X, P, s); break;
    case 7: partial_b<7>(A, G, X, P, s); break;
    case 8: partial_b<8>(A, G, X, P, s); break;
    default: throw Error(SVDS_ERR_ARG, "gram: block width must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}

void gram_combine(const GramPlan& G, int64_t cols, int b, const double* P, double* Z,
                  int64_t ldz, hipStream_t s) {
  if (cols <= 0) return;
  if (G.R <= 0 || G.nblk <= 0) throw Error(SVDS_ERR_ARG, "gram: no plan");
  switch (b) {
    case 1: combine_b<1>(G, cols, P, Z, ldz, s); break;
    case 2: combine_b<2>(G, cols, P, Z, ldz, s); break;
    case 3: combine_b<3>(G, cols, P, Z, ldz, s); break;
    case 4: combine_b<4>(G, cols, P, Z, ldz, s); break;
    case 5: combine_b<5>(G, cols, P, Z, ldz, s); break;
    case 6: combine_b<6>(G, cols, P, Z, ldz, s); break;
    case 7: combine_b<7>(G, cols, P, Z, ldz, s); break;
    case 8: combine_b<8>(G, cols, P, Z, ldz, s); break;
    default: throw Error(SVDS_ERR_ARG, "gram: block width must be 1..8");
  }
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
