// Block-Jacobi preconditioner for C = A^T A: the inverses of the diagonal
// blocks of contiguous column ranges (the generic preconditioner of the
// paper's preconditioned comparison, Section 4), applied block by block.
//
// Setup, one workgroup per block (nb <= 128 columns, the block in LDS):
//   C_j[p][q] = sum_r A[r][c0+p] A[r][c0+q], built row by row of C_j from
//     the transpose (row c of A^T lists the rows r of column c) and the
//     sorted entries of A's row r inside the block: each thread owns rows of
//     C_j, so there are no atomics and the sums have a fixed order;
//   scaling to unit diagonal (zero diagonals -> 1, their rows and columns
//     cleared), right-looking Cholesky in which a pivot <= 1e-12 becomes 1
//     with its column decoupled, in-place inversion of the factor L, and
//     K_j = S L^-T L^-1 S written to HBM (nb x nb, symmetric).
// Apply: T[c0:c1, :] = K_j R[c0:c1, :] for b <= 8 columns.
#include "common.h"

namespace svds {

namespace {

constexpr int kBjT = 256;
constexpr int kBjMax = 128;
constexpr int kBjLd = kBjMax + 1;

__global__ __launch_bounds__(kBjT) void k_bj_setup(const int32_t* __restrict__ arp,
                                                   const int32_t* __restrict__ aci,
                                                   const double* __restrict__ aval,
                                                   const int32_t* __restrict__ trp,
                                                   const int32_t* __restrict__ tci,
                                                   const double* __restrict__ tval, int64_t N,
                                                   int nb, double* __restrict__ K) {
  __shared__ double C[kBjMax * kBjLd];
  __shared__ double sc[kBjMax], tmp[kBjMax];
  __shared__ int empty[kBjMax];
  __shared__ int decouple;
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * nb;
  const int n = (int)((c0 + nb < N) ? nb : N - c0);
  for (int a = t; a < n * kBjLd; a += kBjT) C[a] = 0.0;
  __syncthreads();
  // rows of C_j
  for (int p = t; p < n; p += kBjT) {
    const int64_t c = c0 + p;
    double* Cp = C + p * kBjLd;
    for (int32_t kt = trp[c]; kt < trp[c + 1]; ++kt) {
      const int32_t r = tci[kt];
      const double a = tval[kt];
      // first entry of row r with column >= c0 (sorted columns)
      int32_t lo = arp[r], hi = arp[r + 1];
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (aci[mid] < c0) lo = mid + 1;
        else hi = mid;
      }
      for (int32_t ka = lo; ka < arp[r + 1] && aci[ka] < c0 + n; ++ka)
        Cp[aci[ka] - c0] += a * aval[ka];
    }
  }
  __syncthreads();
  // unit-diagonal scaling; empty columns keep a unit diagonal
  for (int p = t; p < n; p += kBjT) {
    const double d = C[p * kBjLd + p];
    empty[p] = d > 0.0 ? 0 : 1;
    sc[p] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
  }
  __syncthreads();
  for (int a = t; a < n * n; a += kBjT) {
    const int i = a / n, j = a % n;
    double v = C[i * kBjLd + j] * sc[i] * sc[j];
    if (empty[i] || empty[j]) v = (i == j) ? 1.0 : 0.0;
    C[i * kBjLd + j] = v;
  }
  __syncthreads();
  // right-looking Cholesky (lower triangle), pivot rule as stated above
  for (int k = 0; k < n; ++k) {
    if (t == 0) {
      const double p = C[k * kBjLd + k];
      decouple = !(p > 1e-12);
      C[k * kBjLd + k] = decouple ? 1.0 : sqrt(p);
    }
    __syncthreads();
    const double lkk = C[k * kBjLd + k];
    for (int i = k + 1 + t; i < n; i += kBjT)
      C[i * kBjLd + k] = decouple ? 0.0 : C[i * kBjLd + k] / lkk;
    __syncthreads();
    const int m = n - k - 1;
    for (int a = t; a < m * m; a += kBjT) {
      const int i = k + 1 + a / m, j = k + 1 + a % m;
      if (j <= i) C[i * kBjLd + j] -= C[i * kBjLd + k] * C[j * kBjLd + k];
    }
    __syncthreads();
  }
  // in-place inverse of the lower factor, last column first: with the
  // trailing block already inverted, column j below the diagonal becomes
  // -L^-1[j+1:, j+1:] L[j+1:, j] / L[j][j]
  for (int j = n - 1; j >= 0; --j) {
    const double ljj = 1.0 / C[j * kBjLd + j];
    for (int i = j + 1 + t; i < n; i += kBjT) {
      double s = 0.0;
      for (int k = j + 1; k <= i; ++k) s += C[i * kBjLd + k] * C[k * kBjLd + j];
      tmp[i] = -s * ljj;
    }
    __syncthreads();
    for (int i = j + 1 + t; i < n; i += kBjT) C[i * kBjLd + j] = tmp[i];
    if (t == 0) C[j * kBjLd + j] = ljj;
    __syncthreads();
  }
  // K_j = S (L^-T L^-1) S: K[i][j] = sc_i sc_j sum_{k >= max(i, j)} Li[k][i] Li[k][j]
  double* Kj = K + (int64_t)blockIdx.x * nb * nb;
  for (int a = t; a < n * n; a += kBjT) {
    const int i = a / n, j = a % n;
    double s = 0.0;
    for (int k = (i > j ? i : j); k < n; ++k) s += C[k * kBjLd + i] * C[k * kBjLd + j];
    Kj[i * nb + j] = sc[i] * sc[j] * s;
  }
}

// T[c0 + i][col] = sum_k K_j[k][i] R[c0 + k][col]  (K_j symmetric: coalesced reads)
template <int B>
__global__ __launch_bounds__(kBjT) void k_bj_apply(const double* __restrict__ K, int nb, int64_t N,
                                                   const double* __restrict__ R, int64_t ldr,
                                                   double* __restrict__ T, int64_t ldt) {
  __shared__ double rs[kBjMax * B];
  const int t = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * nb;
  const int n = (int)((c0 + nb < N) ? nb : N - c0);
  for (int a = t; a < n * B; a += kBjT) {
    const int k = a / B, c = a % B;
    rs[a] = R[c0 + k + c * ldr];
  }
  __syncthreads();
  const double* Kj = K + (int64_t)blockIdx.x * nb * nb;
  for (int i = t; i < n; i += kBjT) {
    double acc[B];
#pragma unroll
    for (int c = 0; c < B; ++c) acc[c] = 0.0;
    for (int k = 0; k < n; ++k) {
      const double kv = Kj[k * nb + i];
#pragma unroll
      for (int c = 0; c < B; ++c) acc[c] = fma(kv, rs[k * B + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < B; ++c) T[c0 + i + c * ldt] = acc[c];
  }
}

}  // namespace

int bj_max_block() { return kBjMax; }

void bj_setup(const svds_matrix* M, int nb, double* K, hipStream_t s) {
  if (nb < 1 || nb > kBjMax) throw Error(SVDS_ERR_ARG, "block-Jacobi block size 1..128");
  const Csr32& A = M->A;
  const Csr32& At = M->At;
  const int64_t N = A.cols;
  const int64_t nblk = (N + nb - 1) / nb;
  k_bj_setup<<<(unsigned)nblk, kBjT, 0, s>>>(A.rp, A.ci, A.val, At.rp, At.ci, At.val, N, nb, K);
  SVDS_LAUNCH_CHECK();
}

void bj_apply(const double* K, int nb, int64_t N, int b, const double* R, int64_t ldr, double* T,
              int64_t ldt, hipStream_t s) {
  const int64_t nblk = (N + nb - 1) / nb;
  switch (b) {
    case 1: k_bj_apply<1><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 2: k_bj_apply<2><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 3: k_bj_apply<3><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 4: k_bj_apply<4><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 5: k_bj_apply<5><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 6: k_bj_apply<6><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 7: k_bj_apply<7><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    case 8: k_bj_apply<8><<<(unsigned)nblk, kBjT, 0, s>>>(K, nb, N, R, ldr, T, ldt); break;
    default: throw Error(SVDS_ERR_ARG, "bj_apply: block width 1..8");
  }
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds
