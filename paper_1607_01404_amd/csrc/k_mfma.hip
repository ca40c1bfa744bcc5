// Projections of the mixed-precision stage 1 on the matrix cores: the new
// columns of the projected matrix, V^T W, with V and W stored in FP32.
//
// Each FP32 value is split into a BF16 head and a BF16 tail (x ~ hi + lo);
// the product is accumulated in FP32 as hi*hi + hi*lo + lo*hi with
// v_mfma_f32_16x16x32_bf16, which keeps about 16 bits of the operands (the
// omitted lo*lo term is ~2^-16 relative).  The projection is HBM-bound (a few
// flops per byte), so the matrix cores are used to keep it far from any ALU
// limit, not because it is compute-bound.
#include "common.h"

namespace svds {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// Operand layout of v_mfma_f32_16x16x32_bf16 (checked on the device): lane l
// supplies A[m = l%16][k = 8*(l/16) + i] and B[k = 8*(l/16) + i][n = l%16],
// i = 0..7, and receives D[m = 4*(l/16) + i][n = l%16], i = 0..3.
constexpr int kMK = 32;  // rows (K) per MFMA step

__device__ __forceinline__ void split8(const float (&x)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const __bf16 h = (__bf16)x[i];
    hi[i] = h;
    lo[i] = (__bf16)(x[i] - (float)h);
  }
}

// C (nv x nb) = V^T W.  Wavefront w of a workgroup takes the 16-column tile
// blockIdx.y*4 + w of V (the M dimension); the block W (nb <= 8 columns, the
// N dimension padded to 16 with zeros) is shared.  Workgroups stride over
// 32-row steps of the K dimension.
__global__ __launch_bounds__(256) void k_proj_bf16x3(const float* __restrict__ V, int64_t ldv,
                                                     int nv, const float* __restrict__ W,
                                                     int64_t ldw, int nb, int64_t N,
                                                     double* __restrict__ partial) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int mt = blockIdx.y * 4 + w;
  const int j = mt * 16 + (lane & 15);
  const int c = lane & 15;
  const int kq = (lane >> 4) * 8;
  const bool aok = j < nv, bok = c < nb;
  const float* __restrict__ vc = V + (int64_t)(aok ? j : 0) * ldv;
  const float* __restrict__ wc = W + (int64_t)(bok ? c : 0) * ldw;
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int64_t r0 = (int64_t)blockIdx.x * kMK; r0 < N; r0 += (int64_t)gridDim.x * kMK) {
    float a[8], b[8];
    const int64_t rb = r0 + kq;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const bool in = rb + i < N;
      a[i] = (in && aok) ? vc[rb + i] : 0.f;
      b[i] = (in && bok) ? wc[rb + i] : 0.f;
    }
    bf16x8 ahi, alo, bhi, blo;
    split8(a, ahi, alo);
    split8(b, bhi, blo);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, bhi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, blo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, bhi, acc, 0, 0, 0);
  }
  // partial layout: [n * nv + m][block]
  const int nblk = gridDim.x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = mt * 16 + 4 * (lane >> 4) + i;
    const int n = lane & 15;
    if (m < nv && n < nb) partial[((int64_t)n * nv + m) * nblk + blockIdx.x] = (double)acc[i];
  }
}

void proj_bf16x3(const float* V, int64_t ldv, int nv, const float* W, int64_t ldw, int nb,
                 int64_t N, double* partial, double* C, hipStream_t s) {
  if (nv <= 0 || nb <= 0) return;
  if (nb > 16) throw Error(SVDS_ERR_ARG, "proj_bf16x3: block too wide");
  int nblk = (int)std::min<int64_t>(512, std::max<int64_t>(1, (N + 4 * kMK - 1) / (4 * kMK)));
  if (nblk >= 64) nblk = (nblk / 8) * 8;
  dim3 grid(nblk, (nv + 63) / 64);
  k_proj_bf16x3<<<grid, 256, 0, s>>>(V, ldv, nv, W, ldw, nb, N, partial);
  SVDS_LAUNCH_CHECK();
  reduce_partials(partial, nblk, nv * nb, C, s);
}

}  // namespace svds
