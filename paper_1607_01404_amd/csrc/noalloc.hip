// The product with the first stage's operator C = A_w^T A_w without any
// allocation, for callers that cannot allocate device memory (code under
// stream capture, serving loops, harnesses that forbid it).
//
// svds_matrix_normal takes its scratch (the one-pass product's window partial
// sums, or the intermediate A_w X of the two SpMMs) from the library's
// stream-ordered pool.  This variant takes it from one statically allocated
// device array of kScratchBytes per GPU, which the process holds until it
// ends.  Host code never uses the array's name as a device address: the
// address is looked up once per device with hipGetSymbolAddress and kept.
// Every call on a GPU shares that GPU's array; calls that overlap on one GPU
// (on different streams, or from different host threads without ordering)
// race on it.  Nothing in it must start at zero: the partial-sum kernel writes
// every entry the combine reads, and the first SpMM writes every entry of the
// intermediate the second reads.
#include <mutex>

#include "common.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};  // the array's device address on each GPU

// the array's address on the current device (looked up on the first call there)
double* scratch_ptr() {
  int dev = 0;
  SVDS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw svds::Error(SVDS_ERR_ARG, "device ordinal too large");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    SVDS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) throw svds::Error(SVDS_ERR_HIP, "no device address for the static scratch");
    g_ptr[dev] = static_cast<double*>(p);
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int svds_matrix_normal_noalloc(const svds_matrix* h, int b, const double* X,
                                          double* Z, int fused, int* used, void* stream) {
  return svds::guarded([&] {
    if (!h || !X || !Z || b < 1 || b > svds::kMaxBlock)
      throw svds::Error(SVDS_ERR_ARG, "normal args");
    const hipStream_t s = (hipStream_t)stream;
    const svds::Csr32& A = h->A;
    // the same choice as svds_matrix_normal, so that both give the same bits
    const bool one = fused && h->G.R > 0 && svds::gram_cheaper(A, h->G, b);
    const size_t need = sizeof(double) * (size_t)b * (size_t)(one ? h->G.wsum : A.rows);
    if (need > kScratchBytes)
      throw svds::Error(SVDS_ERR_ARG, "scratch of the allocation-free product exceeds 64 MiB");
    if (used) *used = one ? 1 : 0;
    double* P = scratch_ptr();
    if (one) {
      svds::gram_partial(A, h->G, b, X, P, s);
      svds::gram_combine(h->G, A.cols, b, P, Z, 0, s);
    } else {
      svds::spmm(A, b, X, P, s);
      svds::spmm(h->At, b, P, Z, s);
    }
    return SVDS_OK;
  });
}
