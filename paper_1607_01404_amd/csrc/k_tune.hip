// Autotuner for the launch shape of the sparse products.
//
// Candidates: one launch per row-length bin (row lists), or a single launch
// over all rows in natural order with L = 1, 2, ..., 64 lanes per row; each
// with 1, 2 or 4 nonzeros per lane per step.  Each
// candidate is timed with HIP events on the caller's stream for the block
// width the solve will use; the fastest is returned in the caller's copy of
// the matrix descriptor and kept in a process-wide cache keyed by a matrix
// signature (rows, columns, mean and maximum row-length bucket, block width,
// precision), so that matrices of the same shape class skip the search.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace svds {

namespace {
using Key = std::tuple<int, int, int, int, int, int>;
std::mutex g_mu;
std::map<Key, std::pair<int, int>> g_cache;  // (merged bin or -1, unroll)

int log2i(int64_t x) {
  int l = 0;
  while ((int64_t(1) << (l + 1)) <= x) ++l;
  return l;
}

Key signature(const Csr32& A, int b, bool fp32) {
  int hi = 0;
  for (int bn = 0; bn < kNumBins; ++bn)
    if (A.bin_off[bn + 1] > A.bin_off[bn]) hi = bn;
  const int mean_bucket = (int)std::lround(4.0 * std::log2(1.0 + (double)A.nnz / std::max<int64_t>(A.rows, 1)));
  return Key(log2i(A.rows), log2i(A.cols), mean_bucket, hi, b, fp32 ? 1 : 0);
}
}  // namespace

// A is the caller's own copy of a prepared matrix's descriptor: only its
// launch-shape fields are written.
void autotune_spmm(Csr32& A, int b, bool fp32, hipStream_t s) {
  if (A.rows == 0 || A.nnz == 0) return;
  const Key key = signature(A, b, fp32);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      A.merged_bin = it->second.first;
      A.unroll = it->second.second;
      A.tuned_b = b;
      return;
    }
  }
  // candidate shapes: -1 (binned) and single launches with 1..64 lanes per row
  // (only when no row needs the workgroup-per-row kernel)
  const bool has_wg_rows = A.bin_off[kNumBins] > A.bin_off[kNumBins - 1];
  std::vector<std::pair<int, int>> cand;
  for (int u : {1, 2, 4}) {
    cand.push_back({-1, u});
    if (!has_wg_rows)
      for (int bn = 0; bn < kNumBins - 1; ++bn) cand.push_back({bn, u});
  }
  const size_t es = fp32 ? sizeof(float) : sizeof(double);
  // probe blocks and events, released also when a launch throws
  struct Scratch {
    void* p;
    hipStream_t s;
    Scratch(size_t bytes, hipStream_t st) : p(stream_alloc(bytes, st)), s(st) {}
    ~Scratch() { stream_free(p, s); }
  };
  struct Event {
    hipEvent_t e = nullptr;
    Event() { SVDS_HIP(hipEventCreate(&e)); }
    ~Event() { (void)hipEventDestroy(e); }
  };
  const Scratch X(es * (size_t)A.cols * b, s), Y(es * (size_t)A.rows * b, s);
  SVDS_HIP(hipMemsetAsync(X.p, 0, es * (size_t)A.cols * b, s));
  const Event e0, e1;
  std::pair<int, int> best{A.merged_bin, A.unroll};
  float best_ms = 1e30f;
  const bool verbose = std::getenv("SVDS_DEBUG") != nullptr;
  Csr32 T = A;  // the candidate shape under test
  for (const auto& c : cand) {
    T.merged_bin = c.first;
    T.unroll = c.second;
    auto run = [&] {
      if (fp32) spmm_f32(T, b, (const float*)X.p, (float*)Y.p, s);
      else spmm(T, b, (const double*)X.p, (double*)Y.p, s);
    };
    run();  // warm-up
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      SVDS_HIP(hipEventRecord(e0.e, s));
      run();
      SVDS_HIP(hipEventRecord(e1.e, s));
      SVDS_HIP(hipEventSynchronize(e1.e));
      float ms = 0.f;
      SVDS_HIP(hipEventElapsedTime(&ms, e0.e, e1.e));
      tmin = std::min(tmin, ms);
    }
    if (verbose)
      std::fprintf(stderr, "[svds] autotune rows %lld b %d fp32 %d shape %d unroll %d: %.1f us\n",
                   (long long)A.rows, b, fp32 ? 1 : 0, c.first, c.second, tmin * 1e3);
    if (tmin < best_ms) {
      best_ms = tmin;
      best = c;
    }
  }
  // the first result stored for a signature is kept, and used by every solve
  // with it (also by one that tuned at the same time on another stream), so
  // that equal signatures always get equal launch shapes
  std::lock_guard<std::mutex> lk(g_mu);
  const auto kept = g_cache.emplace(key, best).first->second;
  A.merged_bin = kept.first;
  A.unroll = kept.second;
  A.tuned_b = b;
}

}  // namespace svds
