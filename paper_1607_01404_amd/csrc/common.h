// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "svds.h"

namespace svds {

// ---------------------------------------------------------------------------
// errors: thrown inside the library, turned into status codes at the ABI
// ---------------------------------------------------------------------------
struct Error : public std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define SVDS_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::svds::Error(e_ == hipErrorOutOfMemory ? SVDS_ERR_OOM : SVDS_ERR_HIP,       \
                          std::string(#call) + ": " + hipGetErrorString(e_));           \
  } while (0)

#define SVDS_LAUNCH_CHECK() SVDS_HIP(hipGetLastError())

// runs f and turns exceptions into status codes (no exception crosses the ABI)
template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Error& e) {
    if (std::getenv("SVDS_DEBUG")) std::fprintf(stderr, "[svds] error %d: %s\n", e.code, e.what());
    return e.code;
  } catch (const std::bad_alloc&) {
    return SVDS_ERR_OOM;
  } catch (...) {
    return SVDS_ERR_HIP;
  }
}

// the library's stream-ordered memory pool on the current device: created on
// first use with no release threshold, so memory freed at the end of a call
// stays in the pool for the next call instead of going back to the driver
hipMemPool_t device_pool();

// Stream-ordered device blocks with reuse: a block released on stream s is
// kept (up to a byte cap) and handed out again for a request of the same size
// on the same stream, where every earlier use of it is already ordered before
// the new one.  Repeated calls with the same shapes then neither allocate nor
// free (a stream-ordered free costs the host about 0.1 ms).
void* stream_alloc(size_t bytes, hipStream_t s);
void stream_free(void* p, hipStream_t s);
// release every block the cache keeps for stream s (before s is destroyed)
void stream_cache_drop(hipStream_t s);
// device scratch on a stream, returned to the stream-ordered cache when the
// scope ends, also when an error unwinds it
struct StreamScratch {
  void* p;
  hipStream_t s;
  StreamScratch(size_t bytes, hipStream_t st) : p(stream_alloc(bytes, st)), s(st) {}
  ~StreamScratch() { stream_free(p, s); }
  StreamScratch(const StreamScratch&) = delete;
  StreamScratch& operator=(const StreamScratch&) = delete;
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};
// small pinned host blocks (the solvers' control and status records), kept
// for reuse per (device, size, flags): hipHostMalloc and hipHostFree are slow
// and synchronise, which a batch of solves would otherwise pay per solver.
// A block is zeroed when it is handed out.
void* host_record_get(size_t bytes, unsigned flags);
void host_record_put(void* p, size_t bytes, unsigned flags);

// stream-ordered device allocations released together at the end of a call
template <typename T>
T* dalloc(size_t n, hipStream_t s) {
  if (n == 0) n = 1;
  return static_cast<T*>(stream_alloc(sizeof(T) * n, s));
}

// Device arrays of one call.  By default each comes from the stream-ordered
// block cache and is released when the object ends.  With use_workspace()
// they are carved, 256-byte aligned and in request order, from a caller's
// workspace instead (nothing is allocated or released); with count_only set
// nothing is handed out and `used` only sums the aligned sizes (the size
// query of the caller's workspace).
struct DeviceBuffers {
  std::vector<void*> ptrs;
  hipStream_t s;
  char* base = nullptr;  // caller workspace, or null
  size_t cap = 0;        // its size in bytes
  size_t used = 0;       // bytes handed out from it (or counted)
  bool count_only = false;
  void* owned = nullptr;  // one block of the stream-ordered cache holding every array
  explicit DeviceBuffers(hipStream_t st) : s(st) {}
  void use_workspace(void* p, size_t bytes) {
    base = static_cast<char*>(p);
    cap = bytes;
    used = 0;
  }
  // every array from one block of `bytes` taken from the stream-ordered
  // cache (one allocation and one free per solve instead of one per array)
  void own(size_t bytes) {
    owned = stream_alloc(bytes, s);
    use_workspace(owned, bytes);
  }
  template <typename T>
  T* get(size_t n) {
    if (base || count_only) {
      const size_t off = (used + 255) & ~static_cast<size_t>(255);
      used = off + sizeof(T) * n;
      if (count_only) return nullptr;
      if (used > cap) throw Error(SVDS_ERR_ARG, "workspace smaller than the solve needs");
      return reinterpret_cast<T*>(base + off);
    }
    T* p = dalloc<T>(n, s);
    ptrs.push_back(p);
    return p;
  }
  ~DeviceBuffers() {
    for (void* p : ptrs) stream_free(p, s);
    stream_free(owned, s);
  }
};

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kMaxBasis = 64;      // g <= 64 (small problems fit one workgroup)
constexpr int kMaxBlock = 8;       // b <= 8
constexpr int kSmallThreads = 256; // threads of the single-workgroup kernels

// Thresholds shared with the decisions of the method (values, not code, are
// common with the CPU reference: they are part of the method's definition).
constexpr double kEps = 2.220446049250313e-16;  // FP64 machine precision
constexpr double kBreakRatio = 1e-7;    // Cholesky pivot / column norm: dependent
constexpr double kCollapse = 1e-12;     // norm after / before projection: in span
constexpr double kPrevDrop = 1e-10;     // +k direction dropped below this norm
constexpr int kStallRestarts = 3;       // restarts without halving = stalled
constexpr double kFloorGate = 1e4;      // stalled below kFloorGate*eps*||Op||

// Counter streams of the random vectors
constexpr uint64_t kStreamInit = 0, kStreamNorm = 1, kStreamBreak = 2;

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// a value moved between the lanes of a 16-lane row by a DPP pattern
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}

// sum over aligned groups of L lanes (L a power of two, at most 64); every
// lane of a group ends with the same bits.  Inside a 16-lane row the levels
// are DPP moves (the two quad swaps, then the half-row and row mirrors, which
// pair the same partial sums as an exchange with lane i^4 and i^8); only the
// levels across rows go through lane permutes.  A group never reads lanes
// outside itself, so groups that have left a loop may sit beside it.
template <typename TV, int L>
__device__ __forceinline__ TV lane_sum(TV v) {
  if constexpr (L >= 2) v += dpp_row<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  if constexpr (L >= 4) v += dpp_row<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  if constexpr (L >= 8) v += dpp_row<0x141>(v);  // row_half_mirror
  if constexpr (L >= 16) v += dpp_row<0x140>(v);  // row_mirror
  if constexpr (L >= 32) v += __shfl_xor(v, 16, kWave);
  if constexpr (L >= 64) v += __shfl_xor(v, 32, kWave);
  return v;
}

// sum over the 64 lanes of a wavefront (every lane ends with the same bits):
// four DPP levels inside each 16-lane row, then two lane permutes across rows
__device__ __forceinline__ double wave_sum(double v) { return lane_sum<double, 64>(v); }

// Sums of NA values (a power of two, 1..64) over the 64 lanes of a
// wavefront at once, scattered over the lanes: a butterfly whose level j
// pairs every lane with a partner, keeps half of the values still carried
// (chosen by one lane bit) and adds the partner's copies of that half, so
// each level moves half as many values as the one before.  The levels run
// from the cheap DPP patterns inside a 16-lane row (row mirror, half-row
// mirror, the two quad swaps) to the two lane permutes across rows, so the
// permutes carry one value or two; a level's partner always has the same
// values left as the lane itself.  On return v[0] of lane l holds the sum of
// value rs_index<NA>(l); lanes that differ only in bits above the split
// levels hold the same bits, and rs_owner<NA>(l) picks one of them.
namespace rs_detail {
constexpr int kBit[6] = {3, 2, 1, 0, 4, 5};  // lane bit that chooses the half, per level
template <int LEVEL>
__device__ __forceinline__ double partner(double x) {
  if constexpr (LEVEL == 0) return dpp_row<0x140>(x);       // row mirror: 15 - i
  else if constexpr (LEVEL == 1) return dpp_row<0x141>(x);  // half-row mirror: 7 - i
  else if constexpr (LEVEL == 2) return dpp_row<0x4E>(x);   // quad swap: i ^ 2
  else if constexpr (LEVEL == 3) return dpp_row<0xB1>(x);   // quad swap: i ^ 1
  else if constexpr (LEVEL == 4) return __shfl_xor(x, 16, kWave);
  else return __shfl_xor(x, 32, kWave);
}
template <int LEVEL, int S, int NA>
__device__ __forceinline__ void level(double (&v)[NA], int lane) {
  if constexpr (LEVEL < 6) {
    if constexpr (S >= 2) {  // split: keep one half, add the partner's copy of it
      const bool up = (lane >> kBit[LEVEL]) & 1;
#pragma unroll
      for (int k = 0; k < S / 2; ++k) {
        const double keep = up ? v[k + S / 2] : v[k];
        const double send = up ? v[k] : v[k + S / 2];
        v[k] = keep + partner<LEVEL>(send);
      }
      level<LEVEL + 1, S / 2, NA>(v, lane);
    } else {  // one value left: a plain sum with the partner
      v[0] += partner<LEVEL>(v[0]);
      level<LEVEL + 1, 1, NA>(v, lane);
    }
  }
}
}  // namespace rs_detail

template <int NA>
__device__ __forceinline__ double wave_reduce_scatter(double (&v)[NA]) {
  static_assert(NA >= 1 && NA <= 64 && (NA & (NA - 1)) == 0, "NA: a power of two up to 64");
  rs_detail::level<0, NA, NA>(v, (int)(threadIdx.x % kWave));
  return v[0];
}
// the value whose sum lane l holds after wave_reduce_scatter<NA>
template <int NA>
__device__ __forceinline__ int rs_index(int lane) {
  int idx = 0, s = NA;
  for (int j = 0; j < 6 && s >= 2; ++j, s >>= 1)
    if ((lane >> rs_detail::kBit[j]) & 1) idx += s / 2;
  return idx;
}
// whether lane l is the one lane that reports its value (the others holding
// the same value differ from it in the bits of the levels that only added)
template <int NA>
__device__ __forceinline__ bool rs_owner(int lane) {
  int lv = 0;
  for (int s = NA; s >= 2; s >>= 1) ++lv;
  for (int j = lv; j < 6; ++j)
    if ((lane >> rs_detail::kBit[j]) & 1) return false;
  return true;
}

constexpr int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// out[a] = the sum over the wavefront's lanes of acc[a], a < NA (any count):
// reduce-scatters of up to 64 values (zero-padded to a power of two), each
// sum written once by its owner lane.  acc is consumed.
template <int NA>
__device__ __forceinline__ void wave_sums_to(double (&acc)[NA], double* out) {
  const int lane = (int)(threadIdx.x % kWave);
#pragma unroll
  for (int base = 0; base < NA; base += 64) {
    constexpr int kChunk = NA < 64 ? NA : 64;
    constexpr int NP = pow2_at_least(kChunk);
    double v[NP];
#pragma unroll
    for (int a = 0; a < NP; ++a) v[a] = (a < kChunk && base + a < NA) ? acc[(base + a < NA) ? base + a : 0] : 0.0;
    const double r = wave_reduce_scatter<NP>(v);
    const int idx = rs_index<NP>(lane);
    if (rs_owner<NP>(lane) && idx < kChunk && base + idx < NA) out[base + idx] = r;
  }
}

// MI355X dispatches consecutive workgroups round-robin over its 8 XCDs.  This
// maps the hardware block index to a logical one so that logical neighbours
// (adjacent row ranges, which share gathered vector entries) run on the same
// XCD and share its L2.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  constexpr int kXcd = 8;
  if (nblocks < kXcd || (nblocks % kXcd) != 0) return bid;
  return (bid % kXcd) * (nblocks / kXcd) + bid / kXcd;
}

// ---------------------------------------------------------------------------
// Batched launches: one launch per step of the iteration for many problems.
// For each problem p the launch runs exactly the workgroups (x, y), x < gx_p,
// y < gy_p, of that problem's own launch, with the same arguments, so every
// problem gets the same bits as from its own launches.
//
// Placement: workgroup b of a launch runs on XCD b % 8 (the dispatcher deals
// workgroups to the eight XCDs in turn), as slot b / 8 of that XCD.  The
// problems' workgroups, in problem order, are cut into eight runs of equal
// length, run x on XCD x: a problem is on one XCD, or on two or more
// neighbouring XCDs when it is large, so the data a problem re-reads (the
// block X of its sparse product, the block T of its projections) stays in
// the L2 of the XCD that reads it instead of all problems sharing every L2.
// An XCD's run is a list of segments (problem, first local workgroup,
// count); a workgroup finds its segment by binary search over the run's
// prefix counts.  Slots past the end of a run do nothing.
// ---------------------------------------------------------------------------
constexpr int kXcds = 8;

struct BTiles {
  const int* xoff;  // kXcds + 1: first segment of each XCD's run
  const int* xpre;  // nseg + kXcds: per run, 0 and the prefix of its segment counts
  const int* sp;    // nseg: problem of each segment
  const int* sf;    // nseg: its first local workgroup
  const int* gx;    // np: x extent of each problem's grid
  int np;
};

struct BTile {
  int p, x, y, gx;  // p < 0: an idle slot
};

__device__ __forceinline__ BTile batch_tile(const BTiles& t, int bid) {
  const int xc = bid % kXcds, slot = bid / kXcds;
  const int a = t.xoff[xc], n = t.xoff[xc + 1] - a;
  const int* pre = t.xpre + a + xc;  // n + 1 prefix counts of this run
  BTile r;
  if (n <= 0 || slot >= pre[n]) {
    r.p = -1;
    r.x = r.y = r.gx = 0;
    return r;
  }
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= slot) lo = mid;
    else hi = mid - 1;
  }
  r.p = t.sp[a + lo];
  r.gx = t.gx[r.p];
  const int local = t.sf[a + lo] + (slot - pre[lo]);
  r.x = local % r.gx;
  r.y = local / r.gx;
  return r;
}

// Launch arguments of one step for all problems, written to pinned host
// staging by put() (which returns their device address) and copied to device
// memory by flush(), one copy of everything put since the last flush, which
// the launcher calls right before its launch.  The staging is reused from
// the start once the stream has passed the previous round's copies (the
// caller resets it after reading the round's results).
class BatchUpload {
 public:
  BatchUpload() = default;
  BatchUpload(const BatchUpload&) = delete;
  BatchUpload& operator=(const BatchUpload&) = delete;
  ~BatchUpload();
  void init(size_t bytes, hipStream_t s);
  void reset() { used_ = sent_ = 0; }
  void flush();
  template <class T>
  const T* put(const T* v, size_t n) {
    return static_cast<const T*>(put_bytes(v, sizeof(T) * n));
  }
  // placement of a launch whose problem p has gx[p] x gy[p] workgroups;
  // returns the grid size (0: nothing to run)
  int tiles(const std::vector<int>& gx, const std::vector<int>& gy, BTiles& t);

 private:
  const void* put_bytes(const void* v, size_t bytes);
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, used_ = 0, sent_ = 0;
  hipStream_t s_ = nullptr;
};

// SplitMix64 finaliser (Steele, Lea and Flood 2014) on seed + (counter+1)*gamma;
// uniform in [-0.5, 0.5) from the top 53 bits.
__host__ __device__ __forceinline__ double counter_uniform(uint64_t seed, uint64_t stream,
                                                           uint64_t col, uint64_t row) {
  uint64_t ctr = (stream << 40) + (col << 32) + row;
  uint64_t z = seed + (ctr + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53 - 0.5;
}

// ---------------------------------------------------------------------------
// prepared matrix (device)
// ---------------------------------------------------------------------------
constexpr int kNumBins = 8;  // lanes per row 1,2,4,8,16,32,64, and 256 (workgroup)

struct Csr32 {
  int64_t rows = 0, cols = 0, nnz = 0;
  int32_t* rp = nullptr;   // rows+1
  int32_t* ci = nullptr;   // nnz
  double* val = nullptr;   // nnz
  float* val32 = nullptr;  // nnz, FP32 copy for the mixed-precision stage 1
  int32_t* binrows = nullptr;       // rows, grouped by bin, row order kept
  int64_t bin_off[kNumBins + 1] = {0};
  int merged_bin = -1;  // >= 0: one launch over all rows in natural order with the
                        // lane shape of that bin; -1: one launch per row-length bin
  int heuristic_bin = -1;  // the rule-of-thumb choice made when the bins were built
  int tuned_b = 0;         // block width the launch shape was last tuned for
  int unroll = 1;          // nonzeros per lane per step (1, 2 or 4)
  int heuristic_unroll = 1;
};

// Plan of the one-pass normal-equations product Z = A^T (A X) (k_gram.hip)
// for matrices whose blocks of R consecutive rows touch narrow column windows.
// Block b covers rows [b R, min((b+1) R, rows)) and columns [lo[b], hi[b]].
struct GramPlan {
  int R = 0;                  // rows per block (16..128); 0: no plan
  int64_t nblk = 0;           // blocks
  int64_t wsum = 0;           // total window width (rows of the partial sums)
  int32_t* lo = nullptr;      // nblk: first window column, nondecreasing
  int32_t* hi = nullptr;      // nblk: last window column (lo - 1: empty block)
  int64_t* poff = nullptr;    // nblk + 1: window offsets, the prefix of the widths
  int32_t* colptr = nullptr;  // wsum + nblk: block-local column pointers; block
                              //   b's w_b + 1 entries start at poff[b] + b
  uint16_t* cidx = nullptr;   // nnz, CSR order: the nonzero's window column
                              //   (column - lo[b], kGramColBits bits), and
                              //   above them its rank among the block's
                              //   nonzeros in the same column (rows ascending)
  int32_t* cover = nullptr;   // cols: first block whose window holds the column
                              //   (nblk: none)
};
constexpr int kGramMaxNnz = 2048;    // nonzeros per block (staged in LDS)
constexpr int kGramMaxWidth = 512;   // columns per window
constexpr int kGramColBits = 9;      // bits of a window column in GramPlan::cidx
constexpr int kGramMinRows = 16;     // finest block the windows are measured at
constexpr int kGramMaxRows = 128;    // tallest block
static_assert(kGramMaxWidth <= (1 << kGramColBits) && kGramMaxRows <= (1 << (16 - kGramColBits)),
              "a window column and a rank share 16 bits");
// whether the one-pass product moves at most 90 % of the algorithmic bytes of
// the two SpMMs for block width b (the rule of svds_matrix_normal)
bool gram_cheaper(const Csr32& A, const GramPlan& G, int b);

}  // namespace svds

struct svds_matrix {
  int64_t m = 0, n = 0, nnz = 0;  // of the caller's A
  bool transposed = false;         // true when m < n: work matrix is A^T
  svds::Csr32 A;                   // work matrix (tall): rows >= cols
  svds::Csr32 At;                  // its transpose
  double* diagC = nullptr;         // diag(A_w^T A_w) (length A.cols)
  svds::GramPlan G;                // one-pass A_w^T A_w product (G.R = 0: none)
  int device = 0;
  // launch shapes of the two products per (block width, FP32): tuned by the
  // first solve that needs them and fixed from then on, so that every solve
  // on the handle uses the same shapes (the arrays above are never written
  // after preparation; the solvers work on copies of A and At)
  mutable std::mutex shape_mu;
  mutable std::map<std::pair<int, int>, std::array<int, 4>> shapes;
  // set when the arrays were allocated stream-ordered on `owner` (the
  // internal create/solve/destroy sequence of one svds_solve call); they are
  // then released with stream-ordered frees on the same stream
  hipStream_t owner = nullptr;
  bool stream_ordered = false;
  // the device blocks every array above is carved from: the two matrices
  // with diagC, and the plan G
  void* block = nullptr;
  void* gram_block = nullptr;
};

namespace svds {

// ---------------------------------------------------------------------------
// launchers (kernels live in the k_*.hip files)
// ---------------------------------------------------------------------------
// setup
void check_csr(const svds_csr& A, int* d_flag, hipStream_t s);
void rowptr_to32(const int64_t* rp, int32_t* rp32, int64_t m, hipStream_t s);
void copy_csr_arrays(const svds_csr& A, Csr32& out, hipStream_t s);
void transpose_csr(const Csr32& A, Csr32& T, int32_t* d_tmp_cursor, hipStream_t s);
void build_bins(Csr32& A, hipStream_t s);
void row_sqnorms(const Csr32& A, double* out, hipStream_t s);
void to_fp32(const double* in, float* out, int64_t n, hipStream_t s);
void exclusive_scan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s);
void fill_random(double* X, int64_t ld, int64_t N, int ncols, uint64_t seed, uint64_t stream,
                 int col0, hipStream_t s);

// SpMM launch-shape autotuner: times the candidate shapes for block width b
// and keeps the fastest (cached per matrix signature for the process)
void autotune_spmm(Csr32& A, int b, bool fp32, hipStream_t s);

// SpMM: Y (rows x b, row-major) = A X (cols x b, row-major)
void spmm(const Csr32& A, int b, const double* X, double* Y, hipStream_t s);
// one-pass normal-equations product (k_gram.hip)
void gram_windows(const Csr32& A, int64_t nblk, int32_t* lo, int32_t* hi, int32_t* nnzb,
                  hipStream_t s);
void gram_build(const Csr32& A, const GramPlan& G, hipStream_t s);
// P: workspace of G.wsum * b doubles (the windows' partial sums); Z of the
// combine: row-major (ldz = 0) or column-major with leading dimension ldz
void gram_partial(const Csr32& A, const GramPlan& G, int b, const double* X, double* P,
                  hipStream_t s);
void gram_combine(const GramPlan& G, int64_t cols, int b, const double* P, double* Z,
                  int64_t ldz, hipStream_t s);
void spmm_f32(const Csr32& A, int b, const float* X, float* Y, hipStream_t s);

// dense tall-skinny (column-major).  Basis segments may be stored in FP64 or
// FP32 (mixed-precision stage 1); the arithmetic is FP64 throughout.
template <typename TB>
struct SegT {
  const TB* p;
  int ncols;
  int64_t ld;
};
using Seg = SegT<double>;
using Seg32 = SegT<float>;
int reduce_blocks(int64_t N);
// out[o] = sum over blocks of P[o * nblk + block]  (fixed order); with a
// device flag *skip != 0 the outputs are zero (the producing pass was skipped)
void reduce_partials(const double* P, int nblk, int nout, double* out, hipStream_t s,
                     const int* skip = nullptr);
// C ((sum of seg cols) x b, col-major, ld = total) = [segs]^T T; a non-null
// skip points to a device flag that, when set, turns the pass into C = 0
template <typename TB>
void tsgemm_tn(const SegT<TB>* segs, int nseg, int64_t N, const double* T, int64_t ldt, int b,
               double* partial, double* C, hipStream_t s, const int* skip = nullptr);
// the same product left as per-workgroup partial sums, partial[o * nblk + block]
// with o = c * total + col; returns nblk (the consumer reduces them)
int tsgemm_tn_partial(const Seg* segs, int nseg, int64_t N, const double* T, int64_t ldt, int b,
                      double* partial, hipStream_t s);
// T -= [segs] C   (C: total x b, column-major with leading dimension ldc);
// nothing when the device flag *skip is set.  With dgks_out, C also holds the
// block's own Gram matrix in rows total.. (the first Gram-Schmidt pass), and
// *dgks_out receives the second-pass test: 1 (skip the second pass) when
// every column kept at least 1/sqrt(2) of its norm, ||c_j||^2 <= G_jj / 2
template <typename TB>
void ts_update(const SegT<TB>* segs, int nseg, int64_t N, const double* C, int ldc, double* T,
               int64_t ldt, int b, hipStream_t s, const int* skip = nullptr,
               int* dgks_out = nullptr);
// Out (N x nout) = Q (N x nq) Y (nq x nout, ld ldy); Out may not alias Q
template <typename TI, typename TO>
void ts_gemm_nn(const TI* Q, int64_t ldq, int nq, int64_t N, const double* Y, int64_t ldy,
                int nout, TO* Out, int64_t ldo, hipStream_t s);
template <typename TI, typename TO>
void copy_cols_cvt(const TI* A, int64_t lda, int64_t N, int b, TO* B, int64_t ldb, TO* compact,
                   hipStream_t s);
void unpack_rows_f32(const float* compact, int64_t N, int b, float* A, int64_t lda,
                     hipStream_t s);
// H columns of the mixed-precision stage 1: [V]^T W (FP32 storage) with BF16
// MFMA products (hi/lo split) accumulated in FP32, partials summed in FP64
void proj_bf16x3(const float* V, int64_t ldv, int nv, const float* W, int64_t ldw, int nb,
                 int64_t N, double* partial, double* C, hipStream_t s);
// T <- T Rinv (b x b upper), optionally also writes a row-major copy
void ts_scale(double* T, int64_t ldt, int64_t N, int b, const double* Rinv, double* compact,
              hipStream_t s);
// one Cholesky QR step: G = T^T T from the partial sums P (P[o * nblk + k],
// o = c * b + c2), R = chol(G) with the breakdown tests (which = 1: first
// factor, checked against the squared pre-projection norms G0[j * ldg0 + j],
// starts *bad; which = 2: adds to *bad), R and R^-1 stored, T <- T R^-1
// (optionally also row-major into compact) and, when Pout is given, the
// partial sums of the new T's Gram matrix in Pout; returns their count
int cholqr_step(const double* P, int nblk, int which, const double* G0, int ldg0, double* R,
                double* Rinv, int* bad, double* T, int64_t ldt, int64_t N, int b,
                double* compact, double* Pout, hipStream_t s);
// the most partial sums cholqr_step leaves per Gram entry
constexpr int kCholQRMaxBlocks = 256;
// fused residual for nc candidates: R = W Y - V Y diag(theta); per-candidate
// sums (rows < nsplit | rows >= nsplit): ||r||^2, x.r, ||x||^2 each
// (sums = nullptr: the partial sums stay in `partial` as [output][block] and
// the caller reduces them).  Returns the number of blocks.
template <typename TB>
int ts_residual(const TB* V, const TB* W, int64_t ld, int64_t N, int64_t nsplit, int g,
                const double* Y, int64_t ldy, const double* theta, int nc, double* R,
                int64_t ldr, double* partial, double* sums, hipStream_t s);
void pack_rows(const double* A, int64_t lda, const double* B, double beta, int64_t N, int b,
               double* compact, hipStream_t s);  // compact = A + beta*B (B may be null)
void unpack_rows(const double* compact, int64_t N, int b, double* A, int64_t lda, hipStream_t s);
// T[:, j] = R[:, blk[j]] * dinv  (dinv may be null); blk on device
void gather_precond(const double* R, int64_t ldr, const int* d_blk, int nb, const double* dinv,
                    int64_t N, double* T, int64_t ldt, hipStream_t s);
// out = 1 / d elementwise (1 where d <= 0)
void invert_diag(const double* d, int64_t n, double* out, hipStream_t s);
void scale_rows(double* T, int64_t ldt, int64_t N, int b, const double* dinv, hipStream_t s);
void copy_cols(const double* A, int64_t lda, int64_t N, int b, double* B, int64_t ldb,
               hipStream_t s);

// ---- batched steps: one launch for all jobs, each job computed exactly as
// the single launch above would compute it (same workgroups, same sums)
struct BatchProj {  // tsgemm_tn (C = null: partial sums only)
  Seg segs[3];
  int nseg;
  int64_t N;
  const double* T;
  int64_t ldt;
  double* partial;
  double* C;
  const int* skip;
};
// nblk[j]: workgroups of job j (the partial sums' block count)
void tsgemm_tn_batch(int b, const std::vector<BatchProj>& jobs, std::vector<int>& nblk,
                     BatchUpload& up, hipStream_t s);
struct BatchReduce {
  const double* P;
  int nblk, nout;
  double* out;
  const int* skip;
};
void reduce_partials_batch(const std::vector<BatchReduce>& jobs, BatchUpload& up, hipStream_t s);
struct BatchUpdate {
  Seg segs[3];
  int nseg;
  int64_t N;
  const double* C;
  int ldc;
  double* T;
  int64_t ldt;
  const int* skip;
  int* dgks_out;
};
void ts_update_batch(int b, const std::vector<BatchUpdate>& jobs, BatchUpload& up, hipStream_t s);
struct BatchGemm {
  const double* Q;
  int64_t ldq;
  int nq;
  int64_t N;
  const double* Y;
  int64_t ldy;
  int nout;
  double* Out;
  int64_t ldo;
};
void ts_gemm_nn_batch(const std::vector<BatchGemm>& jobs, BatchUpload& up, hipStream_t s);
struct BatchScale {
  double* T;
  int64_t ldt, N;
  const double* Rinv;
  double* compact;
};
void ts_scale_batch(int b, const std::vector<BatchScale>& jobs, BatchUpload& up, hipStream_t s);
struct BatchCholQR {  // cholqr_step
  const double* P;
  int nblk, which;
  const double* G0;
  int ldg0;
  double* R;
  double* Rinv;
  int* bad;
  double* T;
  int64_t ldt, N;
  double* compact;
  double* Pout;
};
// nblk[j]: the partial sums job j leaves in its Pout
void cholqr_batch(int b, const std::vector<BatchCholQR>& jobs, std::vector<int>& nblk,
                  BatchUpload& up, hipStream_t s);
struct BatchResid {  // one sum per candidate (nsplit = N)
  const double* V;
  const double* W;
  int64_t ld, N;
  int g;
  const double* Y;
  int64_t ldy;
  const double* theta;
  int nc;
  double* R;
  int64_t ldr;
  double* partial;
  double* sums;
};
void ts_residual_batch(const std::vector<BatchResid>& jobs, BatchUpload& up, hipStream_t s);
struct BatchGather {
  const double* R;
  int64_t ldr;
  const int* blk;
  const double* dinv;
  int64_t N;
  double* T;
  int64_t ldt;
};
void gather_batch(int nb, const std::vector<BatchGather>& jobs, BatchUpload& up, hipStream_t s);
struct BatchUnpack {
  const double* compact;
  int64_t N;
  double* A;
  int64_t lda;
};
void unpack_batch(int nb, const std::vector<BatchUnpack>& jobs, BatchUpload& up, hipStream_t s);
// the products of jobs whose matrices share one merged launch shape (lanes
// per row, nonzeros per step): Y = A X, row-major blocks of b columns
struct BatchSpmm {
  const Csr32* A;
  const double* X;
  double* Y;
};
void spmm_batch(int b, const std::vector<BatchSpmm>& jobs, BatchUpload& up, hipStream_t s);

// Jacobi-Davidson correction of the second stage: per-column symmetric-QMR state
struct JdCol {
  double tau0, tau, theta, rho;  // |rhs|, quasi-residual norm, smoothing, r.Pr
  double dcoef, acoef, beta;     // coefficients of the current update
  int done, apply;
};
// out[j] = X_j . Y_j (Y null: X_j . X_j) for nb column pairs
void jd_col_dots(const double* X, const double* Y, int64_t ld, int64_t N, int nb, double* partial,
                 double* out, hipStream_t s);
// state from ||r_0||^2 (n2) and r_0 . t_0 (rho0; null: n2); q = t_0, d = x = 0
void jd_start(int64_t N, int nb, int64_t ld, const double* t, const double* n2,
              const double* rho0, JdCol* st, double* q, double* d, double* x, hipStream_t s);
// w = (B q)_compact - s_j q; the product in FP64 or, from the FP32 operator
// of the mixed-precision correction, in FP32 (widened before the shift)
void jd_shift(int64_t N, int nb, const double* Wc, const double* q, int64_t ld,
              const double* shift, double* w, hipStream_t s);
void jd_shift(int64_t N, int nb, const float* Wc, const double* q, int64_t ld,
              const double* shift, double* w, hipStream_t s);
// c (row-major N x nb, FP32) = q (column-major, leading dimension ld), rounded
void jd_pack_f32(const double* q, int64_t ld, int64_t N, int nb, float* c, hipStream_t s);
// r -= alpha w, the scalar step, d and x; then q = r + beta q (t null) or t = r
void jd_step(int64_t N, int nb, int64_t ld, double* r, const double* w, double* q, double* d,
             double* x, double* t, const double* sigma, double* rn2, double tol, JdCol* st,
             double* partial, hipStream_t s);
// preconditioned continuation: beta = rho'/rho, q = t + beta q
void jd_precond_step(int64_t N, int nb, int64_t ld, const double* rho_next, const double* t,
                     double* q, JdCol* st, hipStream_t s);

// block-Jacobi preconditioner of C: K holds ceil(N/nb) blocks of nb x nb
void bj_setup(const svds_matrix* M, int nb, double* K, hipStream_t s);
void bj_apply(const double* K, int nb, int64_t N, int b, const double* R, int64_t ldr, double* T,
              int64_t ldt, hipStream_t s);

// small single-workgroup kernels (all on device, FP64)
struct SmallState;  // defined in small.h
}  // namespace svds
