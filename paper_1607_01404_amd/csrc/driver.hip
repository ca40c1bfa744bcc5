// Host driver of the two-stage hybrid SVD (Algorithm 1) and the C ABI.
//
// Everything numerical runs in the library's kernels on one GPU; the host
// enqueues them on the caller's stream and reads back one small decision
// record per iteration (the Ctl struct written by the control kernel), plus a
// breakdown flag after each block orthogonalisation.
#include <atomic>
#include <map>
#include <memory>
#include <functional>
#include <mutex>
#include <chrono>
#include <thread>
#include <utility>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <vector>

#include "lpc.h"
#include "small.h"

namespace svds {

// launchers defined in k_dense.hip / k_final.hip
void col_residual2(const double* A, int64_t lda, const double* B, int64_t ldb, const double* sc,
                   int64_t N, int k, double* partial, double* out, hipStream_t s);
void col_scale(double* X, int64_t ld, int64_t N, int k, const double* f, hipStream_t s);
void sign_factors(const double* V, int64_t ldv, int64_t N, int k, double* partial, double* f,
                  hipStream_t s);
void sigma_from_lambda(int k, const double* lam, double* sig, double* inv, hipStream_t s);
void stage1_check(int k, const double* rl2, const double* rr2, const double* sig, double normA,
                  double tol, int rel, double* rn, double* taus, int* ok, hipStream_t s);
void sqrt_sum(int k, const double* a, const double* b, double* out, hipStream_t s);
void inv_sqrt(int k, const double* x, double* f, hipStream_t s);
void abs_vec(int k, const double* x, double* y, hipStream_t s);
void cleanup_finish(int k, const double* s, const double* Yq, int ldy, const double* AVq,
                    int ldav, int descending, double* sig, double* P, double* Q, int ldk,
                    hipStream_t st);

// the one-pass product (partial sums, then their per-column sums) against A
// then A^T by two SpMMs, in algorithmic bytes; taken when it moves at most
// 90 % of the two products' bytes
bool gram_cheaper(const Csr32& A, const GramPlan& G, int b) {
  const double fused = 10.0 * (double)A.nnz + 4.0 * (double)(A.rows + 1) + 8.0 * b * (double)A.cols +
                       (4.0 + 8.0 * b) * (double)G.wsum + 20.0 * (double)G.nblk +
                       8.0 * b * (double)G.wsum + (4.0 + 8.0 * b) * (double)A.cols;
  const double two = 24.0 * (double)A.nnz + 4.0 * (double)(A.rows + A.cols + 2) +
                     16.0 * b * (double)(A.rows + A.cols);
  return fused <= 0.9 * two;
}

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// the method's bytes of one product Z = A^T (A X) on n x b blocks: A read
// once in CSR (values, 32-bit column indices, row pointers), X read and Z
// written once.  The one-pass product reads a 16-bit window column and rank
// per nonzero in place of the column index; its other plan data (window
// column pointers, the windows' partial sums) is overhead, not counted here.
double gram_method_bytes(const Csr32& A, int b) {
  return 12.0 * (double)A.nnz + 4.0 * (double)(A.rows + 1) + 16.0 * b * (double)A.cols;
}


}  // namespace

hipMemPool_t device_pool() {
  static std::mutex mu;
  static std::map<int, hipMemPool_t> pools;
  int dev = 0;
  SVDS_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(mu);
  auto it = pools.find(dev);
  if (it != pools.end()) return it->second;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  hipMemPool_t pool = nullptr;
  SVDS_HIP(hipMemPoolCreate(&pool, &props));
  uint64_t keep = UINT64_MAX;
  SVDS_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
  pools[dev] = pool;
  return pool;
}

namespace {
constexpr size_t kCacheCap = (size_t)16 << 30;  // bytes kept for reuse, all streams together
struct BlockCache {
  std::mutex mu;
  std::map<std::pair<hipStream_t, size_t>, std::vector<void*>> free;  // (stream, bytes) -> blocks
  std::map<void*, size_t> size;                                        // every live block
  size_t cached = 0;
};
BlockCache& block_cache() {
  static BlockCache* c = new BlockCache();  // kept to the end of the process
  return *c;
}
}  // namespace

void* stream_alloc(size_t bytes, hipStream_t s) {
  BlockCache& c = block_cache();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.free.find({s, bytes});
    if (it != c.free.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      c.cached -= bytes;
      return p;
    }
  }
  void* p = nullptr;
  SVDS_HIP(hipMallocFromPoolAsync(&p, bytes, device_pool(), s));
  std::lock_guard<std::mutex> lk(c.mu);
  c.size[p] = bytes;
  return p;
}

void stream_free(void* p, hipStream_t s) {
  if (!p) return;
  BlockCache& c = block_cache();
  {
    std::lock_guard<std::mutex> lk(c.mu);
    auto it = c.size.find(p);
    const size_t bytes = it != c.size.end() ? it->second : 0;
    if (bytes && c.cached + bytes <= kCacheCap) {
      c.free[{s, bytes}].push_back(p);
      c.cached += bytes;
      return;
    }
    if (it != c.size.end()) c.size.erase(it);
  }
  (void)hipFreeAsync(p, s);
}

namespace {
struct HostRecords {
  std::mutex mu;
  std::map<std::tuple<int, size_t, unsigned>, std::vector<void*>> free;
};
HostRecords& host_records() {
  static HostRecords* r = new HostRecords;  // lives until the process ends
  return *r;
}
constexpr size_t kHostRecordsKept = 4096;  // blocks kept per (device, size, flags)
}  // namespace

void* host_record_get(size_t bytes, unsigned flags) {
  int dev = 0;
  SVDS_HIP(hipGetDevice(&dev));
  void* p = nullptr;
  {
    HostRecords& r = host_records();
    std::lock_guard<std::mutex> lk(r.mu);
    auto it = r.free.find({dev, bytes, flags});
    if (it != r.free.end() && !it->second.empty()) {
      p = it->second.back();
      it->second.pop_back();
    }
  }
  if (!p) SVDS_HIP(hipHostMalloc(&p, bytes, flags));
  std::memset(p, 0, bytes);
  return p;
}

void host_record_put(void* p, size_t bytes, unsigned flags) {
  if (!p) return;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    HostRecords& r = host_records();
    std::lock_guard<std::mutex> lk(r.mu);
    std::vector<void*>& v = r.free[{dev, bytes, flags}];
    if (v.size() < kHostRecordsKept) {
      v.push_back(p);
      return;
    }
  }
  (void)hipHostFree(p);
}

void stream_cache_drop(hipStream_t s) {
  BlockCache& c = block_cache();
  std::vector<void*> drop;
  {
    std::lock_guard<std::mutex> lk(c.mu);
    for (auto it = c.free.begin(); it != c.free.end();) {
      if (it->first.first != s) {
        ++it;
        continue;
      }
      for (void* p : it->second) {
        drop.push_back(p);
        c.cached -= it->first.second;
        c.size.erase(p);
      }
      it = c.free.erase(it);
    }
  }
  for (void* p : drop) (void)hipFreeAsync(p, s);
}

// ---------------------------------------------------------------------------
// The solver state of one svds call
// ---------------------------------------------------------------------------
class Solver {
 public:
  // a, at: the solve's copies of the work matrix and its transpose with the
  // FP64 launch shapes; a32, at32: the same with the FP32 shapes
  Solver(const svds_matrix* M, const Csr32& a, const Csr32& at, const Csr32& a32,
         const Csr32& at32, int k, int target, double tol, const svds_opts& o, hipStream_t s)
      : M_(M), A_(a), At_(at), A32_(a32), At32_(at32), k_(k), target_(target), tol_(tol), o_(o),
        s_(s), buf_(s) {
    m_ = M->A.rows;
    n_ = M->A.cols;
    largest_ = target == SVDS_LARGEST;
    g_ = o.max_basis_size;
    r_ = o.min_restart_size;
    if (g_ <= 0 || r_ <= 0) {
      const bool small = largest_ && k < 10;
      if (g_ <= 0) g_ = small ? 15 : 35;
      if (r_ <= 0) r_ = small ? 6 : 14;
    }
    b_ = o.block_size > 0 ? o.block_size : 1;
    p_ = o.max_prev_retain >= 0 ? o.max_prev_retain : b_;
    budget_ = o.max_matvecs > 0 ? o.max_matvecs : 2000000;
    tol1_ = o.stage1_tol > 0 ? o.stage1_tol : tol;
    if (b_ > kMaxBlock || g_ > kGmax || k > kKmax || g_ < r_ + p_ + b_ || g_ < k + b_ || r_ < 1 ||
        p_ < 0)
      throw Error(SVDS_ERR_ARG, "basis parameters out of range");
    if (std::min<int64_t>(g_, n_) < k + b_)
      throw Error(SVDS_ERR_ARG, "k + block size exceeds the smaller dimension or the basis");
  }
  ~Solver() {
    for (hipEvent_t e : evpool_) (void)hipEventDestroy(e);
    host_record_put(hctl_, kCtlBytes, kCtlFlags);
    host_record_put(hbad_, sizeof(int), hipHostMallocDefault);
    host_record_put(hjd_, sizeof(JdCol) * kMaxBlock, hipHostMallocDefault);
  }
  Solver(const Solver&) = delete;
  Solver& operator=(const Solver&) = delete;

  int run(double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
          svds_stats* st);
  void prepare(svds_stats* st);
  int complete(double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
               svds_stats* st, bool stage1_done);

  // every device array of the solve, from `a` (the block cache, a caller's
  // workspace, or a count of the bytes); no launch
  void allocate(DeviceBuffers& a);
  // bytes of a caller workspace that holds them
  size_t workspace_bytes() {
    DeviceBuffers c(s_);
    c.count_only = true;
    allocate(c);
    return c.used + 256;  // room to align the workspace's start
  }
  // carve the arrays from a caller's workspace instead of the block cache
  void use_workspace(void* p, size_t bytes) {
    const uintptr_t a = ((uintptr_t)p + 255) & ~(uintptr_t)255;
    const size_t skip = a - (uintptr_t)p;
    if (bytes < skip) throw Error(SVDS_ERR_ARG, "workspace smaller than the solve needs");
    buf_.use_workspace((void*)a, bytes - skip);
  }

  // stage-1 residuals of the block's first target at every `every`-th
  // iteration (training pairs of the learned preconditioner)
  struct Capture {
    int every = 1, max = 0, count = 0;
    double* R = nullptr;
    int64_t ldr = 0;
  };
  void set_capture(Capture* c) { cap_ = c; }

 private:
  Capture* cap_ = nullptr;
  // Jacobi-Davidson second stage
  bool jd_ = false;
  double *jdXb_ = nullptr, *jdR_ = nullptr, *jdQ_ = nullptr, *jdW_ = nullptr, *jdD_ = nullptr;
  double *jdT_ = nullptr, *jdC_ = nullptr, *jdShift_ = nullptr;
  double *jdN2_ = nullptr, *jdSig_ = nullptr, *jdRn2_ = nullptr, *jdRho_ = nullptr;
  JdCol* jdSt_ = nullptr;
  JdCol* hjd_ = nullptr;  // pinned
  void jd_project(double* Z, int nb) {
    count(N8() * (2 * nlock_ + 5 * nb));
    Seg q[2] = {Seg{X_, nlock_, ld_}, Seg{jdXb_, nb, ld_}};
    tsgemm_tn(q, 2, N_, Z, ld_, nb, partial_, jdC_, s_);
    ts_update(q, 2, N_, jdC_, nlock_ + nb, Z, ld_, nb, s_);
  }
  // T (N_ x nb) <- approximate solutions of the correction equations of the
  // block (symmetric QMR from zero with the projected stage-2
  // preconditioner); the Ritz vectors jdXb_ and shifts jdShift_ are set
  void jd_correct(double* T, int nb) {
    const bool pc = o_.precond != SVDS_PC_NONE;
    count(N8() * nb * (3.0 + (pc ? 4.0 : 0.0) + 4.0));
    gather_precond(R_, ld_, d_->blk, nb, nullptr, N_, jdR_, ld_, s_);
    jd_project(jdR_, nb);
    jd_col_dots(jdR_, nullptr, ld_, N_, nb, partial_, jdN2_, s_);
    if (pc) {
      copy_cols(jdR_, ld_, N_, nb, jdT_, ld_, s_);
      apply_pcB(jdT_, nb);
      jd_project(jdT_, nb);
      jd_col_dots(jdR_, jdT_, ld_, N_, nb, partial_, jdRho_, s_);
    }
    jd_start(N_, nb, ld_, pc ? jdT_ : jdR_, jdN2_, pc ? jdRho_ : nullptr, jdSt_, jdQ_, jdD_, T,
             s_);
    const int maxit = o_.jd_max_inner > 0 ? o_.jd_max_inner : 20;
    const double tol = o_.jd_inner_tol > 0.0 ? o_.jd_inner_tol : 0.1;
    for (int it = 0; it < maxit; ++it) {
      // packing, the shifted product, the dots, the QMR step (and with a
      // preconditioner its dots and continuation)
      count(N8() * nb * (2.0 + 3.0 + 2.0 + 9.0 + (pc && it + 1 < maxit ? 5.0 : 0.0)));
      if (jd32_) {  // the product with B through the FP32 copies of A and A^T
        jd_pack_f32(jdQ_, ld_, N_, nb, Tc32_, s_);
        timed_spmm(At(), nb, Tc32_ + n_ * nb, Wc32_);  // v-half: A^T x_u
        timed_spmm(A(), nb, Tc32_, Wc32_ + n_ * nb);   // u-half: A x_v
        mv_ += 2 * nb;
        jd_shift(N_, nb, Wc32_, jdQ_, ld_, jdShift_, jdW_, s_);
      } else {
        pack_rows(jdQ_, ld_, nullptr, 0.0, N_, nb, Tc_, s_);
        apply_op(Tc_, Wc_, nb);
        jd_shift(N_, nb, Wc_, jdQ_, ld_, jdShift_, jdW_, s_);
      }
      jd_project(jdW_, nb);
      jd_col_dots(jdQ_, jdW_, ld_, N_, nb, partial_, jdSig_, s_);
      jd_step(N_, nb, ld_, jdR_, jdW_, jdQ_, jdD_, T, pc ? jdT_ : nullptr, jdSig_, jdRn2_, tol,
              jdSt_, partial_, s_);
      ++jd_inner_;
      if (pc && it + 1 < maxit) {
        apply_pcB(jdT_, nb);
        jd_project(jdT_, nb);
        jd_col_dots(jdR_, jdT_, ld_, N_, nb, partial_, jdRho_, s_);
        jd_precond_step(N_, nb, ld_, jdRho_, jdT_, jdQ_, jdSt_, s_);
      }
      if ((it + 1) % 4 == 0 && it + 1 < maxit) {
        SVDS_HIP(hipMemcpyAsync(hjd_, jdSt_, sizeof(JdCol) * nb, hipMemcpyDeviceToHost, s_));
        SVDS_HIP(hipStreamSynchronize(s_));
        bool all = true;
        for (int j = 0; j < nb; ++j) all = all && hjd_[j].done;
        if (all) break;
      }
    }
  }
  int64_t jd_inner_ = 0;
  // mixed precision, largest values: the correction equation's products with
  // B use the FP32 copies of A and A^T.  The shifts lie far from zero there,
  // so the FP32 rounding of B (relative 6e-8) is small against the inner
  // solve's own target (a reduction of 0.1); the outer residuals, the
  // Rayleigh-Ritz step and every convergence test stay FP64.
  bool jd32_ = false;
  // block-Jacobi preconditioner: inverses of the diagonal blocks of C
  double* bjK_ = nullptr;
  int bjnb_ = 0;
  // learned preconditioner
  bool learned_ = false;
  int ldeg_ = 0;
  LpcOp lop_;
  float* lcoef_ = nullptr;
  LpcScratch lsc_;
  void setup_learned();
  // T (N_ x nb, column-major, stage 1) <- K T
  void learned_apply(double* T, int nb) {
    lpc_apply(lop_, lcoef_, ldeg_, nb, T, ld_, T, ld_, lsc_, s_);
    mv_ += 2 * (int64_t)ldeg_ * nb;
  }
  void capture_residual(int64_t iters, const Ctl& c);

  // ---- configuration
  const svds_matrix* M_;
  const Csr32 A_, At_, A32_, At32_;  // descriptors with this solve's launch shapes
  int k_, target_;
  double tol_, tol1_;
  svds_opts o_;
  hipStream_t s_;
  DeviceBuffers buf_;
  int64_t m_, n_;
  bool largest_;
  int g_, r_, b_, p_;
  int64_t budget_;
  double run_t0_ = 0.0;  // start of run(), for the wall-clock budget
  bool over_budget() const {
    return mv_ >= budget_ || (o_.max_seconds > 0.0 && now() - run_t0_ > o_.max_seconds);
  }
  double normA_ = 0.0;

  // ---- per-stage state
  int stage_ = 1;
  int64_t N_ = 0;      // operator dimension
  int gc_ = 0;         // basis size
  int nlock_ = 0;
  bool refined_ = false;
  double tau_ = 0.0;
  int64_t ld_ = 0;     // leading dimension of the basis arrays
  int rand_count_ = 0;
  int64_t mv_ = 0;     // matrix-vector products (columns times A or A^T)
  int64_t breakdowns_ = 0;

  // ---- device buffers
  double *V_ = nullptr, *W_ = nullptr, *Vt_ = nullptr, *Wt_ = nullptr;
  double *Q_ = nullptr, *Qt_ = nullptr, *X_ = nullptr, *R_ = nullptr, *Z_ = nullptr;
  double *Tc_ = nullptr, *Yc_ = nullptr, *Wc_ = nullptr, *Zc_ = nullptr;
  double* partial_ = nullptr;
  double* cqrP_ = nullptr;  // Gram partial sums between the two Cholesky QR steps
  double* dinv_ = nullptr;  // 1 / diag(A^T A) (ones where zero)
  Small* d_ = nullptr;
  // the control record and the sequence word after it, in pinned coherent
  // host memory mapped for the device
  static constexpr size_t kSeqOff = (sizeof(Ctl) + 63) / 64 * 64;
  static constexpr size_t kCtlBytes = kSeqOff + 64;
  static constexpr unsigned kCtlFlags = hipHostMallocMapped | hipHostMallocCoherent;
  Ctl* hctl_ = nullptr;     // pinned, coherent
  Ctl* dctl_ = nullptr;     // its device address
  int* hseq_ = nullptr;     // sequence word beside the record (pinned, coherent)
  int* dseq_ = nullptr;     // its device address
  int seq_ = 0;             // last sequence number asked of the control kernel
  int* hbad_ = nullptr;     // pinned
  double* vec_ = nullptr;   // small device vectors (k-sized)
  // stage-1 results handed to stage 2 and the clean-up
  double *V1_ = nullptr, *U1_ = nullptr, *sig_ = nullptr, *rn1_ = nullptr, *taus_ = nullptr;
  int* ok_ = nullptr;
  // mixed-precision stage 1: FP32 basis, FP64 work block, FP32 compact blocks
  float *V32_ = nullptr, *W32_ = nullptr, *Vt32_ = nullptr, *Wt32_ = nullptr;
  float *Tc32_ = nullptr, *Yc32_ = nullptr, *Wc32_ = nullptr;
  double* Tb_ = nullptr;
  bool mixed_ = false;

  // ---- operators -----------------------------------------------------------
  const Csr32& A() const { return A_; }
  const Csr32& At() const { return At_; }

  // sparse product with optional event timing.  The events only time the
  // products: they are created without the system-scope fence (a default
  // record writes back and invalidates the caches, which both costs time and
  // hands the next kernel a cold L2), kept in a pool, and read back at the
  // solver's synchronisation points, after which they are reused.
  // timed kernel classes: the SpMM, the one-pass product's partial sums, the
  // basis projections of the FP64 stage-1 iteration and its residual
  enum Timed { kTSpmm = 0, kTGram, kTProj, kTResid, kTKinds };
  struct TimedCall {
    hipEvent_t a, b;
    int kind;
  };
  struct TimedAcc {
    double seconds = 0.0, bytes = 0.0;
    int64_t calls = 0;
    uint64_t seen = 0;  // calls made, timed or not
  };
  std::vector<TimedCall> ev_;                          // recorded since the last harvest
  std::vector<hipEvent_t> evpool_;                     // every event created by this solve
  size_t evnext_ = 0;                                  // first unused event of the pool
  TimedAcc acc_[kTKinds];
  // algorithmic bytes of the streaming kernels of the iterations (every call:
  // sparse products, projections, updates, residuals, restarts, corrections)
  double algb_ = 0.0;
  void count(double bytes) { algb_ += bytes; }
  double N8() const { return 8.0 * (double)N_; }
  double* gramP_ = nullptr;  // partial sums of the one-pass product (wsum x kMaxBlock)
  // profile = 1: one call in kTimeEvery is bracketed by timing events (an
  // event record between two kernels costs a few microseconds of idle time)
  static constexpr uint64_t kTimeEvery = 4;
  // run(): the launches of one call of class `kind`; timed when its turn comes
  template <class F>
  void timed(int kind, double bytes, bool turn, F&& run) {
    if (!o_.profile || !turn) {
      run();
      return;
    }
    hipEvent_t a = pool_event(), b = pool_event();
    SVDS_HIP(hipEventRecord(a, s_));
    run();
    SVDS_HIP(hipEventRecord(b, s_));
    ev_.push_back(TimedCall{a, b, kind});
    acc_[kind].bytes += bytes;
  }
  bool turn(int kind) { return (acc_[kind].seen++ % kTimeEvery) == 0; }
  hipEvent_t pool_event() {
    if (evnext_ == evpool_.size()) {
      hipEvent_t e;
      SVDS_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      evpool_.push_back(e);
    }
    return evpool_[evnext_++];
  }
  // after a stream synchronisation: every recorded pair has completed
  void harvest_events() {
    for (auto& e : ev_) {
      float ms = 0.f;
      SVDS_HIP(hipEventSynchronize(e.b));
      SVDS_HIP(hipEventElapsedTime(&ms, e.a, e.b));
      acc_[e.kind].seconds += ms * 1e-3;
      ++acc_[e.kind].calls;
    }
    ev_.clear();
    evnext_ = 0;
  }
  static double spmm_bytes(const Csr32& Mx, int nb) {
    return (double)Mx.nnz * 12.0 + 4.0 * (double)(Mx.rows + 1) + 8.0 * nb * (double)(Mx.rows + Mx.cols);
  }
  template <typename TV>
  void timed_spmm(const Csr32& Mx, int nb, const TV* X, TV* Y) {
    auto run = [&] {
      if constexpr (std::is_same<TV, double>::value) spmm(Mx, nb, X, Y, s_);
      else spmm_f32(Mx, nb, X, Y, s_);
    };
    // both calls of every kTimeEvery-th pair (A then A^T, or the two halves
    // of B) are timed
    const bool t = ((acc_[kTSpmm].seen++ >> 1) % kTimeEvery) == 0;
    const double sv = (double)sizeof(TV);
    const double bytes = (double)Mx.nnz * (sv + 4.0) + 4.0 * (double)(Mx.rows + 1) +
                         sv * nb * (double)(Mx.rows + Mx.cols);
    count(bytes);
    timed(kTSpmm, bytes, t, run);
  }
  void collect_profile(svds_stats* st) {
    harvest_events();
    st->spmm_calls = acc_[kTSpmm].calls;
    st->spmm_seconds = acc_[kTSpmm].seconds;
    st->spmm_bytes = acc_[kTSpmm].bytes;
    st->gram_calls = acc_[kTGram].calls;
    st->gram_seconds = acc_[kTGram].seconds;
    st->gram_bytes = acc_[kTGram].bytes;
    st->proj_calls = acc_[kTProj].calls;
    st->proj_seconds = acc_[kTProj].seconds;
    st->proj_bytes = acc_[kTProj].bytes;
    st->resid_calls = acc_[kTResid].calls;
    st->resid_seconds = acc_[kTResid].seconds;
    st->resid_bytes = acc_[kTResid].bytes;
    st->alg_bytes = algb_;
  }
  // Z (n x nb) = A^T (A X) by the one-pass product, Z row-major (ldz = 0) or
  // column-major with leading dimension ldz; both kernels (the partial sums,
  // which read A, and their combine) are timed as one call
  void timed_gram(int nb, const double* X, double* Z, int64_t ldz) {
    const GramPlan& G = M_->G;
    const double bytes = gram_method_bytes(A(), nb);
    count(bytes);
    timed(kTGram, bytes, turn(kTGram), [&] {
      gram_partial(A(), G, nb, X, gramP_, s_);
      gram_combine(G, A().cols, nb, gramP_, Z, ldz, s_);
    });
  }
  bool use_gram(int nb) const {
    return o_.fused_gram && M_->G.R > 0 && gram_cheaper(A(), M_->G, nb);
  }

  // W block (compact, N x nb) = Op T block (compact)
  void apply_op(const double* Tc, double* Wc, int nb) {
    if (stage_ == 1 && use_gram(nb)) {
      timed_gram(nb, Tc, Wc, 0);  // n x nb in one pass over A
    } else if (stage_ == 1) {
      timed_spmm(A(), nb, Tc, Yc_);   // m x nb
      timed_spmm(At(), nb, Yc_, Wc);  // n x nb
    } else {
      timed_spmm(At(), nb, Tc + n_ * nb, Wc);  // v-half: A^T x_u
      timed_spmm(A(), nb, Tc, Wc + n_ * nb);   // u-half: A x_v
    }
    mv_ += 2 * nb;
  }

  // ---- orthogonalisation: CGS twice against segs, Cholesky QR twice ----------
  template <typename TB>
  int ortho_once(double* T, int64_t ldt, int nb, const SegT<TB>* segs, int nseg,
                 double* compact) {
    ortho_enqueue(T, ldt, nb, segs, nseg, compact);
    SVDS_HIP(hipMemcpyAsync(hbad_, &d_->bad, sizeof(int), hipMemcpyDeviceToHost, s_));
    SVDS_HIP(hipStreamSynchronize(s_));
    return *hbad_;
  }

  // CGS twice + CholQR twice, enqueued only; d_->bad records dependent columns
  template <typename TB>
  void ortho_enqueue(double* T, int64_t ldt, int nb, const SegT<TB>* segs, int nseg,
                     double* compact) {
    int total = 0;
    for (int i = 0; i < nseg; ++i) total += segs[i].ncols;
    SegT<TB> sb[3];
    int n1 = 0;
    for (int i = 0; i < nseg; ++i)
      if (segs[i].ncols > 0) sb[n1++] = segs[i];
    Seg st{T, nb, ldt};
    const double* G0;
    int ldg0, ldc0;
    if constexpr (std::is_same<TB, double>::value) {
      // pass 1 with the block's own Gram (pre-projection norms) appended
      Seg s1[3];
      for (int i = 0; i < n1; ++i) s1[i] = sb[i];
      s1[n1] = st;
      int nbp = 0;
      count(N8() * (total + nb));
      timed(kTProj, 8.0 * (double)N_ * (total + nb), turn(kTProj),
            [&] { nbp = tsgemm_tn_partial(s1, n1 + 1, N_, T, ldt, nb, partial_, s_); });
      reduce_partials(partial_, nbp, (total + nb) * nb, d_->C0, s_);
      G0 = d_->C0 + total;
      ldg0 = total + nb;
      ldc0 = total + nb;
    } else {
      tsgemm_tn(&st, 1, N_, T, ldt, nb, partial_, d_->G0, s_);
      if (total > 0) tsgemm_tn(sb, n1, N_, T, ldt, nb, partial_, d_->C0, s_);
      // FP32 basis: both passes always run
      count(N8() * nb + (total > 0 ? 2.0 * (4.0 * N_ * total + N8() * nb) : 0.0));
      G0 = d_->G0;
      ldg0 = nb;
      ldc0 = total;
    }
    if (total > 0) {
      // second pass only where the device-side test asks for it (FP64 basis);
      // the FP32 basis of the mixed stage always takes both passes
      const int* sk = std::is_same<TB, double>::value ? &d_->skip2 : nullptr;
      // the first update (the second pass, skipped on the device when the
      // test says so, is not counted for the FP64 basis)
      count((double)sizeof(TB) * N_ * total + 2.0 * N8() * nb);
      if (!std::is_same<TB, double>::value) count((double)sizeof(TB) * N_ * total + 2.0 * N8() * nb);
      // the first update also takes the second-pass test (FP64 basis)
      ts_update(sb, n1, N_, d_->C0, ldc0, T, ldt, nb, s_, nullptr,
                std::is_same<TB, double>::value ? &d_->skip2 : nullptr);
      tsgemm_tn(sb, n1, N_, T, ldt, nb, partial_, d_->C1, s_, sk);
      ts_update(sb, n1, N_, d_->C1, total, T, ldt, nb, s_, sk);
    }
    // Cholesky QR twice: the Gram partial sums of T, then two fused steps
    // (factor, scale, and the first also the partial sums for the second)
    count(N8() * nb * (5.0 + (compact ? 1.0 : 0.0)));
    const int nbk = tsgemm_tn_partial(&st, 1, N_, T, ldt, nb, partial_, s_);
    const int nb2 = cholqr_step(partial_, nbk, 1, G0, ldg0, d_->R1, d_->R1inv, &d_->bad, T, ldt,
                                N_, nb, nullptr, cqrP_, s_);
    cholqr_step(cqrP_, nb2, 2, nullptr, 0, d_->R2, d_->R2inv, &d_->bad, T, ldt, N_, nb, compact,
                nullptr, s_);
  }

  // repair after the control step reported a breakdown of the last block:
  // roll the block back, give its dependent columns fresh random numbers and
  // redo it synchronously
  void repair_block(int nb, int bad, const Seg* segs, int nseg) {
    gc_ -= nb;
    ++breakdowns_;
    double* T = V_ + gc_ * ld_;
    const uint64_t stream = kStreamBreak + (uint64_t)rand_count_++;
    int i = 0;
    for (int j = 0; j < nb; ++j)
      if (bad & (1 << j)) fill_random(T + j * ld_, ld_, N_, 1, o_.seed, stream, i++, s_);
    Seg sg[3];
    for (int q = 0; q < nseg; ++q) sg[q] = segs[q];
    sg[nseg - 1].ncols = gc_;  // the basis segment, rolled back
    ortho(T, ld_, nb, sg, nseg, Tc_);
    append(nb);
    extract_stage();
  }

  // with breakdown repair: dependent columns get fresh counter-based vectors
  template <typename TB>
  void ortho(double* T, int64_t ldt, int nb, const SegT<TB>* segs, int nseg, double* compact) {
    for (int attempt = 0; attempt < 4; ++attempt) {
      int bad = ortho_once(T, ldt, nb, segs, nseg, compact);
      if (!bad) return;
      ++breakdowns_;
      const uint64_t stream = kStreamBreak + (uint64_t)rand_count_++;
      int i = 0;
      for (int j = 0; j < nb; ++j)
        if (bad & (1 << j)) fill_random(T + j * ldt, ldt, N_, 1, o_.seed, stream, i++, s_);
    }
    throw Error(SVDS_ERR_BREAKDOWN, "repeated orthogonalisation breakdown");
  }

  // ---- basis expansion ---------------------------------------------------------
  // V[:, gc:gc+nb] is orthonormal and Tc_ holds it row-major
  void append(int nb) {
    double* Tcol = V_ + gc_ * ld_;
    double* Wcol = W_ + gc_ * ld_;
    if (stage_ == 1 && use_gram(nb)) {  // the combine writes W's columns directly
      timed_gram(nb, Tc_, Wcol, ld_);
      mv_ += 2 * nb;
    } else {
      apply_op(Tc_, Wc_, nb);
      unpack_rows(Wc_, N_, nb, Wcol, ld_, s_);
      count(2.0 * N8() * nb);
    }
    Seg sv{V_, gc_ + nb, ld_};
    count(N8() * (gc_ + 2 * nb));
    int nbp = 0;
    timed(kTProj, 8.0 * (double)N_ * (gc_ + 2 * nb), turn(kTProj),
          [&] { nbp = tsgemm_tn_partial(&sv, 1, N_, Wcol, ld_, nb, partial_, s_); });
    small_h_append(d_, gc_, nb, s_, partial_, nbp);  // sums the partials itself
    if (refined_) {
      // Z = W_new - tau T, orthogonalised against Q: new columns of Rr
      double* Zcol = Q_ + gc_ * ld_;
      pack_rows(Wcol, ld_, Tcol, -tau_, N_, nb, Zc_, s_);
      unpack_rows(Zc_, N_, nb, Zcol, ld_, s_);
      count(5.0 * N8() * nb);
      Seg sq{Q_, gc_, ld_};
      refined_ortho(Zcol, nb, &sq, gc_ > 0 ? 1 : 0);
      small_rr_append(d_, gc_, nb, gc_, s_);
    }
    gc_ += nb;
  }

  // orthogonalisation of a Z block for the refined factor: a dependent
  // column keeps its projection coefficients and gets a fresh orthogonal
  // direction with a zero diagonal entry
  void refined_ortho(double* Zcol, int nb, const Seg* sq, int nseg) {
    int bad = ortho_once(Zcol, ld_, nb, sq, nseg, nullptr);
    if (bad) {
      ++breakdowns_;
      throw Error(SVDS_ERR_BREAKDOWN, "refined factor breakdown");
    }
  }

  void extract_stage() {
    const int desc = (stage_ == 1) ? (largest_ ? 1 : 0) : 1;
    small_extract(d_, gc_, desc, refined_ ? 1 : 0, s_);
  }

  void restart_basis(int nr) {
    count((refined_ ? 3.0 : 2.0) * N8() * (gc_ + nr));
    ts_gemm_nn(V_, ld_, gc_, N_, d_->Yr, kLd, nr, Vt_, ld_, s_);
    ts_gemm_nn(W_, ld_, gc_, N_, d_->Yr, kLd, nr, Wt_, ld_, s_);
    std::swap(V_, Vt_);
    std::swap(W_, Wt_);
    if (refined_) {
      ts_gemm_nn(Q_, ld_, gc_, N_, d_->Qt, kLd, nr, Qt_, ld_, s_);
      std::swap(Q_, Qt_);
    }
    gc_ = nr;
  }

  // rebuild Q, Rr of (W - tau V) for the current basis (after a lock or reset)
  void rebuild_refined() {
    for (int c0 = 0; c0 < gc_; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, gc_ - c0);
      double* Zcol = Q_ + c0 * ld_;
      pack_rows(W_ + c0 * ld_, ld_, V_ + c0 * ld_, -tau_, N_, nb, Zc_, s_);
      unpack_rows(Zc_, N_, nb, Zcol, ld_, s_);
      Seg sq{Q_, c0, ld_};
      refined_ortho(Zcol, nb, &sq, c0 > 0 ? 1 : 0);
      small_rr_append(d_, c0, nb, c0, s_);
    }
  }

  // re-orthonormalise V (against locked vectors) and recompute W, H (Section 3.2)
  void reset() {
    const int gold = gc_;
    std::swap(V_, Vt_);  // old basis now in Vt_
    gc_ = 0;
    const bool was_refined = refined_;
    refined_ = false;  // the refined factor is rebuilt afterwards
    for (int c0 = 0; c0 < gold; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, gold - c0);
      double* T = V_ + gc_ * ld_;
      copy_cols(Vt_ + c0 * ld_, ld_, N_, nb, T, ld_, s_);
      Seg segs[2] = {Seg{X_, nlock_, ld_}, Seg{V_, gc_, ld_}};
      ortho(T, ld_, nb, segs, 2, Tc_);
      append(nb);
    }
    refined_ = was_refined;
    if (refined_) rebuild_refined();
  }

  void residual(int nc, int64_t nsplit) {
    int nbr = 0;
    count(N8() * (2 * gc_ + nc));
    timed(kTResid, 8.0 * (double)N_ * (2 * gc_ + nc), turn(kTResid), [&] {
      nbr = ts_residual(V_, W_, ld_, N_, nsplit, gc_, d_->Y, kLd, d_->theta, nc, R_, ld_,
                        partial_, nullptr, s_);
    });
    reduce_partials(partial_, nbr, (nsplit >= N_ ? 1 : 6) * nc, d_->sums, s_);
  }

  // The control kernel writes its record into pinned host memory, then
  // publishes a sequence number.  The host polls that number instead of
  // synchronising the stream and accepts the record once it carries the
  // number and a matching checksum (the kernel may still be finishing); it
  // checks the stream for errors every few thousand polls.
  Ctl control(const CtlParams& p) {
    ++seq_;
    small_control(d_, p, s_, dctl_, dseq_, seq_);
    return control_wait();
  }
  // the batched driver launches the control steps of many solvers at once
  ControlArgs control_args(const CtlParams& p) {
    ++seq_;
    return ControlArgs{d_, p, dctl_, dseq_, seq_};
  }
  Ctl control_wait() {
    constexpr int nw = (int)(offsetof(Ctl, seq) / sizeof(unsigned int));
    Ctl c;
    // after a short busy spin the poll yields its core (the batched solve runs
    // many of these loops at once); a record that does not appear while the
    // stream is still busy ends the solve after kPollLimit seconds
    constexpr double kPollLimit = 120.0;
    double deadline = 0.0;
    for (uint32_t spins = 1;; ++spins) {
      if (spins > 2048) std::this_thread::yield();
      else __builtin_ia32_pause();
      if (__atomic_load_n(hseq_, __ATOMIC_ACQUIRE) == seq_) {
        std::memcpy(&c, hctl_, sizeof(Ctl));
        if (c.seq == seq_) {
          const unsigned int* w = reinterpret_cast<const unsigned int*>(&c);
          unsigned int sum = ctl_mix((unsigned int)seq_, (unsigned int)nw);
          for (int a = 0; a < nw; ++a) sum += ctl_mix(w[a], (unsigned int)a);
          if (sum == c.sum) break;
        }
      }
      if ((spins & 4095u) == 0) {
        const hipError_t e = hipStreamQuery(s_);
        if (e == hipSuccess) {  // the kernel has ended: the record is whole
          std::memcpy(&c, hctl_, sizeof(Ctl));
          if (c.seq == seq_) break;
          throw Error(SVDS_ERR_HIP, "control record not written");
        }
        if (e != hipErrorNotReady) SVDS_HIP(e);
        const double t = now();
        if (deadline == 0.0) deadline = t + kPollLimit;
        else if (t > deadline)
          throw Error(SVDS_ERR_HIP, "control record not published while the stream stays busy");
      }
    }
    if (ev_.size() >= 64) harvest_events();  // the rest at collect_profile
    return c;
  }

  // stderr trace of the control decisions: every iteration from print level
  // 3, every 2000th at level 2 (progress of long solves)
  void trace(const char* what, int it, const Ctl& c, int nc) {
    if (o_.print_level < 2 || (o_.print_level == 2 && it % 2000 != 0)) return;
    std::fprintf(stderr, "[svds] stage %d %s it %d g %d act %d nb %d rs %d nr %d sweeps %d res0 %.3e maxres %.3e val0 %.12e mv %lld\n",
                 stage_, what, it, gc_, c.action, c.nblock, c.restart, c.nr, c.eig_sweeps,
                 nc > 0 ? c.res[0] : 0.0, c.maxres, nc > 0 ? c.val[0] : 0.0, (long long)mv_);
  }

  // T (the first n_ rows of nb columns, leading dimension ld_) <- K T with
  // the preconditioner of C (point Jacobi, learned polynomial, block Jacobi)
  void apply_pc(double* T, int nb) {
    const double n8 = 8.0 * (double)n_;
    switch (o_.precond) {
      case SVDS_PC_JACOBI: count(n8 * (2 * nb + 1)); break;
      case SVDS_PC_BLOCKJACOBI: count(n8 * (bjnb_ + 2 * nb)); break;
      case SVDS_PC_LEARNED:
        count(ldeg_ * (spmm_bytes(A(), nb) + spmm_bytes(At(), nb) + 6.0 * n8 * nb));
        break;
      default: break;
    }
    switch (o_.precond) {
      case SVDS_PC_JACOBI: scale_rows(T, ld_, n_, nb, dinv_, s_); break;
      case SVDS_PC_LEARNED: learned_apply(T, nb); break;
      case SVDS_PC_BLOCKJACOBI: bj_apply(bjK_, bjnb_, n_, nb, T, ld_, T, ld_, s_); break;
      default: break;
    }
  }

  // preconditioner for the stage-2 block: [K A^T r_u; A K r_v] (pseudo-inverse
  // of B with (A^T A)^-1 ~ K), or the identity
  void precond_stage2(double* T, int nb) {
    count(2.0 * N8() * nb);
    gather_precond(R_, ld_, d_->blk, nb, nullptr, N_, T, ld_, s_);
    apply_pcB(T, nb);
  }
  // T (N_ x nb, the v half first) <- K_B T with the pseudo-inverse composition
  // K_B [y_v; y_u] = [K A^T y_u; A K y_v] of the preconditioner K of C
  void apply_pcB(double* T, int nb) {
    if (o_.precond == SVDS_PC_NONE) return;
    count(4.0 * N8() * nb + spmm_bytes(A(), nb) + spmm_bytes(At(), nb));
    apply_pc(T, nb);                                        // T_v <- K r_v
    pack_rows(T, ld_, nullptr, 0.0, n_, nb, Tc_, s_);       // K r_v (n x nb)
    pack_rows(T + n_, ld_, nullptr, 0.0, m_, nb, Yc_, s_);  // r_u (m x nb)
    spmm(At(), nb, Yc_, Wc_, s_);                           // A^T r_u (n x nb)
    spmm(A(), nb, Tc_, Yc_, s_);                            // A K r_v (m x nb)
    unpack_rows(Wc_, n_, nb, T, ld_, s_);
    apply_pc(T, nb);                                        // K A^T r_u
    unpack_rows(Yc_, m_, nb, T + n_, ld_, s_);
    mv_ += 2 * nb;
  }

  // ---- mixed-precision stage 1 (FP32 basis, FP64 reorthogonalisation) --------
  // the orthonormal FP64 block Tb_ becomes V32[:, gc:gc+nb] and the FP32
  // row-major block for the sparse products
  void commit32(int nb) {
    count(2.0 * N8() * nb);
    copy_cols_cvt<double, float>(Tb_, ld_, N_, nb, V32_ + gc_ * ld_, ld_, Tc32_, s_);
  }
  void append32(int nb) {
    timed_spmm(A32_, nb, (const float*)Tc32_, Yc32_);
    timed_spmm(At32_, nb, (const float*)Yc32_, Wc32_);
    mv_ += 2 * nb;
    float* Wcol = W32_ + gc_ * ld_;
    unpack_rows_f32(Wc32_, N_, nb, Wcol, ld_, s_);
    count(N8() * nb + 4.0 * N_ * (gc_ + 2 * nb));
    proj_bf16x3(V32_, ld_, gc_ + nb, Wcol, ld_, nb, N_, partial_, d_->Hn, s_);
    small_h_append(d_, gc_, nb, s_);
    gc_ += nb;
  }
  void restart32(int nr) {
    count(2.0 * 4.0 * N_ * (gc_ + nr));
    ts_gemm_nn(V32_, ld_, gc_, N_, d_->Yr, kLd, nr, Vt32_, ld_, s_);
    ts_gemm_nn(W32_, ld_, gc_, N_, d_->Yr, kLd, nr, Wt32_, ld_, s_);
    std::swap(V32_, Vt32_);
    std::swap(W32_, Wt32_);
    gc_ = nr;
  }
  void reset32() {
    const int gold = gc_;
    std::swap(V32_, Vt32_);
    gc_ = 0;
    for (int c0 = 0; c0 < gold; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, gold - c0);
      copy_cols_cvt<float, double>(Vt32_ + c0 * ld_, ld_, N_, nb, Tb_, ld_, nullptr, s_);
      Seg32 sv{V32_, gc_, ld_};
      ortho(Tb_, ld_, nb, &sv, 1, (double*)nullptr);
      commit32(nb);
      append32(nb);
    }
  }
  void repair32(int nb, int bad) {
    gc_ -= nb;
    ++breakdowns_;
    const uint64_t stream = kStreamBreak + (uint64_t)rand_count_++;
    int i = 0;
    for (int j = 0; j < nb; ++j)
      if (bad & (1 << j)) fill_random(Tb_ + j * ld_, ld_, N_, 1, o_.seed, stream, i++, s_);
    Seg32 sv{V32_, gc_, ld_};
    ortho(Tb_, ld_, nb, &sv, 1, (double*)nullptr);
    commit32(nb);
    append32(nb);
    extract_stage();
  }

  // ---- stages ------------------------------------------------------------------
  int stage1(double* Vout /*n x k*/, double* Uout /*m x k*/, double* sig, double* rn, double* taus,
             int* ok, int* status1, svds_stats* st);
  // stage 1 in pieces, which the batched driver runs for many solvers in step
 public:
  void s1_start() { s1_begin(); }
  // the stream of the solve's launches; the in-step batched solve moves a
  // prepared solver to its shared stream for stage 1 and back (its arrays
  // stay with the stream they were allocated on)
  void set_stream(hipStream_t s) { s_ = s; }
 private:
  struct S1State {
    int g = 0, r = 0;
    int64_t iters = 0, restarts = 0, resets = 0;
    int since_reset = 0, floor_resets = 0, status = 2, last_nb = 0;
    double t0 = 0.0;
    int64_t mv0 = 0;
  };
  S1State s1_;
  void s1_begin();
  CtlParams s1_params(int nc) const;
  int s1_decide(const Ctl& c);
  void s1_expand(const Ctl& c);
  void s1_restarted(int nr);
  // the random block of a round with nothing to correct, then its
  // orthogonalisation, product, H columns and extraction (as s1_expand)
  void fill_random_block(int nb) {
    fill_random(V_ + gc_ * ld_, ld_, N_, nb, o_.seed, kStreamBreak + (uint64_t)rand_count_++, 0, s_);
  }
  void ortho_and_append(int nb) {
    Seg sv{V_, gc_, ld_};
    ortho_enqueue(V_ + gc_ * ld_, ld_, nb, &sv, 1, Tc_);
    append(nb);
    s1_.last_nb = nb;
    extract_stage();
    ++s1_.iters;
  }
  void s1_end(double* V1, double* U1, double* sig, double* rn, double* taus, int* ok,
              int* status1, svds_stats* st);
 public:
  void s1_end_default(int* status1, svds_stats* st) {
    s1_end(V1_, U1_, sig_, rn1_, taus_, ok_, status1, st);
  }
 private:
  friend struct BatchStage1;
  int stage1_mixed(double* V1, double* U1, double* sig, double* rn, double* taus, int* ok,
                   int* status1, svds_stats* st);
  void final_rr(double* Xk, double* V1, double* U1, double* sig, double* rn, double* taus, int* ok);
  int stage2(const double* taus_h, double* Vout, double* Uout, double* sig, int* nconv,
             svds_stats* st);
  void cleanup_and_output(double* Vw /*n x k*/, double* Uw /*m x k*/, double* sig, double* sigma,
                          double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm);
  void estimate_norm();
  void spmm_cols(const Csr32& Mx, const double* X, int64_t ldx, int64_t nin, int ncols, double* Y,
                 int64_t ldy, int64_t nout) {
    for (int c0 = 0; c0 < ncols; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, ncols - c0);
      pack_rows(X + c0 * ldx, ldx, nullptr, 0.0, nin, nb, Tc_, s_);
      spmm(Mx, nb, Tc_, Yc_, s_);
      unpack_rows(Yc_, nout, nb, Y + c0 * ldy, ldy, s_);
      mv_ += nb;
    }
  }
  // G (k x k, ld k) = X^T Y for N x k blocks
  void gram(const double* X, int64_t ldx, const double* Yb, int64_t ldy, int64_t N, int k,
            double* G) {
    Seg sx{X, k, ldx};
    for (int c0 = 0; c0 < k; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, k - c0);
      tsgemm_tn(&sx, 1, N, Yb + c0 * ldy, ldy, nb, partial_, G + (int64_t)c0 * k, s_);
    }
  }
  // orthonormalise the k columns of X (N rows) in blocks of up to 8
  void orthonormalise(double* X, int64_t ldx, int64_t N, int k) {
    const int64_t Nsave = N_;
    N_ = N;
    for (int c0 = 0; c0 < k; c0 += kMaxBlock) {
      const int nb = std::min(kMaxBlock, k - c0);
      Seg sx{X, c0, ldx};
      ortho(X + c0 * ldx, ldx, nb, &sx, c0 > 0 ? 1 : 0, nullptr);
    }
    N_ = Nsave;
  }
};

// ---------------------------------------------------------------------------
// ||A|| estimate: sqrt of the largest Ritz value of C on a 30-dimensional
// Krylov space with full reorthogonalisation (single-vector block)
// ---------------------------------------------------------------------------
void Solver::estimate_norm() {
  stage_ = 1;
  N_ = n_;
  gc_ = 0;
  refined_ = false;
  const int steps = (int)std::min<int64_t>(std::min(30, kGmax), n_);
  fill_random(V_, ld_, N_, 1, o_.seed, kStreamNorm, 0, s_);
  ortho<double>(V_, ld_, 1, nullptr, 0, Tc_);
  append(1);
  // all steps are enqueued without host synchronisation; each records its
  // breakdown flag, and the space ends before the first step that broke down
  // (an invariant subspace).  Later steps only add rows and columns to H
  // beyond the valid leading block.
  const int first = gc_;
  while (gc_ < steps) {
    double* T = V_ + gc_ * ld_;
    copy_cols(W_ + (gc_ - 1) * ld_, ld_, N_, 1, T, ld_, s_);
    Seg sv{V_, gc_, ld_};
    ortho_enqueue(T, ld_, 1, &sv, 1, Tc_);
    small_record_bad(d_, gc_, s_);
    append(1);
  }
  if (gc_ > first) {
    int hb[kGmax];
    SVDS_HIP(hipMemcpyAsync(hb, d_->stepbad, sizeof(int) * gc_, hipMemcpyDeviceToHost, s_));
    SVDS_HIP(hipStreamSynchronize(s_));
    for (int st = first; st < gc_; ++st)
      if (hb[st]) {
        gc_ = st;
        break;
      }
  }
  small_extract(d_, gc_, 1, 0, s_);
  double lam = 0.0;
  SVDS_HIP(hipMemcpyAsync(&lam, d_->theta, sizeof(double), hipMemcpyDeviceToHost, s_));
  SVDS_HIP(hipStreamSynchronize(s_));
  normA_ = std::sqrt(std::max(lam, 0.0));
}

// ---------------------------------------------------------------------------
// Stage 1: GD+k on C with soft locking (Algorithm 1, first stage)
// ---------------------------------------------------------------------------
// stage 1 up to the first extraction: small state, random block, Krylov fill
void Solver::s1_begin() {
  stage_ = 1;
  N_ = n_;
  gc_ = 0;
  nlock_ = 0;
  refined_ = false;
  s1_ = S1State{};
  s1_.t0 = now();
  s1_.mv0 = mv_;
  // reset the small state
  SVDS_HIP(hipMemsetAsync(d_, 0, sizeof(Small), s_));
  {
    std::vector<double> best(kKmax + 8, INFINITY);
    SVDS_HIP(hipMemcpyAsync(d_->best, best.data(), sizeof(double) * best.size(),
                            hipMemcpyHostToDevice, s_));
    double nc = normA_ * normA_;
    SVDS_HIP(hipMemcpyAsync(&d_->normop, &nc, sizeof(double), hipMemcpyHostToDevice, s_));
    SVDS_HIP(hipStreamSynchronize(s_));
  }
  s1_.g = (int)std::min<int64_t>(g_, n_);
  s1_.r = std::min(r_, std::max(1, s1_.g - b_ - p_));
  const int fill = std::min(std::max(s1_.r, k_ + b_), s1_.g - b_);
  fill_random(V_, ld_, N_, b_, o_.seed, kStreamInit, 0, s_);
  ortho<double>(V_, ld_, b_, nullptr, 0, Tc_);
  append(b_);
  while (gc_ < fill && gc_ + b_ <= s1_.g) {
    double* T = V_ + gc_ * ld_;
    copy_cols(W_ + (gc_ - b_) * ld_, ld_, N_, b_, T, ld_, s_);
    Seg sv{V_, gc_, ld_};
    ortho(T, ld_, b_, &sv, 1, Tc_);
    append(b_);
  }
  extract_stage();
}

CtlParams Solver::s1_params(int nc) const {
  CtlParams P{};
  P.stage = 1;
  P.gc = gc_;
  P.g = s1_.g;
  P.r = s1_.r;
  P.p = p_;
  P.b = b_;
  P.k = k_;
  P.nc = nc;
  P.since_reset = s1_.since_reset;
  P.floor_resets = s1_.floor_resets;
  P.budget_hit = over_budget() ? 1 : 0;
  P.tol = tol1_;
  P.rel = o_.relative_tol ? 1 : 0;
  P.normA = normA_;
  P.eps = kEps;
  P.gate = kFloorGate * kEps;
  return P;
}

// the host's part of a control decision: 1 = stage 1 ends, 2 = the step was
// a breakdown repair or a reset (done here; the next round starts with the
// residual), 0 = expand the basis (after a restart when c.restart)
int Solver::s1_decide(const Ctl& c) {
  if (c.action == kBreakdown) {
    Seg sv{V_, gc_, ld_};
    repair_block(s1_.last_nb, c.bad, &sv, 1);
    return 2;
  }
  if (c.action == kExitConverged || c.action == kExitFloor || c.action == kExitBudget) {
    s1_.status = c.action == kExitConverged ? 0 : (c.action == kExitFloor ? 1 : 2);
    normA_ = std::max(normA_, std::sqrt(c.normop));
    return 1;
  }
  if (c.action == kReset) {
    reset();
    ++s1_.resets;
    s1_.since_reset = 0;
    s1_.floor_resets += c.floor_reset;
    extract_stage();
    return 2;
  }
  return 0;
}

// the basis after a restart: V <- V Y_r, W <- W Y_r (the products launched by the caller)
void Solver::s1_restarted(int nr) {
  std::swap(V_, Vt_);
  std::swap(W_, Wt_);
  gc_ = nr;
  ++s1_.restarts;
  ++s1_.since_reset;
}

void Solver::s1_expand(const Ctl& c) {
  if (c.restart) {
    restart_basis(c.nr);
    ++s1_.restarts;
    ++s1_.since_reset;
  }
  int nb = c.nblock;
  double* T = V_ + gc_ * ld_;
  if (nb == 0) {
    nb = b_;
    count(N8() * nb);
    fill_random(T, ld_, N_, nb, o_.seed, kStreamBreak + (uint64_t)rand_count_++, 0, s_);
  } else {
    count(N8() * (2 * nb + (o_.precond == SVDS_PC_JACOBI ? 1 : 0)));
    gather_precond(R_, ld_, d_->blk, nb, o_.precond == SVDS_PC_JACOBI ? dinv_ : nullptr, N_, T,
                   ld_, s_);
    if (o_.precond != SVDS_PC_JACOBI) apply_pc(T, nb);
  }
  Seg sv{V_, gc_, ld_};
  ortho_enqueue(T, ld_, nb, &sv, 1, Tc_);
  append(nb);
  s1_.last_nb = nb;
  extract_stage();
  ++s1_.iters;
}

// final Rayleigh-Ritz on A X (Algorithm 1, end of the first stage)
void Solver::s1_end(double* V1, double* U1, double* sig, double* rn, double* taus, int* ok,
                    int* status1, svds_stats* st) {
  double* Xk = X_;  // n x k (ld ld_)
  ts_gemm_nn(V_, ld_, gc_, N_, d_->Y, kLd, k_, Xk, ld_, s_);
  final_rr(Xk, V1, U1, sig, rn, taus, ok);
  SVDS_HIP(hipStreamSynchronize(s_));
  st->iters[0] = s1_.iters;
  st->restarts[0] = s1_.restarts;
  st->resets += s1_.resets;
  st->matvecs[0] = mv_ - s1_.mv0;
  st->seconds[0] = now() - s1_.t0;
  *status1 = s1_.status;
}

int Solver::stage1(double* V1, double* U1, double* sig, double* rn, double* taus, int* ok,
                   int* status1, svds_stats* st) {
  s1_begin();
  for (;;) {
    const int nc = std::min(gc_, k_ + b_);
    residual(nc, N_);
    Ctl c = control(s1_params(nc));
    trace("s1", (int)s1_.iters, c, nc);
    if (cap_) capture_residual(s1_.iters, c);
    const int what = s1_decide(c);
    if (what == 1) break;
    if (what == 2) continue;
    s1_expand(c);
  }
  s1_end(V1, U1, sig, rn, taus, ok, status1, st);
  return 0;
}

// ---------------------------------------------------------------------------
// Stage 2: GD+k on B with hard locking and, for the smallest values, the
// simplified refined projection (Algorithm 1, second stage)
// ---------------------------------------------------------------------------
int Solver::stage2(const double* taus_h, double* V1, double* U1, double* sig, int* nconv,
                   svds_stats* st) {
  stage_ = 2;
  jd_ = o_.stage2_solver == SVDS_STAGE2_JD;
  jd32_ = jd_ && mixed_ && largest_;
  N_ = n_ + m_;
  gc_ = 0;
  nlock_ = 0;
  refined_ = !largest_;
  tau_ = taus_h[0];
  const double t0 = now();
  const int64_t mv0 = mv_;
  SVDS_HIP(hipMemsetAsync(d_, 0, sizeof(Small), s_));
  {
    double nb = normA_;
    SVDS_HIP(hipMemcpyAsync(&d_->normop, &nb, sizeof(double), hipMemcpyHostToDevice, s_));
  }
  const int g = (int)std::min<int64_t>(g_, N_);
  const int r = std::min(r_, std::max(1, g - b_ - p_));
  // initial basis [v; u] (the 1/sqrt(2) is absorbed by the normalisation)
  for (int c0 = 0; c0 < k_; c0 += kMaxBlock) {
    const int nb = std::min(kMaxBlock, k_ - c0);
    double* T = V_ + gc_ * ld_;
    copy_cols(V1 + c0 * ld_, ld_, n_, nb, T, ld_, s_);
    copy_cols(U1 + c0 * ld_, ld_, m_, nb, T + n_, ld_, s_);
    Seg sv{V_, gc_, ld_};
    ortho(T, ld_, nb, &sv, gc_ > 0 ? 1 : 0, Tc_);
    append(nb);
  }
  extract_stage();
  int64_t iters = 0, restarts = 0, resets = 0;
  int since_reset = 0;
  int exit_action = kExitBudget;
  int last_nb = 0;
  for (;;) {
    const int nc = std::min(gc_, b_);
    residual(nc, n_);
    CtlParams P{};
    P.stage = 2;
    P.gc = gc_;
    P.g = g;
    P.r = r;
    P.p = p_;
    P.b = b_;
    P.k = k_;
    P.nc = nc;
    P.nlock = nlock_;
    P.since_reset = since_reset;
    P.budget_hit = over_budget() ? 1 : 0;
    P.refined = refined_ ? 1 : 0;
    P.tol = tol_;
    P.normA = normA_;
    P.eps = kEps;
    P.gate = kFloorGate * kEps;
    Ctl c = control(P);
    trace("s2", (int)iters, c, nc);
    if (c.action == kBreakdown) {
      Seg segs[2] = {Seg{X_, nlock_, ld_}, Seg{V_, gc_, ld_}};
      repair_block(last_nb, c.bad, segs, 2);
      continue;
    }
    if (c.nlockable > 0) {
      // x = V y for the converged prefix -> locked vectors
      count(N8() * (gc_ + c.nlockable));
      ts_gemm_nn(V_, ld_, gc_, N_, d_->Y, kLd, c.nlockable, X_ + nlock_ * ld_, ld_, s_);
      nlock_ += c.nlockable;
    }
    if (c.action == kExitConverged || c.action == kExitBudget) {
      exit_action = c.action;
      break;
    }
    if (c.action == kLock) {
      restart_basis(c.nr);
      ++restarts;
      ++since_reset;
      if (refined_) {
        tau_ = taus_h[std::min(nlock_, k_ - 1)];
        rebuild_refined();
      }
      extract_stage();
      continue;
    }
    if (c.action == kReset) {
      reset();
      ++resets;
      since_reset = 0;
      extract_stage();
      continue;
    }
    const int nb = c.nblock;
    if (jd_) {
      // Ritz vectors of the block and the shifts, before a restart changes V
      count(N8() * (gc_ + nb));
      ts_gemm_nn(V_, ld_, gc_, N_, d_->Y, kLd, nb, jdXb_, ld_, s_);
      if (refined_) {
        double sh[kMaxBlock];
        for (int j = 0; j < nb; ++j) sh[j] = tau_;
        SVDS_HIP(hipMemcpyAsync(jdShift_, sh, sizeof(double) * nb, hipMemcpyHostToDevice, s_));
      } else {
        SVDS_HIP(hipMemcpyAsync(jdShift_, d_->theta, sizeof(double) * nb, hipMemcpyDeviceToDevice,
                                s_));
      }
    }
    if (c.restart) {
      restart_basis(c.nr);
      ++restarts;
      ++since_reset;
    }
    double* T = V_ + gc_ * ld_;
    if (jd_) jd_correct(T, nb);
    else precond_stage2(T, nb);
    Seg segs[2] = {Seg{X_, nlock_, ld_}, Seg{V_, gc_, ld_}};
    if (refined_) {
      ortho(T, ld_, nb, segs, 2, Tc_);  // the refined factor update needs a valid block
    } else {
      ortho_enqueue(T, ld_, nb, segs, 2, Tc_);
    }
    append(nb);
    last_nb = nb;
    extract_stage();
    ++iters;
  }
  *nconv = nlock_;
  int have = nlock_;
  if (have < k_) {  // budget: complete with the current best approximations
    const int extra = std::min(k_ - have, gc_);
    ts_gemm_nn(V_, ld_, gc_, N_, d_->Y, kLd, extra, X_ + have * ld_, ld_, s_);
    SVDS_HIP(hipMemcpyAsync(d_->lockval + have, d_->theta, sizeof(double) * extra,
                            hipMemcpyDeviceToDevice, s_));
    have += extra;
  }
  // halves: v = x(1:n)/||.||, u = x(n+1:)/||.||, sigma = |lambda| (Algorithm 1)
  double* nv = vec_;
  double* nu = nv + kKmax;
  double* fv = nu + kKmax;
  double* fu = fv + kKmax;
  copy_cols(X_, ld_, n_, have, V1, ld_, s_);
  copy_cols(X_ + n_, ld_, m_, have, U1, ld_, s_);
  col_residual2(V1, ld_, nullptr, 0, nullptr, n_, have, partial_, nv, s_);
  col_residual2(U1, ld_, nullptr, 0, nullptr, m_, have, partial_, nu, s_);
  inv_sqrt(have, nv, fv, s_);
  inv_sqrt(have, nu, fu, s_);
  col_scale(V1, ld_, n_, have, fv, s_);
  col_scale(U1, ld_, m_, have, fu, s_);
  abs_vec(have, d_->lockval, sig, s_);
  SVDS_HIP(hipStreamSynchronize(s_));
  st->iters[1] = iters;
  st->restarts[1] = restarts;
  st->resets += resets;
  st->matvecs[1] = mv_ - mv0;
  st->seconds[1] = now() - t0;
  (void)exit_action;
  return 0;
}

// ---------------------------------------------------------------------------
// two-sided clean-up: orthonormalise U and V, SVD of U^T A V, rotate; then
// eq. (res), sign convention and output in the caller's orientation
// ---------------------------------------------------------------------------
void Solver::cleanup_and_output(double* Vw, double* Uw, double* sig, double* sigma, double* U,
                                int64_t ldu, double* V, int64_t ldv, double* rnorm) {
  double* P = vec_;                    // k x k (ld kLd)
  double* Qm = P + kLd * kLd;
  double* sv = Qm + kLd * kLd;
  double* Yq = sv + kLd;
  double* AVq = Yq + kLd * kLd;
  double* H2 = AVq + kLd * kLd;
  double* rl2 = H2 + kLd * kLd;
  double* rr2 = rl2 + kLd;
  double* f = rr2 + kLd;
  double* sgn = f + kLd;
  double* U2 = Wt_;  // m x k
  double* V2 = Vt_;  // n x k
  double* AV = R_;   // m x k
  double* AtU = Q_ ? Q_ : W_;
  if (o_.two_sided_cleanup) {
    orthonormalise(Uw, ld_, m_, k_);
    orthonormalise(Vw, ld_, n_, k_);
    spmm_cols(A(), Vw, ld_, n_, k_, AV, ld_, m_);
    gram(Uw, ld_, AV, ld_, m_, k_, H2);  // H2 = U^T A V (k x k, ld k)
    small_svd(k_, H2, k_, sv, Yq, kLd, AVq, kLd, s_);
    cleanup_finish(k_, sv, Yq, kLd, AVq, kLd, largest_ ? 1 : 0, sig, P, Qm, kLd, s_);
    ts_gemm_nn(Uw, ld_, k_, m_, P, kLd, k_, U2, ld_, s_);
    ts_gemm_nn(Vw, ld_, k_, n_, Qm, kLd, k_, V2, ld_, s_);
  } else {
    copy_cols(Uw, ld_, m_, k_, U2, ld_, s_);
    copy_cols(Vw, ld_, n_, k_, V2, ld_, s_);
  }
  // eq. (res)
  spmm_cols(A(), V2, ld_, n_, k_, AV, ld_, m_);
  spmm_cols(At(), U2, ld_, m_, k_, AtU, ld_, n_);
  col_residual2(AV, ld_, U2, ld_, sig, m_, k_, partial_, rl2, s_);
  col_residual2(AtU, ld_, V2, ld_, sig, n_, k_, partial_, rr2, s_);
  sqrt_sum(k_, rl2, rr2, rnorm, s_);
  // caller orientation: right vectors of the caller's A
  double* Vc = M_->transposed ? U2 : V2;
  double* Uc = M_->transposed ? V2 : U2;
  const int64_t nV = M_->transposed ? m_ : n_;
  const int64_t nU = M_->transposed ? n_ : m_;
  sign_factors(Vc, ld_, nV, k_, partial_, sgn, s_);
  col_scale(Vc, ld_, nV, k_, sgn, s_);
  col_scale(Uc, ld_, nU, k_, sgn, s_);
  copy_cols(Vc, ld_, nV, k_, V, ldv, s_);
  copy_cols(Uc, ld_, nU, k_, U, ldu, s_);
  SVDS_HIP(hipMemcpyAsync(sigma, sig, sizeof(double) * k_, hipMemcpyDeviceToDevice, s_));
}

// Rayleigh-Ritz on the returned basis through A X (Algorithm 1, first stage):
// G = (A X)^T (A X), sigma = |lambda|^(1/2), v = X z, u = A v / sigma, then
// eq. (res) and the stage-2 shifts
void Solver::final_rr(double* Xk, double* V1, double* U1, double* sig, double* rn, double* taus,
                      int* ok) {
  double* AX = R_;  // m x k, ld ld_
  spmm_cols(A(), Xk, ld_, n_, k_, AX, ld_, m_);
  double* G = vec_;                 // k x k
  double* lam = vec_ + kKmax * kKmax;
  double* Z = lam + kKmax;          // k x k (ld kLd)
  double* inv = Z + kLd * kLd;
  double* rl2 = inv + kKmax;
  double* rr2 = rl2 + kKmax;
  gram(AX, ld_, AX, ld_, m_, k_, G);
  small_eig(k_, G, k_, largest_ ? 1 : 0, lam, Z, kLd, s_);
  ts_gemm_nn(Xk, ld_, k_, n_, Z, kLd, k_, V1, ld_, s_);      // v = X z
  ts_gemm_nn(AX, ld_, k_, m_, Z, kLd, k_, Wt_, ld_, s_);     // A v
  sigma_from_lambda(k_, lam, sig, inv, s_);
  copy_cols(Wt_, ld_, m_, k_, U1, ld_, s_);
  col_scale(U1, ld_, m_, k_, inv, s_);                      // u = A v / sigma
  double* AtU = Vt_;
  spmm_cols(At(), U1, ld_, m_, k_, AtU, ld_, n_);
  col_residual2(Wt_, ld_, U1, ld_, sig, m_, k_, partial_, rl2, s_);   // ||A v - s u||^2
  col_residual2(AtU, ld_, V1, ld_, sig, n_, k_, partial_, rr2, s_);   // ||A^T u - s v||^2
  stage1_check(k_, rl2, rr2, sig, normA_, tol_, o_.relative_tol ? 1 : 0, rn, taus, ok, s_);
}

// ---------------------------------------------------------------------------
// Stage 1 in mixed precision: the basis V, W = C V and the sparse products in
// FP32, the new columns of H = V^T W with BF16 matrix-core products (FP32
// accumulation); reorthogonalisation, Cholesky QR Gram matrices, the
// projected eigenproblem and the residual norms in FP64.  The stage-1 floor
// uses the unit roundoff of the projections (2^-16 for the split BF16
// product); stage 2 and the final Rayleigh-Ritz are FP64.
// ---------------------------------------------------------------------------
constexpr double kEpsMixed = 1.52587890625e-05;  // 2^-16

int Solver::stage1_mixed(double* V1, double* U1, double* sig, double* rn, double* taus, int* ok,
                         int* status1, svds_stats* st) {
  stage_ = 1;
  N_ = n_;
  gc_ = 0;
  nlock_ = 0;
  refined_ = false;
  const double t0 = now();
  const int64_t mv0 = mv_;
  SVDS_HIP(hipMemsetAsync(d_, 0, sizeof(Small), s_));
  {
    std::vector<double> best(kKmax + 8, INFINITY);
    SVDS_HIP(hipMemcpyAsync(d_->best, best.data(), sizeof(double) * best.size(),
                            hipMemcpyHostToDevice, s_));
    double nc = normA_ * normA_;
    SVDS_HIP(hipMemcpyAsync(&d_->normop, &nc, sizeof(double), hipMemcpyHostToDevice, s_));
    SVDS_HIP(hipStreamSynchronize(s_));
  }
  const int g = (int)std::min<int64_t>(g_, n_);
  const int r = std::min(r_, std::max(1, g - b_ - p_));
  const int fill = std::min(std::max(r, k_ + b_), g - b_);
  fill_random(Tb_, ld_, N_, b_, o_.seed, kStreamInit, 0, s_);
  ortho<double>(Tb_, ld_, b_, nullptr, 0, nullptr);
  commit32(b_);
  append32(b_);
  while (gc_ < fill && gc_ + b_ <= g) {
    copy_cols_cvt<float, double>(W32_ + (gc_ - b_) * ld_, ld_, N_, b_, Tb_, ld_, nullptr, s_);
    Seg32 sv{V32_, gc_, ld_};
    ortho(Tb_, ld_, b_, &sv, 1, (double*)nullptr);
    commit32(b_);
    append32(b_);
  }
  extract_stage();
  int64_t iters = 0, restarts = 0, resets = 0;
  int since_reset = 0, floor_resets = 0;
  int status = 2;
  int last_nb = 0;
  for (;;) {
    const int nc = std::min(gc_, k_ + b_);
    count(4.0 * N_ * 2 * gc_ + N8() * nc);
    ts_residual(V32_, W32_, ld_, N_, N_, gc_, d_->Y, kLd, d_->theta, nc, R_, ld_, partial_,
                d_->sums, s_);
    CtlParams P{};
    P.stage = 1;
    P.gc = gc_;
    P.g = g;
    P.r = r;
    P.p = p_;
    P.b = b_;
    P.k = k_;
    P.nc = nc;
    P.since_reset = since_reset;
    P.floor_resets = floor_resets;
    P.budget_hit = over_budget() ? 1 : 0;
    P.tol = tol1_;
    P.rel = o_.relative_tol ? 1 : 0;
    P.normA = normA_;
    P.eps = kEpsMixed;
    P.gate = std::min(kFloorGate * kEpsMixed, 1e-2);
    Ctl c = control(P);
    trace("s1m", (int)iters, c, nc);
    if (c.action == kBreakdown) {
      repair32(last_nb, c.bad);
      continue;
    }
    if (c.action == kExitConverged || c.action == kExitFloor || c.action == kExitBudget) {
      status = c.action == kExitConverged ? 0 : (c.action == kExitFloor ? 1 : 2);
      normA_ = std::max(normA_, std::sqrt(c.normop));
      break;
    }
    if (c.action == kReset) {
      reset32();
      ++resets;
      since_reset = 0;
      floor_resets += c.floor_reset;
      extract_stage();
      continue;
    }
    if (c.restart) {
      restart32(c.nr);
      ++restarts;
      ++since_reset;
    }
    int nb = c.nblock;
    if (nb == 0) {
      nb = b_;
      count(N8() * nb);
      fill_random(Tb_, ld_, N_, nb, o_.seed, kStreamBreak + (uint64_t)rand_count_++, 0, s_);
    } else {
      count(N8() * (2 * nb + (o_.precond == SVDS_PC_JACOBI ? 1 : 0)));
      gather_precond(R_, ld_, d_->blk, nb, o_.precond == SVDS_PC_JACOBI ? dinv_ : nullptr, N_,
                     Tb_, ld_, s_);
      if (o_.precond != SVDS_PC_JACOBI) apply_pc(Tb_, nb);
    }
    Seg32 sv{V32_, gc_, ld_};
    ortho_enqueue(Tb_, ld_, nb, &sv, 1, (double*)nullptr);
    commit32(nb);
    append32(nb);
    last_nb = nb;
    extract_stage();
    ++iters;
  }
  double* Xk = X_;
  ts_gemm_nn(V32_, ld_, gc_, N_, d_->Y, kLd, k_, Xk, ld_, s_);
  final_rr(Xk, V1, U1, sig, rn, taus, ok);
  SVDS_HIP(hipStreamSynchronize(s_));
  st->iters[0] = iters;
  st->restarts[0] = restarts;
  st->resets += resets;
  st->matvecs[0] = mv_ - mv0;
  st->seconds[0] = now() - t0;
  *status1 = status;
  return 0;
}

// coefficients of the learned preconditioner for this matrix (one forward
// pass of the network; its activations are freed right after)
void Solver::setup_learned() {
  if (!o_.pc_model) throw Error(SVDS_ERR_ARG, "learned preconditioner without pc_model");
  lpc_compute(lop_, s_);
  DeviceBuffers tmp(s_);
  float* feat = tmp.get<float>((size_t)n_ * kLpcNF);
  float* cache = tmp.get<float>((size_t)n_ * kLpcCacheRow);
  float* gbuf = tmp.get<float>((size_t)m_ * kLpcHid);
  lpc_features(lop_, feat, s_);
  lpc_forward(lop_, o_.pc_model, feat, ldeg_, lcoef_, cache, gbuf, s_);
  learned_ = true;
}

// enqueue a copy of R_[:, blk[0]] (blk on the device) into the capture array
void Solver::capture_residual(int64_t iters, const Ctl& c) {
  const bool expand = c.action != kBreakdown && c.action != kExitConverged &&
                      c.action != kExitFloor && c.action != kExitBudget && c.action != kReset;
  if (!expand || c.nblock <= 0 || cap_->count >= cap_->max || iters % cap_->every != 0) return;
  gather_precond(R_, ld_, d_->blk, 1, nullptr, N_, cap_->R + (int64_t)cap_->count * cap_->ldr,
                 cap_->ldr, s_);
  ++cap_->count;
}

void Solver::allocate(DeviceBuffers& a) {
  const int64_t Nmax = m_ + n_;
  ld_ = round_up(Nmax, 64);
  // basis arrays hold g columns (and the 30 of the norm estimate)
  const size_t basis = (size_t)ld_ * std::min(kGmax, std::max(g_, 30));
  const size_t blk = (size_t)ld_ * kMaxBlock;
  V_ = a.get<double>(basis);
  W_ = a.get<double>(basis);
  Vt_ = a.get<double>(basis);
  Wt_ = a.get<double>(basis);
  if (!largest_) {
    Q_ = a.get<double>(basis);
    Qt_ = a.get<double>(basis);
  }
  X_ = a.get<double>((size_t)ld_ * std::max(kKmax, kLd));
  R_ = a.get<double>((size_t)ld_ * std::max(kKmax + 8, kLd));
  Tc_ = a.get<double>(blk);
  Yc_ = a.get<double>(blk);
  Wc_ = a.get<double>(blk);
  Zc_ = a.get<double>(blk);
  partial_ = a.get<double>((size_t)2048 * 264 * kMaxBlock + 4096);
  cqrP_ = a.get<double>((size_t)kCholQRMaxBlocks * kMaxBlock * kMaxBlock);
  d_ = a.get<Small>(1);
  vec_ = a.get<double>(16 * kLd * kLd);
  V1_ = a.get<double>((size_t)ld_ * kKmax);
  U1_ = a.get<double>((size_t)ld_ * kKmax);
  sig_ = a.get<double>(kKmax);
  rn1_ = a.get<double>(kKmax);
  taus_ = a.get<double>(kKmax);
  ok_ = a.get<int>(1);
  if (o_.precision == SVDS_MIXED) {
    V32_ = a.get<float>(basis);
    W32_ = a.get<float>(basis);
    Vt32_ = a.get<float>(basis);
    Wt32_ = a.get<float>(basis);
    Tc32_ = a.get<float>(blk);
    Yc32_ = a.get<float>(blk);
    Wc32_ = a.get<float>(blk);
    Tb_ = a.get<double>(blk);
  }
  if (o_.fused_gram && M_->G.R > 0) gramP_ = a.get<double>((size_t)M_->G.wsum * kMaxBlock);
  if (o_.precond == SVDS_PC_JACOBI) dinv_ = a.get<double>(n_);
  if (o_.precond == SVDS_PC_LEARNED) {
    ldeg_ = o_.pc_degree > 0 ? o_.pc_degree : kLpcDefaultDegree;
    if (ldeg_ > kLpcMaxDegree) throw Error(SVDS_ERR_ARG, "pc_degree out of range");
    lpc_alloc(M_, lop_, a);
    lcoef_ = a.get<float>((size_t)n_ * kLpcCoef);
    lpc_scratch(lop_, kMaxBlock, lsc_, a);
  }
  if (o_.precond == SVDS_PC_BLOCKJACOBI) {
    bjnb_ = o_.pc_block > 0 ? o_.pc_block : 64;
    bjK_ = a.get<double>((size_t)((n_ + bjnb_ - 1) / bjnb_) * bjnb_ * bjnb_);
  }
  if (o_.stage2_solver == SVDS_STAGE2_JD && o_.method != SVDS_METHOD_NORMAL) {
    jdXb_ = a.get<double>(blk);
    jdR_ = a.get<double>(blk);
    jdQ_ = a.get<double>(blk);
    jdW_ = a.get<double>(blk);
    jdD_ = a.get<double>(blk);
    jdT_ = a.get<double>(blk);
    jdC_ = a.get<double>((size_t)(kKmax + kMaxBlock) * kMaxBlock);
    jdShift_ = a.get<double>(kMaxBlock);
    jdN2_ = a.get<double>(kMaxBlock);
    jdSig_ = a.get<double>(kMaxBlock);
    jdRn2_ = a.get<double>(kMaxBlock);
    jdRho_ = a.get<double>(kMaxBlock);
    jdSt_ = a.get<JdCol>(kMaxBlock);
  }
}

// everything before the first stage: the solver's arrays, the pinned control
// records, the preconditioner, ||A||
void Solver::prepare(svds_stats* st) {
  std::memset(st, 0, sizeof(*st));
  const double t0 = now();
  run_t0_ = t0;
  if (!buf_.base) buf_.own(workspace_bytes());  // no caller workspace: one block
  allocate(buf_);
  mixed_ = o_.precision == SVDS_MIXED;
  hctl_ = static_cast<Ctl*>(host_record_get(kCtlBytes, kCtlFlags));
  SVDS_HIP(hipHostGetDevicePointer((void**)&dctl_, hctl_, 0));
  hseq_ = reinterpret_cast<int*>(reinterpret_cast<char*>(hctl_) + kSeqOff);
  dseq_ = reinterpret_cast<int*>(reinterpret_cast<char*>(dctl_) + kSeqOff);
  __atomic_store_n(hseq_, 0, __ATOMIC_RELEASE);
  hbad_ = static_cast<int*>(host_record_get(sizeof(int), hipHostMallocDefault));
  hjd_ = static_cast<JdCol*>(host_record_get(sizeof(JdCol) * kMaxBlock, hipHostMallocDefault));
  if (o_.precond == SVDS_PC_JACOBI)
    invert_diag(M_->diagC, n_, dinv_, s_);  // 1/diag(C), with 1 where the column is empty
  if (o_.precond == SVDS_PC_LEARNED) setup_learned();
  if (o_.precond == SVDS_PC_BLOCKJACOBI) bj_setup(M_, bjnb_, bjK_, s_);
  SVDS_HIP(hipMemsetAsync(d_, 0, sizeof(Small), s_));
  // ---- ||A||
  if (o_.norm_A > 0) {
    normA_ = o_.norm_A;
  } else {
    estimate_norm();
    mv_ = 0;
  }
  st->setup_seconds = now() - t0;
}

int Solver::run(double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
                svds_stats* st) {
  prepare(st);
  return complete(sigma, U, ldu, V, ldv, rnorm, st, false);
}

// the stages (stage 1 unless a batched driver already ran it and its end),
// the clean-up and the statistics
int Solver::complete(double* sigma, double* U, int64_t ldu, double* V, int64_t ldv,
                     double* rnorm, svds_stats* st, bool stage1_done) {
  double *V1 = V1_, *U1 = U1_, *sig = sig_, *rn1 = rn1_, *taus = taus_;
  int* ok = ok_;
  int nconv = 0;
  if (o_.method == SVDS_METHOD_AUGMENTED) {
    // stage 2 alone (largest values) from one counter-based block [v; u]
    // of length n + m; no stage-1 bounds
    fill_random(X_, ld_, n_ + m_, k_, o_.seed, kStreamInit, 0, s_);
    copy_cols(X_, ld_, n_, k_, V1, ld_, s_);
    copy_cols(X_ + n_, ld_, m_, k_, U1, ld_, s_);
    std::vector<double> th(k_, normA_ * kEps);
    st->stage1_status = 0;
    stage2(th.data(), V1, U1, sig, &nconv, st);
    st->stage_exit = 2;
  } else {
    // ---- stage 1
    int okh = 0, status1 = 2;
    if (stage1_done) {
      status1 = st->stage1_status;
    } else if (mixed_) {
      stage1_mixed(V1, U1, sig, rn1, taus, ok, &status1, st);
    } else {
      stage1(V1, U1, sig, rn1, taus, ok, &status1, st);
    }
    SVDS_HIP(hipMemcpyAsync(&okh, ok, sizeof(int), hipMemcpyDeviceToHost, s_));
    SVDS_HIP(hipStreamSynchronize(s_));
    st->stage1_status = status1;
    st->stage_exit = 1;
    if (o_.method == SVDS_METHOD_HYBRID && status1 != 2 && (o_.force_stage2 || !okh)) {
      std::vector<double> th(k_);
      SVDS_HIP(hipMemcpyAsync(th.data(), taus, sizeof(double) * k_, hipMemcpyDeviceToHost, s_));
      SVDS_HIP(hipStreamSynchronize(s_));
      stage2(th.data(), V1, U1, sig, &nconv, st);
      st->stage_exit = 2;
    }
  }
  cleanup_and_output(V1, U1, sig, sigma, U, ldu, V, ldv, rnorm);
  std::vector<double> hr(k_), hs(k_);
  SVDS_HIP(hipMemcpyAsync(hr.data(), rnorm, sizeof(double) * k_, hipMemcpyDeviceToHost, s_));
  SVDS_HIP(hipMemcpyAsync(hs.data(), sigma, sizeof(double) * k_, hipMemcpyDeviceToHost, s_));
  SVDS_HIP(hipStreamSynchronize(s_));
  int good = 0;
  bool finite = true;
  for (int i = 0; i < k_; ++i) {
    // eq. (res), or the relative rule of the condition estimate
    const double lim = (o_.relative_tol ? hs[i] : normA_) * tol_;
    good += hr[i] < lim;
    finite = finite && std::isfinite(hr[i]);
  }
  st->nconv = good;
  st->inner_iters = jd_inner_;
  st->norm_A_used = normA_;
  collect_profile(st);
  st->breakdowns = breakdowns_;
  if (!finite && good == 0) return SVDS_ERR_BREAKDOWN;
  return good >= k_ ? SVDS_OK : SVDS_NOT_CONVERGED;
}

// ---------------------------------------------------------------------------
// Batched launches: argument upload
// ---------------------------------------------------------------------------
BatchUpload::~BatchUpload() {
  if (dev_) stream_free(dev_, s_);
  if (host_) (void)hipHostFree(host_);
}

void BatchUpload::init(size_t bytes, hipStream_t s) {
  s_ = s;
  cap_ = bytes;
  SVDS_HIP(hipHostMalloc((void**)&host_, bytes, hipHostMallocDefault));
  dev_ = static_cast<char*>(stream_alloc(bytes, s));
}

const void* BatchUpload::put_bytes(const void* v, size_t bytes) {
  const size_t off = (used_ + 255) & ~static_cast<size_t>(255);
  if (off + bytes > cap_) throw Error(SVDS_ERR_ARG, "batched launch arguments exceed the staging");
  std::memcpy(host_ + off, v, bytes);
  used_ = off + bytes;
  return dev_ + off;
}

void BatchUpload::flush() {
  if (used_ <= sent_) return;
  SVDS_HIP(hipMemcpyAsync(dev_ + sent_, host_ + sent_, used_ - sent_, hipMemcpyHostToDevice, s_));
  sent_ = used_;
}

int BatchUpload::tiles(const std::vector<int>& gx, const std::vector<int>& gy, BTiles& t) {
  const int np = (int)gx.size();
  std::vector<int> g(np), cnt(np);
  int64_t total = 0;
  for (int p = 0; p < np; ++p) {
    g[p] = std::max(gx[p], 1);
    cnt[p] = (gx[p] > 0 && gy[p] > 0) ? gx[p] * gy[p] : 0;
    total += cnt[p];
  }
  if (total > (int64_t)INT32_MAX / 2) throw Error(SVDS_ERR_ARG, "batched launch too large");
  const int per = (int)((total + kXcds - 1) / kXcds);  // run length of each XCD
  std::vector<int> xoff(kXcds + 1, 0), xpre, sp, sf;
  int xc = 0, fill = 0;  // current XCD and the workgroups already in its run
  xpre.push_back(0);
  for (int p = 0; p < np && per > 0; ++p) {
    int done = 0;
    while (done < cnt[p]) {
      if (fill == per) {  // run full: the next XCD starts its own
        ++xc;
        xoff[xc] = (int)sp.size();
        xpre.push_back(0);
        fill = 0;
      }
      const int take = std::min(cnt[p] - done, per - fill);
      sp.push_back(p);
      sf.push_back(done);
      fill += take;
      xpre.push_back(fill);
      done += take;
    }
  }
  for (int x = xc + 1; x <= kXcds; ++x) {
    xoff[x] = (int)sp.size();
    if (x < kXcds) xpre.push_back(0);
  }
  if (sp.empty()) sp.push_back(0), sf.push_back(0);  // keep the arrays non-empty
  t.xoff = put(xoff.data(), xoff.size());
  t.xpre = put(xpre.data(), xpre.size());
  t.sp = put(sp.data(), sp.size());
  t.sf = put(sf.data(), sf.size());
  t.gx = put(g.data(), g.size());
  t.np = np;
  return total > 0 ? per * kXcds : 0;
}

// ---------------------------------------------------------------------------
// Stage 1 of many solvers in step (svds_solve_batched): every step of an
// iteration is one launch for all solvers that take it, with each solver's
// own arguments and launch geometry, so every solver computes exactly what
// its own stage1() would.  The host reads all control records of a round
// and takes each solver's decision; breakdown repairs and resets, which
// synchronise, run per solver.
// ---------------------------------------------------------------------------
struct BatchStage1 {
  std::vector<Solver*> sv;
  hipStream_t s;
  BatchUpload up;

  // solvers that can run in step: FP64 stage 1 through two SpMMs with a
  // merged launch shape, no preconditioner or point Jacobi
  static bool eligible(const Solver& x) {
    return x.o_.precision == SVDS_FP64 && x.o_.method != SVDS_METHOD_AUGMENTED &&
           (x.o_.precond == SVDS_PC_NONE || x.o_.precond == SVDS_PC_JACOBI) &&
           !(x.o_.fused_gram && x.M_->G.R > 0) && !x.cap_ && !x.o_.profile;
  }

  void residual(const std::vector<Solver*>& a) {
    std::vector<BatchResid> jobs;
    for (Solver* x : a) {
      const int nc = std::min(x->gc_, x->k_ + x->b_);
      x->count(x->N8() * (2 * x->gc_ + nc));
      jobs.push_back(BatchResid{x->V_, x->W_, x->ld_, x->N_, x->gc_, x->d_->Y, kLd,
                                x->d_->theta, nc, x->R_, x->ld_, x->partial_, x->d_->sums});
    }
    ts_residual_batch(jobs, up, s);
  }

  // products with A then A^T of the compact blocks, grouped by launch shape
  void products(const std::vector<Solver*>& a, int nb) {
    for (int pass = 0; pass < 2; ++pass) {
      std::map<std::pair<int, int>, std::vector<BatchSpmm>> groups;
      for (Solver* x : a) {
        const Csr32& M = pass == 0 ? x->A_ : x->At_;
        const double* X = pass == 0 ? x->Tc_ : x->Yc_;
        double* Y = pass == 0 ? x->Yc_ : x->Wc_;
        x->count(Solver::spmm_bytes(M, nb));
        if (M.merged_bin < 0 || M.merged_bin >= kNumBins - 1) {
          spmm(M, nb, X, Y, s);  // binned rows: the matrix's own launches
          continue;
        }
        groups[{M.merged_bin, M.unroll}].push_back(BatchSpmm{&M, X, Y});
      }
      for (auto& g : groups) spmm_batch(nb, g.second, up, s);
    }
    for (Solver* x : a) x->mv_ += 2 * nb;
  }

  // correction, orthogonalisation, products, H columns, extraction of
  // solvers with the same block width (their control steps chose expand)
  void expand(const std::vector<Solver*>& a, int nb) {
    std::vector<BatchGather> ga;
    for (Solver* x : a) {
      const bool jac = x->o_.precond == SVDS_PC_JACOBI;
      x->count(x->N8() * (2 * nb + (jac ? 1 : 0)));
      ga.push_back(BatchGather{x->R_, x->ld_, x->d_->blk, jac ? x->dinv_ : nullptr, x->N_,
                               x->V_ + x->gc_ * x->ld_, x->ld_});
    }
    gather_batch(nb, ga, up, s);
    // classical Gram-Schmidt pass 1 with the block's own Gram matrix appended
    std::vector<BatchProj> p1;
    std::vector<Solver*> wb;  // solvers with a basis to project against
    for (Solver* x : a) {
      double* T = x->V_ + x->gc_ * x->ld_;
      BatchProj q{};
      q.nseg = 0;
      if (x->gc_ > 0) q.segs[q.nseg++] = Seg{x->V_, x->gc_, x->ld_};
      q.segs[q.nseg++] = Seg{T, nb, x->ld_};
      q.N = x->N_;
      q.T = T;
      q.ldt = x->ld_;
      q.partial = x->partial_;
      p1.push_back(q);
      x->count(x->N8() * (x->gc_ + nb));
      if (x->gc_ > 0) wb.push_back(x);
    }
    std::vector<int> nblk;
    tsgemm_tn_batch(nb, p1, nblk, up, s);
    std::vector<BatchReduce> r1;
    for (size_t j = 0; j < a.size(); ++j)
      r1.push_back(BatchReduce{a[j]->partial_, nblk[j], (a[j]->gc_ + nb) * nb, a[j]->d_->C0,
                               nullptr});
    reduce_partials_batch(r1, up, s);
    if (!wb.empty()) {
      std::vector<BatchUpdate> u1, u2;
      std::vector<BatchProj> p2;
      for (Solver* x : wb) {
        const int total = x->gc_, ldc0 = total + nb;
        double* T = x->V_ + x->gc_ * x->ld_;
        BatchUpdate u{};
        u.segs[0] = Seg{x->V_, total, x->ld_};
        u.nseg = 1;
        u.N = x->N_;
        u.C = x->d_->C0;
        u.ldc = ldc0;
        u.T = T;
        u.ldt = x->ld_;
        u.skip = nullptr;
        u.dgks_out = &x->d_->skip2;  // the first update takes the second-pass test
        u1.push_back(u);
        u.dgks_out = nullptr;
        BatchProj q{};
        q.segs[0] = Seg{x->V_, total, x->ld_};
        q.nseg = 1;
        q.N = x->N_;
        q.T = T;
        q.ldt = x->ld_;
        q.partial = x->partial_;
        q.C = x->d_->C1;
        q.skip = &x->d_->skip2;
        p2.push_back(q);
        u.C = x->d_->C1;
        u.ldc = total;
        u.skip = &x->d_->skip2;
        u2.push_back(u);
        x->count(8.0 * x->N_ * total + 2.0 * x->N8() * nb);
      }
      ts_update_batch(nb, u1, up, s);
      std::vector<int> nb2;
      tsgemm_tn_batch(nb, p2, nb2, up, s);
      ts_update_batch(nb, u2, up, s);
    }
    // Cholesky QR twice: the Gram partial sums of T, then two fused steps
    {
      std::vector<BatchProj> pg;
      for (Solver* x : a) {
        double* T = x->V_ + x->gc_ * x->ld_;
        BatchProj q{};
        q.segs[0] = Seg{T, nb, x->ld_};
        q.nseg = 1;
        q.N = x->N_;
        q.T = T;
        q.ldt = x->ld_;
        q.partial = x->partial_;
        pg.push_back(q);
        x->count(x->N8() * nb * 6.0);
      }
      std::vector<int> nbk, nb2, unused;
      tsgemm_tn_batch(nb, pg, nbk, up, s);
      std::vector<BatchCholQR> c1, c2;
      for (size_t j = 0; j < a.size(); ++j) {
        Solver* x = a[j];
        double* T = x->V_ + x->gc_ * x->ld_;
        const int total = x->gc_;
        c1.push_back(BatchCholQR{x->partial_, nbk[j], 1, x->d_->C0 + total, total + nb, x->d_->R1,
                                 x->d_->R1inv, &x->d_->bad, T, x->ld_, x->N_, nullptr, x->cqrP_});
      }
      cholqr_batch(nb, c1, nb2, up, s);
      for (size_t j = 0; j < a.size(); ++j) {
        Solver* x = a[j];
        double* T = x->V_ + x->gc_ * x->ld_;
        c2.push_back(BatchCholQR{x->cqrP_, nb2[j], 2, nullptr, 0, x->d_->R2, x->d_->R2inv,
                                 &x->d_->bad, T, x->ld_, x->N_, x->Tc_, nullptr});
      }
      cholqr_batch(nb, c2, unused, up, s);
    }
    // W's new columns: C T by A then A^T, then into the basis layout
    products(a, nb);
    std::vector<BatchUnpack> un;
    std::vector<BatchProj> ph;
    for (Solver* x : a) {
      double* Wcol = x->W_ + x->gc_ * x->ld_;
      un.push_back(BatchUnpack{x->Wc_, x->N_, Wcol, x->ld_});
      BatchProj q{};
      q.segs[0] = Seg{x->V_, x->gc_ + nb, x->ld_};
      q.nseg = 1;
      q.N = x->N_;
      q.T = Wcol;
      q.ldt = x->ld_;
      q.partial = x->partial_;
      ph.push_back(q);
      x->count(2.0 * x->N8() * nb + x->N8() * (x->gc_ + 2 * nb));
    }
    unpack_batch(nb, un, up, s);
    std::vector<int> nbh;
    tsgemm_tn_batch(nb, ph, nbh, up, s);
    std::vector<HAppendArgs> ha;
    std::vector<ExtractArgs> ex;
    for (size_t j = 0; j < a.size(); ++j) {
      Solver* x = a[j];
      ha.push_back(HAppendArgs{x->d_, x->gc_, nb, x->partial_, nbh[j]});
    }
    small_h_append_batch(ha, up, s);
    for (Solver* x : a) {
      x->gc_ += nb;
      x->s1_.last_nb = nb;
      ++x->s1_.iters;
      ex.push_back(ExtractArgs{x->d_, x->gc_, x->largest_ ? 1 : 0});
    }
    small_extract_batch(ex, up, s);
  }

  // stage 1 of every solver, from s1_begin (done) to the round its control
  // step ends it
  void run() {
    up.init((size_t)64 << 20, s);
    std::vector<Solver*> act = sv;  // solvers still in stage 1
    std::vector<Solver*> live = sv; // solvers whose residual and control run this round
    const bool verbose = std::getenv("SVDS_DEBUG") != nullptr;
    double t_enq = 0.0, t_wait = 0.0;
    int64_t rounds = 0;
    while (!act.empty()) {
      const double ta = now();
      ++rounds;
      residual(live);
      std::vector<ControlArgs> ca;
      for (Solver* x : live) ca.push_back(x->control_args(x->s1_params(std::min(x->gc_, x->k_ + x->b_))));
      small_control_batch(ca, up, s);
      const double tb = now();
      t_enq += tb - ta;
      std::vector<std::pair<Solver*, Ctl>> go;
      std::vector<Solver*> next;
      for (Solver* x : live) {
        const Ctl c = x->control_wait();
        x->trace("s1b", (int)x->s1_.iters, c, std::min(x->gc_, x->k_ + x->b_));
        const int what = x->s1_decide(c);
        if (what == 1) continue;  // stage 1 ends for this solver
        next.push_back(x);
        if (what == 0) go.push_back({x, c});
      }
      up.reset();  // every copy of this round has executed (the records were read)
      const double tc = now();
      t_wait += tc - tb;
      act = next;
      // restarts, then the corrections of each block width
      std::vector<BatchGemm> rs;
      std::vector<std::pair<Solver*, int>> restarted;
      for (auto& q : go) {
        Solver* x = q.first;
        const Ctl& c = q.second;
        if (!c.restart) continue;
        x->count(2.0 * x->N8() * (x->gc_ + c.nr));
        rs.push_back(BatchGemm{x->V_, x->ld_, x->gc_, x->N_, x->d_->Yr, kLd, c.nr, x->Vt_, x->ld_});
        rs.push_back(BatchGemm{x->W_, x->ld_, x->gc_, x->N_, x->d_->Yr, kLd, c.nr, x->Wt_, x->ld_});
        restarted.push_back({x, c.nr});
      }
      ts_gemm_nn_batch(rs, up, s);
      for (auto& q : restarted) q.first->s1_restarted(q.second);
      std::map<int, std::vector<Solver*>> byb;
      for (auto& q : go) {
        Solver* x = q.first;
        int nb = q.second.nblock;
        if (nb == 0) {  // nothing left to correct: a random block (rare)
          nb = x->b_;
          x->count(x->N8() * nb);
          x->fill_random_block(nb);
          x->ortho_and_append(nb);
          continue;
        }
        byb[nb].push_back(x);
      }
      for (auto& g : byb) expand(g.second, g.first);
      live = act;
      t_enq += now() - tc;
    }
    SVDS_HIP(hipStreamSynchronize(s));
    if (verbose)
      std::fprintf(stderr, "[svds] in step: %zu solvers, %lld rounds, host %.3f s enqueuing, "
                           "%.3f s waiting for control records\n",
                   sv.size(), (long long)rounds, t_enq, t_wait);
  }
};

}  // namespace svds

// ===========================================================================
// C ABI
// ===========================================================================
using svds::Error;
using svds::guarded;

namespace {

// Device arrays of a prepared matrix: plain allocations for handles made by
// svds_matrix_create, stream-ordered ones (on the call's stream) for the
// transient handle inside svds_solve, so that concurrent solves on different
// streams do not synchronise the device on every allocation and release.
struct MemMode {
  bool async;
  hipStream_t s;
  template <class T>
  void alloc(T** p, size_t count) const {
    const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
    if (async) *p = static_cast<T*>(svds::stream_alloc(bytes, s));
    else SVDS_HIP(hipMalloc((void**)p, bytes));
  }
  void release(void* p) const {
    if (!p) return;
    if (async) svds::stream_free(p, s);
    else (void)hipFree(p);
  }
};

// Arrays carved, 256-byte aligned and in request order, from one block: a
// first pass with no block only sums the sizes, a second hands out pointers.
// A handle's arrays live in two blocks (the matrices with diag(C), the
// one-pass product's plan), one allocation and one release each.
struct Carve {
  char* base = nullptr;
  size_t used = 0;
  template <class T>
  void take(T** p, size_t count) {
    const size_t off = (used + 255) & ~static_cast<size_t>(255);
    used = off + sizeof(T) * std::max<size_t>(count, 1);
    *p = base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
};

using svds::StreamScratch;

void carve_csr(svds::Csr32& c, int64_t rows, int64_t cols, int64_t nnz, Carve& k) {
  c.rows = rows;
  c.cols = cols;
  c.nnz = nnz;
  k.take(&c.rp, rows + 1);
  k.take(&c.ci, nnz);
  k.take(&c.val, nnz);
  k.take(&c.binrows, rows);
  k.take(&c.val32, nnz);
}

// Plan of the one-pass A^T A product (k_gram.hip).  The windows are measured
// on blocks of kGramMinRows rows and merged on the host for the candidate
// block heights; the tallest block height whose blocks stay within the LDS
// limits is kept.  No plan when the windows' first columns decrease, or when
// the windows together would exceed four times the column count (their
// partial sums would cost more traffic than the second product saves).
void build_gram_plan(svds_matrix* h, const MemMode& mm, hipStream_t s) {
  const svds::Csr32& A = h->A;
  constexpr int F = svds::kGramMinRows;
  const int64_t nf = (A.rows + F - 1) / F;
  if (A.nnz <= 0 || nf <= 0) return;
  std::vector<int32_t> flo(nf), fhi(nf), fnz(nf);
  {
    const StreamScratch w(sizeof(int32_t) * 3 * nf, s);
    int32_t* d = w.as<int32_t>();
    svds::gram_windows(A, nf, d, d + nf, d + 2 * nf, s);
    SVDS_HIP(hipMemcpyAsync(flo.data(), d, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
    SVDS_HIP(hipMemcpyAsync(fhi.data(), d + nf, sizeof(int32_t) * nf, hipMemcpyDeviceToHost, s));
    SVDS_HIP(hipMemcpyAsync(fnz.data(), d + 2 * nf, sizeof(int32_t) * nf, hipMemcpyDeviceToHost,
                            s));
  }
  SVDS_HIP(hipStreamSynchronize(s));
  for (int R = svds::kGramMaxRows; R >= F; R /= 2) {
    const int64_t k = R / F;
    const int64_t nb = (nf + k - 1) / k;
    std::vector<int32_t> lo(nb), hi(nb);
    std::vector<int64_t> poff(nb + 1, 0);
    bool ok = true;
    int32_t prev = 0;
    for (int64_t b = 0; b < nb && ok; ++b) {
      int32_t mn = INT32_MAX, mx = -1;
      int64_t nz = 0;
      for (int64_t f = b * k; f < std::min(nf, (b + 1) * k); ++f) {
        mn = std::min(mn, flo[f]);
        mx = std::max(mx, fhi[f]);
        nz += fnz[f];
      }
      if (mx < 0) {  // empty block: an empty window at the previous start
        mn = prev;
        mx = prev - 1;
      }
      ok = nz <= svds::kGramMaxNnz && mx - mn + 1 <= svds::kGramMaxWidth && mn >= prev;
      lo[b] = mn;
      hi[b] = mx;
      prev = mn;
      poff[b + 1] = poff[b] + (mx - mn + 1);
    }
    if (!ok) continue;
    if (poff[nb] > 4 * A.cols) return;  // shorter blocks only add overlap
    svds::GramPlan& g = h->G;
    g.R = R;
    g.nblk = nb;
    g.wsum = poff[nb];
    auto lay = [&](Carve& c) {
      c.take(&g.lo, nb);
      c.take(&g.hi, nb);
      c.take(&g.poff, nb + 1);
      c.take(&g.colptr, g.wsum + nb);
      c.take(&g.cidx, A.nnz);
      c.take(&g.cover, A.cols);
    };
    Carve size;
    lay(size);
    Carve c;
    mm.alloc(&c.base, size.used);
    h->gram_block = c.base;
    lay(c);
    SVDS_HIP(hipMemcpyAsync(g.lo, lo.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
    SVDS_HIP(hipMemcpyAsync(g.hi, hi.data(), sizeof(int32_t) * nb, hipMemcpyHostToDevice, s));
    SVDS_HIP(hipMemcpyAsync(g.poff, poff.data(), sizeof(int64_t) * (nb + 1),
                            hipMemcpyHostToDevice, s));
    svds::gram_build(A, g, s);
    SVDS_HIP(hipStreamSynchronize(s));  // the host vectors above end here
    return;
  }
}

void destroy_matrix(svds_matrix* h) {
  if (!h) return;
  const MemMode mm{h->stream_ordered, h->owner};
  mm.release(h->block);
  mm.release(h->gram_block);
  delete h;
}

int create_matrix(const svds_csr* A, svds_matrix** out, hipStream_t s, bool stream_ordered) {
  if (!A || !out) throw Error(SVDS_ERR_ARG, "null argument");
  if (A->m <= 0 || A->n <= 0 || A->nnz < 0 || !A->rowptr || (A->nnz > 0 && (!A->colind || !A->values)))
    throw Error(SVDS_ERR_ARG, "bad sizes or pointers");
  if (A->nnz >= (int64_t)INT32_MAX || A->m >= (int64_t)INT32_MAX || A->n >= (int64_t)INT32_MAX)
    throw Error(SVDS_ERR_ARG, "matrix too large for 32-bit indices");
  // row pointer ends and the structure check
  int64_t ends[2] = {0, 0};
  SVDS_HIP(hipMemcpyAsync(&ends[0], A->rowptr, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  SVDS_HIP(hipMemcpyAsync(&ends[1], A->rowptr + A->m, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  int flag = 0;
  {
    const StreamScratch f(sizeof(int), s);
    SVDS_HIP(hipMemsetAsync(f.p, 0, sizeof(int), s));
    svds::check_csr(*A, f.as<int>(), s);
    SVDS_HIP(hipMemcpyAsync(&flag, f.p, sizeof(int), hipMemcpyDeviceToHost, s));
  }
  SVDS_HIP(hipStreamSynchronize(s));
  if (ends[0] != 0 || ends[1] != A->nnz || flag) throw Error(SVDS_ERR_CSR, "malformed CSR");

  auto* h = new svds_matrix();
  const MemMode mm{stream_ordered, s};
  h->owner = s;
  h->stream_ordered = stream_ordered;
  try {
    SVDS_HIP(hipGetDevice(&h->device));
    h->m = A->m;
    h->n = A->n;
    h->nnz = A->nnz;
    h->transposed = A->m < A->n;
    // A and its transpose, owned by the handle from their allocation on (so
    // that destroy_matrix releases them if a later step fails); swapped
    // into A_w and A_w^T at the end
    svds::Csr32& a = h->A;
    svds::Csr32& at = h->At;
    double* diag = nullptr;  // diag(A_w^T A_w): A_w has min(m, n) columns
    auto lay = [&](Carve& k) {
      carve_csr(a, A->m, A->n, A->nnz, k);
      carve_csr(at, A->n, A->m, A->nnz, k);
      k.take(&diag, std::min(A->m, A->n));
    };
    Carve size;
    lay(size);
    Carve k;
    mm.alloc(&k.base, size.used);
    h->block = k.base;
    lay(k);
    svds::copy_csr_arrays(*A, a, s);
    {
      const StreamScratch cursor(sizeof(int32_t) * (A->n + 1), s);
      svds::transpose_csr(a, at, cursor.as<int32_t>(), s);
    }
    svds::build_bins(a, s);
    svds::build_bins(at, s);
    // FP32 copies of the values for the mixed-precision stage 1
    svds::to_fp32(a.val, a.val32, A->nnz, s);
    svds::to_fp32(at.val, at.val32, A->nnz, s);
    if (h->transposed) std::swap(h->A, h->At);
    h->diagC = diag;
    svds::row_sqnorms(h->At, h->diagC, s);  // rows of A_w^T = columns of A_w
    build_gram_plan(h, mm, s);
    SVDS_HIP(hipStreamSynchronize(s));
  } catch (...) {
    destroy_matrix(h);
    throw;
  }
  *out = h;
  return SVDS_OK;
}

svds_opts default_opts() {
  svds_opts o;
  std::memset(&o, 0, sizeof(o));
  o.max_prev_retain = -1;
  o.two_sided_cleanup = 1;
  o.autotune = 1;
  o.fused_gram = 1;
  o.stage2_solver = SVDS_STAGE2_JD;
  return o;
}

// Launch shapes of the products with A_w and A_w^T for block width b (FP32
// products when fp32): the handle's table entry if a solve already fixed one,
// else tuned on the copies a, at (or the rule of thumb when tune is false,
// which is not stored) and published; when two solves tune at once, the first
// to publish wins and both use its shapes.
void launch_shapes(const svds_matrix* h, int b, bool fp32, bool tune, svds::Csr32& a,
                   svds::Csr32& at, hipStream_t s) {
  if (!tune) {
    a.merged_bin = a.heuristic_bin;
    a.unroll = a.heuristic_unroll;
    at.merged_bin = at.heuristic_bin;
    at.unroll = at.heuristic_unroll;
    return;
  }
  const std::pair<int, int> key(b, fp32 ? 1 : 0);
  auto apply = [&](const std::array<int, 4>& v) {
    a.merged_bin = v[0];
    a.unroll = v[1];
    at.merged_bin = v[2];
    at.unroll = v[3];
  };
  {
    std::lock_guard<std::mutex> lk(h->shape_mu);
    auto it = h->shapes.find(key);
    if (it != h->shapes.end()) {
      apply(it->second);
      return;
    }
  }
  svds::autotune_spmm(a, b, fp32, s);
  svds::autotune_spmm(at, b, fp32, s);
  std::lock_guard<std::mutex> lk(h->shape_mu);
  auto ins = h->shapes.emplace(key, std::array<int, 4>{a.merged_bin, a.unroll, at.merged_bin,
                                                       at.unroll});
  apply(ins.first->second);
}

// options with their defaults and range checks
svds_opts checked_opts(const svds_matrix* h, int k, int target, const svds_opts* opts) {
  if (!h) throw Error(SVDS_ERR_ARG, "null argument");
  if (target != SVDS_LARGEST && target != SVDS_SMALLEST) throw Error(SVDS_ERR_ARG, "target");
  const int64_t mn = std::min(h->m, h->n);
  if (k < 1 || k > mn || k > svds::kKmax) throw Error(SVDS_ERR_ARG, "k out of range");
  svds_opts o = opts ? *opts : default_opts();
  if (o.precision != SVDS_FP64 && o.precision != SVDS_MIXED) throw Error(SVDS_ERR_ARG, "precision");
  if (o.precond != SVDS_PC_NONE && o.precond != SVDS_PC_JACOBI && o.precond != SVDS_PC_LEARNED &&
      o.precond != SVDS_PC_BLOCKJACOBI)
    throw Error(SVDS_ERR_ARG, "precond");
  if (o.precond == SVDS_PC_BLOCKJACOBI && (o.pc_block < 0 || o.pc_block > 128))
    throw Error(SVDS_ERR_ARG, "block-Jacobi block size 1..128");
  if (o.precond == SVDS_PC_LEARNED && (!o.pc_model || o.pc_degree < 0 || o.pc_degree > 15))
    throw Error(SVDS_ERR_ARG, "learned preconditioner: pc_model / pc_degree");
  if (o.method != SVDS_METHOD_HYBRID && o.method != SVDS_METHOD_NORMAL &&
      o.method != SVDS_METHOD_AUGMENTED)
    throw Error(SVDS_ERR_ARG, "method");
  if (o.method == SVDS_METHOD_AUGMENTED && target != SVDS_LARGEST)
    throw Error(SVDS_ERR_ARG, "the augmented method alone seeks the largest values only");
  if (o.stage2_solver != SVDS_STAGE2_GDK && o.stage2_solver != SVDS_STAGE2_JD)
    throw Error(SVDS_ERR_ARG, "stage2_solver");
  if (o.relative_tol && o.method != SVDS_METHOD_NORMAL)
    throw Error(SVDS_ERR_ARG, "the relative stopping rule needs the normal-equations method");
  return o;
}

int solve_prepared(const svds_matrix* h, int k, int target, double tol, const svds_opts* opts,
                   double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
                   void* workspace, size_t workspace_bytes, svds_stats* stats, hipStream_t s,
                   svds::Solver::Capture* cap = nullptr) {
  const svds_opts o = checked_opts(h, k, target, opts);
  if (!sigma || !U || !V || !rnorm) throw Error(SVDS_ERR_ARG, "null argument");
  if (!(tol > 0.0 && tol < 1.0)) throw Error(SVDS_ERR_ARG, "tol must be in (0, 1)");
  if (ldu < h->m || ldv < h->n) throw Error(SVDS_ERR_ARG, "leading dimension too small");
  svds_stats local;
  svds_stats* st = stats ? stats : &local;
  const int b = o.block_size > 0 ? o.block_size : 1;
  svds::Csr32 a = h->A, at = h->At, a32 = h->A, at32 = h->At;
  launch_shapes(h, b, false, o.autotune != 0, a, at, s);
  if (o.precision == SVDS_MIXED) launch_shapes(h, b, true, o.autotune != 0, a32, at32, s);
  svds::Solver solver(h, a, at, a32, at32, k, target, tol, o, s);
  if (cap) {
    if (o.precision != SVDS_FP64) throw Error(SVDS_ERR_ARG, "residual capture needs FP64");
    solver.set_capture(cap);
  }
  if (workspace) solver.use_workspace(workspace, workspace_bytes);
  return solver.run(sigma, U, ldu, V, ldv, rnorm, st);
}

}  // namespace

extern "C" {

int svds_opts_init(svds_opts* opts) {
  if (!opts) return SVDS_ERR_ARG;
  *opts = default_opts();
  return SVDS_OK;
}

const char* svds_error_string(int code) {
  switch (code) {
    case SVDS_OK: return "ok";
    case SVDS_NOT_CONVERGED: return "not converged within the matrix-vector budget";
    case SVDS_ERR_ARG: return "invalid argument";
    case SVDS_ERR_CSR: return "malformed CSR matrix";
    case SVDS_ERR_OOM: return "device out of memory";
    case SVDS_ERR_HIP: return "HIP runtime error";
    case SVDS_ERR_BREAKDOWN: return "numerical breakdown";
    default: return "unknown status";
  }
}

int svds_matrix_create(const svds_csr* A, svds_matrix** out, void* stream) {
  return guarded([&] { return create_matrix(A, out, (hipStream_t)stream, false); });
}

int svds_matrix_destroy(svds_matrix* h) {
  destroy_matrix(h);
  return SVDS_OK;
}

int svds_matrix_normal(const svds_matrix* h, int b, const double* X, double* Z, int fused,
                       int* used, void* stream) {
  return guarded([&] {
    if (!h || !X || !Z || b < 1 || b > svds::kMaxBlock) throw Error(SVDS_ERR_ARG, "normal args");
    const hipStream_t s = (hipStream_t)stream;
    const svds::Csr32& A = h->A;
    const bool one = fused && h->G.R > 0 && svds::gram_cheaper(A, h->G, b);
    if (used) *used = one ? 1 : 0;
    if (one) {
      const StreamScratch P(sizeof(double) * h->G.wsum * b, s);
      svds::gram_partial(A, h->G, b, X, P.as<double>(), s);
      svds::gram_combine(h->G, A.cols, b, P.as<double>(), Z, 0, s);
    } else {
      const StreamScratch Y(sizeof(double) * A.rows * b, s);
      svds::spmm(A, b, X, Y.as<double>(), s);
      svds::spmm(h->At, b, Y.as<double>(), Z, s);
    }
    return SVDS_OK;
  });
}

int svds_matrix_spmm(const svds_matrix* h, int trans, int b, const double* X, double* Y,
                     void* stream) {
  return guarded([&] {
    if (!h || !X || !Y || b < 1 || b > svds::kMaxBlock) throw Error(SVDS_ERR_ARG, "spmm args");
    // the caller's A: A = A_w (not transposed) or A_w^T (transposed)
    const bool use_w = (trans == 0) != h->transposed;
    svds::spmm(use_w ? h->A : h->At, b, X, Y, (hipStream_t)stream);
    return SVDS_OK;
  });
}

int svds_solve_prepared(const svds_matrix* h, int k, int target, double tol,
                        const svds_opts* opts, double* sigma, double* U, int64_t ldu, double* V,
                        int64_t ldv, double* rnorm, void* workspace, size_t workspace_bytes,
                        svds_stats* stats, void* stream) {
  return guarded([&] {
    return solve_prepared(h, k, target, tol, opts, sigma, U, ldu, V, ldv, rnorm, workspace,
                          workspace_bytes, stats, (hipStream_t)stream);
  });
}

int svds_workspace_size(const svds_matrix* h, int k, int target, const svds_opts* opts,
                        size_t* bytes) {
  return guarded([&] {
    if (!bytes) throw Error(SVDS_ERR_ARG, "null argument");
    const svds_opts o = checked_opts(h, k, target, opts);
    // the launch shapes do not change the arrays: the handle's descriptors serve
    svds::Solver solver(h, h->A, h->At, h->A, h->At, k, target, 0.5, o, nullptr);
    *bytes = solver.workspace_bytes();
    return SVDS_OK;
  });
}

int svds_stream_release(void* stream) {
  return guarded([&] {
    svds::stream_cache_drop((hipStream_t)stream);
    return SVDS_OK;
  });
}

int svds_solve(const svds_csr* A, int k, int target, double tol, const svds_opts* opts,
               double* sigma, double* U, int64_t ldu, double* V, int64_t ldv, double* rnorm,
               svds_stats* stats, void* stream) {
  return guarded([&] {
    const double t0 = svds::now();
    svds_matrix* h = nullptr;
    create_matrix(A, &h, (hipStream_t)stream, true);
    struct Guard {
      svds_matrix* h;
      ~Guard() { destroy_matrix(h); }
    } g{h};
    const double t1 = svds::now();
    int rc = solve_prepared(h, k, target, tol, opts, sigma, U, ldu, V, ldv, rnorm, nullptr, 0,
                            stats, (hipStream_t)stream);
    if (stats) stats->setup_seconds += t1 - t0;
    return rc;
  });
}

namespace {

// the previous design of the batched solve: host workers, each driving its
// own stream through whole solves (used when the options do not allow the
// solves to run in step)
int solve_batched_workers(int nprob, const svds_csr* A, int k, int target, double tol,
                          const svds_opts* opts, double* const* sigma, double* const* U,
                          const int64_t* ldu, double* const* V, const int64_t* ldv,
                          double* const* rnorm, svds_stats* stats, int nworkers, void* stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return SVDS_ERR_HIP;
  const int nw = std::max(1, std::min(nprob, nworkers > 0 ? nworkers : 16));
  std::vector<int> rc(nprob, SVDS_OK);
  std::atomic<int> next{0};
  std::vector<hipStream_t> streams(nw, nullptr);
  for (int w = 0; w < nw; ++w)
    if (hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess) {
      for (int q = 0; q < w; ++q) (void)hipStreamDestroy(streams[q]);
      return SVDS_ERR_HIP;
    }
  // the problems' inputs were produced on the caller's stream
  if (stream) {
    hipEvent_t ready;
    if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(ready, (hipStream_t)stream);
      for (int w = 0; w < nw; ++w) (void)hipStreamWaitEvent(streams[w], ready, 0);
      (void)hipEventDestroy(ready);
    }
  }
  auto work = [&](int w) {
    (void)hipSetDevice(dev);
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= nprob) break;
      rc[i] = svds_solve(&A[i], k, target, tol, opts, sigma[i], U[i], ldu[i], V[i], ldv[i],
                         rnorm[i], stats ? &stats[i] : nullptr, streams[w]);
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& t : pool) t.join();
  // make the caller's stream wait for every worker stream
  for (int w = 0; w < nw; ++w) {
    hipEvent_t done;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) == hipSuccess) {
      (void)hipEventRecord(done, streams[w]);
      if (stream) (void)hipStreamWaitEvent((hipStream_t)stream, done, 0);
      else (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    (void)hipStreamSynchronize(streams[w]);
    svds::stream_cache_drop(streams[w]);  // blocks kept for a stream that ends here
    (void)hipStreamSynchronize(streams[w]);
    (void)hipStreamDestroy(streams[w]);
  }
  int worst = SVDS_OK;
  for (int x : rc) {
    if (x < 0 && (worst >= 0 || x < worst)) worst = x;
    else if (worst >= 0 && x > worst) worst = x;
  }
  return worst;
}

// problems solved in step per group: the group's arrays live together
constexpr int kStepGroup = 256;
// host threads (and streams) of the in-step solve's set-up and clean-up,
// unless the caller names a number
constexpr int kStepWorkers = 16;

// f(w, j) for problem j of [0, np) on worker w, problems dealt round-robin
// over nw host threads (worker 0 is the calling thread); the first exception
// is rethrown after every worker has finished
void deal(int nw, int np, int dev, const std::function<void(int, int)>& f) {
  std::mutex mu;
  std::exception_ptr first;
  auto work = [&](int w) {
    try {
      (void)hipSetDevice(dev);
      for (int j = w; j < np; j += nw) f(w, j);
    } catch (...) {
      std::lock_guard<std::mutex> lk(mu);
      if (!first) first = std::current_exception();
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < nw; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& t : pool) t.join();
  if (first) std::rethrow_exception(first);
}

// the solves of problems [i0, i1) in step (their inputs checked): matrix
// set-up, norm estimates and the first block on the worker streams ws, one
// host thread each; stage 1 of every eligible solver in step on stream s;
// clean-up again on the worker streams.  rc: per-problem status
void solve_in_step(int i0, int i1, const svds_csr* A, int k, int target, double tol,
                   const svds_opts& o, double* const* sigma, double* const* U,
                   const int64_t* ldu, double* const* V, const int64_t* ldv,
                   double* const* rnorm, svds_stats* stats, hipStream_t s,
                   const std::vector<hipStream_t>& ws, int dev, std::vector<int>& rc) {
  const int np = i1 - i0;
  const int nw = std::max(1, std::min<int>((int)ws.size(), np));
  std::vector<svds_matrix*> hs(np, nullptr);
  struct Guard {
    std::vector<svds_matrix*>& h;
    ~Guard() {
      for (svds_matrix* x : h) destroy_matrix(x);
    }
  } guard{hs};
  std::vector<std::unique_ptr<svds::Solver>> sol(np);
  std::vector<svds_stats> local(np);
  const int b = o.block_size > 0 ? o.block_size : 1;
  const bool verbose = std::getenv("SVDS_DEBUG") != nullptr;
  const double t0 = svds::now();
  deal(nw, np, dev, [&](int w, int j) {
    const int i = i0 + j;
    create_matrix(&A[i], &hs[j], ws[w], true);
    if (ldu[i] < hs[j]->m || ldv[i] < hs[j]->n)
      throw Error(SVDS_ERR_ARG, "leading dimension too small");
    checked_opts(hs[j], k, target, &o);
    svds::Csr32 a = hs[j]->A, at = hs[j]->At;
    launch_shapes(hs[j], b, false, o.autotune != 0, a, at, ws[w]);
    sol[j].reset(new svds::Solver(hs[j], a, at, a, at, k, target, tol, o, ws[w]));
    sol[j]->prepare(stats ? &stats[i] : &local[j]);
  });
  for (int w = 0; w < nw; ++w) SVDS_HIP(hipStreamSynchronize(ws[w]));
  const double t1 = svds::now();
  std::vector<svds::Solver*> step;
  for (int j = 0; j < np; ++j)
    if (svds::BatchStage1::eligible(*sol[j])) step.push_back(sol[j].get());
  for (svds::Solver* x : step) {
    x->set_stream(s);
    x->s1_start();
  }
  if (!step.empty()) {
    svds::BatchStage1 bs;
    bs.sv = step;
    bs.s = s;
    bs.run();  // ends with s synchronised
  }
  const double t2 = svds::now();
  deal(nw, np, dev, [&](int w, int j) {
    const int i = i0 + j;
    svds_stats* st = stats ? &stats[i] : &local[j];
    svds::Solver* x = sol[j].get();
    x->set_stream(ws[w]);
    const bool done = svds::BatchStage1::eligible(*x);
    if (done) {
      int status1 = 2;
      x->s1_end_default(&status1, st);
      st->stage1_status = status1;
    }
    rc[i] = x->complete(sigma[i], U[i], ldu[i], V[i], ldv[i], rnorm[i], st, done);
  });
  for (int w = 0; w < nw; ++w) SVDS_HIP(hipStreamSynchronize(ws[w]));
  const double t3 = svds::now();
  sol.clear();  // the solvers' arrays back to their streams' caches
  for (svds_matrix*& h : hs) {
    destroy_matrix(h);
    h = nullptr;
  }
  if (verbose)
    std::fprintf(stderr, "[svds] in step group of %d: set-up %.3f s, stage 1 %.3f s, "
                         "clean-up %.3f s on %d host threads, release %.3f s\n",
                 np, t1 - t0, t2 - t1, t3 - t2, nw, svds::now() - t3);
}

}  // namespace

int svds_solve_batched(int nprob, const svds_csr* A, int k, int target, double tol,
                       const svds_opts* opts, double* const* sigma, double* const* U,
                       const int64_t* ldu, double* const* V, const int64_t* ldv,
                       double* const* rnorm, svds_stats* stats, int nworkers, void* stream) {
  if (nprob < 0 || (nprob > 0 && (!A || !sigma || !U || !ldu || !V || !ldv || !rnorm)))
    return SVDS_ERR_ARG;
  if (nprob == 0) return SVDS_OK;
  const svds_opts o = opts ? *opts : default_opts();
  // in step: FP64 stage 1 with no preconditioner or point Jacobi, no timing
  const bool step = nworkers <= 0 && o.precision == SVDS_FP64 &&
                    o.method != SVDS_METHOD_AUGMENTED &&
                    (o.precond == SVDS_PC_NONE || o.precond == SVDS_PC_JACOBI) && !o.profile;
  if (!step)
    return solve_batched_workers(nprob, A, k, target, tol, opts, sigma, U, ldu, V, ldv, rnorm,
                                 stats, nworkers < 0 ? -nworkers : nworkers, stream);
  std::vector<int> rc(nprob, SVDS_OK);
  const int code = guarded([&] {
    if (target != SVDS_LARGEST && target != SVDS_SMALLEST) throw Error(SVDS_ERR_ARG, "target");
    if (!(tol > 0.0 && tol < 1.0)) throw Error(SVDS_ERR_ARG, "tol must be in (0, 1)");
    int dev = 0;
    SVDS_HIP(hipGetDevice(&dev));
    const hipStream_t s = (hipStream_t)stream;
    // the worker streams of set-up and clean-up; they wait for the caller's
    // stream (the problems' inputs) and the caller's stream waits for them
    const int nw = std::min(nprob, nworkers < 0 ? -nworkers : kStepWorkers);
    const bool verbose = std::getenv("SVDS_DEBUG") != nullptr;
    const double ta = svds::now();
    struct Streams {
      std::vector<hipStream_t> v;
      bool verbose;
      ~Streams() {
        const double t = svds::now();
        for (hipStream_t x : v) {
          (void)hipStreamSynchronize(x);
          svds::stream_cache_drop(x);  // blocks kept for a stream that ends here
          (void)hipStreamSynchronize(x);
          (void)hipStreamDestroy(x);
        }
        if (verbose)
          std::fprintf(stderr, "[svds] batched: worker streams released in %.3f s\n", svds::now() - t);
      }
    } ws{{}, verbose};
    for (int w = 0; w < nw; ++w) {
      hipStream_t x = nullptr;
      SVDS_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
      ws.v.push_back(x);
    }
    {
      hipEvent_t ready;
      SVDS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
      (void)hipEventRecord(ready, s);
      for (hipStream_t x : ws.v) (void)hipStreamWaitEvent(x, ready, 0);
      (void)hipEventDestroy(ready);
    }
    const double tb = svds::now();
    for (int i0 = 0; i0 < nprob; i0 += kStepGroup)
      solve_in_step(i0, std::min(nprob, i0 + kStepGroup), A, k, target, tol, o, sigma, U, ldu,
                    V, ldv, rnorm, stats, s, ws.v, dev, rc);
    if (verbose)
      std::fprintf(stderr, "[svds] batched: streams created in %.3f s, groups %.3f s\n", tb - ta,
                   svds::now() - tb);
    return SVDS_OK;
  });
  if (code != SVDS_OK) return code;
  int worst = SVDS_OK;
  for (int x : rc) {
    if (x < 0 && (worst >= 0 || x < worst)) worst = x;
    else if (worst >= 0 && x > worst) worst = x;
  }
  return worst;
}


// ---- learned preconditioner ------------------------------------------------
namespace {
void check_degree(int degree) {
  if (degree < 0 || degree > svds::kLpcMaxDegree) throw Error(SVDS_ERR_ARG, "degree out of range");
}
}  // namespace

int svds_lpc_init(float* params, uint64_t seed, const float* out_bias, void* stream) {
  return guarded([&] {
    if (!params) throw Error(SVDS_ERR_ARG, "null params");
    using namespace svds;
    std::vector<float> h(kLpcNParams, 0.0f);
    auto fill = [&](int off, int fan_in, int count, uint64_t strm) {
      // uniform on [-sqrt(3/fan_in), sqrt(3/fan_in)): variance 1/fan_in
      const double a = 2.0 * std::sqrt(3.0 / fan_in);
      for (int i = 0; i < count; ++i) h[off + i] = (float)(a * counter_uniform(seed, strm, 0, i));
    };
    fill(kW1, 2 * kLpcNF, 2 * kLpcNF * kLpcHid, 101);
    fill(kW2, 2 * kLpcHid, 2 * kLpcHid * kLpcHid, 102);
    if (out_bias)
      for (int m = 0; m < kLpcOut; ++m) h[kB3 + m] = out_bias[m];
    hipStream_t s = (hipStream_t)stream;
    SVDS_HIP(hipMemcpyAsync(params, h.data(), sizeof(float) * kLpcNParams, hipMemcpyHostToDevice, s));
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_features(const svds_matrix* A, float* feat, void* stream) {
  return guarded([&] {
    if (!A || !feat) throw Error(SVDS_ERR_ARG, "null argument");
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    svds::LpcOp op;
    svds::lpc_prepare(A, op, buf, s);
    svds::lpc_features(op, feat, s);
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_forward(const svds_matrix* A, const float* params, const float* feat, int degree,
                     float* coef, float* cache, void* stream) {
  return guarded([&] {
    if (!A || !params || !feat || !coef) throw Error(SVDS_ERR_ARG, "null argument");
    check_degree(degree);
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    svds::LpcOp op;
    svds::lpc_prepare(A, op, buf, s);
    float* c = cache ? cache : buf.get<float>((size_t)op.N * svds::kLpcCacheRow);
    float* gbuf = buf.get<float>((size_t)op.mw * svds::kLpcHid);
    svds::lpc_forward(op, params, feat, degree, coef, c, gbuf, s);
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_backward(const svds_matrix* A, const float* params, const float* cache, int degree,
                      const float* dcoef, float* grad, void* stream) {
  return guarded([&] {
    if (!A || !params || !cache || !dcoef || !grad) throw Error(SVDS_ERR_ARG, "null argument");
    check_degree(degree);
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    svds::LpcOp op;
    svds::lpc_prepare(A, op, buf, s);
    float* work = buf.get<float>((size_t)op.N * (svds::kLpcOut + 3 * svds::kLpcHid));
    float* gbuf = buf.get<float>((size_t)op.mw * svds::kLpcHid);
    float* part = buf.get<float>((size_t)svds::lpc_partial_floats(op.N));
    svds::lpc_backward(op, params, cache, degree, dcoef, grad, false, work, gbuf, part, s);
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_loss(const svds_matrix* A, int np, const double* R, int64_t ldr, const float* coef,
                  int degree, float* dcoef, double* loss, void* stream) {
  return guarded([&] {
    if (!A || !R || !coef || !dcoef || !loss || np < 1) throw Error(SVDS_ERR_ARG, "bad argument");
    check_degree(degree);
    const int64_t N = A->A.cols;
    if (ldr < N) throw Error(SVDS_ERR_ARG, "leading dimension too small");
    hipStream_t s = (hipStream_t)stream;
    svds::LpcSet st(A, np, R, ldr, degree, s);
    SVDS_HIP(hipMemcpyAsync(st.coef, coef, sizeof(float) * N * svds::kLpcCoef,
                            hipMemcpyDeviceToDevice, s));
    svds::DeviceBuffers buf(s);
    double* dl = buf.get<double>(1);
    SVDS_HIP(hipMemsetAsync(dl, 0, sizeof(double), s));
    svds::lpc_loss(st, degree, 1.0, dl, s);
    SVDS_HIP(hipMemcpyAsync(dcoef, st.dcoef, sizeof(float) * N * svds::kLpcCoef,
                            hipMemcpyDeviceToDevice, s));
    SVDS_HIP(hipMemcpyAsync(loss, dl, sizeof(double), hipMemcpyDeviceToHost, s));
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_apply(const svds_matrix* A, const float* coef, int degree, int nb, const double* R,
                   int64_t ldr, double* T, int64_t ldt, void* stream) {
  return guarded([&] {
    if (!A || !coef || !R || !T || nb < 1 || nb > svds::kMaxBlock)
      throw Error(SVDS_ERR_ARG, "bad argument");
    check_degree(degree);
    if (ldr < A->A.cols || ldt < A->A.cols) throw Error(SVDS_ERR_ARG, "leading dimension");
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    svds::LpcOp op;
    svds::lpc_prepare(A, op, buf, s);
    svds::LpcScratch sc;
    svds::lpc_scratch(op, nb, sc, buf);
    svds::lpc_apply(op, coef, degree, nb, R, ldr, T, ldt, sc, s);
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_lpc_adam(int n, float* params, const float* grad, float* m, float* v, int step, float lr,
                  float beta1, float beta2, float eps, void* stream) {
  return guarded([&] {
    if (n < 0 || (n > 0 && (!params || !grad || !m || !v)) || step < 1)
      throw Error(SVDS_ERR_ARG, "bad argument");
    if (n == 0) return SVDS_OK;
    svds::lpc_adam(n, params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    SVDS_HIP(hipStreamSynchronize((hipStream_t)stream));
    return SVDS_OK;
  });
}

int svds_lpc_train(int nsets, const svds_lpc_set* sets, int degree, int steps, float lr,
                   float* params, double* loss_history, void* stream) {
  return guarded([&] {
    if (nsets < 1 || !sets || !params || steps < 0) throw Error(SVDS_ERR_ARG, "bad argument");
    check_degree(degree);
    hipStream_t s = (hipStream_t)stream;
    std::vector<std::unique_ptr<svds::LpcSet>> own;
    std::vector<svds::LpcSet*> ptrs;
    for (int i = 0; i < nsets; ++i) {
      const svds_lpc_set& q = sets[i];
      if (!q.A || q.npairs < 0 || (q.npairs > 0 && (!q.R || q.ldr < q.A->A.cols)))
        throw Error(SVDS_ERR_ARG, "bad training set");
      own.emplace_back(new svds::LpcSet(q.A, q.npairs, q.R, q.ldr, degree, s));
      ptrs.push_back(own.back().get());
    }
    svds::lpc_train(ptrs, degree, steps, lr, params, loss_history, s);
    return SVDS_OK;
  });
}

int svds_collect_residuals(const svds_matrix* A, int k, int target, double tol,
                           const svds_opts* opts, int every, int max_pairs, double* R,
                           int64_t ldr, int* npairs, svds_stats* stats, void* stream) {
  return guarded([&] {
    if (!A || !R || !npairs || every < 1 || max_pairs < 0 || ldr < A->A.cols)
      throw Error(SVDS_ERR_ARG, "bad argument");
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    const int kk = std::max(k, 1);
    double* sig = buf.get<double>(kk);
    double* rn = buf.get<double>(kk);
    double* U = buf.get<double>((size_t)A->m * kk);
    double* V = buf.get<double>((size_t)A->n * kk);
    svds::Solver::Capture cap;
    cap.every = every;
    cap.max = max_pairs;
    cap.R = R;
    cap.ldr = ldr;
    const int rc = solve_prepared(A, k, target, tol, opts, sig, U, A->m, V, A->n, rn, nullptr, 0,
                                  stats, s, &cap);
    SVDS_HIP(hipStreamSynchronize(s));
    *npairs = cap.count;
    return rc;
  });
}

int svds_condest(const svds_matrix* A, double rtol, const svds_opts* opts, double* sigma_max,
                 double* sigma_min, double* kappa, svds_stats* stats, void* stream) {
  return guarded([&] {
    if (!A || !sigma_max || !sigma_min || !kappa) throw Error(SVDS_ERR_ARG, "null argument");
    if (!(rtol > 0.0 && rtol < 1.0)) rtol = 0.1;
    svds_opts o = opts ? *opts : default_opts();
    o.method = SVDS_METHOD_NORMAL;
    o.relative_tol = 1;
    o.block_size = 1;
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    double* sig = buf.get<double>(1);
    double* rn = buf.get<double>(1);
    double* U = buf.get<double>((size_t)A->m);
    double* V = buf.get<double>((size_t)A->n);
    double h[2] = {0.0, 0.0};
    int worst = SVDS_OK;
    for (int t = 0; t < 2; ++t) {
      const int rc = solve_prepared(A, 1, t == 0 ? SVDS_LARGEST : SVDS_SMALLEST, rtol, &o, sig, U,
                                    A->m, V, A->n, rn, nullptr, 0, stats ? &stats[t] : nullptr, s);
      if (rc < 0) return rc;
      worst = std::max(worst, rc);
      SVDS_HIP(hipMemcpyAsync(&h[t], sig, sizeof(double), hipMemcpyDeviceToHost, s));
      SVDS_HIP(hipStreamSynchronize(s));
    }
    *sigma_max = h[0];
    *sigma_min = h[1];
    *kappa = h[1] > 0.0 ? h[0] / h[1] : INFINITY;
    return worst;
  });
}

int svds_blockjacobi_apply(const svds_matrix* A, int nb, int b, const double* R, int64_t ldr,
                           double* T, int64_t ldt, void* stream) {
  return guarded([&] {
    if (!A || !R || !T || b < 1 || b > svds::kMaxBlock || nb < 1 || nb > 128)
      throw Error(SVDS_ERR_ARG, "bad argument");
    const int64_t N = A->A.cols;
    if (ldr < N || ldt < N) throw Error(SVDS_ERR_ARG, "leading dimension");
    hipStream_t s = (hipStream_t)stream;
    svds::DeviceBuffers buf(s);
    double* K = buf.get<double>((size_t)((N + nb - 1) / nb) * nb * nb);
    svds::bj_setup(A, nb, K, s);
    svds::bj_apply(K, nb, N, b, R, ldr, T, ldt, s);
    SVDS_HIP(hipStreamSynchronize(s));
    return SVDS_OK;
  });
}

int svds_small_eig(int g, const double* H, int64_t ldh, int descending, double* theta, double* Y,
                   int64_t ldy, void* stream) {
  return guarded([&] {
    if (!H || !theta || !Y || ldh < g || ldy < g) throw Error(SVDS_ERR_ARG, "small_eig args");
    svds::small_eig(g, H, (int)ldh, descending, theta, Y, (int)ldy, (hipStream_t)stream);
    return SVDS_OK;
  });
}

int svds_small_svd(int g, const double* R, int64_t ldr, double* s, double* Y, int64_t ldy,
                   void* stream) {
  return guarded([&] {
    if (!R || !s || !Y || ldr < g || ldy < g) throw Error(SVDS_ERR_ARG, "small_svd args");
    svds::small_svd(g, R, (int)ldr, s, Y, (int)ldy, nullptr, 0, (hipStream_t)stream);
    return SVDS_OK;
  });
}

}  // extern "C"
