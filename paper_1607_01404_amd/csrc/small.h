// Small replicated objects of the eigensolver (Section 3.3: the projected
// matrix, its eigenvectors, the refined R factor, restart coefficients) and
// the decisions taken from them.  They live in device memory and are worked
// on by single-workgroup kernels, so the iteration never needs the host to do
// arithmetic; the host only reads the decision record back.
#pragma once

#include <cstddef>

#include "common.h"

namespace svds {

constexpr int kLd = 48;          // leading dimension of the small matrices
constexpr int kGmax = 48;        // largest basis the small kernels accept
constexpr int kKmax = 48;        // largest number of wanted triplets

enum Action : int {
  kExpand = 0,      // correct the block and append it
  kExitConverged = 1,
  kExitFloor = 2,   // stage 1 stopped at its attainable accuracy
  kExitBudget = 3,
  kReset = 4,       // recompute W = Op V from a re-orthonormalised V
  kLock = 5,        // stage 2: lock the converged prefix, then restart
  kBreakdown = 6,   // the last block orthogonalisation broke down: roll it back
};

struct Ctl {
  int action;
  int nblock;       // block columns to append
  int restart;      // 1: restart coefficients are in Yr (gc x nr)
  int nr;           // basis size after the restart
  int nlockable;    // stage 2: converged prefix length
  int nconv, npc;   // converged / practically converged among candidates
  int floor_reset;  // the reset confirms the attainable floor
  int eig_sweeps;   // Jacobi sweeps of the last extraction (trace)
  int bad;          // breakdown bitmask of the last block orthogonalisation
  double normop;    // ||Op|| used by the tests
  double maxres;    // largest residual of the wanted pairs
  double minres;
  double res[kKmax + 8];  // candidate residual norms (trace)
  double val[kKmax + 8];  // candidate Ritz values (trace)
  int seq;                // host copy only: the control step's sequence number
  unsigned int sum;       // host copy only: checksum of the words before seq
};

// checksum of a control record's words and its sequence number: a sum of
// per-word mixes, so any order of summation gives it
__host__ __device__ inline unsigned int ctl_mix(unsigned int w, unsigned int i) {
  return (w ^ (i * 0x9E3779B9u)) * (2u * i + 1u);
}

struct Small {
  double H[kLd * kLd];     // V^T Op V
  double Y[kLd * kLd];     // extraction vectors (eigen- or right singular vectors)
  double Yw[kLd * kLd];    // warm start for the eigensolver: H is nearly diagonal in it
  int warm_g;              // its size (-1: none)
  int warm_diag;           // leading block of Yw^T H Yw that is diagonal to rounding
  double theta[kLd];       // Ritz values (refined: y^T H y)
  double sv[kLd];          // refined: singular values of Rr
  double Rr[kLd * kLd];    // refined: R of (W - tau V) = Q Rr
  double Yr[kLd * kLd];    // restart coefficients
  double Qt[kLd * kLd];    // refined restart: R Yr = Qt Rt
  double yprev[kLd * kMaxBlock];  // +k coefficient vectors
  double Hn[(256 + kMaxBlock) * kMaxBlock];  // new columns of the projected matrix
  double C0[(256 + kMaxBlock) * kMaxBlock];  // orthogonalisation coefficients, pass 1
  double C1[256 * kMaxBlock];                // pass 2
  double G[kMaxBlock * kMaxBlock];           // Gram of the block
  double G0[kMaxBlock * kMaxBlock];          // Gram before projection (FP32 bases)
  double R1[kMaxBlock * kMaxBlock], R1inv[kMaxBlock * kMaxBlock];
  double R2[kMaxBlock * kMaxBlock], R2inv[kMaxBlock * kMaxBlock];
  double sums[6 * (kKmax + 8)];              // residual sums
  double best[kKmax + 8];
  int stall[kKmax + 8];
  int blk[kMaxBlock];
  int bad;                // orthogonalisation breakdown bitmask
  int skip2;              // 1: the second Gram-Schmidt pass is not needed
  int stepbad[kGmax];     // breakdown record of each step of the norm estimate
  int nprev, gprev;       // +k vectors: count and rows
  double normop;          // running ||Op||
  int eig_sweeps;
  double res_min;         // smallest candidate residual of the last control step
  double lockval[kKmax];  // stage 2: locked Ritz values
};

// parameters of a control step (by value)
struct CtlParams {
  int stage;        // 1 or 2
  int gc, g, r, p, b, k;
  int nc;           // candidates whose residuals were computed
  int nlock;        // stage 2: vectors locked so far
  int since_reset, floor_resets, budget_hit;
  int refined;
  int rel;          // stage 1: converged when ||r^C|| <= tol |lambda| (relative rule)
  double tol, normA, eps;
  double gate;      // stalled pairs count as at the floor below gate * ||Op||
};

void small_eig(int g, const double* H, int ldh, int descending, double* theta, double* Y, int ldy,
               hipStream_t s);
void small_svd(int g, const double* R, int ldr, double* s, double* Y, int ldy, double* AV,
               int ldav, hipStream_t st);
// H <- [H, Hn; Hn^T] (the new columns Hn, tot = gc + nb by nb, symmetrised
// in the new diagonal block) and the warm start extended by the identity;
// with partial non-null, Hn is first summed from the projection's nblk
// per-workgroup partial sums (partial[o * nblk + block])
void small_h_append(Small* d, int gc, int nb, hipStream_t s, const double* partial = nullptr,
                    int nblk = 0);
// d->stepbad[step] = d->bad (the breakdown record of the last orthogonalisation)
void small_record_bad(Small* d, int step, hipStream_t s);
void small_extract(Small* d, int gc, int descending, int refined, hipStream_t s);
void small_rr_append(Small* d, int gc, int nb, int total, hipStream_t s);
// the control step: its decision record is built in LDS; host (may be null)
// is the device address of a pinned, coherent host copy that the kernel
// fills at its end; seqp (device address of a pinned host word) receives
// seq after the record has been written
void small_control(Small* d, const CtlParams& p, hipStream_t s, Ctl* host = nullptr,
                   int* seqp = nullptr, int seq = 0);

// batched single-workgroup steps: workgroup p runs problem p's step
struct HAppendArgs {
  Small* d;
  int gc, nb;
  const double* P;  // null: Hn already summed
  int nblk;
};
struct ExtractArgs {
  Small* d;
  int gc, descending;
};
struct ControlArgs {
  Small* d;
  CtlParams P;
  Ctl* host;
  int* seqp;
  int seq;
};
void small_h_append_batch(const std::vector<HAppendArgs>& a, BatchUpload& up, hipStream_t s);
void small_extract_batch(const std::vector<ExtractArgs>& a, BatchUpload& up, hipStream_t s);
void small_control_batch(const std::vector<ControlArgs>& a, BatchUpload& up, hipStream_t s);
void small_rtr_accumulate(const double* C0, int ldc0, const double* C1, int total, int nb,
                          double* Cout, hipStream_t s);
void small_final_rr(int k, double* G, int ldg, int descending, double* lam, double* Z, int ldz,
                    hipStream_t s);

}  // namespace svds
