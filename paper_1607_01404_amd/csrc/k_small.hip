// Single-workgroup FP64 kernels for the small replicated problems of the
// eigensolver (Section 3.3 treats their cost as minor next to the tall
// products): the projected eigenproblem (bordered secular solver and cyclic
// two-sided Jacobi), the SVD of the refined R factor (one-sided Jacobi),
// Householder QR for the refined restart (Section 3.2), and the control step
// that applies the convergence tests, picks the block and builds the GD+k
// restart coefficients.  (The Cholesky factors of the block Gram matrices
// are formed inside the fused Cholesky QR steps of k_dense.hip.)
#include "small.h"

namespace svds {

constexpr int kT = kSmallThreads;
constexpr int kLs = kLd + 1;  // padded leading dimension in LDS
constexpr int kEigT = 1024;   // threads of the eigensolver kernels

// round-robin pairing for np (even) indices, round r in [0, np-1)
__device__ __forceinline__ void rr_pair(int np, int r, int k, int& p, int& q) {
  if (k == 0) {
    p = np - 1;
    q = r;
  } else {
    p = (r + k) % (np - 1);
    q = (r - k + np - 1) % (np - 1);
  }
}

// C (M x N) = op(A) B with op(A) (M x K) and B (K x N), all in LDS with
// leading dimension kLs; op(A) = A^T when TA.  Each thread forms a 2 x 2 tile
// (half the LDS reads of one output per thread); every output is summed over
// the inner index in order.
template <bool TA, int NT = kEigT>
__device__ void lds_gemm(int M, int N, int K, const double* A, const double* B, double* C) {
  const int mt = (M + 1) >> 1, nt = (N + 1) >> 1;
  for (int a = threadIdx.x; a < mt * nt; a += NT) {
    const int i0 = 2 * (a % mt), j0 = 2 * (a / mt);
    const int i1 = min(i0 + 1, M - 1), j1 = min(j0 + 1, N - 1);
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
    for (int c = 0; c < K; ++c) {
      const double a0 = TA ? A[c * kLs + i0] : A[i0 * kLs + c];
      const double a1 = TA ? A[c * kLs + i1] : A[i1 * kLs + c];
      const double b0 = B[c * kLs + j0], b1 = B[c * kLs + j1];
      c00 = fma(a0, b0, c00);
      c01 = fma(a0, b1, c01);
      c10 = fma(a1, b0, c10);
      c11 = fma(a1, b1, c11);
    }
    C[i0 * kLs + j0] = c00;
    if (j0 + 1 < N) C[i0 * kLs + j0 + 1] = c01;
    if (i0 + 1 < M) {
      C[(i0 + 1) * kLs + j0] = c10;
      if (j0 + 1 < N) C[(i0 + 1) * kLs + j0 + 1] = c11;
    }
  }
}

// ---------------------------------------------------------------------------
// symmetric eigenproblem by cyclic Jacobi with a round-robin parallel order.
// A (n x n, ld kLs) in LDS is destroyed; Z must hold an orthonormal matrix W
// on entry (identity, or the previous eigenvectors when H was expressed in a
// basis close to its eigenbasis) and receives W J, the eigenvectors; d the
// eigenvalues (unsorted).  Each round applies the disjoint rotations of all
// pairs as independent 2 x 2 block updates of A (one barrier) and the column
// rotations of Z.
// ---------------------------------------------------------------------------
__device__ void make_pairs(int np, unsigned char* pp, unsigned char* pq) {
  for (int a = threadIdx.x; a < (np - 1) * (np / 2); a += kT) {
    const int r = a / (np / 2), k = a % (np / 2);
    int p, q;
    rr_pair(np, r, k, p, q);
    pp[a] = (unsigned char)p;
    pq[a] = (unsigned char)q;
  }
}

template <int NT>
__device__ int jacobi_eig_lds(int n, double* A, double* Z, double* d, double* cs, double* sn,
                              int* flag, double thr_floor = 0.0, double thr_rel = 0.25) {
  __shared__ double tt_[kLd / 2 + 1], apq_[kLd / 2 + 1];
  __shared__ int zero_[kLd / 2 + 1];
  __shared__ double red_[NT / kWave];
  __shared__ unsigned char pp[(kLd - 1) * (kLd / 2)], pq[(kLd - 1) * (kLd / 2)];
  __shared__ unsigned char active[kLd];
  __shared__ int nactive;
  const int t = threadIdx.x;
  const int np = n + (n & 1);
  const int npair = np / 2;
  if (n & 1) {  // padding index: zero row and column of A, unit vector in Z
    for (int j = t; j < np; j += NT) {
      A[n * kLs + j] = 0.0;
      A[j * kLs + n] = 0.0;
      Z[n * kLs + j] = (j == n) ? 1.0 : 0.0;
      Z[j * kLs + n] = (j == n) ? 1.0 : 0.0;
    }
  }
  for (int a = t; a < (np - 1) * npair; a += NT) {
    const int r = a / npair, k = a % npair;
    int p, q;
    rr_pair(np, r, k, p, q);
    pp[a] = (unsigned char)p;
    pq[a] = (unsigned char)q;
  }
  double f = 0.0;
  for (int a = t; a < n * n; a += NT) {
    const double v = A[(a / n) * kLs + (a % n)];
    f += v * v;
  }
  f = wave_sum(f);
  if (t % kWave == 0) red_[t / kWave] = f;
  __syncthreads();
  double fr = 0.0;
  for (int w = 0; w < NT / kWave; ++w) fr += red_[w];
  const double frob = sqrt(fr);
  // off-diagonal entries below thr_rel * eps * ||A||_F are dropped (by
  // default eps ||A|| / 4): they move eigenvalues and residuals of the Ritz
  // pairs by less than the rounding level of the projected matrix itself
  const double thr = fmax(thr_rel * kEps * frob, thr_floor);
  // Threshold cyclic Jacobi on active rounds only: each sweep first scans all
  // off-diagonal entries and marks the rounds of the parallel ordering that
  // hold an entry above the threshold; only those rounds are processed.
  // Rotations create fill-in in other rounds, which the next sweep's scan
  // picks up; the iteration ends when a scan finds nothing.  A round's 2 x 2
  // block updates of A and its rotations of Z are one flat work list over
  // the workgroup.
  int sweep = 0;
  for (; sweep < 60 && np > 1; ++sweep) {
    if (t < np - 1) active[t] = 0;
    if (t == 0) nactive = 0;
    __syncthreads();
    for (int e = t; e < (np - 1) * npair; e += NT)
      if (fabs(A[pp[e] * kLs + pq[e]]) > thr) active[e / npair] = 1;
    __syncthreads();
    if (t < np - 1 && active[t]) atomicAdd(&nactive, 1);
    __syncthreads();
    if (nactive == 0) break;
    for (int r = 0; r < np - 1; ++r) {
      if (!active[r]) continue;  // uniform: read after a barrier
      const unsigned char* P = pp + r * npair;
      const unsigned char* Q = pq + r * npair;
      if (t < npair) {
        const int p = P[t], q = Q[t];
        const double apq = A[p * kLs + q];
        double c = 1.0, sv = 0.0, tt = 0.0;
        const double app = A[p * kLs + p], aqq = A[q * kLs + q];
        if (fabs(apq) > thr) {
          const double th = (aqq - app) / (2.0 * apq);
          tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          sv = tt * c;
        }
        cs[t] = c;
        sn[t] = sv;
        tt_[t] = tt;
        apq_[t] = apq;
        zero_[t] = (sv == 0.0 && apq != 0.0) ? 1 : 0;
      }
      __syncthreads();
      const int nA = npair * npair;
      for (int idx = t; idx < nA + npair * np; idx += NT) {
        if (idx < nA) {  // A <- J^T A J, block (K, L)
          const int K = idx / npair, L = idx % npair;
          const int pK = P[K], qK = Q[K];
          if (K == L) {
            if (sn[K] != 0.0) {
              A[pK * kLs + pK] -= tt_[K] * apq_[K];
              A[qK * kLs + qK] += tt_[K] * apq_[K];
              A[pK * kLs + qK] = 0.0;
              A[qK * kLs + pK] = 0.0;
            } else if (zero_[K]) {
              A[pK * kLs + qK] = 0.0;
              A[qK * kLs + pK] = 0.0;
            }
            continue;
          }
          const double cK = cs[K], sK = sn[K], cL = cs[L], sL = sn[L];
          if (sK == 0.0 && sL == 0.0) continue;
          const int pL = P[L], qL = Q[L];
          const double a11 = A[pK * kLs + pL], a12 = A[pK * kLs + qL];
          const double a21 = A[qK * kLs + pL], a22 = A[qK * kLs + qL];
          const double b11 = cK * a11 - sK * a21, b12 = cK * a12 - sK * a22;
          const double b21 = sK * a11 + cK * a21, b22 = sK * a12 + cK * a22;
          A[pK * kLs + pL] = cL * b11 - sL * b12;
          A[pK * kLs + qL] = sL * b11 + cL * b12;
          A[qK * kLs + pL] = cL * b21 - sL * b22;
          A[qK * kLs + qL] = sL * b21 + cL * b22;
        } else {  // Z <- Z J, row i of rotation L
          const int e2 = idx - nA;
          const int L = e2 / np, i = e2 % np;
          const double sL = sn[L];
          if (sL == 0.0) continue;
          const double cL = cs[L];
          const int pL = P[L], qL = Q[L];
          const double x = Z[i * kLs + pL], y = Z[i * kLs + qL];
          Z[i * kLs + pL] = cL * x - sL * y;
          Z[i * kLs + qL] = sL * x + cL * y;
        }
      }
      __syncthreads();
    }
  }
  if (t == 0) *flag = 0;
  for (int i = t; i < n; i += NT) d[i] = A[i * kLs + i];
  __syncthreads();
  return sweep + 1;
}

// ---------------------------------------------------------------------------
// symmetric eigenproblem of a bordered diagonal matrix.  A (g x g, ld kLs):
// its leading g0 x g0 block is diagonal to rounding (the projected matrix in
// the previous eigenbasis, or after a restart in the retained Ritz vectors),
// the last g - g0 <= kBordMax columns are dense.  The border columns are
// added one at a time; each step is the arrowhead eigenproblem
// [[diag(lam), z], [z^T, alpha]] in the current eigenbasis, whose eigenvalues
// are the roots of  alpha - mu - sum_j z_j^2 / (lam_j - mu) = 0,  one in each
// gap between consecutive poles and one beyond each end.  Couplings below
// 8 eps ||.|| deflate their pole; two poles closer than that (after a
// rotation that moves the coupling onto the upper one) deflate the lower.
// Each root is found by 16 lanes (the sums split over them) with a
// safeguarded iteration that keeps its nearest pole exact and linearises
// the rest, in coordinates relative to that pole.  The eigenvectors come
// from Loewner's formula for the coupling vector that the computed roots
// solve exactly (Gu and Eisenstat), which keeps them orthogonal.
// Z holds an orthonormal W on entry and W U on return; d receives the
// eigenvalues (ascending).  A is destroyed; U0, V (kLd x kLs) and Bc
// (kLd x kBordMax) are scratch.
// ---------------------------------------------------------------------------
constexpr int kBordMax = 16;
constexpr int kRootLanes = 16;

// 1/x to about one ulp for normal x: the hardware estimate refined by two
// Newton steps (each at least doubles the correct bits).  The secular sums
// use it; their error bound already allows a few ulps per term.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// sum over the 16 lanes of a row (a root's group); all lanes hold the same bits
__device__ __forceinline__ double group16_sum(double v) { return lane_sum<double, 16>(v); }

__device__ __forceinline__ double group16_prod(double v) {
  v *= dpp_row<0xB1>(v);
  v *= dpp_row<0x4E>(v);
  v *= dpp_row<0x141>(v);
  v *= dpp_row<0x140>(v);
  return v;
}

template <int NT>
__device__ void bordered_eig_lds(int g, int g0, double* A, double* Z, double* d, double* U0,
                                 double* V, double* Bc) {
  __shared__ double lam[kLd + 1], zv[kLd], dk[kLd], zk[kLd], zh[kLd], tau[kLd + 1];
  __shared__ double nrm[kLd + 1], vals[kLd + 1];
  __shared__ int kidx[kLd], defl[kLd], Kk[kLd + 1], pos[kLd + 1];
  __shared__ int rot_p[kLd], rot_j[kLd];
  __shared__ double rot_c[kLd], rot_s[kLd];
  __shared__ int s_m, s_nrot;
  __shared__ double s_lo, s_hi;
  const int t = threadIdx.x;
  const int nbd = g - g0;
  for (int a = t; a < g * nbd; a += NT) {
    const int r = a % g, c = a / g;
    Bc[c * kLd + r] = A[r * kLs + g0 + c];
  }
  for (int i = t; i < g0; i += NT) vals[i] = A[i * kLs + i];
  for (int a = t; a < g0 * g0; a += NT) U0[(a / g0) * kLs + (a % g0)] = 0.0;
  __syncthreads();
  for (int i = t; i < g0; i += NT) {  // ascending order: U = a permutation
    const double v = vals[i];
    int rank = 0;
    for (int j = 0; j < g0; ++j) rank += (vals[j] < v || (vals[j] == v && j < i));
    lam[rank] = v;
    U0[i * kLs + rank] = 1.0;
  }
  __syncthreads();
  double* U = U0;
  double* Un = A;
  for (int c = 0; c < nbd; ++c) {
    const int n = g0 + c;  // size before this step
    const double alpha = Bc[c * kLd + n];
    for (int a = t; a < n * kRootLanes; a += NT) {  // z = U^T x, 16 lanes per entry
      const int i = a / kRootLanes, l = a % kRootLanes;
      double acc = 0.0;
      for (int r = l; r < n; r += kRootLanes) acc = fma(U[r * kLs + i], Bc[c * kLd + r], acc);
      acc = group16_sum(acc);
      if (l == 0) zv[i] = acc;
    }
    __syncthreads();
    if (t < kWave) {
      // deflation in wave 0 (lane i: pole i); nearly equal poles are rare and
      // take the serial path below
      const int i = t;
      const double zi = (i < n) ? zv[i] : 0.0;
      const double li = (i < n) ? lam[i] : 0.0;
      const double zn = wave_sum(zi * zi);
      // the poles are in ascending order: the largest magnitude is at an end
      const double lm = (n > 0) ? fmax(fabs(lam[0]), fabs(lam[n - 1])) : 0.0;
      const double tol = 8.0 * kEps * fmax(fmax(lm, fabs(alpha)), sqrt(zn));
      const bool keep = i < n && fabs(zi) > tol;
      const unsigned long long kmask = __ballot(keep);
      const unsigned long long below = (i == 0) ? 0ull : (kmask & ((1ull << i) - 1ull));
      bool close = false;
      if (keep && below) {
        const int p = 63 - __clzll((long long)below);
        const double zp = zv[p];
        const double r = hypot(zp, zi);
        close = fabs((zi / r) * (zp / r) * (li - lam[p])) <= tol;
      }
      const unsigned long long cmask = __ballot(close);
      if (cmask == 0ull) {
        const unsigned long long lower = (i == 0) ? 0ull : ((1ull << i) - 1ull);
        const int m = __popcll(kmask);
        if (keep) {
          const int q = __popcll(kmask & lower);
          kidx[q] = i;
          dk[q] = li;
          zk[q] = zi;
        } else if (i < n) {
          defl[__popcll(~kmask & lower)] = i;
        }
        const double zk2 = wave_sum(keep ? zi * zi : 0.0);
        if (i == 0) {
          const double znk = sqrt(zk2);
          const double lo0 = m ? lam[__ffsll((long long)kmask) - 1] : alpha;
          const double hi0 = m ? lam[63 - __clzll((long long)kmask)] : alpha;
          s_lo = fmin(lo0, alpha) - znk - tol;
          s_hi = fmax(hi0, alpha) + znk + tol;
          s_m = m;
          s_nrot = 0;
        }
      } else if (i == 0) {
        int m = 0, nrot = 0;
        for (int j = 0; j < n; ++j) {
          if (!(fabs(zv[j]) > tol)) continue;
          if (m > 0) {
            const int p = kidx[m - 1];
            const double r = hypot(zv[p], zv[j]);
            const double cc = zv[j] / r, ss = zv[p] / r;
            if (fabs(cc * ss * (lam[j] - lam[p])) <= tol) {
              const double lp = cc * cc * lam[p] + ss * ss * lam[j];
              const double lj = ss * ss * lam[p] + cc * cc * lam[j];
              lam[p] = lp;
              lam[j] = lj;
              zv[p] = 0.0;
              zv[j] = r;
              rot_p[nrot] = p;
              rot_j[nrot] = j;
              rot_c[nrot] = cc;
              rot_s[nrot] = ss;
              ++nrot;
              --m;
            }
          }
          kidx[m++] = j;
        }
        double zk2 = 0.0;
        for (int j = 0; j < m; ++j) {
          dk[j] = lam[kidx[j]];
          zk[j] = zv[kidx[j]];
          zk2 = fma(zk[j], zk[j], zk2);
        }
        int q = 0, nd = 0;
        for (int j = 0; j < n; ++j) {
          if (q < m && kidx[q] == j) ++q;
          else defl[nd++] = j;
        }
        const double znk = sqrt(zk2);
        s_lo = (m ? fmin(dk[0], alpha) : alpha) - znk - tol;
        s_hi = (m ? fmax(dk[m - 1], alpha) : alpha) + znk + tol;
        s_m = m;
        s_nrot = nrot;
      }
    }
    __syncthreads();
    const int m = s_m;
    const int nrot = s_nrot;
    for (int r = t; r < n && nrot > 0; r += NT) {  // deflation rotations on U's columns
      for (int q = 0; q < nrot; ++q) {
        const int p = rot_p[q], j = rot_j[q];
        const double up = U[r * kLs + p], uj = U[r * kLs + j];
        U[r * kLs + p] = rot_c[q] * up - rot_s[q] * uj;
        U[r * kLs + j] = rot_s[q] * up + rot_c[q] * uj;
      }
    }
    if (m == 0) {
      if (t == 0) {
        Kk[0] = -1;
        tau[0] = alpha;
      }
    } else if (t < (m + 1) * kRootLanes) {  // whole 16-lane groups
      const int k = t / kRootLanes, l = t % kRootLanes;
      int K;
      double a, b, t0 = 0.0;
      bool guess = false;
      if (k == 0) {
        K = 0;
        a = s_lo - dk[0];
        b = 0.0;
      } else if (k == m) {
        K = m - 1;
        a = 0.0;
        b = s_hi - dk[m - 1];
      } else {
        const double base = dk[k - 1];
        const double del = dk[k] - base;
        const double mid = 0.5 * del;
        double s = 0.0;
        for (int j = l; j < m; j += kRootLanes) s += zk[j] * zk[j] / ((dk[j] - base) - mid);
        s = group16_sum(s);
        const double fm = (alpha - base) - mid - s;
        if (fm < 0.0) {  // root left of the middle: origin dk[k-1]
          K = k - 1;
          a = 0.0;
          b = mid;
        } else {
          K = k;
          a = -mid;
          b = 0.0;
        }
        // first guess: the gap's two poles exact, every other term (and the
        // linear one) frozen at the middle, tau offset from dk[k-1]:
        //   c + zl^2 / tau - zh^2 / (del - tau) = 0,
        //   i.e. -c tau^2 + (c del - zl^2 - zh^2) tau + zl^2 del = 0,
        // whose one root in (0, del) is formed without cancellation
        const double zl2 = zk[k - 1] * zk[k - 1], zh2 = zk[k] * zk[k];
        const double c = fm - zl2 / mid + zh2 / mid;
        const double Bq = c * del - zl2 - zh2;
        const double sq = sqrt(fmax(Bq * Bq + 4.0 * c * zl2 * del, 0.0));
        const double r1 = (Bq >= 0.0) ? (Bq + sq) / (2.0 * c) : (Bq - sq) / (2.0 * c);
        const double r2 = (Bq >= 0.0) ? -2.0 * zl2 * del / (Bq + sq) : 2.0 * zl2 * del / (sq - Bq);
        const double tau0 = (r1 > 0.0 && r1 < del) ? r1 : r2;
        t0 = (K == k - 1) ? tau0 : tau0 - del;
        guess = true;
      }
      const double dK = dk[K], zK2 = zk[K] * zk[K], aK = alpha - dK;
      double tt = (guess && a < t0 && t0 < b) ? t0 : 0.5 * (a + b);
      for (int it = 0; it < 200; ++it) {
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int j = l; j < m; j += kRootLanes) {
          if (j == K) continue;
          const double qj = zk[j] * rcp_nr((dk[j] - dK) - tt);
          s1 = fma(zk[j], qj, s1);
          s2 = fma(qj, qj, s2);
          s3 += fabs(zk[j] * qj);
        }
        s1 = group16_sum(s1);
        s2 = group16_sum(s2);
        s3 = group16_sum(s3);
        const double R = aK - tt - s1;  // the secular function without the origin pole
        const double Rp = -1.0 - s2;
        const double zt = zK2 / tt;
        const double f = R + zt;
        if (fabs(f) <= 8.0 * kEps * (fabs(aK) + fabs(tt) + s3 + fabs(zt))) break;
        if (f > 0.0) a = tt;
        else b = tt;
        // R + Rp (x - tt) + zK2 / x = 0, i.e. Rp x^2 + B x + zK2 = 0.  With
        // Rp < 0 < zK2 it has one positive and one negative root; the bracket
        // lies on one side of the origin pole, so only that side's root is
        // formed, each in its cancellation-free form
        const double B = R - Rp * tt;
        const double sq = sqrt(B * B - 4.0 * Rp * zK2);
        const bool right = a >= 0.0;
        double rq;
        if (B >= 0.0) {
          const double w = -B - sq;
          rq = right ? w / (2.0 * Rp) : 2.0 * zK2 / w;
        } else {
          const double w = -B + sq;
          rq = right ? 2.0 * zK2 / w : w / (2.0 * Rp);
        }
        double tn = 0.5 * (a + b);
        if (a < rq && rq < b) tn = rq;
        const bool stop = fabs(tn - tt) <= 4.0 * kEps * fabs(tn) ||
                          (b - a) <= 4.0 * kEps * fmax(fabs(a), fabs(b));
        tt = tn;
        if (stop) break;
      }
      if (l == 0) {
        Kk[k] = K;
        tau[k] = tt;
      }
    }
    __syncthreads();
    // roots mu_k = dk[Kk[k]] + tau[k]; Loewner's coupling vector
    if (t < m * kRootLanes) {  // 16 lanes per pole j, whole groups
      const int j = t / kRootLanes, l = t % kRootLanes;
      const double dj = dk[j];
      double p = (l == 0) ? (dk[Kk[m]] - dj) + tau[m] : 1.0;
      for (int k = l; k < m; k += kRootLanes) {
        const double num = (dk[Kk[k]] - dj) + tau[k];
        p *= (k == j) ? num : num / (dk[k] - dj);
      }
      p = group16_prod(p);
      if (l == 0) zh[j] = copysign(sqrt(fabs(p)), zk[j]);
    }
    // the new eigenvalues in ascending order: roots first, then deflated poles
    for (int q = t; q <= n; q += NT) {
      const double v = (q <= m) ? ((m == 0) ? alpha : dk[Kk[q]] + tau[q]) : lam[defl[q - m - 1]];
      vals[q] = v;
    }
    __syncthreads();
    // arrowhead eigenvectors (unnormalised) without their last entry, -1: row
    // i of V belongs to pole i of U, zero for the deflated poles, so that the
    // product with U needs no index gather
    for (int a = t; a < n * (m + 1); a += NT) {
      const int k = a / n, e = a % n;
      if (e < m) V[kidx[e] * kLs + k] = zh[e] / ((dk[e] - dk[Kk[k]]) - tau[k]);
      else V[defl[e - m] * kLs + k] = 0.0;
    }
    for (int a = t; a < (n + 1) * kRootLanes; a += NT) {  // ranks, 16 lanes per entry
      const int q = a / kRootLanes, l = a % kRootLanes;
      const double v = vals[q];
      double rank = 0.0;
      for (int j = l; j <= n; j += kRootLanes)
        rank += (vals[j] < v || (vals[j] == v && j < q)) ? 1.0 : 0.0;
      rank = group16_sum(rank);
      if (l == 0) pos[q] = (int)rank;
    }
    __syncthreads();
    if (t < (m + 1) * kRootLanes) {  // 16 lanes per column k
      const int k = t / kRootLanes, l = t % kRootLanes;
      double s = (l == 0) ? 1.0 : 0.0;  // the last entry, -1
      for (int i = l; i < n; i += kRootLanes) s = fma(V[i * kLs + k], V[i * kLs + k], s);
      s = group16_sum(s);
      if (l == 0) nrm[k] = 1.0 / sqrt(s);
    }
    __syncthreads();
    // Un = [U 0; 0 1] [arrowhead eigenvectors | deflated unit vectors], columns in order
    {
      const int mt = (n + 1) >> 1, qt = (m + 2) >> 1;  // 2 x 2 tiles of rows < n, columns <= m
      const int ntile = mt * qt;
      const int nd = n - m;  // deflated columns
      for (int a = t; a < ntile + (m + 1) + (n + 1) * nd; a += NT) {
        if (a < ntile) {
          const int r0 = 2 * (a % mt), q0 = 2 * (a / mt);
          const int r1 = min(r0 + 1, n - 1), q1 = min(q0 + 1, m);
          double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
          for (int j = 0; j < n; ++j) {
            const double u0 = U[r0 * kLs + j], u1 = U[r1 * kLs + j];
            const double v0 = V[j * kLs + q0], v1 = V[j * kLs + q1];
            c00 = fma(u0, v0, c00);
            c01 = fma(u0, v1, c01);
            c10 = fma(u1, v0, c10);
            c11 = fma(u1, v1, c11);
          }
          Un[r0 * kLs + pos[q0]] = c00 * nrm[q0];
          if (q0 + 1 <= m) Un[r0 * kLs + pos[q0 + 1]] = c01 * nrm[q0 + 1];
          if (r0 + 1 < n) {
            Un[(r0 + 1) * kLs + pos[q0]] = c10 * nrm[q0];
            if (q0 + 1 <= m) Un[(r0 + 1) * kLs + pos[q0 + 1]] = c11 * nrm[q0 + 1];
          }
        } else if (a < ntile + m + 1) {  // the new last row of the root columns
          const int q = a - ntile;
          Un[n * kLs + pos[q]] = -nrm[q];
        } else {  // deflated unit vectors: columns of U, zero in the new row
          const int e = a - ntile - (m + 1);
          const int r = e / nd, q = m + 1 + e % nd;
          Un[r * kLs + pos[q]] = (r < n) ? U[r * kLs + defl[q - m - 1]] : 0.0;
        }
      }
    }
    __syncthreads();
    for (int q = t; q <= n; q += NT) lam[pos[q]] = vals[q];
    double* tmp = U;
    U = Un;
    Un = tmp;
    __syncthreads();
  }
  for (int i = t; i < g; i += NT) d[i] = lam[i];
  // Z <- W U
  lds_gemm<false>(g, g, g, Z, U, Un);
  __syncthreads();
  for (int a = t; a < g * g; a += NT) {
    const int r = a / g, c = a % g;
    Z[r * kLs + c] = Un[r * kLs + c];
  }
  __syncthreads();
}

// sort eigenpairs: theta[rank] = d[i], Y[:, rank] = Z[0:n, i]
__device__ void sort_pairs(int n, const double* d, const double* Z, int descending,
                           double* theta, double* Y, int ldy) {
  const int t = threadIdx.x;
  for (int i = t; i < n; i += kT) {
    const double di = d[i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double dj = d[j];
      const bool before = descending ? (dj > di || (dj == di && j < i)) : (dj < di || (dj == di && j < i));
      rank += before;
    }
    theta[rank] = di;
    for (int r = 0; r < n; ++r) Y[(int64_t)rank * ldy + r] = Z[r * kLs + i];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kEigT) void k_eig(int g, const double* H, int ldh, int descending,
                                            double* theta, double* Y, int ldy) {
  __shared__ double A[kLd * kLs];
  __shared__ double Z[kLd * kLs];
  __shared__ double d[kLd], cs[kLd], sn[kLd];
  __shared__ int flag;
  for (int a = threadIdx.x; a < g * g; a += kEigT) {
    const int i = a % g, j = a / g;
    A[i * kLs + j] = 0.5 * (H[(int64_t)j * ldh + i] + H[(int64_t)i * ldh + j]);
    Z[i * kLs + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  jacobi_eig_lds<kEigT>(g, A, Z, d, cs, sn, &flag);
  sort_pairs(g, d, Z, descending, theta, Y, ldy);
}

void small_eig(int g, const double* H, int ldh, int descending, double* theta, double* Y, int ldy,
               hipStream_t s) {
  if (g < 1 || g > kGmax) throw Error(SVDS_ERR_ARG, "small_eig: 1 <= g <= 48");
  k_eig<<<1, kEigT, 0, s>>>(g, H, ldh, descending, theta, Y, ldy);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// one-sided Jacobi SVD of A (n x n, ld kLs, LDS): on return the columns of A
// are U*Sigma (unsorted) and Vm the right singular vectors (unsorted)
// ---------------------------------------------------------------------------
__device__ void jacobi_svd_lds(int n, double* A, double* Vm, double* cs, double* sn, int* flag) {
  const int t = threadIdx.x;
  const int np = n + (n & 1);
  for (int a = t; a < np * kLs; a += kT) Vm[a] = 0.0;
  __syncthreads();
  if (n & 1)
    for (int j = t; j < np; j += kT) A[j * kLs + n] = 0.0;  // zero padding column
  for (int j = t; j < np; j += kT) Vm[j * kLs + j] = 1.0;
  __syncthreads();
  const int npair = np / 2;
  constexpr int G = 8;  // lanes per pair
  __shared__ unsigned char pp[(kLd - 1) * (kLd / 2)], pq[(kLd - 1) * (kLd / 2)];
  make_pairs(np, pp, pq);
  __syncthreads();
  for (int sweep = 0; sweep < 80 && np > 1; ++sweep) {
    if (t == 0) *flag = 0;
    __syncthreads();
    for (int r = 0; r < np - 1; ++r) {
      const int k = t / G, l = t % G;
      double al = 0.0, be = 0.0, ga = 0.0;
      int p = 0, q = 0;
      if (k < npair) {
        p = pp[r * npair + k];
        q = pq[r * npair + k];
        for (int i = l; i < n; i += G) {
          const double x = A[i * kLs + p], y = A[i * kLs + q];
          al += x * x;
          be += y * y;
          ga += x * y;
        }
      }
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) {
        al += __shfl_xor(al, off, kWave);
        be += __shfl_xor(be, off, kWave);
        ga += __shfl_xor(ga, off, kWave);
      }
      if (k < npair && l == 0) {
        double c = 1.0, s = 0.0;
        if (fabs(ga) > kEps * (double)n * sqrt(al * be) && ga != 0.0) {
          const double zeta = (be - al) / (2.0 * ga);
          const double tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = c * tt;
          *flag = 1;
        }
        cs[k] = c;
        sn[k] = s;
      }
      __syncthreads();
      for (int kk = t >> 6; kk < npair; kk += kT / kWave) {
        const int i = t & 63;
        const double c = cs[kk], s = sn[kk];
        if (i >= np || s == 0.0) continue;
        const int p2 = pp[r * npair + kk], q2 = pq[r * npair + kk];
        double x = A[i * kLs + p2], y = A[i * kLs + q2];
        A[i * kLs + p2] = c * x - s * y;
        A[i * kLs + q2] = s * x + c * y;
        x = Vm[i * kLs + p2];
        y = Vm[i * kLs + q2];
        Vm[i * kLs + p2] = c * x - s * y;
        Vm[i * kLs + q2] = s * x + c * y;
      }
      __syncthreads();
    }
    if (*flag == 0) break;
    __syncthreads();
  }
}

// columns norms of A -> sv, sorted ascending; Y[:, rank] = Vm[:, j]; AV likewise
__device__ void svd_finish(int n, const double* A, const double* Vm, double* sbuf, double* s,
                           double* Y, int ldy, double* AV, int ldav) {
  const int t = threadIdx.x;
  for (int j = t; j < n; j += kT) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += A[i * kLs + j] * A[i * kLs + j];
    sbuf[j] = sqrt(acc);
  }
  __syncthreads();
  for (int j = t; j < n; j += kT) {
    const double sj = sbuf[j];
    int rank = 0;
    for (int i = 0; i < n; ++i) rank += (sbuf[i] < sj) || (sbuf[i] == sj && i < j);
    s[rank] = sj;
    for (int i = 0; i < n; ++i) Y[(int64_t)rank * ldy + i] = Vm[i * kLs + j];
    if (AV)
      for (int i = 0; i < n; ++i) AV[(int64_t)rank * ldav + i] = A[i * kLs + j];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kT) void k_svd(int g, const double* R, int ldr, double* s, double* Y,
                                            int ldy, double* AV, int ldav) {
  __shared__ double A[kLd * kLs];
  __shared__ double Vm[kLd * kLs];
  __shared__ double cs[kLd], sn[kLd], sb[kLd];
  __shared__ int flag;
  for (int a = threadIdx.x; a < g * g; a += kT) {
    const int i = a % g, j = a / g;
    A[i * kLs + j] = R[(int64_t)j * ldr + i];
  }
  __syncthreads();
  jacobi_svd_lds(g, A, Vm, cs, sn, &flag);
  svd_finish(g, A, Vm, sb, s, Y, ldy, AV, ldav);
}

void small_svd(int g, const double* R, int ldr, double* s, double* Y, int ldy, double* AV,
               int ldav, hipStream_t st) {
  if (g < 1 || g > kGmax) throw Error(SVDS_ERR_ARG, "small_svd: 1 <= g <= 48");
  k_svd<<<1, kT, 0, st>>>(g, R, ldr, s, Y, ldy, AV, ldav);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// projected matrix: append the new columns Hn ((gc+nb) x nb, ld gc+nb)
// ---------------------------------------------------------------------------
// P non-null: the new columns are first summed from the projection's nblk
// per-workgroup partial sums (P[o * nblk + block], o = c * tot + i), 16
// lanes per entry (64 entries at a time, their loads unrolled), and also
// stored in d->Hn
constexpr int kHAppT = 1024;  // threads of the append kernels

__device__ __forceinline__ void h_append_body(Small* d, int gc, int nb, const double* P, int nblk) {
  const int tot = gc + nb;
  __shared__ double hn[kLd * kMaxBlock];
  if (P) {
    const int l = threadIdx.x % 16, grp = threadIdx.x / 16;
    for (int o = grp; o < tot * nb; o += kHAppT / 16) {  // uniform per 16-lane group
      const double* p = P + (int64_t)o * nblk;
      double sum = 0.0;
#pragma unroll 8
      for (int k = l; k < nblk; k += 16) sum += p[k];
      sum = lane_sum<double, 16>(sum);
      if (l == 0) {
        hn[o] = sum;
        d->Hn[o] = sum;
      }
    }
  } else {
    for (int o = threadIdx.x; o < tot * nb; o += blockDim.x) hn[o] = d->Hn[o];
  }
  // previous eigenvectors stay a good start: W <- diag(W, I); a projected
  // matrix built from nothing starts from W = I with no diagonal block
  const bool warm = d->warm_g == gc || gc == 0;
  for (int a = threadIdx.x; a < tot * tot; a += blockDim.x) {
    const int i = a % tot, j = a / tot;
    if (i < gc && j < gc) continue;
    d->Yw[j * kLd + i] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    d->warm_g = warm ? tot : -1;
    if (gc == 0) d->warm_diag = 0;
  }
  for (int a = threadIdx.x; a < tot * nb; a += blockDim.x) {
    const int i = a % tot, c = a / tot;
    const int j = gc + c;
    double v = hn[c * tot + i];
    if (i >= gc) {  // symmetrise the new diagonal block
      const int ci = i - gc;
      v = 0.5 * (v + hn[ci * tot + j]);
    }
    d->H[j * kLd + i] = v;
    d->H[i * kLd + j] = v;
  }
}

__global__ __launch_bounds__(kHAppT) void k_h_append(Small* d, int gc, int nb, const double* P,
                                                     int nblk) {
  h_append_body(d, gc, nb, P, nblk);
}
__global__ __launch_bounds__(kHAppT) void k_h_append_batch(const HAppendArgs* a) {
  const HAppendArgs q = a[blockIdx.x];
  h_append_body(q.d, q.gc, q.nb, q.P, q.nblk);
}

__global__ void k_record_bad(Small* d, int step) {
  if (threadIdx.x == 0) d->stepbad[step] = d->bad;
}

void small_record_bad(Small* d, int step, hipStream_t s) {
  if (step < 0 || step >= kGmax) throw Error(SVDS_ERR_ARG, "record_bad: step");
  k_record_bad<<<1, kWave, 0, s>>>(d, step);
  SVDS_LAUNCH_CHECK();
}

void small_h_append(Small* d, int gc, int nb, hipStream_t s, const double* partial, int nblk) {
  k_h_append<<<1, kHAppT, 0, s>>>(d, gc, nb, partial, nblk);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// extraction: Rayleigh-Ritz (eigenpairs of H in target order) or, for the
// refined projection, right singular vectors of Rr in ascending order with
// theta_j = y_j^T H y_j (Section 3.2)
// ---------------------------------------------------------------------------
// A (g x g) <- Z^T A Z, symmetrised; Mx scratch
__device__ void project_lds(int g, double* A, const double* Z, double* Mx) {
  const int t = threadIdx.x;
  lds_gemm<false>(g, g, g, A, Z, Mx);
  __syncthreads();
  lds_gemm<true>(g, g, g, Z, Mx, A);
  __syncthreads();
  for (int a = t; a < g * g; a += kEigT) {
    const int i = a % g, j = a / g;
    if (i < j) {
      const double v = 0.5 * (A[i * kLs + j] + A[j * kLs + i]);
      A[i * kLs + j] = v;
      A[j * kLs + i] = v;
    }
  }
  __syncthreads();
}

__device__ void load_sym_h(const Small* d, int g, double* A) {
  for (int a = threadIdx.x; a < g * g; a += kEigT) {
    const int i = a % g, j = a / g;
    A[i * kLs + j] = 0.5 * (d->H[j * kLd + i] + d->H[i * kLd + j]);
  }
}

// Rayleigh-Ritz extraction.  H is expressed in the warm basis W (the
// previous eigenvectors, padded with the identity for new columns), where its
// leading block is diagonal to rounding.  When the dense border is narrow the
// bordered solver gives eigenvectors W U of that form; H is then projected on
// them again and the threshold Jacobi finishes on the exact projection, so
// the rounding of the warm basis never accumulates from one extraction to the
// next.  That projection, g-term dot products in FP64, carries off-diagonal
// rounding of about sqrt(g) eps ||H|| by itself, so the finishing Jacobi
// leaves entries below sqrt(g) eps ||H||_F alone: they are indistinguishable
// from that rounding, change the Ritz values by their square over the gap and
// the residuals by about their own size, below the eps ||C|| floor of the
// convergence test (Section 3.2).  Otherwise Jacobi runs from W to eps/4.
__device__ __forceinline__ void extract_rr_body(Small* d, int gc, int descending) {
  __shared__ double A[kLd * kLs];
  __shared__ double Z[kLd * kLs];
  __shared__ double Mx[kLd * kLs];
  __shared__ double Vb[kLd * kLs];
  __shared__ double Bc[kLd * kBordMax];
  __shared__ double dd[kLd], cs[kLd], sn[kLd];
  __shared__ int flag;
  const int t = threadIdx.x;
  const bool warm = d->warm_g == gc;
  load_sym_h(d, gc, A);
  for (int a = t; a < gc * gc; a += kEigT) {
    const int i = a % gc, j = a / gc;
    Z[i * kLs + j] = warm ? d->Yw[j * kLd + i] : (i == j ? 1.0 : 0.0);
  }
  __syncthreads();
  if (warm) project_lds(gc, A, Z, Mx);
  const int g0 = warm ? d->warm_diag : -1;
  const bool bordered = warm && g0 >= 0 && g0 <= gc && gc - g0 <= kBordMax;
  if (bordered) {
    bordered_eig_lds<kEigT>(gc, g0, A, Z, dd, Mx, Vb, Bc);
    load_sym_h(d, gc, A);
    __syncthreads();
    project_lds(gc, A, Z, Mx);
  }
  const int nsw = jacobi_eig_lds<kEigT>(gc, A, Z, dd, cs, sn, &flag, 0.0,
                                        bordered ? sqrt((double)gc) : 0.25);
  if (t == 0) d->eig_sweeps = nsw;
  sort_pairs(gc, dd, Z, descending, d->theta, d->Y, kLd);
  for (int a = t; a < gc * gc; a += kEigT) {
    const int i = a % gc, j = a / gc;
    d->Yw[j * kLd + i] = d->Y[j * kLd + i];
  }
  if (t == 0) {
    d->warm_g = gc;
    d->warm_diag = gc;
  }
}

__global__ __launch_bounds__(kEigT) void k_extract_rr(Small* d, int gc, int descending) {
  extract_rr_body(d, gc, descending);
}
__global__ __launch_bounds__(kEigT) void k_extract_rr_batch(const ExtractArgs* a) {
  const ExtractArgs q = a[blockIdx.x];
  extract_rr_body(q.d, q.gc, q.descending);
}

__global__ __launch_bounds__(kT) void k_extract_refined(Small* d, int gc) {
  __shared__ double A[kLd * kLs];
  __shared__ double Z[kLd * kLs];
  __shared__ double Mx[kLd * kLs];
  __shared__ double dd[kLd];
  __shared__ double cs[kLd], sn[kLd];
  __shared__ int flag;
  const int t = threadIdx.x;
  for (int a = t; a < gc * gc; a += kT) {
    const int i = a % gc, j = a / gc;
    A[i * kLs + j] = (i <= j) ? d->Rr[j * kLd + i] : 0.0;
  }
  __syncthreads();
  jacobi_svd_lds(gc, A, Z, cs, sn, &flag);
  svd_finish(gc, A, Z, dd, d->sv, d->Y, kLd, nullptr, 0);
  // theta_j = y_j^T H y_j with H and the sorted Y staged in LDS
  for (int a = t; a < gc * gc; a += kT) {
    const int i = a % gc, j = a / gc;
    A[i * kLs + j] = d->H[j * kLd + i];
    Z[i * kLs + j] = d->Y[j * kLd + i];
  }
  __syncthreads();
  for (int a = t; a < gc * gc; a += kT) {  // M = H Y
    const int i = a % gc, j = a / gc;
    double acc = 0.0;
    for (int c = 0; c < gc; ++c) acc += A[i * kLs + c] * Z[c * kLs + j];
    Mx[i * kLs + j] = acc;
  }
  __syncthreads();
  for (int j = t; j < gc; j += kT) {
    double acc = 0.0;
    for (int r = 0; r < gc; ++r) acc += Z[r * kLs + j] * Mx[r * kLs + j];
    d->theta[j] = acc;
  }
}

void small_extract(Small* d, int gc, int descending, int refined, hipStream_t s) {
  if (gc < 1 || gc > kGmax) throw Error(SVDS_ERR_ARG, "extract: basis size");
  if (refined) k_extract_refined<<<1, kT, 0, s>>>(d, gc);
  else k_extract_rr<<<1, kEigT, 0, s>>>(d, gc, descending);
  SVDS_LAUNCH_CHECK();
}


// ---------------------------------------------------------------------------
// refined factor: Rr[0:gc, gc:gc+nb] = C0 + C1 (projection coefficients),
// Rr[gc:, gc:] = R2 R1, below-diagonal entries zero
// ---------------------------------------------------------------------------
__global__ void k_rr_append(Small* d, int gc, int nb) {
  const int ld0 = gc + nb;
  for (int a = threadIdx.x; a < (gc + nb) * nb; a += blockDim.x) {
    const int i = a % (gc + nb), c = a / (gc + nb);
    double v;
    if (i < gc) {
      v = d->C0[(int64_t)c * ld0 + i] + d->C1[(int64_t)c * gc + i];
    } else {
      const int ii = i - gc;
      v = 0.0;
      for (int j = ii; j <= c; ++j) v += d->R2[j * nb + ii] * d->R1[c * nb + j];
    }
    d->Rr[(gc + c) * kLd + i] = v;
    if (i < gc) d->Rr[i * kLd + gc + c] = 0.0;
  }
}

void small_rr_append(Small* d, int gc, int nb, int total, hipStream_t s) {
  (void)total;
  k_rr_append<<<1, kT, 0, s>>>(d, gc, nb);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// control step
// ---------------------------------------------------------------------------
__device__ __forceinline__ double halves_res(const double* sums, int nc, int c, double theta) {
  // eq. (res) of the normalised halves from the fused sums (see k_residual):
  // A v - s u = r_u/a + x_u (theta/a - s/c),  A^T u - s v = r_v/c + x_v (theta/c - s/a)
  const double rv2 = sums[0 * nc + c], xrv = sums[1 * nc + c], xv2 = sums[2 * nc + c];
  const double ru2 = sums[3 * nc + c], xru = sums[4 * nc + c], xu2 = sums[5 * nc + c];
  const double a = sqrt(fmax(xv2, 0.0)), cc = sqrt(fmax(xu2, 0.0));
  if (!(a > 0.0) || !(cc > 0.0)) return INFINITY;
  const double s = fabs(theta);
  const double e1 = theta / a - s / cc;
  const double e2 = theta / cc - s / a;
  const double t1 = ru2 / (a * a) + 2.0 * e1 * xru / a + e1 * e1 * xu2;
  const double t2 = rv2 / (cc * cc) + 2.0 * e2 * xrv / cc + e2 * e2 * xv2;
  return sqrt(fmax(t1, 0.0) + fmax(t2, 0.0));
}

__device__ void control_body(Small* d, const CtlParams& P, Ctl& C) {
  __shared__ int s_action, s_nblock, s_restart, s_reff, s_off, s_peff, s_lock, s_bad;
  __shared__ int s_blk[kMaxBlock];
  __shared__ double Yr[kLd * kLs];
  __shared__ double M[kLd * kLs];
  const int t = threadIdx.x;
  const int gc = P.gc, nc = P.nc;
  __shared__ double th_s[kLd], sums_s[6 * (kKmax + 8)], best_s[kKmax + 8];
  __shared__ int stall_s[kKmax + 8];
  __shared__ bool conv[kKmax + 8], done[kKmax + 8];
  __shared__ double rn[kKmax + 8];
  __shared__ bool pcf[kKmax + 8];
  __shared__ double mx_s, s_nop0;
  __shared__ int s_nprev, s_gprev, s_sweeps;
  {  // the record starts zeroed (C lives in LDS)
    unsigned int* w = reinterpret_cast<unsigned int*>(&C);
    for (int a = t; a < (int)(sizeof(Ctl) / sizeof(unsigned int)); a += kT) w[a] = 0u;
  }
  if (t == 0) s_bad = d->bad;
  // the scalars of the decision, loaded in parallel with the arrays so that
  // the serial decision below reads only LDS
  if (t == kWave) {
    s_nop0 = d->normop;
    s_nprev = d->nprev;
    s_gprev = d->gprev;
    s_sweeps = d->eig_sweeps;
  }
  for (int j = t; j < gc; j += kT) th_s[j] = d->theta[j];
  for (int j = t; j < (P.stage == 1 ? nc : 6 * nc); j += kT) sums_s[j] = d->sums[j];
  for (int j = t; j < nc; j += kT) {
    best_s[j] = d->best[j];
    stall_s[j] = d->stall[j];
  }
  if (t < kWave) {
    double mx = 0.0;
    for (int j = t; j < gc; j += kWave) mx = fmax(mx, fabs(d->theta[j]));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
    if (t == 0) mx_s = mx;
  }
  __syncthreads();
  if (s_bad) {  // leave every state untouched: the host rolls the block back
    if (t == 0) {
      C.action = kBreakdown;
      C.bad = s_bad;
    }
    return;
  }
  const double nop = fmax(s_nop0, mx_s);
  // the convergence tests of the candidates, one thread each
  for (int c = t; c < nc; c += kT) {
    const double r = sqrt(fmax(P.stage == 1 ? sums_s[c] : sums_s[0 * nc + c] + sums_s[3 * nc + c], 0.0));
    rn[c] = r;
    C.res[c] = r;
    C.val[c] = th_s[c];
    bool cv, pc = false;
    if (P.stage == 1) {
      const double thr = P.rel ? fmax(P.tol * fabs(th_s[c]), P.eps * nop)
                               : fmax(sqrt(fabs(th_s[c]) * nop) * P.tol, P.eps * nop);
      cv = r <= thr;
      pc = !cv && stall_s[c] >= kStallRestarts && r <= P.gate * nop;
    } else {
      cv = false;
      if (r <= 1.4142135623730951 * nop * P.tol)
        cv = halves_res(sums_s, nc, c, th_s[c]) < P.normA * P.tol;
    }
    conv[c] = cv;
    pcf[c] = pc;
    done[c] = cv || pc;
  }
  __syncthreads();
  if (t == 0) {
    C.bad = 0;
    d->normop = nop;
    int ncv = 0, npc = 0;
    for (int c = 0; c < nc; ++c) {
      ncv += conv[c];
      npc += pcf[c];
    }
    int action = kExpand, nblock = 0, restart = 0, reff = 0, off = 0, peff = 0, lock = 0;
    int floor_reset = 0;
    double maxres = 0.0, minres = INFINITY;
    const int kk = min(P.k, nc);
    for (int c = 0; c < kk; ++c) maxres = fmax(maxres, rn[c]);
    if (P.stage == 1) {
      bool all = (kk == P.k);
      bool anypc = false;
      for (int c = 0; c < kk; ++c) {
        all = all && done[c];
        anypc = anypc || (done[c] && !conv[c]);
      }
      if (all) {
        if (anypc && P.floor_resets < 1) {
          action = kReset;
          floor_reset = 1;
          for (int c = 0; c < kKmax + 8; ++c) {
            d->best[c] = INFINITY;
            d->stall[c] = 0;
          }
        } else {
          action = anypc ? kExitFloor : kExitConverged;
        }
      } else if (P.budget_hit) {
        action = kExitBudget;
      } else {
        for (int c = 0; c < nc && nblock < P.b; ++c)
          if (!done[c]) s_blk[nblock++] = c;
        for (int j = 0; j < nblock; ++j) minres = fmin(minres, rn[s_blk[j]]);
        if (nblock > 0 && P.since_reset > 0 && minres < sqrt((double)P.since_reset) * nop * P.eps) {
          action = kReset;
        } else {
          const int nb_next = nblock > 0 ? nblock : P.b;
          if (gc + nb_next > P.g) {
            restart = 1;
            for (int c = 0; c < nc; ++c) {
              if (rn[c] < 0.5 * best_s[c]) {
                d->best[c] = rn[c];
                d->stall[c] = 0;
              } else {
                d->stall[c] = stall_s[c] + 1;
              }
            }
            int nd = 0;
            for (int c = 0; c < nc; ++c) nd += done[c];
            reff = min(max(P.r, nd + P.b), P.g - P.b);
            off = 0;
          }
        }
      }
    } else {
      int L = 0;
      while (L < nc && conv[L]) ++L;
      if (L > 0) {
        for (int i = 0; i < L; ++i) d->lockval[P.nlock + i] = th_s[i];
        lock = L;
        if (P.nlock + L >= P.k) {
          action = kExitConverged;
        } else {
          action = kLock;
          restart = 1;
          reff = min(P.r, gc - L);
          off = L;
        }
      } else if (P.budget_hit) {
        action = kExitBudget;
      } else {
        for (int c = 0; c < nc; ++c) s_blk[nblock++] = c;
        for (int j = 0; j < nblock; ++j) minres = fmin(minres, rn[s_blk[j]]);
        if (P.since_reset > 0 && minres < sqrt((double)P.since_reset) * nop * P.eps) {
          action = kReset;
        } else if (gc + nblock > P.g) {
          restart = 1;
          reff = min(P.r, gc);
          off = 0;
        }
      }
    }
    if (restart) {
      const int room = max(0, P.g - P.b - reff);
      peff = (P.p > 0) ? min(min(P.p, s_nprev), room) : 0;
    }
    if (action == kReset) d->nprev = 0;
    {
      double rmin = INFINITY;
      for (int c = 0; c < nc; ++c) rmin = fmin(rmin, rn[c]);
      d->res_min = (action == kExpand && isfinite(rmin)) ? rmin : 0.0;
    }
    s_action = action;
    s_nblock = nblock;
    s_restart = restart;
    s_reff = reff;
    s_off = off;
    s_peff = peff;
    s_lock = lock;
    C.action = action;
    C.nblock = nblock;
    C.nlockable = lock;
    C.nconv = ncv;
    C.npc = npc;
    C.floor_reset = floor_reset;
    C.normop = nop;
    C.eig_sweeps = s_sweeps;
    C.maxres = maxres;
    C.minres = minres;
  }
  __syncthreads();
  const int action = s_action;
  const int nblock = s_nblock;
  if (s_restart) {
    const int reff = s_reff, off = s_off, peff = s_peff;
    // the extraction vectors staged in M (free until H is rotated below),
    // the retained ones also in Yr
    for (int a = t; a < gc * gc; a += kT) {
      const int i = a % gc, j = a / gc;
      const double y = d->Y[j * kLd + i];
      M[i * kLs + j] = y;
      if (j >= off && j < off + reff) Yr[i * kLs + (j - off)] = y;
    }
    __syncthreads();
    // +k: previous block coefficient vectors (zero padded), classical
    // Gram-Schmidt twice against Y[:, 0:off], the retained vectors and the
    // accepted ones: all projections of a pass at once, 16 lanes per product
    __shared__ double yv[kLd], dots[2 * kLd], s_ny;
    int nr = reff;
    for (int pv = 0; pv < peff; ++pv) {
      for (int i = t; i < kLd; i += kT)
        yv[i] = (i < gc && i < s_gprev) ? d->yprev[pv * kLd + i] : 0.0;
      __syncthreads();
      const int nq = off + nr;
      for (int rep = 0; rep < 2; ++rep) {
        for (int a = t; a < nq * 16; a += kT) {
          const int q = a / 16, l = a % 16;
          double acc = 0.0;
          for (int i = l; i < gc; i += 16)
            acc = fma(yv[i], (q < off) ? M[i * kLs + q] : Yr[i * kLs + (q - off)], acc);
          acc = lane_sum<double, 16>(acc);
          if (l == 0) dots[q] = acc;
        }
        __syncthreads();
        for (int i = t; i < gc; i += kT) {
          double y = yv[i];
          for (int q = 0; q < nq; ++q)
            y -= dots[q] * ((q < off) ? M[i * kLs + q] : Yr[i * kLs + (q - off)]);
          yv[i] = y;
        }
        __syncthreads();
      }
      if (t < kWave) {
        double v = (t < gc) ? yv[t] : 0.0;
        v = wave_sum(v * v);
        if (t == 0) s_ny = sqrt(v);
      }
      __syncthreads();
      const double ny = s_ny;
      if (ny > kPrevDrop) {  // uniform: read after a barrier
        for (int i = t; i < gc; i += kT) Yr[i * kLs + nr] = yv[i] / ny;
        ++nr;
      }
      __syncthreads();
    }
    // H <- Yr^T H Yr (M = H Yr first), from H staged in LDS
    __shared__ double Hl[kLd * kLs];
    for (int a = t; a < gc * gc; a += kT) {
      const int i = a % gc, c = a / gc;
      Hl[i * kLs + c] = d->H[c * kLd + i];
    }
    __syncthreads();
    lds_gemm<false, kT>(gc, nr, gc, Hl, Yr, M);
    __syncthreads();
    lds_gemm<true, kT>(nr, nr, gc, Yr, M, Hl);
    __syncthreads();
    for (int a = t; a < nr * nr; a += kT) {
      const int i = a % nr, j = a / nr;
      d->H[j * kLd + i] = 0.5 * (Hl[i * kLs + j] + Hl[j * kLs + i]);
    }
    __syncthreads();
    // next +k vectors: the block's coefficients in the new basis (the
    // block's extraction vectors staged in LDS first)
    if (action == kExpand) {
      __shared__ double Yb[kMaxBlock * kLd];
      for (int a = t; a < gc * nblock; a += kT) {
        const int r = a % gc, c = a / gc;
        Yb[c * kLd + r] = d->Y[s_blk[c] * kLd + r];
      }
      __syncthreads();
      for (int a = t; a < nr * nblock; a += kT) {
        const int i = a % nr, c = a / nr;
        double acc = 0.0;
        for (int r = 0; r < gc; ++r) acc += Yr[r * kLs + i] * Yb[c * kLd + r];
        d->yprev[c * kLd + i] = acc;
      }
    }
    // refined factor restart: Rr Yr = Qt Rt (Householder), Rr <- Rt
    if (P.refined) {
      for (int a = t; a < gc * nr; a += kT) {
        const int i = a % gc, j = a / gc;
        double acc = 0.0;
        for (int c = i; c < gc; ++c) acc += d->Rr[c * kLd + i] * Yr[c * kLs + j];
        M[i * kLs + j] = acc;
      }
      __syncthreads();
      // Householder QR of M (gc x nr); reflectors kept below the diagonal
      __shared__ double vnorm2[kLd];
      __shared__ double diag[kLd];
      for (int j = 0; j < nr; ++j) {
        if (t == 0) {
          double s2 = 0.0;
          for (int i = j; i < gc; ++i) s2 += M[i * kLs + j] * M[i * kLs + j];
          const double x0 = M[j * kLs + j];
          const double nx = sqrt(s2);
          const double alpha = (x0 >= 0.0) ? -nx : nx;
          M[j * kLs + j] = x0 - alpha;  // v_j (v = x - alpha e1)
          const double v2 = s2 - x0 * x0 + (x0 - alpha) * (x0 - alpha);
          vnorm2[j] = v2;
          diag[j] = alpha;
        }
        __syncthreads();
        const double v2 = vnorm2[j];
        for (int c = j + 1 + t; c < nr; c += kT) {
          if (v2 > 0.0) {
            double w = 0.0;
            for (int i = j; i < gc; ++i) w += M[i * kLs + j] * M[i * kLs + c];
            const double f = 2.0 * w / v2;
            for (int i = j; i < gc; ++i) M[i * kLs + c] -= f * M[i * kLs + j];
          }
        }
        __syncthreads();
      }
      // Qt = H_0 ... H_{nr-1} I[:, 0:nr]; columns independent
      for (int c = t; c < nr; c += kT) {
        for (int i = 0; i < gc; ++i) d->Qt[c * kLd + i] = (i == c) ? 1.0 : 0.0;
        for (int j = nr - 1; j >= 0; --j) {
          const double v2 = vnorm2[j];
          if (!(v2 > 0.0)) continue;
          double w = 0.0;
          for (int i = j; i < gc; ++i) w += M[i * kLs + j] * d->Qt[c * kLd + i];
          const double f = 2.0 * w / v2;
          for (int i = j; i < gc; ++i) d->Qt[c * kLd + i] -= f * M[i * kLs + j];
        }
      }
      __syncthreads();
      for (int a = t; a < nr * nr; a += kT) {
        const int i = a % nr, j = a / nr;
        double v = 0.0;
        if (i == j) v = diag[j];
        else if (i < j) v = M[i * kLs + j];
        d->Rr[j * kLd + i] = v;
      }
    }
    __syncthreads();
    // restart coefficients for the host's V <- V Yr
    for (int a = t; a < gc * nr; a += kT) {
      const int i = a % gc, j = a / gc;
      d->Yr[j * kLd + i] = Yr[i * kLs + j];
    }
    // the retained extraction vectors are eigenvectors of H (Rayleigh-Ritz), so
    // the leading reff x reff block of the restarted H is diagonal: warm start
    // from the identity with that block known diagonal
    for (int a = t; a < nr * nr; a += kT) {
      const int i = a % nr, j = a / nr;
      d->Yw[j * kLd + i] = (i == j) ? 1.0 : 0.0;
    }
    if (t == 0) {
      d->warm_g = P.refined ? -1 : nr;
      d->warm_diag = reff;
      C.restart = 1;
      C.nr = nr;
      if (action == kExpand) {
        d->nprev = nblock;
        d->gprev = nr;
      } else {
        d->nprev = 0;
      }
    }
  } else {
    if (action == kExpand) {
      for (int a = t; a < gc * nblock; a += kT) {
        const int i = a % gc, c = a / gc;
        d->yprev[c * kLd + i] = d->Y[s_blk[c] * kLd + i];
      }
    }
    if (t == 0) {
      C.restart = 0;
      C.nr = gc;
      if (action == kExpand) {
        d->nprev = nblock;
        d->gprev = gc;
      }
    }
  }
  if (t < kMaxBlock) d->blk[t] = (t < nblock) ? s_blk[t] : 0;
}

// the control step; with a non-null host record (pinned, coherent host memory
// mapped for the device) the decision record is also written there with
// ordinary vector stores, so the host reads it without a separate copy.
// Publication order: the lanes of wavefront 0 write the record's words and a
// checksum of them; each lane then executes a system-scope release fence, so
// that its own words are visible to the host before the workgroup barrier
// completes; after the barrier thread 0 writes the sequence number and the
// checksum and publishes the sequence number with a system-scope release
// store.  A host that reads the published number therefore reads every word
// of the same record.  (A release store orders only the storing lane's own
// earlier stores: without the fences of the other lanes, words written by
// lanes 1..63 could reach host memory after the sequence word, and a host
// polling that word could take the new number with words of the previous
// record.)  The host also checks the checksum before it accepts the record.
__device__ __forceinline__ void control_kernel_body(Small* d, const CtlParams& P, Ctl* host,
                                                    int* seqp, int seq) {
  __shared__ Ctl rec;
  control_body(d, P, rec);
  if (host) {
    __syncthreads();
    constexpr int nw = (int)(offsetof(Ctl, seq) / sizeof(unsigned int));
    unsigned int part = 0;
    if (threadIdx.x < kWave) {
      const unsigned int* src = reinterpret_cast<const unsigned int*>(&rec);
      unsigned int* dst = reinterpret_cast<unsigned int*>(host);
      for (int a = threadIdx.x; a < nw; a += kWave) {
        const unsigned int w = src[a];
        dst[a] = w;
        part += ctl_mix(w, (unsigned int)a);
      }
#pragma unroll
      for (int off = kWave / 2; off > 0; off >>= 1) part += __shfl_xor(part, off, kWave);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");  // system scope: this lane's words
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      host->seq = seq;
      host->sum = part + ctl_mix((unsigned int)seq, (unsigned int)nw);
      if (seqp) __hip_atomic_store(seqp, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

__global__ __launch_bounds__(kT) void k_control(Small* d, CtlParams P, Ctl* host, int* seqp,
                                               int seq) {
  control_kernel_body(d, P, host, seqp, seq);
}
__global__ __launch_bounds__(kT) void k_control_batch(const ControlArgs* a) {
  const ControlArgs& q = a[blockIdx.x];
  control_kernel_body(q.d, q.P, q.host, q.seqp, q.seq);
}

void small_control(Small* d, const CtlParams& p, hipStream_t s, Ctl* host, int* seqp, int seq) {
  if (p.nc > kKmax + 8 || p.gc > kGmax) throw Error(SVDS_ERR_ARG, "control: sizes");
  k_control<<<1, kT, 0, s>>>(d, p, host, seqp, seq);
  SVDS_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// stage-1 final Rayleigh-Ritz on A X: eigenpairs of the k x k Gram matrix
// ---------------------------------------------------------------------------
void small_final_rr(int k, double* G, int ldg, int descending, double* lam, double* Z, int ldz,
                    hipStream_t s) {
  small_eig(k, G, ldg, descending, lam, Z, ldz, s);
}

// batched single-workgroup steps
void small_h_append_batch(const std::vector<HAppendArgs>& a, BatchUpload& up, hipStream_t s) {
  if (a.empty()) return;
  const auto* d = up.put(a.data(), a.size());
  up.flush();
  k_h_append_batch<<<(unsigned)a.size(), kHAppT, 0, s>>>(d);
  SVDS_LAUNCH_CHECK();
}

void small_extract_batch(const std::vector<ExtractArgs>& a, BatchUpload& up, hipStream_t s) {
  if (a.empty()) return;
  for (const ExtractArgs& q : a)
    if (q.gc < 1 || q.gc > kGmax) throw Error(SVDS_ERR_ARG, "extract: basis size");
  const auto* d = up.put(a.data(), a.size());
  up.flush();
  k_extract_rr_batch<<<(unsigned)a.size(), kEigT, 0, s>>>(d);
  SVDS_LAUNCH_CHECK();
}

void small_control_batch(const std::vector<ControlArgs>& a, BatchUpload& up, hipStream_t s) {
  if (a.empty()) return;
  for (const ControlArgs& q : a)
    if (q.P.nc > kKmax + 8 || q.P.gc > kGmax) throw Error(SVDS_ERR_ARG, "control: sizes");
  const auto* d = up.put(a.data(), a.size());
  up.flush();
  k_control_batch<<<(unsigned)a.size(), kT, 0, s>>>(d);
  SVDS_LAUNCH_CHECK();
}

}  // namespace svds

