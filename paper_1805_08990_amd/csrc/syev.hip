// Symmetric eigen-decomposition of the small k x k matrix M = R Dhat R^T of
// the column compression, with truncation: only eigenpairs with
// |lambda| > tol * max|lambda| are formed, ordered by |lambda| descending.
//
//   1. tridiag_kernel   : Householder reduction to tridiagonal form
//                         (one workgroup, 256 row lanes x 4 column groups).
//   2. bisect_kernel    : every eigenvalue by Sturm-count bisection, one
//                         thread per eigenvalue index (embarrassingly parallel).
//   3. select_kernel    : threshold, |lambda|-descending order of the kept set
//                         and the clusters of kept eigenvalues whose gaps are
//                         below 1e-3 ||T|| (the absolute criterion of LAPACK's
//                         inverse iteration).
//   4. invit_kernel     : inverse iteration with a partially pivoted
//                         tridiagonal LU, one workgroup per kept eigenvalue,
//                         all independent.
//   5. orth_kernel      : one workgroup per cluster orthonormalises the
//                         cluster's vectors (right-looking modified Gram-Schmidt,
//                         two passes).
//   6. backtr_kernel    : V = H_0 ... H_{k-3} Z, one workgroup per column.
//
// An inverse-iteration vector is off its eigenvector by O(u ||M|| / gap) in
// the directions of nearby eigenvectors; orthonormalising a cluster mixes its
// vectors by that much, which changes sum_i lam_i v_i v_i^T by O(u ||M||) per
// pair (the mixing times the eigenvalue difference), so the kept part is
// reproduced to roundoff and the vectors are orthonormal to roundoff.
#include "common.h"

namespace dme {
namespace {

constexpr int kTriT = 1024;
constexpr int kRowLanes = 256;
constexpr int kColGroups = kTriT / kRowLanes;
constexpr double kOrtol = 1e-3;  // gaps below kOrtol ||T|| join a cluster
constexpr int kInvitIters = 3;
constexpr int kInvitLdsMaxK = 2048;  // inverse-iteration arrays in LDS up to this k

__device__ inline double block_sum_1024(double v, double* red) {
  // red: kTriT doubles of LDS; returns the total to every thread
  const int t = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) tot += red[w];
  __syncthreads();
  return tot;
}

// Householder tridiagonalisation with the whole matrix in registers, for
// k <= 32 RB: the 1024 threads form a 32 x 32 grid and thread (a, b) holds the
// RB x RB block of rows a RB .. and columns b RB ..  A step broadcasts column j
// through LDS, wave 0 forms the reflector, the product p = tau A22 v is summed
// across the 32 column owners of a row block with lane shuffles (they share a
// wave), and the rank-2 update touches registers only.  The reflector vectors
// are written to A(j+2:, j) at the end, as in tridiag_kernel.
template <int RBR, int RBC, int NT>
__global__ __launch_bounds__(NT) void tridiag_reg_kernel(double* A, int64_t lda, int k, double* d,
                                                           double* e, double* tau) {
  constexpr int G = 32;         // column blocks (one half-wave per row block)
  constexpr int KM = G * RBC;   // largest k
  static_assert((NT / G) * RBR == KM, "row and column blocks must cover the same k");
  __shared__ double col[KM];    // column j, then v
  __shared__ double sp[KM];     // p, then w
  __shared__ double coef[4];    // beta, tau, scale, K
  const int t = threadIdx.x;
  const int a = t / G, b = t % G;  // a: row block, b: column block (b runs along the wave)
  const int lane = t & 63;
  double blk[RBR][RBC];
#pragma unroll
  for (int ii = 0; ii < RBR; ++ii)
#pragma unroll
    for (int jj = 0; jj < RBC; ++jj) {
      const int i = a * RBR + ii, l = b * RBC + jj;
      blk[ii][jj] = (i < k && l < k) ? A[i + (int64_t)l * lda] : 0.0;
    }
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1;
    // broadcast column j
    if (b == j / RBC) {
#pragma unroll
      for (int jj = 0; jj < RBC; ++jj)
        if (jj == j % RBC) {
#pragma unroll
          for (int ii = 0; ii < RBR; ++ii) col[a * RBR + ii] = blk[ii][jj];
        }
    }
    __syncthreads();
    if (t < 64) {
      double s2 = 0.0;
      for (int i = j + 2 + lane; i < k; i += 64) s2 += col[i] * col[i];
      for (int off = 32; off > 0; off >>= 1) s2 += __shfl_xor(s2, off, 64);
      if (lane == 0) {
        const double alpha = col[r0];
        if (s2 == 0.0) {
          coef[0] = alpha; coef[1] = 0.0; coef[2] = 0.0;
        } else {
          const double beta = -copysign(sqrt(alpha * alpha + s2), alpha);
          coef[0] = beta;
          coef[1] = (beta - alpha) / beta;
          coef[2] = 1.0 / (alpha - beta);
        }
        d[j] = col[j];
        e[j] = coef[0];
        tau[j] = coef[1];
      }
    }
    __syncthreads();
    const double tj = coef[1], sc = coef[2];
    if (tj == 0.0) continue;  // uniform: nothing to annihilate
    // v (in place of col): v(r0) = 1, v(i) = sc col(i) below, 0 above
    for (int i = t; i < KM; i += NT) {
      double v = 0.0;
      if (i == r0) v = 1.0;
      else if (i > r0 && i < k) v = sc * col[i];
      col[i] = v;  // each entry written by its own thread after every read above
    }
    __syncthreads();
    // p = tau A22 v: row-block partial over this thread's columns, summed
    // across the 32 threads of the row block (one half of a wave)
#pragma unroll
    for (int ii = 0; ii < RBR; ++ii) {
      double acc = 0.0;
#pragma unroll
      for (int jj = 0; jj < RBC; ++jj) acc += blk[ii][jj] * col[b * RBC + jj];
      for (int off = 16; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      const int i = a * RBR + ii;
      if (b == 0) sp[i] = (i >= r0 && i < k) ? tj * acc : 0.0;
    }
    __syncthreads();
    if (t < 64) {
      double pv = 0.0;
      for (int i = r0 + lane; i < k; i += 64) pv += sp[i] * col[i];
      for (int off = 32; off > 0; off >>= 1) pv += __shfl_xor(pv, off, 64);
      if (lane == 0) coef[3] = 0.5 * tj * pv;
    }
    __syncthreads();
    const double Kc = coef[3];
    // rank-2 update of the trailing block: A22 -= v w^T + w v^T, w = p - K v
    // (v, w of this thread's columns in registers, of its rows read per row)
    double vl[RBC], wl[RBC];
#pragma unroll
    for (int q = 0; q < RBC; ++q) {
      const int l = b * RBC + q;
      vl[q] = col[l];
      wl[q] = sp[l] - Kc * col[l];
    }
#pragma unroll
    for (int ii = 0; ii < RBR; ++ii) {
      const int i = a * RBR + ii;
      const double vi = col[i];
      const double wi = sp[i] - Kc * vi;
#pragma unroll
      for (int jj = 0; jj < RBC; ++jj) blk[ii][jj] -= vi * wl[jj] + wi * vl[jj];
    }
    // keep the reflector in column j (rows >= j + 2) and beta at (r0, j)
    if (b == j / RBC) {
#pragma unroll
      for (int jj = 0; jj < RBC; ++jj)
        if (jj == j % RBC) {
#pragma unroll
          for (int ii = 0; ii < RBR; ++ii) {
            const int i = a * RBR + ii;
            if (i == r0) blk[ii][jj] = coef[0];
            else if (i > r0) blk[ii][jj] = col[i];
          }
        }
    }
    __syncthreads();
  }
  // write back; d, e of the last 2 x 2 block
#pragma unroll
  for (int ii = 0; ii < RBR; ++ii)
#pragma unroll
    for (int jj = 0; jj < RBC; ++jj) {
      const int i = a * RBR + ii, l = b * RBC + jj;
      if (i < k && l < k) A[i + (int64_t)l * lda] = blk[ii][jj];
    }
  __syncthreads();
  if (t == 0) {
    if (k >= 2) {
      d[k - 2] = A[(k - 2) + (int64_t)(k - 2) * lda];
      e[k - 2] = A[(k - 1) + (int64_t)(k - 2) * lda];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = A[(k - 1) + (int64_t)(k - 1) * lda];
    tau[k - 1] = 0.0;
  }
}

// Householder tridiagonalisation for k <= kTriMaxK, same outputs as
// tridiag_kernel.  Wave w owns the columns l = r0 + w, r0 + w + 16, ... of the
// trailing block and lane i its rows r0 + i, r0 + i + 64, ..., so the products
// with the trailing block read whole column segments (coalesced) with many
// independent loads per lane; v, w and the product p live in LDS.
constexpr int kTriMaxK = 512;
constexpr int kTriRows = kTriMaxK / 64;  // row blocks per lane

__global__ __launch_bounds__(kTriT) void tridiag_small_kernel(double* A, int64_t lda, int k, double* d,
                                                              double* e, double* tau) {
  extern __shared__ double sm[];
  double* sv = sm;             // v (rows r0 .. k-1; sv[r0] = 1)
  double* sw = sm + k;         // w
  double* sp = sm + 2 * k;     // p
  double* pp = sm + 3 * k;     // [16][k] per-wave partial products
  __shared__ double red[kTriT / 64];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  constexpr int NW = kTriT / 64;
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1;
    const double alpha = A[r0 + (int64_t)j * lda];
    double part = 0.0;
    for (int i = j + 2 + t; i < k; i += kTriT) {
      const double a = A[i + (int64_t)j * lda];
      part += a * a;
    }
    const double sig2 = block_sum_1024(part, red);
    if (sig2 == 0.0) {
      if (t == 0) { tau[j] = 0.0; e[j] = alpha; d[j] = A[j + (int64_t)j * lda]; }
      __syncthreads();
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
    const double tj = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    for (int i = r0 + t; i < k; i += kTriT) {
      double vi = 1.0;
      if (i > r0) {
        vi = A[i + (int64_t)j * lda] * scale;
        A[i + (int64_t)j * lda] = vi;
      }
      sv[i] = vi;
    }
    if (t == 0) {
      tau[j] = tj;
      e[j] = beta;
      d[j] = A[j + (int64_t)j * lda];
      A[r0 + (int64_t)j * lda] = beta;
    }
    __syncthreads();
    // p = tau * A22 v: per-wave column sums, then across waves
    {
      double acc[kTriRows];
#pragma unroll
      for (int q = 0; q < kTriRows; ++q) acc[q] = 0.0;
      for (int l = r0 + wv; l < k; l += NW) {
        const double vl = sv[l];
        const double* col = A + (int64_t)l * lda;
#pragma unroll
        for (int q = 0; q < kTriRows; ++q) {
          const int i = r0 + lane + 64 * q;
          if (i < k) acc[q] += col[i] * vl;
        }
      }
#pragma unroll
      for (int q = 0; q < kTriRows; ++q) {
        const int i = r0 + lane + 64 * q;
        if (i < k) pp[wv * k + i] = acc[q];
      }
    }
    __syncthreads();
    part = 0.0;
    for (int i = r0 + t; i < k; i += kTriT) {
      double sacc = 0.0;
      for (int g = 0; g < NW; ++g) sacc += pp[g * k + i];
      const double pi = tj * sacc;
      sp[i] = pi;
      part += pi * sv[i];
    }
    // K = tau/2 * p^T v ; w = p - K v
    const double pv = block_sum_1024(part, red);
    const double Kc = 0.5 * tj * pv;
    for (int i = r0 + t; i < k; i += kTriT) sw[i] = sp[i] - Kc * sv[i];
    __syncthreads();
    // A22 -= v w^T + w v^T
    for (int l = r0 + wv; l < k; l += NW) {
      const double vl = sv[l], wl = sw[l];
      double* col = A + (int64_t)l * lda;
#pragma unroll
      for (int q = 0; q < kTriRows; ++q) {
        const int i = r0 + lane + 64 * q;
        if (i < k) col[i] -= sv[i] * wl + sw[i] * vl;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (k >= 2) {
      d[k - 2] = A[(k - 2) + (int64_t)(k - 2) * lda];
      e[k - 2] = A[(k - 1) + (int64_t)(k - 2) * lda];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = A[(k - 1) + (int64_t)(k - 1) * lda];
    tau[k - 1] = 0.0;
  }
}

// Householder tridiagonalisation of A (k x k, ld lda, full symmetric storage,
// overwritten).  Outputs d[k], e[k-1], tau[k]; v_j is left in A(j+2:, j) with
// an implicit 1 at row j + 1.
__global__ __launch_bounds__(kTriT) void tridiag_kernel(double* A, int64_t lda, int k, double* d,
                                                        double* e, double* tau, double* pbuf) {
  __shared__ double red[kTriT / 64];
  __shared__ double scal[4];
  __shared__ double ppart[kColGroups][kRowLanes];
  const int t = threadIdx.x;
  const int rl = t % kRowLanes, cg = t / kRowLanes;
  double* p = pbuf;        // length k
  double* w = pbuf + k;    // length k
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1;  // first row of x
    // sigma^2 = sum_{i >= j+2} A(i, j)^2
    // alpha is read before the reduction's barriers: thread 0 overwrites
    // A(r0, j) with beta below, after every wave has passed them.
    const double alpha = A[r0 + (int64_t)j * lda];
    double part = 0.0;
    for (int i = j + 2 + t; i < k; i += kTriT) {
      const double a = A[i + (int64_t)j * lda];
      part += a * a;
    }
    const double sig2 = block_sum_1024(part, red);
    if (sig2 == 0.0) {
      if (t == 0) { tau[j] = 0.0; e[j] = alpha; d[j] = A[j + (int64_t)j * lda]; }
      __syncthreads();
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + sig2), alpha);
    const double tj = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    // v stored in place (rows >= j+2); v(r0) = 1
    for (int i = j + 2 + t; i < k; i += kTriT) A[i + (int64_t)j * lda] *= scale;
    if (t == 0) {
      tau[j] = tj;
      e[j] = beta;
      d[j] = A[j + (int64_t)j * lda];
      A[r0 + (int64_t)j * lda] = beta;
    }
    __syncthreads();
    // p = tau * A22 v over rows/cols [r0, k)
    for (int i0 = r0; i0 < k; i0 += kRowLanes) {
      const int i = i0 + rl;
      double acc = 0.0;
      if (i < k) {
        for (int l = r0 + cg; l < k; l += kColGroups) {
          const double vl = (l == r0) ? 1.0 : A[l + (int64_t)j * lda];
          acc += A[i + (int64_t)l * lda] * vl;
        }
      }
      ppart[cg][rl] = acc;
      __syncthreads();
      if (cg == 0 && i < k) {
        double s = 0.0;
        for (int g = 0; g < kColGroups; ++g) s += ppart[g][rl];
        p[i] = tj * s;
      }
      __syncthreads();
    }
    // K = tau/2 * p^T v ; w = p - K v
    part = 0.0;
    for (int i = r0 + t; i < k; i += kTriT) {
      const double vi = (i == r0) ? 1.0 : A[i + (int64_t)j * lda];
      part += p[i] * vi;
    }
    const double pv = block_sum_1024(part, red);
    const double Kc = 0.5 * tj * pv;
    for (int i = r0 + t; i < k; i += kTriT) {
      const double vi = (i == r0) ? 1.0 : A[i + (int64_t)j * lda];
      w[i] = p[i] - Kc * vi;
    }
    __syncthreads();
    // A22 -= v w^T + w v^T
    for (int i0 = r0; i0 < k; i0 += kRowLanes) {
      const int i = i0 + rl;
      if (i < k) {
        const double vi = (i == r0) ? 1.0 : A[i + (int64_t)j * lda];
        const double wi = w[i];
        for (int l = r0 + cg; l < k; l += kColGroups) {
          const double vl = (l == r0) ? 1.0 : A[l + (int64_t)j * lda];
          A[i + (int64_t)l * lda] -= vi * w[l] + wi * vl;
        }
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (k >= 2) {
      d[k - 2] = A[(k - 2) + (int64_t)(k - 2) * lda];
      e[k - 2] = A[(k - 1) + (int64_t)(k - 2) * lda];
      tau[k - 2] = 0.0;
    }
    d[k - 1] = A[(k - 1) + (int64_t)(k - 1) * lda];
    tau[k - 1] = 0.0;
  }
  (void)scal;
}

// Number of eigenvalues of the tridiagonal (d, e) strictly below x.
__device__ inline int sturm_count(const double* d, const double* e2, int k, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += (q < 0.0);
  for (int i = 1; i < k; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += (q < 0.0);
  }
  return cnt;
}

// bounds[0..1] = Gershgorin interval, bounds[2] = pivmin, bounds[3] = ||T||_inf;
// e2 = e^2.
__global__ void tri_prep_kernel(const double* d, const double* e, int k, double* e2, double* bounds) {
  __shared__ double slo[256], shi[256], se2[256], snrm[256];
  double lo = INFINITY, hi = -INFINITY, me2 = 0.0, nrm = 0.0;
  for (int i = threadIdx.x; i < k; i += 256) {
    const double el = (i > 0) ? fabs(e[i - 1]) : 0.0;
    const double er = (i + 1 < k) ? fabs(e[i]) : 0.0;
    lo = fmin(lo, d[i] - el - er);
    hi = fmax(hi, d[i] + el + er);
    nrm = fmax(nrm, fabs(d[i]) + el + er);
    if (i + 1 < k) {
      const double v = e[i] * e[i];
      e2[i] = v;
      me2 = fmax(me2, v);
    }
  }
  slo[threadIdx.x] = lo; shi[threadIdx.x] = hi; se2[threadIdx.x] = me2; snrm[threadIdx.x] = nrm;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      slo[threadIdx.x] = fmin(slo[threadIdx.x], slo[threadIdx.x + s]);
      shi[threadIdx.x] = fmax(shi[threadIdx.x], shi[threadIdx.x + s]);
      se2[threadIdx.x] = fmax(se2[threadIdx.x], se2[threadIdx.x + s]);
      snrm[threadIdx.x] = fmax(snrm[threadIdx.x], snrm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double nrmT = snrm[0];
    const double slack = 2.0 * DBL_EPSILON * nrmT * k + 1e-300;
    bounds[0] = slo[0] - slack;
    bounds[1] = shi[0] + slack;
    bounds[2] = DBL_MIN * fmax(1.0, se2[0]);
    bounds[3] = nrmT;
  }
}

// Eigenvalue i (ascending) by multisection on the Sturm count: wave i
// evaluates the count at 63 interior points of its interval and keeps the
// sub-interval where the count passes i, so each round shrinks the interval
// 64-fold.  Stops at the width the reduction determines the eigenvalue to.
__global__ __launch_bounds__(64) void bisect_kernel(const double* d, const double* e2, int k,
                                                    const double* bounds, double* lam) {
  const int i = blockIdx.x;
  const int lane = threadIdx.x;
  if (i >= k) return;
  double lo = bounds[0], hi = bounds[1];
  const double pivmin = bounds[2];
  const double atol = DBL_EPSILON * bounds[3] + 2.0 * DBL_MIN;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + atol) break;
    const double h = (hi - lo) / 64.0;
    const double x = (lane < 63) ? lo + h * (double)(lane + 1) : hi;
    const bool above = (lane < 63) ? (sturm_count(d, e2, k, x, pivmin) > i) : true;
    const uint64_t mask = __ballot(above);
    const int first = __ffsll((unsigned long long)mask) - 1;  // lane 63 is always set
    const double nlo = (first == 0) ? lo : lo + h * (double)first;
    const double nhi = (first == 63) ? hi : lo + h * (double)(first + 1);
    if (!(nhi - nlo < hi - lo)) break;  // no progress in floating point
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[i] = 0.5 * (lo + hi);
}

// One thread: threshold, ordering by |lambda| descending (negatives first on
// ties), clusters of the kept set.  Outputs:
//   order[c]  : ascending index of the c-th kept eigenvalue
//   lam_out   : kept eigenvalues (|lambda| desc), then the rest
//   clusters  : (start, len) runs in ascending order over kept eigenvalues
//               with consecutive gaps <= kOrtol ||T||;
//               cl_count[0] = number of clusters
//   keep[0]   : kept count (capped at max_keep, flag |= 2 when capped)
__global__ void select_kernel(const double* lam, int k, double tol, int64_t max_keep,
                              const double* bounds, int* order, int* pos_of, double* lam_out,
                              int* clusters, int* cl_count, int64_t* keep, int* flag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  // eigenvalues are known to about u ||T||; a zero matrix has no nonzero ones
  double amax = 0.0;
  if (k > 0 && bounds[3] > 0.0) amax = fmax(fabs(lam[0]), fabs(lam[k - 1]));
  const double thr = tol * amax;
  int lo = 0, hi = k - 1, c = 0;
  int kept = 0;
  // merge from both ends of the ascending list
  while (lo <= hi) {
    const double al = fabs(lam[lo]), ah = fabs(lam[hi]);
    int take;
    if (al >= ah) take = lo++;
    else take = hi--;
    const double a = fabs(lam[take]);
    if (amax > 0.0 && a > thr) {
      order[c] = take;
      ++c;
    }
    pos_of[take] = -1;
  }
  kept = c;
  int64_t cap = kept;
  if (cap > max_keep) {
    cap = max_keep;
    atomicOr(flag, 2);
  }
  for (int q = 0; q < k; ++q) pos_of[q] = -1;
  for (int q = 0; q < cap; ++q) pos_of[order[q]] = q;
  // lam_out: kept first (in order), then the remaining ones in ascending order
  int o = 0;
  for (int q = 0; q < cap; ++q) lam_out[o++] = lam[order[q]];
  for (int q = 0; q < k; ++q)
    if (pos_of[q] < 0) lam_out[o++] = lam[q];
  // clusters among kept eigenvalues, scanning in ascending order
  int ncl = 0;
  int q = 0;
  while (q < k) {
    if (pos_of[q] < 0) { ++q; continue; }
    int start = q, len = 1;
    while (q + len < k && pos_of[q + len] >= 0) {
      const double a = lam[q + len - 1], b = lam[q + len];
      if (b - a <= kOrtol * bounds[3]) ++len;
      else break;
    }
    clusters[2 * ncl] = start;
    clusters[2 * ncl + 1] = len;
    ++ncl;
    q = start + len;
  }
  cl_count[0] = ncl;
  keep[0] = cap;
}

// Deterministic start vector in (-1, 1).
__device__ inline double start_entry(int idx, int i) {
  uint32_t h = (uint32_t)(idx * 0x9E3779B9u) ^ (uint32_t)(i * 0x85EBCA6Bu) ^ 0x27D4EB2Fu;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)(h & 0xFFFFFF) / (double)0x1000000) * 2.0 - 1.0;
}

// Inverse iteration for kept eigenvalue number `blockIdx.x` (ascending index
// idx, output column pos_of[idx]); the tridiagonal LU and the solves are
// sequential (thread 0), the rescaling and normalisation use the block.
// Eigenvalues inside one cluster get shifts nudged apart by a few ulps of
// ||T|| and distinct start vectors, so their iterates differ.  Z is column-
// major: Z[i + c * ldz] is entry i of output column c.
__global__ void invit_kernel(const double* d, const double* e, int k, const double* lam,
                             const int* order, const int64_t* keep, const double* bounds,
                             double* work, double* Z, int64_t ldz, int use_lds) {
  const int c = blockIdx.x;
  if (c >= keep[0]) return;
  const int idx = order[c];
  extern __shared__ double ism[];
  __shared__ double red[256 / 64];
  __shared__ double sscale;
  // the sequential LU and solves touch these arrays element by element:
  // keep them in LDS when they fit
  double* u0 = use_lds ? ism : work + (int64_t)c * 6 * k;
  double* u1 = u0 + k;
  double* u2 = u1 + k;
  double* lm = u2 + k;
  double* x = lm + k;
  int* sw = reinterpret_cast<int*>(x + k);
  const double nrmT = bounds[3];
  const double eps = DBL_EPSILON;
  const double small = eps * fmax(nrmT, DBL_MIN);
  // nudge equal neighbours apart: count earlier eigenvalues within a few ulps
  double lamq = lam[idx];
  {
    int rank_in_tie = 0;
    for (int q = idx - 1; q >= 0 && lam[idx] - lam[q] <= 4.0 * eps * nrmT; --q) ++rank_in_tie;
    lamq += 4.0 * rank_in_tie * eps * fmax(nrmT, DBL_MIN);
  }
  if (threadIdx.x == 0) {
    // LU with partial pivoting of T - lamq I: rows i, i+1 may swap.
    // After elimination row i holds u0[i] (diag), u1[i], u2[i] (super-diags).
    double a = d[0] - lamq;
    double b = (k > 1) ? e[0] : 0.0;
    for (int i = 0; i + 1 < k; ++i) {
      const double sub = e[i];
      const double dn = d[i + 1] - lamq;
      const double sn = (i + 2 < k) ? e[i + 1] : 0.0;
      if (fabs(a) >= fabs(sub)) {
        sw[i] = 0;
        const double piv = (a == 0.0) ? small : a;
        const double mlt = sub / piv;
        u0[i] = piv; u1[i] = b; u2[i] = 0.0; lm[i] = mlt;
        a = dn - mlt * b;
        b = sn;
      } else {
        sw[i] = 1;
        const double mlt = a / sub;
        u0[i] = sub; u1[i] = dn; u2[i] = sn; lm[i] = mlt;
        a = b - mlt * dn;
        b = -mlt * sn;
      }
    }
    u0[k - 1] = (a == 0.0) ? small : a;
    u1[k - 1] = 0.0; u2[k - 1] = 0.0;
  }
  for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] = start_entry(idx, i);
  __syncthreads();
  for (int it = 0; it < kInvitIters; ++it) {
    if (threadIdx.x == 0) {
      for (int i = 0; i + 1 < k; ++i) {
        if (sw[i]) { const double tmp = x[i]; x[i] = x[i + 1]; x[i + 1] = tmp; }
        x[i + 1] -= lm[i] * x[i];
      }
      for (int i = k - 1; i >= 0; --i) {
        double v = x[i];
        if (i + 1 < k) v -= u1[i] * x[i + 1];
        if (i + 2 < k) v -= u2[i] * x[i + 2];
        const double piv = (fabs(u0[i]) < small) ? copysign(small, u0[i] == 0.0 ? 1.0 : u0[i]) : u0[i];
        x[i] = v / piv;
      }
      double mx = 0.0;
      for (int i = 0; i < k; ++i) mx = fmax(mx, fabs(x[i]));
      sscale = (mx > 0.0) ? 1.0 / mx : 1.0;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += blockDim.x) x[i] *= sscale;
    __syncthreads();
  }
  double part = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) part += x[i] * x[i];
  for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
  __syncthreads();
  double nn = 0.0;
  for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) nn += red[wv];
  const double inv = (nn > 0.0) ? 1.0 / sqrt(nn) : 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) Z[i + (int64_t)c * ldz] = x[i] * inv;
}

// Orthonormalise the vectors of one cluster (blockIdx.x), in ascending
// eigenvalue order, by right-looking modified Gram-Schmidt done twice: at
// step j every later vector loses its component along z_j.  Each wave
// handles a subset of the later vectors and recomputes ||z_j|| itself, so a
// step needs one barrier.  The cluster is staged in LDS when it fits
// (lds_doubles entries of dynamic shared memory).
__global__ __launch_bounds__(1024) void orth_kernel(int k, const int* clusters, const int* cl_count,
                                                    const int* pos_of, double* Z, int64_t ldz,
                                                    int lds_doubles) {
  extern __shared__ double zs[];
  const int cl = blockIdx.x;
  if (cl >= cl_count[0]) return;
  const int start = clusters[2 * cl], len = clusters[2 * cl + 1];
  if (len < 2) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const bool staged = (int64_t)len * k <= (int64_t)lds_doubles;
  // vector q of the cluster: zs[q * k + i] when staged, else Z column pos_of[start + q]
  auto vec = [&](int q) -> double* {
    return staged ? zs + (int64_t)q * k : Z + (int64_t)pos_of[start + q] * ldz;
  };
  if (staged) {
    for (int q = wv; q < len; q += nw) {
      const double* src = Z + (int64_t)pos_of[start + q] * ldz;
      for (int i = lane; i < k; i += 64) zs[(int64_t)q * k + i] = src[i];
    }
    __syncthreads();
  }
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = 0; j < len; ++j) {
      const double* zj = vec(j);
      double nj = 0.0;
      for (int i = lane; i < k; i += 64) nj += zj[i] * zj[i];
      for (int off = 32; off > 0; off >>= 1) nj += __shfl_xor(nj, off, 64);
      const double inv2 = (nj > 0.0) ? 1.0 / nj : 0.0;
      for (int l = j + 1 + wv; l < len; l += nw) {
        double* zl = vec(l);
        double dt = 0.0;
        for (int i = lane; i < k; i += 64) dt += zj[i] * zl[i];
        for (int off = 32; off > 0; off >>= 1) dt += __shfl_xor(dt, off, 64);
        const double f = dt * inv2;
        for (int i = lane; i < k; i += 64) zl[i] -= f * zj[i];
      }
      __syncthreads();
    }
    // normalise every vector of the cluster
    for (int j = wv; j < len; j += nw) {
      double* zj = vec(j);
      double nj = 0.0;
      for (int i = lane; i < k; i += 64) nj += zj[i] * zj[i];
      for (int off = 32; off > 0; off >>= 1) nj += __shfl_xor(nj, off, 64);
      const double inv = (nj > 0.0) ? 1.0 / sqrt(nj) : 0.0;
      for (int i = lane; i < k; i += 64) zj[i] *= inv;
    }
    __syncthreads();
  }
  if (staged) {
    for (int q = wv; q < len; q += nw) {
      double* dst = Z + (int64_t)pos_of[start + q] * ldz;
      for (int i = lane; i < k; i += 64) dst[i] = zs[(int64_t)q * k + i];
    }
  }
}

// V(:, c) = H_0 H_1 ... H_{k-3} z_c, with z_c = Z[i + c * ldz]; one block per
// column, z staged in LDS.  Also fixes the sign so that the largest-|entry| is
// positive.
__global__ void backtr_kernel(const double* A, int64_t lda, const double* tau, int k,
                              const double* Z, int64_t ldz, const int64_t* keep, double* V,
                              int64_t ldv) {
  extern __shared__ double z[];
  __shared__ double red[256 / 64];
  const int c = blockIdx.x;
  if (c >= keep[0]) return;
  for (int i = threadIdx.x; i < k; i += blockDim.x) z[i] = Z[i + (int64_t)c * ldz];
  __syncthreads();
  for (int j = k - 3; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const int r0 = j + 1;
    double part = 0.0;
    for (int i = r0 + threadIdx.x; i < k; i += blockDim.x) {
      const double vi = (i == r0) ? 1.0 : A[i + (int64_t)j * lda];
      part += vi * z[i];
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    double s = 0.0;
    for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) s += red[wv];
    __syncthreads();
    s *= tj;
    for (int i = r0 + threadIdx.x; i < k; i += blockDim.x) {
      const double vi = (i == r0) ? 1.0 : A[i + (int64_t)j * lda];
      z[i] -= s * vi;
    }
    __syncthreads();
  }
  // sign convention: largest |entry| positive (first one on ties)
  if (threadIdx.x == 0) {
    double best = -1.0, sgn = 1.0;
    for (int i = 0; i < k; ++i) {
      const double a = fabs(z[i]);
      if (a > best) { best = a; sgn = (z[i] < 0.0) ? -1.0 : 1.0; }
    }
    red[0] = sgn;
  }
  __syncthreads();
  const double sgn = red[0];
  for (int i = threadIdx.x; i < k; i += blockDim.x) V[i + (int64_t)c * ldv] = sgn * z[i];
}

}  // namespace

size_t syev_workspace(int64_t k) {
  size_t b = 0;
  b += (size_t)k * k * sizeof(double) + 256;      // A copy
  b += 8 * ((size_t)k * sizeof(double) + 256);    // d, e, tau, p, w, e2, lam, bounds
  b += 4 * ((size_t)k * sizeof(int) + 256);       // order, pos_of, clusters(2k), count
  b += (size_t)k * 2 * sizeof(int) + 256;
  b += (size_t)k * 6 * k * sizeof(double) + 256;  // invit scratch (per cluster)
  b += (size_t)k * k * sizeof(double) + 256;      // Zt
  return b;
}

void syev_trunc_f64(hipStream_t s, int64_t k, const double* M, int64_t ldm, double tol,
                    int64_t max_keep, double* lam_out, double* V_out, int64_t ldv,
                    int64_t* keep_dev, int* flag_dev, Arena& ws) {
  DME_REQUIRE(k >= 0 && k <= 16384, DME_EINVAL, "syev: k out of range");
  if (k == 0) {
    fill_f64(s, reinterpret_cast<double*>(keep_dev), 1, 1, 1, 0.0);  // all-zero bits
    return;
  }
  const int ki = (int)k;
  double* A = ws.get<double>((size_t)k * k);
  double* d = ws.get<double>(k);
  double* e = ws.get<double>(k);
  double* tau = ws.get<double>(k);
  double* pw = ws.get<double>(2 * k);
  double* e2 = ws.get<double>(k);
  double* lam = ws.get<double>(k);
  double* bounds = ws.get<double>(8);
  int* order = ws.get<int>(k);
  int* pos_of = ws.get<int>(k);
  int* clusters = ws.get<int>(2 * k);
  int* cl_count = ws.get<int>(4);
  double* work = ws.get<double>((size_t)k * 6 * k);
  double* Zt = ws.get<double>((size_t)k * k);

  copy_f64(s, M, ldm, A, k, k, k);
  if (k == 1) {
    // trivial: d = M(0,0)
    copy_f64(s, A, 1, d, 1, 1, 1);
    fill_f64(s, e, 1, 1, 1, 0.0);
    fill_f64(s, tau, 1, 1, 1, 0.0);
  } else {
    if (k <= 128) {
      hipLaunchKernelGGL((tridiag_reg_kernel<4, 4, 1024>), dim3(1), dim3(1024), 0, s, A, k, ki, d, e, tau);
    } else if (k <= 160) {
      hipLaunchKernelGGL((tridiag_reg_kernel<5, 5, 1024>), dim3(1), dim3(1024), 0, s, A, k, ki, d, e, tau);
    } else if (k <= 192) {
      hipLaunchKernelGGL((tridiag_reg_kernel<12, 6, 512>), dim3(1), dim3(512), 0, s, A, k, ki, d, e, tau);
    } else if (k <= kTriMaxK) {
      const size_t lds = (size_t)(3 + kTriT / 64) * k * sizeof(double);
      hipLaunchKernelGGL(tridiag_small_kernel, dim3(1), dim3(kTriT), lds, s, A, k, ki, d, e, tau);
    } else {
      hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(kTriT), 0, s, A, k, ki, d, e, tau, pw);
    }
    DME_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(tri_prep_kernel, dim3(1), dim3(256), 0, s, d, e, ki, e2, bounds);
  DME_HIP(hipGetLastError());
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)k), dim3(64), 0, s, d, e2, ki, bounds, lam);
  DME_HIP(hipGetLastError());
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(64), 0, s, lam, ki, tol, max_keep, bounds, order,
                     pos_of, lam_out, clusters, cl_count, keep_dev, flag_dev);
  DME_HIP(hipGetLastError());
  // Z: k x (kept) column-major with ld = k (kept <= k)
  const unsigned nkeep = (unsigned)std::min<int64_t>(k, max_keep);
  const int invit_lds = (k <= kInvitLdsMaxK) ? 1 : 0;
  hipLaunchKernelGGL(invit_kernel, dim3(nkeep), dim3(64), invit_lds ? (size_t)6 * k * sizeof(double) : 0,
                     s, d, e, ki, lam, order, keep_dev, bounds, work, Zt, k, invit_lds);
  DME_HIP(hipGetLastError());
  // cluster staging in LDS: up to 144 KiB, never more than the whole k x k set
  const int64_t orth_lds = std::min<int64_t>(k * k, (144 * 1024) / (int64_t)sizeof(double));
  hipLaunchKernelGGL(orth_kernel, dim3((unsigned)k), dim3(1024), (size_t)orth_lds * sizeof(double), s,
                     ki, clusters, cl_count, pos_of, Zt, k, (int)orth_lds);
  DME_HIP(hipGetLastError());
  hipLaunchKernelGGL(backtr_kernel, dim3((unsigned)std::min<int64_t>(k, max_keep)), dim3(256),
                     (size_t)k * sizeof(double), s, A, k, tau, ki, Zt, k, keep_dev, V_out, ldv);
  DME_HIP(hipGetLastError());
}

}  // namespace dme
