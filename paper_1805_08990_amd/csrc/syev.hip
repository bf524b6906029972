// Symmetric eigen-decomposition of the small k x k matrix M = R Dhat R^T of
// the column compression, with truncation: only eigenpairs with
// |lambda| > tol * max|lambda| are formed, ordered by |lambda| descending.
//
//   1. tridiagonalisation: Householder reduction to tridiagonal form in one
//                         workgroup: tridiag_tiles_kernel holds the matrix in
//                         registers by tiles (k <= 192), tridiag_small_kernel
//                         keeps the vectors in LDS (k <= 512), tridiag_kernel
//                         works from global memory (larger k).
//   2. bisect_wg_kernel : every eigenvalue by Sturm-count multisection, one
//                         four-wave workgroup per eigenvalue index (all
//                         independent); the tiled tridiagonalisation leaves
//                         its spectrum bounds, tri_prep_kernel forms them
//                         otherwise.
//   3. select_kernel    : threshold, |lambda|-descending order of the kept set
//                         and the clusters of kept eigenvalues whose gaps are
//                         below 1e-3 ||T|| (the absolute criterion of LAPACK's
//                         inverse iteration), one workgroup with prefix sums.
//   4. twist_kernel     : eigenvector from a twisted factorisation, one
//                         wave per kept eigenvalue, all independent;
//      invit_kernel     : inverse iteration with a partially pivoted
//                         tridiagonal LU for tied eigenvalues (and k > 512).
//   5. polar steps      : clusters whose vectors are nearly orthonormal get
//                         three Newton-Schulz steps Z <- Z (3I - Z^T Z) / 2
//                         (restricted to each cluster's block), two MFMA
//                         products a step: Z^T Z (the first one also checks
//                         the clusters) and Z B with B formed as it is read;
//      orth_kernel      : one workgroup per remaining cluster orthonormalises
//                         its vectors (right-looking modified Gram-Schmidt,
//                         two passes).
//   6. backtr_kernel    : Q = H_0 ... H_{k-3} formed one wave per column, on a
//                         second stream beside steps 2-5; then V = Q Z (GEMM).
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
constexpr int kInvitArrays = 8;      // k-long arrays per inverse iteration

__device__ inline double block_sum_1024(double v, double* red) {
  // red: kTriT doubles of LDS; returns the total to every thread
  const int t = threadIdx.x;
  v = wave_sum_f64(v);
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double tot = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) tot += red[w];
  __syncthreads();
  return tot;
}

// sum over aligned groups of G lanes (G = 4, 8 or 16), the same in every lane
template <int G>
__device__ inline double group_sum_f64(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "group size");
  if constexpr (G == 16) return group16_sum_f64(v);
  if constexpr (G == 8) return group8_sum_f64(v);
  v += dpp_mov_f64<kDppXor1>(v);
  return v + dpp_mov_f64<kDppXor2>(v);
}

// Reduce-scatter steps over a half-wave (32 lanes).  rs16: lanes 0-15 of the
// half get a + a of the lane 16 away, lanes 16-31 get b + b of theirs (one
// permlane swap per dword).  rs_dpp: lanes whose bit `hi` is clear get
// a + a of the partner lane, the others b + b of theirs, the partner given by
// the DPP pattern CTRL.
__device__ __forceinline__ double rs16(double a, double b) {
  const uint64_t ua = (uint64_t)__double_as_longlong(a), ub = (uint64_t)__double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)ua, (uint32_t)ub, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(ua >> 32), (uint32_t)(ub >> 32), false, false);
  const double x = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
  const double y = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
  return x + y;
}
template <int CTRL>
__device__ __forceinline__ double rs_dpp(double a, double b, bool hi) {
  const double send = hi ? a : b;  // what the partner keeps
  return (hi ? b : a) + dpp_mov_f64<CTRL>(send);
}
// Row sums of an RT-row tile (RT <= 16) over the 32 lanes of a half-wave: on
// return lane c holds the sum of row c / (32 / S) for S = 8 slots (RT <= 8)
// or 16 slots, zero for the slots past RT.
template <int RT>
__device__ __forceinline__ double tile_row_sums(const double (&sp)[RT], int c) {
  static_assert(RT <= 16, "rows per tile");
  constexpr int S = (RT <= 8) ? 8 : 16;
  double x[S];
#pragma unroll
  for (int u = 0; u < S; ++u) x[u] = (u < RT) ? sp[u] : 0.0;
  double y[S / 2];
#pragma unroll
  for (int t = 0; t < S / 2; ++t) y[t] = rs16(x[t], x[t + S / 2]);  // bit 4 picks t or t + S/2
  const bool b3 = (c >> 3) & 1, b2 = (c >> 2) & 1;
  double z[S / 4];
#pragma unroll
  for (int t = 0; t < S / 4; ++t) z[t] = rs_dpp<kDppRor8>(y[t], y[t + S / 4], b3);  // bit 3
  double w[S / 8];
#pragma unroll
  for (int t = 0; t < S / 8; ++t) w[t] = rs_dpp<kDppHalfMirror>(z[t], z[t + S / 8], b2);  // bit 2
  double v;
  if constexpr (S == 16) {
    v = rs_dpp<kDppXor2>(w[0], w[1], (c >> 1) & 1);  // bit 1
  } else {
    v = w[0];
    v += dpp_mov_f64<kDppXor2>(v);
  }
  return v + dpp_mov_f64<kDppXor1>(v);
}
// sp[u] = sum over m >= M0 of a[u][m] x[m], for the first live chunk m0
// (uniform) taken as a compile-time start by dispatch, so that the skipped
// chunks cost no instructions.
template <int NC, int RT, int M0 = 0>
__device__ __forceinline__ void tile_matvec(int m0, const double (&a)[RT][NC], const double (&x)[NC],
                                            double (&sp)[RT]) {
  if constexpr (M0 + 1 < NC) {
    if (m0 > M0) {
      tile_matvec<NC, RT, M0 + 1>(m0, a, x, sp);
      return;
    }
  }
#pragma unroll
  for (int u = 0; u < RT; ++u) {
    double acc = 0.0;
#pragma unroll
    for (int m = M0; m < NC; ++m) acc += a[u][m] * x[m];
    sp[u] = acc;
  }
}
// The rank-2 update of a tile, a[u][m] -= v_u w_m + w_u v_m, with the row
// values v_u (from vr) and w_u = p_u - K v_u (p_u from pr) read from LDS a pair
// of rows at a time, so that only the column values stay in registers.  The
// chunks before the trailing part change by zero (v and w vanish there); they
// are updated anyway: skipping them by a branch or a dispatch costs more in
// selects or registers than the fused multiply-adds it saves.
template <int NC, int RT>
__device__ __forceinline__ void tile_rank2(double (&a)[RT][NC], const double* vr, const double* pr, double K,
                                           const double (&vC)[NC], const double (&wC)[NC]) {
  static_assert(RT % 2 == 0, "row pairs");
#pragma unroll
  for (int u = 0; u < RT; u += 2) {
    const double2 v2 = *reinterpret_cast<const double2*>(vr + u);
    const double2 p2 = *reinterpret_cast<const double2*>(pr + u);
    const double w0 = p2.x - K * v2.x, w1 = p2.y - K * v2.y;
#pragma unroll
    for (int m = 0; m < NC; ++m) {  // two fused steps in place: no temporaries
      a[u][m] = fma(-v2.x, wC[m], fma(-w0, vC[m], a[u][m]));
      a[u + 1][m] = fma(-v2.y, wC[m], fma(-w1, vC[m], a[u + 1][m]));
    }
  }
}

// e2 = e^2 and the spectrum bounds of the tridiagonal (d, e) (what
// tri_prep_kernel computes), by the whole workgroup from d and e in LDS;
// red holds at least 4 x (waves) doubles.  Called after a barrier.
__device__ inline void tri_bounds_block(const double* sd, const double* se, int k, double* e2, double* bounds,
                                        double* red) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, nw = blockDim.x >> 6;
  double lo = INFINITY, hi = -INFINITY, me2 = 0.0, nrm = 0.0;
  for (int i = t; i < k; i += blockDim.x) {
    const double el = (i > 0) ? fabs(se[i - 1]) : 0.0;
    const double er = (i + 1 < k) ? fabs(se[i]) : 0.0;
    lo = fmin(lo, sd[i] - el - er);
    hi = fmax(hi, sd[i] + el + er);
    nrm = fmax(nrm, fabs(sd[i]) + el + er);
    if (i + 1 < k) {
      const double v = se[i] * se[i];
      e2[i] = v;
      me2 = fmax(me2, v);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off, 64));
    hi = fmax(hi, __shfl_xor(hi, off, 64));
    me2 = fmax(me2, __shfl_xor(me2, off, 64));
    nrm = fmax(nrm, __shfl_xor(nrm, off, 64));
  }
  __syncthreads();  // red may alias LDS the caller used before
  if (lane == 0) {
    red[4 * w] = lo;
    red[4 * w + 1] = hi;
    red[4 * w + 2] = me2;
    red[4 * w + 3] = nrm;
  }
  __syncthreads();
  if (t == 0) {
    for (int q = 1; q < nw; ++q) {
      lo = fmin(lo, red[4 * q]);
      hi = fmax(hi, red[4 * q + 1]);
      me2 = fmax(me2, red[4 * q + 2]);
      nrm = fmax(nrm, red[4 * q + 3]);
    }
    const double slack = 2.0 * DBL_EPSILON * nrm * k + 1e-300;
    bounds[0] = lo - slack;
    bounds[1] = hi + slack;
    bounds[2] = DBL_MIN * fmax(1.0, me2);
    bounds[3] = nrm;
  }
}

// Householder tridiagonalisation with the whole matrix in registers, in
// RT x NC tiles: the 32 lanes of a half-wave share the rows RT h .. RT h + RT - 1
// (h = 2 wave + half) and lane c of them holds the columns c + 32 m (m < NC),
// so a half-wave holds whole rows.  Step j takes two barriers:
//   product phase: p = tau A v by row sums (a reduce-scatter over the 32
//     lanes), the per-wave parts of p^T v, and column j + 1 as it stands
//     (by symmetry the lane q & 31 of every half-wave holds its rows), all to
//     LDS;
//   update phase: every wave applies A -= v w^T + w v^T,
//     w = p - (tau/2)(p^T v) v, to its tiles, while wave 0 forms the
//     reflector of step j + 1 from the column in LDS with the same update
//     applied to it (so the reflector does not wait for the owner of the row).
// The product and the update are issue-bound on the SIMDs' FP64 VALU; the
// reflector (a wave sum, a reciprocal square root and a reciprocal) runs
// beside the update.  The input Min is read once, into the registers; the
// reflector of step j goes to A(j+2:, j) and d, e, tau as in tridiag_kernel.
template <int NC, int RT>
__global__ __launch_bounds__(32 * 32 * NC / RT) void tridiag_tiles_kernel(const double* Min, int64_t ldm,
                                                                          double* A, int64_t lda, int k,
                                                                          double* d, double* e, double* tau,
                                                                          double* e2, double* bounds) {
  constexpr int KM = 32 * NC;        // largest k
  constexpr int NW = KM / (2 * RT);  // waves: two RT-row tiles each
  static_assert(KM % (2 * RT) == 0 && NW <= 16 && RT % 2 == 0, "whole waves, at most 16, row pairs");
  constexpr int NC2 = (KM + 63) / 64;  // entries per lane of wave 0 when it forms a reflector
  constexpr int KP = 64 * NC2;
  __shared__ double vbuf[2][KP];  // reflector of step j in vbuf[j & 1]
  __shared__ double tjs[2];       // and its tau
  __shared__ double pb[KP];       // p
  __shared__ double cb[KP];       // column j + 1 before the update of step j
  __shared__ double wpart[NW];
  __shared__ double sd[KM], se[KM];  // d and e as formed, for the bounds at the end
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int c = lane & 31;
  const int rbase = RT * (2 * wv + (lane >> 5));
  const int wrow_last = 2 * RT * wv + 2 * RT - 1;  // last row of this wave
  double a[RT][NC];
  // entry (rbase + u, c + 32 m) of the input, read as Min(c + 32 m, rbase + u)
  // by symmetry so that the lanes of a half-wave read consecutive addresses
#pragma unroll
  for (int u = 0; u < RT; ++u) {
    const int i = rbase + u;
    const double* Mi = Min + (int64_t)i * ldm + c;
#pragma unroll
    for (int m = 0; m < NC; ++m) a[u][m] = (i < k && c + 32 * m < k) ? Mi[32 * m] : 0.0;
  }
  // Reflector of step q (by wave 0) from column q as it stands, entries
  // l = lane + 64 m in y, with its diagonal entry dq and subdiagonal entry
  // alpha; q = k - 2 leaves the last 2 x 2 block.  With S = alpha^2 + s2,
  // r = 1/sqrt(S) and n = S r: beta = -sign(alpha) n,
  // tau = (beta - alpha)/beta = 1 + |alpha| r and
  // 1/(alpha - beta) = sign(alpha)/(|alpha| + n), the reciprocal square root
  // and the reciprocal from the hardware estimates by two Newton steps each.
  auto form = [&](int q, const double (&y)[NC2], double dq, double alpha) {
    const bool refl = q + 2 < k;
    double s2 = 0.0;
#pragma unroll
    for (int m = 0; m < NC2; ++m) {
      const int l = lane + 64 * m;
      s2 += (l >= q + 2 && l < k) ? y[m] * y[m] : 0.0;
    }
    s2 = wave_sum_f64(s2);
    double beta = alpha, tq = 0.0, sc = 0.0;
    if (refl && s2 != 0.0) {
      const double S = fma(alpha, alpha, s2), hS = 0.5 * S;
      double r = __builtin_amdgcn_rsq(S);
      r = r * fma(-hS * r, r, 1.5);
      r = r * fma(-hS * r, r, 1.5);
      const double n = S * r, aa = fabs(alpha);
      beta = -copysign(n, alpha);
      tq = fma(aa, r, 1.0);
      const double den = aa + n;
      double ri = __builtin_amdgcn_rcp(den);
      ri = fma(ri, fma(-den, ri, 1.0), ri);
      ri = fma(ri, fma(-den, ri, 1.0), ri);
      sc = copysign(ri, alpha);
    }
    double vv[NC2];
#pragma unroll
    for (int m = 0; m < NC2; ++m) {
      const int l = lane + 64 * m;
      vv[m] = (l == q + 1) ? 1.0 : ((l > q + 1 && l < k) ? sc * y[m] : 0.0);
    }
    if (refl) {
#pragma unroll
      for (int m = 0; m < NC2; ++m) vbuf[q & 1][lane + 64 * m] = vv[m];
    }
    if (lane == 0) {
      d[q] = dq;
      sd[q] = dq;
      e[q] = beta;
      se[q] = beta;
      tau[q] = tq;
      if (refl) tjs[q & 1] = tq;
    }
    if (tq != 0.0) {
#pragma unroll
      for (int m = 0; m < NC2; ++m) {
        const int l = lane + 64 * m;
        if (l > q + 1 && l < k) A[l + (int64_t)q * lda] = vv[m];
      }
    }
  };
  if (c == 0) {  // column 0 (every half-wave its rows)
#pragma unroll
    for (int u = 0; u < RT; ++u) cb[rbase + u] = a[u][0];
  }
  __syncthreads();
  if (wv == 0) {
    double y0[NC2];
#pragma unroll
    for (int m = 0; m < NC2; ++m) y0[m] = cb[lane + 64 * m];
    form(0, y0, cb[0], k > 1 ? cb[1] : 0.0);
  }
  __syncthreads();
  for (int j = 0; j + 2 < k; ++j) {
    const int r0 = j + 1, q = j + 1;
    const int mq = q >> 5;  // chunk of column q (chunks m < mq lie before the trailing part)
    const double tj = tjs[j & 1];
    const double* v = vbuf[j & 1];
    const bool live = wrow_last >= r0;  // wave-uniform
    if (tj != 0.0) {                    // uniform across the workgroup
      double vC[NC];
#pragma unroll
      for (int m = 0; m < NC; ++m) vC[m] = v[c + 32 * m];
      constexpr int SL = (RT <= 8) ? 4 : 2;  // lanes per row sum
      const int srow = c / SL;               // the row whose sum this lane gets
      double pu = 0.0;                       // p of row rbase + srow (zero before the trailing part)
      if (live) {
        double sp[RT];
        tile_matvec<NC, RT>(mq, a, vC, sp);
        const double sum = tile_row_sums<RT>(sp, c);
        const int i = rbase + srow;
        pu = (srow < RT && i >= r0 && i < k) ? tj * sum : 0.0;
      }
      const bool lead = (c % SL) == 0;  // one lane per row
      if (lead && srow < RT) pb[rbase + srow] = pu;
      const double vs = (srow < RT) ? v[rbase + min(srow, RT - 1)] : 0.0;
      const double pv = wave_sum_f64(lead ? pu * vs : 0.0);  // both half-waves
      if (lane == 0) wpart[wv] = pv;
    }
    if (live && c == (q & 31)) {
#pragma unroll
      for (int m = 0; m < NC; ++m)
        if (m == mq) {
#pragma unroll
          for (int u = 0; u < RT; ++u) cb[rbase + u] = a[u][m];
        }
    }
    __syncthreads();
    double Kc = 0.0;
    if (tj != 0.0) {
      constexpr int G = NW <= 4 ? 4 : (NW <= 8 ? 8 : 16);  // NW <= 16
      const int gi = lane & (G - 1);
      const double pvt = group_sum_f64<G>(gi < NW ? wpart[gi] : 0.0);
      Kc = 0.5 * tj * pvt;
    }
    if (wv == 0) {
      // column q after step j: y_l = x_l - v_l w_q - w_l v_q with v_q = 1
      // (the entry (l, q) of the tile update); unchanged when the step had no
      // reflector.  Every load is issued before the arithmetic.
      const bool upd = tj != 0.0;
      const double pq = pb[q], vq1 = v[q + 1], pq1 = pb[q + 1], cq = cb[q], cq1 = cb[q + 1];
      double xl[NC2], vl[NC2], pl[NC2];
#pragma unroll
      for (int m = 0; m < NC2; ++m) {
        const int l = lane + 64 * m;
        xl[m] = cb[l];
        vl[m] = v[l];
        pl[m] = pb[l];
      }
      const double wq = pq - Kc, wq1 = pq1 - Kc * vq1;
      const double dq = upd ? fma(-1.0, wq, fma(-wq, 1.0, cq)) : cq;
      const double alpha = upd ? fma(-vq1, wq, fma(-wq1, 1.0, cq1)) : cq1;
      double y[NC2];
#pragma unroll
      for (int m = 0; m < NC2; ++m)
        y[m] = upd ? fma(-vl[m], wq, fma(-(pl[m] - Kc * vl[m]), 1.0, xl[m])) : xl[m];
      form(q, y, dq, alpha);
    }
    if (tj != 0.0 && live) {
      double vC2[NC], wC[NC];
#pragma unroll
      for (int m = 0; m < NC; ++m) {
        vC2[m] = v[c + 32 * m];  // read again rather than held across the barrier
        wC[m] = pb[c + 32 * m] - Kc * vC2[m];
      }
      tile_rank2<NC, RT>(a, v + rbase, pb + rbase, Kc, vC2, wC);
    }
    __syncthreads();
  }
  // the last diagonal entry
  if (k - 1 >= rbase && k - 1 < rbase + RT) {
    const int uu = k - 1 - rbase;
#pragma unroll
    for (int u = 0; u < RT; ++u)
      if (u == uu) {
#pragma unroll
        for (int m = 0; m < NC; ++m)
          if (c + 32 * m == k - 1) {
            d[k - 1] = a[u][m];
            sd[k - 1] = a[u][m];
          }
      }
    if (c == 0) tau[k - 1] = 0.0;
  }
  __syncthreads();
  tri_bounds_block(sd, se, k, e2, bounds, pb);  // pb (KM >= 4 NW doubles) is free by now
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

// Sturm counts (eigenvalues of the tridiagonal (d, e) strictly below x) at
// two shifts x1 < x2 at once (two independent recurrences interleaved, so
// each hides the other's latency).  1/q comes from the
// hardware reciprocal refined by one Newton step; the count only needs the
// signs of q, which such a perturbation (a relative change of a few ulps of
// the pivots, i.e. of d) leaves as correct as the exact division.
__device__ inline double rcp_f64(double q) {
#if defined(__HIP_DEVICE_COMPILE__)
  double r = __builtin_amdgcn_rcp(q);
  const double e = fma(-q, r, 1.0);
  return fma(r, e, r);
#else
  return 1.0 / q;
#endif
}

__device__ inline void sturm_count2(const double* __restrict__ d, const double* __restrict__ e2, int k,
                                    double x1, double x2, double pivmin, int& c1, int& c2) {
  double q1 = d[0] - x1, q2 = d[0] - x2;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  if (fabs(q2) < pivmin) q2 = -pivmin;
  int n1 = (q1 < 0.0), n2 = (q2 < 0.0);
#pragma unroll 4
  for (int i = 1; i < k; ++i) {
    const double di = d[i], ei = e2[i - 1];
    q1 = (di - x1) - ei * rcp_f64(q1);
    q2 = (di - x2) - ei * rcp_f64(q2);
    if (fabs(q1) < pivmin) q1 = -pivmin;
    if (fabs(q2) < pivmin) q2 = -pivmin;
    n1 += (q1 < 0.0);
    n2 += (q2 < 0.0);
  }
  c1 = n1;
  c2 = n2;
}

// Eigenvalue i (ascending) by multisection on the Sturm count: workgroup i
// (four waves) evaluates the count at 511 interior points of its interval (two
// per lane, p = t + 1 and t + 257 for thread t; p = 512 is hi) and keeps the
// sub-interval where the count passes i, so each round shrinks the interval
// 512-fold (four waves gain 9 bits a round where one gains 7, for the same
// Sturm-count work per wave).  Each wave's first point above the index goes
// through LDS and one barrier.  Stops at the width the reduction determines the
// eigenvalue to.  d and e2 are read with scalar loads (the same entry for
// every lane of a wave).
constexpr int kBisWaves = 4;
__global__ __launch_bounds__(64 * kBisWaves) void bisect_wg_kernel(const double* __restrict__ d,
                                                                   const double* __restrict__ e2, int k,
                                                                   const double* __restrict__ bounds,
                                                                   double* lam) {
  constexpr int P = 128 * kBisWaves;  // points per round
  __shared__ int first[2][2][kBisWaves];  // [round parity][half][wave]: first point above, or P
  const int i = blockIdx.x;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  double lo = bounds[0], hi = bounds[1];
  const double pivmin = bounds[2];
  const double atol = DBL_EPSILON * bounds[3] + 2.0 * DBL_MIN;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + atol) break;
    const double h = (hi - lo) / (double)P;
    const double x1 = lo + h * (double)(t + 1);
    const double x2 = (t < P / 2 - 1) ? lo + h * (double)(t + P / 2 + 1) : hi;
    int c1, c2;
    sturm_count2(d, e2, k, x1, x2, pivmin, c1, c2);
    const uint64_t m1 = __ballot(c1 > i);
    const uint64_t m2 = __ballot((t == P / 2 - 1) || c2 > i);  // hi is always above
    const int par = it & 1;
    if (lane == 0) {
      first[par][0][w] = (m1 != 0) ? 64 * w + __ffsll((unsigned long long)m1) - 1 : P;
      first[par][1][w] = (m2 != 0) ? P / 2 + 64 * w + __ffsll((unsigned long long)m2) - 1 : P;
    }
    __syncthreads();
    int f = P;
    for (int q = 0; q < kBisWaves; ++q) f = min(f, first[par][0][q]);
    if (f == P)
      for (int q = 0; q < kBisWaves; ++q) f = min(f, first[par][1][q]);
    // f: first point above (0-based), the same in every thread
    const double nlo = (f == 0) ? lo : lo + h * (double)f;
    const double nhi = (f == P - 1) ? hi : lo + h * (double)(f + 1);
    if (!(nhi - nlo < hi - lo)) break;  // no progress in floating point (uniform)
    lo = nlo;
    hi = nhi;
  }
  if (t == 0) lam[i] = 0.5 * (lo + hi);
}

// Selection, by one block of kSelT threads.  Outputs:
//   order[c]  : ascending index of the c-th kept eigenvalue, kept ones ordered
//               by |lambda| descending, ties by ascending index (so negatives
//               come first)
//   pos_of[i] : output column of eigenvalue i, -1 when not kept
//   lam_out   : kept eigenvalues (in that order), then the rest ascending
//   clusters  : (start, len) runs in ascending order over kept eigenvalues
//               with consecutive gaps <= kOrtol ||T||;
//               cl_count[0] = number of clusters
//   keep[0]   : kept count (capped at max_keep, flag |= 2 when capped)
//   cl_of[c]  : cluster of kept column c (c < ncol) when it has two or more
//               members, else -1; cl_fail[0 .. ncol) cleared
// The counts that place the unkept eigenvalues and the clusters come from
// block-wide prefix sums over contiguous chunks of the index range.
constexpr int kSelT = 1024;
constexpr int kSelLds = 4096;  // eigenvalues staged in LDS up to this k

__device__ inline int block_scan_incl(int v, int* sh) {
  // inclusive prefix sum of v over the block: within each wave by lane
  // shifts, then over the wave totals (two barriers)
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  int before = 0;
  for (int q = 0; q < w; ++q) before += sh[q];
  __syncthreads();  // sh is reused by the next scan
  return x + before;
}

__global__ __launch_bounds__(kSelT) void select_kernel(const double* lam, int k, double tol,
                                                       int64_t max_keep, const double* bounds,
                                                       int* order, int* pos_of, double* lam_out,
                                                       int* clusters, int* cl_count, int64_t* keep,
                                                       int* flag, int ncol, int* cl_of, int* cl_fail) {
  __shared__ int sh[kSelT];
  __shared__ double slam[kSelLds];  // the eigenvalues, for the O(k) rank loops
  const int t = threadIdx.x;
  for (int c = t; c < ncol; c += kSelT) {  // cluster of each kept column: none yet
    cl_of[c] = -1;
    cl_fail[c] = 0;
  }
  const bool staged = k <= kSelLds;
  if (staged)
    for (int j = t; j < k; j += kSelT) slam[j] = lam[j];
  __syncthreads();
  const double* lamv = staged ? (const double*)slam : lam;
  // eigenvalues are known to about u ||T||; a zero matrix has no nonzero ones
  const double nrmT = bounds[3];
  double amax = 0.0;
  if (k > 0 && nrmT > 0.0) amax = fmax(fabs(lam[0]), fabs(lam[k - 1]));
  const double thr = tol * amax;
  const bool any = amax > 0.0;
  // contiguous chunk of indices of this thread
  const int per = (k + kSelT - 1) / kSelT;
  const int i0 = min(k, t * per), i1 = min(k, i0 + per);
  int cnt = 0;
  for (int i = i0; i < i1; ++i) cnt += (any && fabs(lam[i]) > thr) ? 1 : 0;
  const int nkept = block_scan_incl(cnt, sh);
  __shared__ int tot_kept;
  if (t == kSelT - 1) tot_kept = nkept;
  __syncthreads();
  const int kept = tot_kept;
  const int cap = (int)min<int64_t>(kept, max_keep);
  if (t == 0 && kept > max_keep) atomicOr(flag, 2);
  // rank of every kept eigenvalue (every |lambda_j| >= |lambda_i| is kept too)
  for (int i = i0; i < i1; ++i) {
    int pos = -1;
    const double a = fabs(lam[i]);
    if (any && a > thr) {
      int rk = 0;
      for (int j = 0; j < k; ++j) {
        const double b = fabs(lamv[j]);
        rk += (b > a || (b == a && j < i)) ? 1 : 0;
      }
      if (rk < cap) {
        pos = rk;
        order[rk] = i;
        lam_out[rk] = lam[i];
      }
    }
    pos_of[i] = pos;
  }
  __syncthreads();  // pos_of (global) visible to the block
  // the unkept ones, ascending, after the kept ones
  int un = 0;
  for (int i = i0; i < i1; ++i) un += (pos_of[i] < 0) ? 1 : 0;
  int o = cap + block_scan_incl(un, sh) - un;
  for (int i = i0; i < i1; ++i)
    if (pos_of[i] < 0) lam_out[o++] = lam[i];
  // clusters: a run starts at a kept eigenvalue whose lower neighbour is not
  // kept or lies more than kOrtol ||T|| below
  auto starts = [&](int i) {
    return pos_of[i] >= 0 && (i == 0 || pos_of[i - 1] < 0 || lam[i] - lam[i - 1] > kOrtol * nrmT);
  };
  // ... and ends at a kept eigenvalue whose upper neighbour starts a run or
  // is not kept; a run's id is the number of starts up to it, minus one
  auto ends = [&](int i) { return pos_of[i] >= 0 && (i + 1 == k || pos_of[i + 1] < 0 || starts(i + 1)); };
  int ns = 0;
  for (int i = i0; i < i1; ++i) ns += starts(i) ? 1 : 0;
  const int incl = block_scan_incl(ns, sh);
  int id = incl - ns;  // runs started before this chunk
  for (int i = i0; i < i1; ++i) {
    if (starts(i)) clusters[2 * id++] = i;
    if (ends(i)) clusters[2 * (id - 1) + 1] = i;  // the end index for now
  }
  __shared__ int tot_runs;
  if (t == kSelT - 1) tot_runs = incl;
  __syncthreads();  // every run's start and end are written, and the run count is known
  const int runs = tot_runs;
  for (int q = t; q < runs; q += kSelT) clusters[2 * q + 1] = clusters[2 * q + 1] - clusters[2 * q] + 1;
  if (t == kSelT - 1) {
    cl_count[0] = runs;
    keep[0] = cap;
  }
  __syncthreads();  // run lengths final
  // cl_of[col] = run of kept column col when the run has two or more members
  id = incl - ns;
  for (int i = i0; i < i1; ++i) {
    if (starts(i)) ++id;
    if (pos_of[i] >= 0 && pos_of[i] < ncol && clusters[2 * (id - 1) + 1] >= 2) cl_of[pos_of[i]] = id - 1;
  }
}

// Deterministic start vector in (-1, 1).
__device__ inline double start_entry(int idx, int i) {
  uint32_t h = (uint32_t)(idx * 0x9E3779B9u) ^ (uint32_t)(i * 0x85EBCA6Bu) ^ 0x27D4EB2Fu;
  h ^= h >> 15; h *= 0x2C1B3C6Du; h ^= h >> 12; h *= 0x297A2D39u; h ^= h >> 15;
  return ((double)(h & 0xFFFFFF) / (double)0x1000000) * 2.0 - 1.0;
}

// Inverse iteration for kept eigenvalue number `blockIdx.x` (ascending index
// idx, output column pos_of[idx]), one wave per eigenvalue.  The tridiagonal
// LU with partial pivoting and the solves are sequential (lane 0); their
// recurrences carry their state in registers and read only the arrays that do
// not depend on it, and the pivots are stored as reciprocals, so the critical
// path is a few floating-point operations per row.  Eigenvalues inside one
// cluster get shifts nudged apart by a few ulps of ||T|| and distinct start
// vectors, so their iterates differ.  Z is column-major: Z[i + c * ldz] is
// entry i of output column c.
template <bool LDS>
__global__ __launch_bounds__(64) void invit_kernel(const double* d, const double* e, int k,
                                                   const double* lam, const int* order,
                                                   const int64_t* keep, const double* bounds,
                                                   double* work, double* Z, int64_t ldz,
                                                   int ties_only) {
  const int c = blockIdx.x;
  if (c >= keep[0]) {  // unused column: zero (the polar step multiplies it by 0)
    if (!ties_only)
      for (int i = threadIdx.x; i < k; i += 64) Z[i + (int64_t)c * ldz] = 0.0;
    return;
  }
  const int idx = order[c];
  const int lane = threadIdx.x;
  extern __shared__ double ism[];
  __shared__ double sscale;
  if (ties_only && !(idx > 0 && lam[idx] - lam[idx - 1] <= 4.0 * DBL_EPSILON * bounds[3])) return;
  // keep the arrays in LDS when they fit (a compile-time choice, so that
  // every access has a known address space)
  double* dd;
  if constexpr (LDS) dd = ism;
  else dd = work + (int64_t)c * kInvitArrays * k;
  double* ee = dd + k;   // e (0 past the end)
  double* u1 = ee + k;   // first super-diagonal of U
  double* u2 = u1 + k;   // second super-diagonal of U
  double* lm = u2 + k;   // multipliers
  double* rp = lm + k;   // 1 / pivots
  double* x = rp + k;    // iterate
  double* swd = x + k;   // row swap flags (0 or 1)
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
  for (int i = lane; i < k; i += 64) {
    dd[i] = d[i] - lamq;
    ee[i] = (i + 1 < k) ? e[i] : 0.0;
    x[i] = start_entry(idx, i);
  }
  __syncthreads();
  if (lane == 0) {
    // LU with partial pivoting of T - lamq I: rows i, i+1 may swap.  After
    // elimination row i holds the pivot, u1[i], u2[i].
    // (each loop loads the next row's operands before it works on this one)
    double a = dd[0];
    double b = (k > 1) ? ee[0] : 0.0;
    double sub_n = ee[0], dn_n = (k > 1) ? dd[1] : 0.0, sn_n = (k > 1) ? ee[1] : 0.0;
    for (int i = 0; i + 1 < k; ++i) {
      const double sub = sub_n, dn = dn_n, sn = sn_n;
      if (i + 2 < k) {
        sub_n = ee[i + 1];
        dn_n = dd[i + 2];
        sn_n = ee[i + 2];
      }
      double piv, mlt, na, nb, w1, w2, sw;
      if (fabs(a) >= fabs(sub)) {
        piv = (a == 0.0) ? small : a;
        mlt = sub / piv;
        w1 = b; w2 = 0.0; sw = 0.0;
        na = dn - mlt * b;
        nb = sn;
      } else {
        piv = sub;
        mlt = a / sub;
        w1 = dn; w2 = sn; sw = 1.0;
        na = b - mlt * dn;
        nb = -mlt * sn;
      }
      const double pv = (fabs(piv) < small) ? copysign(small, piv) : piv;
      rp[i] = 1.0 / pv;
      u1[i] = w1; u2[i] = w2; lm[i] = mlt; swd[i] = sw;
      a = na;
      b = nb;
    }
    {
      const double piv = (a == 0.0) ? small : a;
      const double pv = (fabs(piv) < small) ? copysign(small, piv) : piv;
      rp[k - 1] = 1.0 / pv;
      u1[k - 1] = 0.0; u2[k - 1] = 0.0;
    }
  }
  __syncthreads();
  for (int it = 0; it < kInvitIters; ++it) {
    if (lane == 0) {
      // forward: apply the row swaps and multipliers; (xa, xb) = rows i, i+1
      double xa = x[0];
      double xb_n = (k > 1) ? x[1] : 0.0, sw_n = swd[0], lm_n = lm[0];
      for (int i = 0; i + 1 < k; ++i) {
        double xb = xb_n;
        const double swv = sw_n, lmv = lm_n;
        if (i + 2 < k) {
          xb_n = x[i + 2];
          sw_n = swd[i + 1];
          lm_n = lm[i + 1];
        }
        if (swv != 0.0) { const double tmp = xa; xa = xb; xb = tmp; }
        xb -= lmv * xa;
        x[i] = xa;
        xa = xb;
      }
      x[k - 1] = xa;
      // backward: (x1, x2) = solved rows i + 1, i + 2
      double x1 = 0.0, x2 = 0.0, mx = 0.0;
      double xi_n = x[k - 1], a1_n = u1[k - 1], a2_n = u2[k - 1], r_n = rp[k - 1];
      for (int i = k - 1; i >= 0; --i) {
        const double xi = xi_n, a1 = a1_n, a2 = a2_n, ri = r_n;
        if (i > 0) {
          xi_n = x[i - 1];
          a1_n = u1[i - 1];
          a2_n = u2[i - 1];
          r_n = rp[i - 1];
        }
        const double v = (xi - a1 * x1 - a2 * x2) * ri;
        x[i] = v;
        mx = fmax(mx, fabs(v));
        x2 = x1;
        x1 = v;
      }
      sscale = (mx > 0.0) ? 1.0 / mx : 1.0;
    }
    __syncthreads();
    const double sc = sscale;
    for (int i = lane; i < k; i += 64) x[i] *= sc;
    __syncthreads();
  }
  double part = 0.0;
  for (int i = lane; i < k; i += 64) part += x[i] * x[i];
  part = wave_sum_f64(part);
  const double inv = (part > 0.0) ? 1.0 / sqrt(part) : 0.0;
  for (int i = lane; i < k; i += 64) Z[i + (int64_t)c * ldz] = x[i] * inv;
}

// Eigenvector of T for kept eigenvalue number `blockIdx.x` from a twisted
// factorisation (Fernando 1997; Parlett & Dhillon 1997), one wave per
// eigenvalue.  With the shift lam:
//   dp_0 = d_0 - lam,          dp_i = (d_i - lam) - e_{i-1}^2 / dp_{i-1}
//   dm_{k-1} = d_{k-1} - lam,  dm_i = (d_i - lam) - e_i^2 / dm_{i+1}
//   gamma_i = dp_i + dm_i - (d_i - lam)
// (T - lam I = N_r diag(..., gamma_r, ...) N_r^T twisted at r), and with
// r = argmin |gamma_i|: z_r = 1, z_i = -e_i z_{i+1} / dp_i below the twist,
// z_i = -e_{i-1} z_{i-1} / dm_i above it.  Two sweeps down and up instead of
// a factorisation and repeated solves.  d - lam and e are staged in LDS; the
// sweeps are scalar recurrences that every lane of a wave runs alike, reading
// the current row's values by LDS broadcast (independent of the recurrence,
// so they are read ahead) and leaving their results (1 / dp, 1 / dm, the two
// parts of gamma, z) in LDS by lane 0.  Pivots below eps ||T|| in magnitude
// are replaced by +-eps ||T||, as in the LU of the inverse iteration.  Tied
// eigenvalues (within 4 ulps of ||T|| of the previous one) are left to the
// inverse iteration, whose distinct start vectors separate them.
template <int NS>
__global__ __launch_bounds__(128) void twist_kernel(const double* __restrict__ d, const double* __restrict__ e,
                                                    int k, const double* __restrict__ lam,
                                                    const int* __restrict__ order,
                                                    const int64_t* __restrict__ keep,
                                                    const double* __restrict__ bounds, double* Z,
                                                    int64_t ldz) {
  // wave 0 runs the forward sweep and then z below the twist, wave 1 the
  // backward sweep and then z above it
  constexpr int KM = 64 * NS;
  __shared__ double dn[KM];   // d_i - lam
  __shared__ double en[KM];   // e_i (0 past the last coupling)
  __shared__ double rf[KM];   // 1 / dp_i (wave 0)
  __shared__ double rb[KM];   // 1 / dm_i (wave 1)
  __shared__ double gsh[KM];  // dp_i - (d_i - lam) (wave 0)
  __shared__ double dsh[KM];  // dm_i (wave 1)
  __shared__ double zs[KM];   // z
  __shared__ double part2[2];
  __shared__ double spow[2];
  __shared__ int rsh;
  const int c = blockIdx.x;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (c >= keep[0]) {  // unused column: zero (the polar step multiplies it by 0)
    for (int i = threadIdx.x; i < k; i += 128) Z[i + (int64_t)c * ldz] = 0.0;
    return;
  }
  const int idx = order[c];
  const double nrmT = bounds[3];
  const double small = DBL_EPSILON * fmax(nrmT, DBL_MIN);
  if (idx > 0 && lam[idx] - lam[idx - 1] <= 4.0 * DBL_EPSILON * nrmT) return;  // a tie
  const double lamq = lam[idx];
  for (int i = threadIdx.x; i < KM; i += 128) {
    dn[i] = (i < k) ? d[i] - lamq : 0.0;
    en[i] = (i + 1 < k) ? e[i] : 0.0;
  }
  __syncthreads();
  auto guard = [&](double p) { return (fabs(p) < small) ? copysign(small, p) : p; };
  // The sweeps take the rows in blocks of kTwB: a block's inputs are read from
  // LDS one block ahead (LDS latency off the recurrence) and its results are
  // gathered into lanes 0 .. kTwB - 1 and stored once per block.
  constexpr int kTwB = 8;
  auto put = [&](double acc, double v, int u) { return (lane == u) ? v : acc; };  // lane u takes v
  if (w == 0) {
    // forward: dp (kept as 1 / dp) and the gamma part dp_i - (d_i - lam)
    double ep = 0.0, rprev = 0.0;
    double dA[kTwB], eA[kTwB];
#pragma unroll
    for (int u = 0; u < kTwB; ++u) {
      dA[u] = dn[u];
      eA[u] = en[u];
    }
    for (int i0 = 0; i0 < k; i0 += kTwB) {
      double dB[kTwB], eB[kTwB];
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        const int ii = min(i0 + kTwB + u, KM - 1);
        dB[u] = dn[ii];
        eB[u] = en[ii];
      }
      double rr = 0.0, gg = 0.0;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        if (i0 + u < k) {  // uniform
          const double di = dA[u];
          const double p = guard(di - ep * ep * rprev);
          const double r = rcp_f64(p);
          rr = put(rr, r, u);
          gg = put(gg, p - di, u);
          ep = eA[u];
          rprev = r;
        }
      }
      if (lane < kTwB && i0 + lane < k) {
        rf[i0 + lane] = rr;
        gsh[i0 + lane] = gg;
      }
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        dA[u] = dB[u];
        eA[u] = eB[u];
      }
    }
  } else {
    // backward: dm (kept as 1 / dm); blocks from the top
    double rprev = 0.0;
    const int top = k - 1;
    double dA[kTwB], eA[kTwB];
#pragma unroll
    for (int u = 0; u < kTwB; ++u) {
      const int ii = max(top - u, 0);
      dA[u] = dn[ii];
      eA[u] = en[ii];
    }
    for (int i0 = top; i0 >= 0; i0 -= kTwB) {
      double dB[kTwB], eB[kTwB];
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        const int ii = max(i0 - kTwB - u, 0);
        dB[u] = dn[ii];
        eB[u] = en[ii];
      }
      double rr = 0.0, pp = 0.0;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        if (i0 - u >= 0) {  // uniform
          const double di = dA[u];
          const double ei = eA[u];  // coupling of rows i and i + 1 (0 for the last)
          const double p = guard(di - ei * ei * rprev);
          const double r = rcp_f64(p);
          rr = put(rr, r, u);
          pp = put(pp, p, u);
          rprev = r;
        }
      }
      if (lane < kTwB && i0 - lane >= 0) {
        rb[i0 - lane] = rr;
        dsh[i0 - lane] = pp;
      }
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        dA[u] = dB[u];
        eA[u] = eB[u];
      }
    }
  }
  __syncthreads();  // both parts of gamma are in LDS
  // twist r = argmin |gamma_i| (lowest i among equals), by wave 1
  if (w == 1) {
    double best = DBL_MAX;
    int bi = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int i = 64 * m + lane;
      const double g = (i < k) ? fabs(gsh[i] + dsh[i]) : DBL_MAX;
      if (i < k && (g < best || (g == best && i < bi))) { best = g; bi = i; }
    }
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob < best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) rsh = bi;
  }
  __syncthreads();
  const int r = rsh;
  // z_r = 1; z below the twist by wave 0 (1 / dp), above by wave 1 (1 / dm);
  // a running rescale keeps the entries in range (the stored part of the
  // sweep is rescaled with it)
  double scale_pow = 0.0;  // number of 1e-150 rescales of this wave's part
  if (w == 0) {
    if (lane == 0) zs[r] = 1.0;
    double zc = 1.0;  // z_{i+1}
    double fA[kTwB], eA[kTwB];
#pragma unroll
    for (int u = 0; u < kTwB; ++u) {
      const int ii = max(r - 1 - u, 0);
      fA[u] = rf[ii];
      eA[u] = en[ii];
    }
    for (int i0 = r - 1; i0 >= 0; i0 -= kTwB) {
      double fB[kTwB], eB[kTwB];
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        const int ii = max(i0 - kTwB - u, 0);
        fB[u] = rf[ii];
        eB[u] = en[ii];
      }
      double zz = 0.0;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        if (i0 - u >= 0) {  // uniform
          zc = -eA[u] * zc * fA[u];
          if (fabs(zc) > 1e150) {  // uniform; the stored part and this block's rescale with it
            for (int q = i0 + 1 + lane; q <= r; q += 64) zs[q] *= 1e-150;
            zz *= 1e-150;
            zc *= 1e-150;
            scale_pow += 1.0;
          }
          zz = put(zz, zc, u);
        }
      }
      if (lane < kTwB && i0 - lane >= 0) zs[i0 - lane] = zz;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        fA[u] = fB[u];
        eA[u] = eB[u];
      }
    }
  } else {
    double zc = 1.0;  // z_{i-1}
    double bA[kTwB], eA[kTwB];
#pragma unroll
    for (int u = 0; u < kTwB; ++u) {
      const int ii = min(r + 1 + u, KM - 1);
      bA[u] = rb[ii];
      eA[u] = en[ii - 1];
    }
    for (int i0 = r + 1; i0 < k; i0 += kTwB) {
      double bB[kTwB], eB[kTwB];
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        const int ii = min(i0 + kTwB + u, KM - 1);
        bB[u] = rb[ii];
        eB[u] = en[ii - 1];
      }
      double zz = 0.0;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        if (i0 + u < k) {  // uniform
          zc = -eA[u] * zc * bA[u];
          if (fabs(zc) > 1e150) {  // uniform
            for (int q = r + 1 + lane; q < i0; q += 64) zs[q] *= 1e-150;
            zz *= 1e-150;
            zc *= 1e-150;
            scale_pow += 1.0;
          }
          zz = put(zz, zc, u);
        }
      }
      if (lane < kTwB && i0 + lane < k) zs[i0 + lane] = zz;
#pragma unroll
      for (int u = 0; u < kTwB; ++u) {
        bA[u] = bB[u];
        eA[u] = eB[u];
      }
    }
  }
  // the two parts share z_r = 1; a part that was rescaled is scaled back
  // relative to the other before the norm
  if (lane == 0) spow[w] = scale_pow;
  __syncthreads();
  const double mine = spow[w], other = spow[1 - w];
  const double rel = (mine >= other) ? 1.0 : pow(1e-150, other - mine);
  double z[NS];
  double sq = 0.0;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int i = 64 * m + lane;
    const bool mine_row = (w == 0) ? (i <= r) : (i > r);
    z[m] = (i < k && mine_row) ? zs[i] * rel : 0.0;
    sq += z[m] * z[m];
  }
  sq = wave_sum_f64(sq);
  if (lane == 0) part2[w] = sq;
  __syncthreads();
  const double tot = part2[0] + part2[1];
  const double inv = (tot > 0.0) ? 1.0 / sqrt(tot) : 0.0;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int i = 64 * m + lane;
    const bool mine_row = (w == 0) ? (i <= r) : (i > r);
    if (i < k && mine_row) Z[i + (int64_t)c * ldz] = z[m] * inv;
  }
}

// Polar (Newton-Schulz) orthonormalisation of the clusters, by GEMMs: with
// G = Z^T Z, Z <- Z B, B = I + (same cluster ? (I - G) / 2 : 0), three times.
// A step takes e = ||Z^T Z - I|| to about (3/4) e^2, so a cluster whose
// vectors are nearly orthonormal (len * max |G - I| below kPolarTol; the
// vectors are off by O(eps ||T|| / gap)) ends below 1e-16 (1e-2, 7.5e-5,
// 4.2e-9, 1.3e-17); the others (cl_fail set) keep their vectors for modified
// Gram-Schmidt.  The polar factor mixes a cluster's vectors least.
constexpr double kPolarTol = 1e-2;
constexpr int kPolarSteps = 3;

// The products of a polar step on FP64 MFMA, one 16 x 16 tile of the result
// a workgroup, the inner dimension over its four waves (as the small GEMMs):
//   kPolarGram:  G = Z^T Z (ncol x ncol, Z k x ncol), and on the first step
//                (check) cl_fail[c] |= 1 for a cluster c with an entry of
//                len * |G - I| not below kPolarTol;
//   kPolarApply: Zo = Z B, B = I + (i, j in one cluster that passed ?
//                (I - G) / 2 : 0), B formed from G as it is read.
typedef double pv4d __attribute__((ext_vector_type(4)));
constexpr int kPolarGram = 0, kPolarApply = 1;
template <int MODE>
__global__ __launch_bounds__(256) void polar_gemm_kernel(int k, int ncol, const double* __restrict__ Z,
                                                         const double* __restrict__ G, const int* cl_of,
                                                         const int* clusters, int* cl_fail, bool check,
                                                         double* __restrict__ out) {
  __shared__ pv4d red[3][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int M = (MODE == kPolarGram) ? ncol : k;  // rows of the result
  const int K = (MODE == kPolarGram) ? k : ncol;  // inner dimension
  const int m = blockIdx.x * 16 + r16, n = blockIdx.y * 16 + r16;
  const bool min_ = m < M, nin = n < ncol;
  const int cn = nin ? cl_of[n] : -1;
  const bool nlive = (MODE == kPolarApply) && cn >= 0 && !cl_fail[cn];
  auto opA = [&](int q) -> double {  // (m, q) of Z^T or of Z
    if (!min_ || q >= K) return 0.0;
    return (MODE == kPolarGram) ? Z[q + (int64_t)m * k] : Z[m + (int64_t)q * k];
  };
  auto opB = [&](int q) -> double {  // (q, n) of Z or of B
    if (!nin || q >= K) return 0.0;
    if (MODE == kPolarGram) return Z[q + (int64_t)n * k];
    const double dl = (q == n) ? 1.0 : 0.0;
    return (nlive && cl_of[q] == cn) ? dl + 0.5 * (dl - G[q + (int64_t)n * ncol]) : dl;
  };
  pv4d acc = pv4d{0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  for (int k0 = 4 * wave; k0 < K; k0 += 16 * U) {
    double fa[U], fb[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int q = k0 + 16 * u + kq;
      fa[u] = opB(q);
      fb[u] = opA(q);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[u], acc, 0, 0, 0);
  }
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w) acc += red[w][lane];
    const int cm = (MODE == kPolarGram && check && min_) ? cl_of[m] : -1;
    bool bad = false;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nn = blockIdx.y * 16 + v * 4 + kq;
      if (min_ && nn < ncol) {
        out[m + (int64_t)nn * M] = acc[v];
        if (cm >= 0 && cl_of[nn] == cm) {
          const double dev = fabs(acc[v] - (m == nn ? 1.0 : 0.0));
          if (!(dev * clusters[2 * cm + 1] < kPolarTol)) bad = true;
        }
      }
    }
    if (bad) atomicOr(&cl_fail[cm], 1);
  }
}

// Orthonormalise the vectors of one cluster (blockIdx.x), in ascending
// eigenvalue order, by right-looking modified Gram-Schmidt done twice: at
// step j every later vector loses its component along z_j.  The later vectors
// are spread over the 32 half-waves of the block (a half-wave sums its dot
// products with lane moves only), the half-wave that updates z_{j+1} also
// forms its new squared norm for the next step, so a step needs one barrier.
// The cluster is staged in LDS when it fits (lds_doubles entries of dynamic
// shared memory); the two cases are separate instantiations so that every
// access has a known address space.
template <bool STAGED>
__device__ void orth_cluster(int k, int start, int len, const int* pos_of, double* Z, int64_t ldz,
                             double* zs, double* nrm) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
  const int hw = 2 * wv + (lane >> 5), hl = lane & 31;  // half-wave index, lane in it
  const int nhw = 2 * nw;
  // vector q of the cluster: zs[q * k + i] when staged, else Z column pos_of[start + q]
  auto vec = [&](int q) -> double* {
    if constexpr (STAGED) return zs + (int64_t)q * k;
    else return Z + (int64_t)pos_of[start + q] * ldz;
  };
  if constexpr (STAGED) {
    for (int q = wv; q < len; q += nw) {
      const double* src = Z + (int64_t)pos_of[start + q] * ldz;
      for (int i = lane; i < k; i += 64) zs[(int64_t)q * k + i] = src[i];
    }
    __syncthreads();
  }
  for (int pass = 0; pass < 2; ++pass) {
    if (wv == 0) {
      const double* z0 = vec(0);
      double n0 = 0.0;
      for (int i = lane; i < k; i += 64) n0 += z0[i] * z0[i];
      n0 = wave_sum_f64(n0);
      if (lane == 0) nrm[0] = n0;
    }
    __syncthreads();
    for (int j = 0; j < len; ++j) {
      const double* zj = vec(j);
      const double nj = nrm[j & 1];
      const double inv2 = (nj > 0.0) ? 1.0 / nj : 0.0;
      for (int l = j + 1 + hw; l < len; l += nhw) {
        double* zl = vec(l);
        double dt = 0.0;
        for (int i = hl; i < k; i += 32) dt += zj[i] * zl[i];
        dt = half_wave_sum_f64(dt);
        const double f = dt * inv2;
        double nn = 0.0;
        for (int i = hl; i < k; i += 32) {
          const double v = zl[i] - f * zj[i];
          zl[i] = v;
          nn += v * v;
        }
        if (l == j + 1) {
          nn = half_wave_sum_f64(nn);
          if (hl == 0) nrm[(j + 1) & 1] = nn;
        }
      }
      __syncthreads();
    }
    // normalise every vector of the cluster
    for (int j = wv; j < len; j += nw) {
      double* zj = vec(j);
      double nj = 0.0;
      for (int i = lane; i < k; i += 64) nj += zj[i] * zj[i];
      nj = wave_sum_f64(nj);
      const double inv = (nj > 0.0) ? 1.0 / sqrt(nj) : 0.0;
      for (int i = lane; i < k; i += 64) zj[i] *= inv;
    }
    __syncthreads();
  }
  if constexpr (STAGED) {
    for (int q = wv; q < len; q += nw) {
      double* dst = Z + (int64_t)pos_of[start + q] * ldz;
      for (int i = lane; i < k; i += 64) dst[i] = zs[(int64_t)q * k + i];
    }
  }
}

__global__ __launch_bounds__(1024) void orth_kernel(int k, const int* clusters, const int* cl_count,
                                                    const int* pos_of, const int* cl_fail, double* Z,
                                                    int64_t ldz, int lds_doubles) {
  extern __shared__ double zs[];
  __shared__ double nrm[2];  // squared norm of the pivot of step j in nrm[j & 1]
  const int cl = blockIdx.x;
  if (cl >= cl_count[0]) return;
  const int start = clusters[2 * cl], len = clusters[2 * cl + 1];
  if (len < 2 || !cl_fail[cl]) return;
  if ((int64_t)len * k <= (int64_t)lds_doubles) orth_cluster<true>(k, start, len, pos_of, Z, ldz, zs, nrm);
  else orth_cluster<false>(k, start, len, pos_of, Z, ldz, zs, nrm);
}

// V(:, c) = H_0 H_1 ... H_{k-3} z_c, with z_c = Z[i + c * ldz]; one wave per
// column (kBtCols columns per block).  With LDS the block stages each
// chunk of kBtChunk reflectors (with the implicit unit entry) and z in LDS,
// so the reflectors are read from HBM once per block and every wave applies
// them with wave reductions only; otherwise z stays in its output column and
// the reflectors are read from A.  (Z == nullptr stands for I, which forms Q.)
constexpr int kBtCols = 4;
constexpr int kBtChunk = 16;
constexpr int kBtLdsMaxK = 960;  // LDS staging up to this k (20 k doubles)

template <bool LDS>
__global__ __launch_bounds__(64 * kBtCols) void backtr_kernel(const double* A, int64_t lda,
                                                              const double* tau, int k,
                                                              const double* Z, int64_t ldz,
                                                              const int64_t* keep, int ncols,
                                                              double* V, int64_t ldv) {
  constexpr bool use_lds = LDS;
  extern __shared__ double bsh[];  // z of the block's columns, then a chunk of reflectors
  __shared__ double tch[kBtChunk];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = blockIdx.x * kBtCols + wv;
  // columns: ncols, or keep[0] when ncols < 0; Z == nullptr stands for I
  const bool active = c < (ncols >= 0 ? (int64_t)ncols : keep[0]);  // wave-uniform; no early return
  double* z;
  if constexpr (LDS) z = bsh + (int64_t)wv * k;
  else z = V + (int64_t)c * ldv;
  double* vch = bsh + (int64_t)kBtCols * k;
  if (active)
    for (int i = lane; i < k; i += 64) z[i] = Z ? Z[i + (int64_t)c * ldz] : (i == c ? 1.0 : 0.0);
  for (int jhi = k - 3; jhi >= 0; jhi -= kBtChunk) {
    const int jlo = max(0, jhi - kBtChunk + 1);
    if (use_lds) {
      __syncthreads();  // the previous chunk is consumed
      const int nj = jhi - jlo + 1;
      for (int idx = threadIdx.x; idx < nj * k; idx += blockDim.x) {
        const int jj = idx / k, i = idx % k;
        const int j = jlo + jj;
        const double v = A[i + (int64_t)j * lda];  // unconditional load, masked below
        vch[idx] = (i == j + 1) ? 1.0 : ((i > j + 1) ? v : 0.0);
      }
      if ((int)threadIdx.x < nj) tch[threadIdx.x] = tau[jlo + threadIdx.x];
      __syncthreads();
    }
    if (!active) continue;
    for (int j = jhi; j >= jlo; --j) {
      const double tj = use_lds ? tch[j - jlo] : tau[j];
      if (tj == 0.0) continue;
      const int r0 = j + 1;
      double part = 0.0;
      if (use_lds) {
        const double* vj = vch + (int64_t)(j - jlo) * k;
        for (int i = r0 + lane; i < k; i += 64) part += vj[i] * z[i];
        part = wave_sum_f64(part);
        const double s = tj * part;
        for (int i = r0 + lane; i < k; i += 64) z[i] -= s * vj[i];
      } else {
        const double* vj = A + (int64_t)j * lda;
        for (int i = r0 + lane; i < k; i += 64) part += ((i == r0) ? 1.0 : vj[i]) * z[i];
        part = wave_sum_f64(part);
        const double s = tj * part;
        for (int i = r0 + lane; i < k; i += 64) z[i] -= s * ((i == r0) ? 1.0 : vj[i]);
      }
    }
  }
  if (!active) return;
  for (int i = lane; i < k; i += 64) V[i + (int64_t)c * ldv] = z[i];
}

// Sign convention of the eigenvectors: in each column c < keep[0] of V the
// largest |entry| is positive (the first one on ties).  One wave per column.
__global__ __launch_bounds__(64) void sign_columns_kernel(double* V, int64_t ldv, int k, const int64_t* keep) {
  const int c = blockIdx.x, lane = threadIdx.x;
  if (c >= keep[0]) return;
  double* z = V + (int64_t)c * ldv;
  double best = -1.0;
  int bi = k;
  for (int i = lane; i < k; i += 64) {
    const double a = fabs(z[i]);
    if (a > best) { best = a; bi = i; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if (bi < k && z[bi] < 0.0)
    for (int i = lane; i < k; i += 64) z[i] = -z[i];
}

}  // namespace

size_t syev_workspace(int64_t k) {
  size_t b = 0;
  b += (size_t)k * k * sizeof(double) + 256;      // A copy
  b += 8 * ((size_t)k * sizeof(double) + 256);    // d, e, tau, p, w, e2, lam, bounds
  b += 4 * ((size_t)k * sizeof(int) + 256);       // order, pos_of, clusters(2k), count
  b += (size_t)k * 2 * sizeof(int) + 256;
  b += (size_t)k * kInvitArrays * k * sizeof(double) + 256;  // inverse-iteration arrays
  b += (size_t)k * k * sizeof(double) + 256;      // Zt
  b += 2 * ((size_t)k * k * sizeof(double) + 256);  // polar steps: G, Z1
  b += 2 * ((size_t)k * sizeof(int) + 256);          // cl_of, cl_fail
  b += gemm_f64_workspace(k, k, k);
  b += (size_t)k * k * sizeof(double) + 256;      // Q
  return b;
}

void syev_trunc_f64(hipStream_t s, int64_t k, const double* M, int64_t ldm, double tol,
                    int64_t max_keep, double* lam_out, double* V_out, int64_t ldv,
                    int64_t* keep_dev, int* flag_dev, Arena& ws, const SyevPost& post) {
  DME_REQUIRE(k >= 0 && k <= 16384, DME_EINVAL, "syev: k out of range");
  if (k == 0) {
    fill_f64(s, reinterpret_cast<double*>(keep_dev), 1, 1, 1, 0.0);  // all-zero bits
    if (post.rank_seq) *post.rank_seq = value_to_host_launch(s, keep_dev, post.rank_veto);
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
  double* work = ws.get<double>((size_t)k * kInvitArrays * k);
  double* Zt = ws.get<double>((size_t)k * k);

  const bool tiles = k >= 2 && k <= 192;  // the register-tiled reduction reads M itself
  if (!tiles) copy_f64(s, M, ldm, A, k, k, k);
  if (k == 1) {
    // trivial: d = M(0,0)
    copy_f64(s, A, 1, d, 1, 1, 1);
    fill_f64(s, e, 1, 1, 1, 0.0);
    fill_f64(s, tau, 1, 1, 1, 0.0);
  } else {
    if (k <= 64) {
      hipLaunchKernelGGL((tridiag_tiles_kernel<2, 8>), dim3(1), dim3(256), 0, s, M, ldm, A, k, ki, d, e, tau,
                         e2, bounds);
    } else if (k <= 128) {
      hipLaunchKernelGGL((tridiag_tiles_kernel<4, 8>), dim3(1), dim3(512), 0, s, M, ldm, A, k, ki, d, e, tau,
                         e2, bounds);
    } else if (k <= 160) {
      hipLaunchKernelGGL((tridiag_tiles_kernel<5, 8>), dim3(1), dim3(640), 0, s, M, ldm, A, k, ki, d, e, tau,
                         e2, bounds);
    } else if (k <= 192) {
      hipLaunchKernelGGL((tridiag_tiles_kernel<6, 12>), dim3(1), dim3(512), 0, s, M, ldm, A, k, ki, d, e, tau,
                         e2, bounds);
    } else if (k <= kTriMaxK) {
      const size_t lds = (size_t)(3 + kTriT / 64) * k * sizeof(double);
      hipLaunchKernelGGL(tridiag_small_kernel, dim3(1), dim3(kTriT), lds, s, A, k, ki, d, e, tau);
    } else {
      hipLaunchKernelGGL(tridiag_kernel, dim3(1), dim3(kTriT), 0, s, A, k, ki, d, e, tau, pw);
    }
    DME_HIP(hipGetLastError());
  }
  // Q = H_0 ... H_{k-3} (the tridiagonalisation's reflectors applied to I) on
  // the second stream, beside the eigenvalue and eigenvector work below
  double* Qm = ws.get<double>((size_t)k * k);
  AuxStream& ax = aux_stream();
  DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
  {
    const dim3 bt_grid((unsigned)cdiv(k, kBtCols));
    if (k <= kBtLdsMaxK)
      hipLaunchKernelGGL(backtr_kernel<true>, bt_grid, dim3(64 * kBtCols),
                         (size_t)(kBtCols + kBtChunk) * k * sizeof(double), ax.s2, A, k, tau, ki,
                         (const double*)nullptr, k, keep_dev, ki, Qm, k);
    else
      hipLaunchKernelGGL(backtr_kernel<false>, bt_grid, dim3(64 * kBtCols), 0, ax.s2, A, k, tau, ki,
                         (const double*)nullptr, k, keep_dev, ki, Qm, k);
    DME_HIP(hipGetLastError());
  }
  const hipEvent_t q_done = ax.record(ax.s2);
  if (k == 1 || k > 192) {  // the register-tiled reductions leave e2 and the bounds themselves
    hipLaunchKernelGGL(tri_prep_kernel, dim3(1), dim3(256), 0, s, d, e, ki, e2, bounds);
    DME_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(bisect_wg_kernel, dim3((unsigned)k), dim3(64 * kBisWaves), 0, s, d, e2, ki, bounds, lam);
  DME_HIP(hipGetLastError());
  const unsigned nkeep_sel = (unsigned)std::min<int64_t>(k, max_keep);
  int* cl_of = ws.get<int>(k);
  int* cl_fail = ws.get<int>(k);
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelT), 0, s, lam, ki, tol, max_keep, bounds, order,
                     pos_of, lam_out, clusters, cl_count, keep_dev, flag_dev, (int)nkeep_sel, cl_of, cl_fail);
  DME_HIP(hipGetLastError());
  if (post.rank_seq) {  // the kept count to the host from the second stream, beside the vectors
    DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
    *post.rank_seq = value_to_host_launch(ax.s2, keep_dev, post.rank_veto);
  }
  // Z: k x (kept) column-major with ld = k (kept <= k)
  const unsigned nkeep = (unsigned)std::min<int64_t>(k, max_keep);
  // twisted factorisations for k <= 512, inverse iteration for ties (and larger k)
  int ties_only = 1;
  switch (cdiv(k, 64)) {
#define DME_TWIST(NS)                                                                             \
  case NS:                                                                                        \
    hipLaunchKernelGGL(twist_kernel<NS>, dim3(nkeep), dim3(128), 0, s, d, e, ki, lam, order, keep_dev, \
                       bounds, Zt, k);                                                            \
    break;
    DME_TWIST(1) DME_TWIST(2) DME_TWIST(3) DME_TWIST(4) DME_TWIST(5) DME_TWIST(6) DME_TWIST(7)
    DME_TWIST(8)
#undef DME_TWIST
    default: ties_only = 0;
  }
  DME_HIP(hipGetLastError());
  if (k <= kInvitLdsMaxK)
    hipLaunchKernelGGL(invit_kernel<true>, dim3(nkeep), dim3(64), (size_t)kInvitArrays * k * sizeof(double),
                       s, d, e, ki, lam, order, keep_dev, bounds, work, Zt, k, ties_only);
  else
    hipLaunchKernelGGL(invit_kernel<false>, dim3(nkeep), dim3(64), 0, s, d, e, ki, lam, order, keep_dev,
                       bounds, work, Zt, k, ties_only);
  DME_HIP(hipGetLastError());
  // clusters: polar steps where the vectors are nearly orthonormal,
  // modified Gram-Schmidt for the rest; the result ends in Zf
  double* Zf = Zt;
  {
    const int nc = (int)nkeep;
    double* G = ws.get<double>((size_t)nc * nc);
    double* Z1 = ws.get<double>((size_t)k * nc);
    double* Zo = Z1;  // Zf -> Zo each step
    const dim3 gg((unsigned)cdiv(nc, 16), (unsigned)cdiv(nc, 16)), ga((unsigned)cdiv(k, 16), (unsigned)cdiv(nc, 16));
    for (int step = 0; step < kPolarSteps; ++step) {
      hipLaunchKernelGGL(polar_gemm_kernel<kPolarGram>, gg, dim3(256), 0, s, ki, nc, Zf, (const double*)nullptr,
                         cl_of, clusters, cl_fail, step == 0, G);
      DME_HIP(hipGetLastError());
      hipLaunchKernelGGL(polar_gemm_kernel<kPolarApply>, ga, dim3(256), 0, s, ki, nc, Zf, G, cl_of, clusters,
                         cl_fail, false, Zo);
      DME_HIP(hipGetLastError());
      std::swap(Zf, Zo);
    }
    // cluster staging in LDS: up to 144 KiB, never more than the whole k x k set
    const int64_t orth_lds = std::min<int64_t>(k * k, (144 * 1024) / (int64_t)sizeof(double));
    hipLaunchKernelGGL(orth_kernel, dim3((unsigned)k), dim3(1024), (size_t)orth_lds * sizeof(double), s,
                       ki, clusters, cl_count, pos_of, cl_fail, Zf, k, (int)orth_lds);
    DME_HIP(hipGetLastError());
  }
  // V = Q Z with Q formed beside the eigenvalue work
  DME_HIP(hipStreamWaitEvent(s, q_done, 0));
  gemm_f64(s, 'N', 'N', k, (int64_t)nkeep, k, 1.0, Qm, k, Zf, k, 0.0, V_out, ldv, &ws);
  if (post.signs) {
    hipLaunchKernelGGL(sign_columns_kernel, dim3(nkeep), dim3(64), 0, s, V_out, ldv, ki, keep_dev);
    DME_HIP(hipGetLastError());
  }
}

}  // namespace dme
