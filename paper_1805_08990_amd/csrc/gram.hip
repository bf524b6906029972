// Column compression through the Gram matrix (Sec. 3, the compression after
// Alg. 2) for P = W Dhat W^T with Dhat symmetric positive definite, which is
// what every compression of a DLE / DRE solve sees (Dhat is block diagonal
// from D, the weights of the quadrature factor, t I or copies of D, all
// positive definite when P0 is positive semidefinite):
//
//     Dhat = F F^T (Cholesky),  G = F^T (W^T W) F  (k x k),
//     G = V Lam V^T, keep lam_i > tol max lam (sorted descending),
//     L = W F V_I Lam_I^-1/2,  D = Lam_I,
//
// so P = (W F)(W F)^T = L D L^T on the kept part: the nonzero eigenvalues of
// G are those of P and L = W F V_I Lam_I^-1/2 its eigenvectors.  Compared with
// Householder QR of W (M = R Dhat R^T) this needs one product W^T W (an FP64
// MFMA GEMM, split over n) instead of a tree of column steps, and leaves W
// intact.  Forming W^T W squares the condition number of W: the eigenvalues of
// G carry absolute errors of order u ||G||, which is the accuracy the
// truncation at tol ||G|| >> u ||G|| needs, and P is reproduced to
// O(u ||P||); the columns of L belonging to eigenvalues near tol max lam are
// orthonormal only to about u / tol-level accuracy (~1e-7 measured), which no
// later step relies on (every later compression forms W^T W itself).
#include <thread>

#include "common.h"

namespace dme {
namespace {

constexpr int kCT = 256;    // Cholesky threads (4 waves)

// v from lane `l` (a constant) to every lane, through the scalar unit
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
constexpr int kCB = 32;     // Cholesky block width
constexpr int kCPanel = 192;  // rows below a block staged in LDS (larger k read them from L2)

// In-place lower Cholesky factor of a k x k symmetric positive definite A (ld
// lda; only the lower triangle is read), one workgroup, blocked right-looking,
// three barriers per 32-column block:
//   (a) wave 0 factors the diagonal block column by column with row i in
//       lane i's registers, column c of L broadcast by readlane (no
//       workgroup barrier inside the block);
//   (b) every thread solves rows below the block against it (one row each)
//       and stages them in LDS;
//   (c) the trailing lower triangle is updated in 4 x 4 register tiles
//       (A22 -= L21 L21^T, 32 terms per entry).
// The strict upper triangle is set to zero.  A non-positive (or non-finite)
// pivot sets *status = -1 and zeroes A (what follows then sees a zero matrix,
// not NaNs); otherwise *status = 0.
__global__ __launch_bounds__(kCT) void chol_lower_kernel(int k, double* A, int64_t lda, int64_t* status) {
  __shared__ double blk[kCB][kCB + 1];
  __shared__ double pan[kCPanel][kCB + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  if (tid == 0) bad = 0;
  for (int j = 1; j < k; ++j)
    for (int i = tid; i < j; i += kCT) A[i + (int64_t)j * lda] = 0.0;
  __syncthreads();
  for (int j0 = 0; j0 < k; j0 += kCB) {
    const int jb = min(kCB, k - j0);
    const int rest = k - j0 - jb;
    // (a) diagonal block: loaded by every thread, factored by wave 0
    for (int idx = tid; idx < kCB * kCB; idx += kCT) {
      const int r = idx % kCB, c = idx / kCB;
      blk[r][c] = (r < jb && c <= r) ? A[(j0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
    }
    __syncthreads();
    if (tid < 64) {
      // lane i holds row i of the block in registers; column c of L reaches
      // the other lanes by readlane (constant lane index: no LDS round trip)
      double row[kCB];
#pragma unroll
      for (int c = 0; c < kCB; ++c) row[c] = (lane < jb) ? blk[lane][c] : 0.0;
      bool okall = true;
#pragma unroll
      for (int c = 0; c < kCB; ++c) {
        if (c < jb) {
          const double p = readlane_f64(row[c], c);
          const bool ok = p > 0.0 && isfinite(p);
          okall = okall && ok;
          const double dc = ok ? sqrt(p) : 1.0;
          if (lane == c) row[c] = dc;
          if (lane > c) row[c] = row[c] / dc;
#pragma unroll
          for (int l = c + 1; l < kCB; ++l) {
            if (l < jb) {
              const double llc = readlane_f64(row[c], l);
              if (lane >= l) row[l] -= row[c] * llc;
            }
          }
        }
      }
      if (lane == 0 && !okall) bad = 1;
      if (lane < jb) {
#pragma unroll
        for (int c = 0; c < kCB; ++c) blk[lane][c] = (c <= lane) ? row[c] : 0.0;
      }
    }
    __syncthreads();
    for (int idx = tid; idx < jb * jb; idx += kCT) {
      const int r = idx % jb, c = idx / jb;
      if (r >= c) A[(j0 + r) + (int64_t)(j0 + c) * lda] = blk[r][c];
    }
    if (rest > 0) {
      // (b) rows below the block: x L11^T = a, one thread per row
      const bool staged = rest <= kCPanel;
      for (int i = tid; i < rest; i += kCT) {
        double x[kCB];
        const int64_t row = j0 + jb + i;
#pragma unroll
        for (int c = 0; c < kCB; ++c) x[c] = (c < jb) ? A[row + (int64_t)(j0 + c) * lda] : 0.0;
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
          if (c < jb) {
            double v = x[c];
#pragma unroll
            for (int l = 0; l < c; ++l) v -= x[l] * blk[c][l];
            x[c] = v / blk[c][c];
          }
        }
#pragma unroll
        for (int c = 0; c < kCB; ++c) {
          if (c < jb) {
            A[row + (int64_t)(j0 + c) * lda] = x[c];
            if (staged) pan[i][c] = x[c];
          }
        }
      }
      __syncthreads();
      // (c) trailing lower triangle in 4 x 4 tiles (tile (ti, tl), ti >= tl)
      const int nt = (rest + 3) / 4;
      const int ntiles = nt * (nt + 1) / 2;
      for (int t = tid; t < ntiles; t += kCT) {
        int tl = (int)((2.0 * nt + 1.0 - sqrt((2.0 * nt + 1.0) * (2.0 * nt + 1.0) - 8.0 * t)) / 2.0);
        while (tl > 0 && tl * (2 * nt - tl + 1) / 2 > t) --tl;
        while ((tl + 1) * (2 * nt - tl) / 2 <= t) ++tl;
        const int ti = tl + (t - tl * (2 * nt - tl + 1) / 2);
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
        for (int c = 0; c < jb; ++c) {
          double xi[4], xl[4];
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int ri = 4 * ti + a, rl = 4 * tl + a;
            if (staged) {
              xi[a] = ri < rest ? pan[ri][c] : 0.0;
              xl[a] = rl < rest ? pan[rl][c] : 0.0;
            } else {
              xi[a] = ri < rest ? A[(j0 + jb + ri) + (int64_t)(j0 + c) * lda] : 0.0;
              xl[a] = rl < rest ? A[(j0 + jb + rl) + (int64_t)(j0 + c) * lda] : 0.0;
            }
          }
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] += xi[a] * xl[b];
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int ri = 4 * ti + a, rl = 4 * tl + b;
            if (ri < rest && rl < rest && ri >= rl) {
              const int64_t gi = j0 + jb + ri, gl = j0 + jb + rl;
              A[gi + gl * lda] -= acc[a][b];
            }
          }
      }
    }
    __syncthreads();
  }
  if (bad) {
    for (int j = 0; j < k; ++j)
      for (int i = tid; i < k; i += kCT) A[i + (int64_t)j * lda] = 0.0;
  }
  if (tid == 0) *status = bad ? -1 : 0;
}

// F for a Dhat whose D blocks are diag(lam) - t Z Z^T (see LowRankD), one
// workgroup: Zh = sqrt(t) Lam^-1/2 Z and G = Zh^T Zh (m x m, one lane per
// entry) in LDS, G = U g U^T by cyclic Jacobi in registers of one thread
// (m = M <= 8 at compile time), K = U diag(1 / (1 + sqrt(1 - g))) U^T,
// Mz = Zh K, then F_D(i, j) = sqrt(lam_i) (delta_ij - Mz(i, :) Zh(j, :)^T) in
// every D block and sqrt(Dhat_ii) on the rest of the diagonal.  lam <= 0,
// g >= 1 or a non-positive diagonal entry make *status = -1 (and F zero).
constexpr int kLrMaxM = 8;
constexpr int kLrMaxR = 256;
constexpr int kLrT = 256;

template <int M>
__global__ __launch_bounds__(kLrT) void lowrank_factor_kernel(int k, const double* Dhat, int64_t lddh,
                                                              const double* lam, const double* Z, double t,
                                                              int r, int ncopies, double* F, int64_t* status) {
  static_assert(M >= 1 && M <= kLrMaxM, "m");
  __shared__ double Zh[kLrMaxR][M];
  __shared__ double Mz[kLrMaxR][M];
  __shared__ double sl[kLrMaxR];
  __shared__ double Gs[M * M];
  __shared__ double Ks[M][M];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  __syncthreads();
  const double st = sqrt(t);
  for (int i = tid; i < r; i += kLrT) {
    const double l = lam[i];
    if (!(l > 0.0) || !isfinite(l)) bad = 1;
    const double s = (l > 0.0) ? sqrt(l) : 1.0;
    sl[i] = s;
#pragma unroll
    for (int a = 0; a < M; ++a) Zh[i][a] = st * Z[i + (int64_t)a * r] / s;
  }
  __syncthreads();
  if (tid < M * M) {  // G = Zh^T Zh, entry (a, b) by lane a + M b
    const int a = tid % M, b = tid / M;
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc = fma(Zh[i][a], Zh[i][b], acc);
    Gs[tid] = acc;
  }
  __syncthreads();
  if (tid == 0) {
    double G[M][M], U[M][M];
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = 0; b < M; ++b) {
        G[a][b] = Gs[a + b * M];
        U[a][b] = (a == b) ? 1.0 : 0.0;
      }
    // cyclic Jacobi on the symmetric M x M G; a rotation zeroes its pair
    // exactly, and pairs below 1e-17 sqrt(|G_pp G_qq|) are dropped, so the
    // sweeps end once every off-diagonal entry is at that level
    for (int sweep = 0; sweep < 30; ++sweep) {
      bool rotated = false;
#pragma unroll
      for (int p = 0; p < M; ++p)
#pragma unroll
        for (int q = p + 1; q < M; ++q) {
          if (fabs(G[p][q]) <= 1e-17 * sqrt(fabs(G[p][p] * G[q][q]))) {
            G[p][q] = G[q][p] = 0.0;
            continue;
          }
          rotated = true;
          const double theta = (G[q][q] - G[p][p]) / (2.0 * G[p][q]);
          const double tn = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
          const double c = 1.0 / sqrt(tn * tn + 1.0), sn = tn * c;
#pragma unroll
          for (int x = 0; x < M; ++x) {  // G <- J^T G J, U <- U J
            const double gp = G[x][p], gq = G[x][q];
            G[x][p] = c * gp - sn * gq;
            G[x][q] = sn * gp + c * gq;
          }
#pragma unroll
          for (int x = 0; x < M; ++x) {
            const double gp = G[p][x], gq = G[q][x];
            G[p][x] = c * gp - sn * gq;
            G[q][x] = sn * gp + c * gq;
          }
#pragma unroll
          for (int x = 0; x < M; ++x) {
            const double up = U[x][p], uq = U[x][q];
            U[x][p] = c * up - sn * uq;
            U[x][q] = sn * up + c * uq;
          }
          G[p][q] = G[q][p] = 0.0;
        }
      if (!rotated) break;
    }
    double f[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      const double g = G[a][a];
      if (!(g < 1.0) || !isfinite(g)) bad = 1;
      f[a] = 1.0 / (1.0 + sqrt(fmax(1.0 - g, 0.0)));
    }
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
      for (int b = 0; b < M; ++b) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) v += U[a][q] * f[q] * U[b][q];
        Ks[a][b] = v;
      }
  }
  __syncthreads();
  for (int i = tid; i < r; i += kLrT)
#pragma unroll
    for (int a = 0; a < M; ++a) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b) v += Zh[i][b] * Ks[b][a];
      Mz[i][a] = v;
    }
  // the rest of the diagonal
  const int nd = ncopies * r;
  for (int i = nd + tid; i < k; i += kLrT) {
    const double d = Dhat[i + (int64_t)i * lddh];
    if (!(d > 0.0) || !isfinite(d)) bad = 1;
  }
  __syncthreads();
  const bool ok = !bad;
  for (int j = tid >> 6; j < k; j += kLrT / 64) {  // a wave per column
    const bool inblk = j < nd;                     // D block jb, rows i0 .. i0 + r - 1
    const int jb = inblk ? j / r : 0, jj = j - jb * r, i0 = jb * r;
    double zj[M];
#pragma unroll
    for (int a = 0; a < M; ++a) zj[a] = inblk ? Zh[jj][a] : 0.0;
    for (int i = tid & 63; i < k; i += 64) {
      double v = 0.0;
      if (ok) {
        if (inblk && i >= i0 && i < i0 + r) {
          const int ii = i - i0;
          double acc = 0.0;
#pragma unroll
          for (int a = 0; a < M; ++a) acc += Mz[ii][a] * zj[a];
          v = sl[ii] * ((ii == jj ? 1.0 : 0.0) - acc);
        } else if (i == j) {
          v = sqrt(Dhat[i + (int64_t)i * lddh]);
        }
      }
      F[i + (int64_t)j * k] = v;
    }
  }
  if (tid == 0) *status = ok ? 0 : -1;
}

__global__ void copy_lower_kernel(int k, const double* Dhat, int64_t ldd, double* F) {
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < (int64_t)k * k; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % k), j = (int)(idx / k);
    F[idx] = Dhat[i + (int64_t)j * ldd];
  }
}

// S = (G + G^T) / 2; a non-finite entry sets bit 1 of *flag
// S = F sym(G) F for a diagonal Dhat, F = diag(sqrt(Dhat_ii)): every block
// checks the diagonal (k entries) so that a non-positive or non-finite entry
// zeroes S everywhere, and block 0 writes *status (-1 then, else 0).
__global__ void gram_scale_sym_kernel(int k, const double* G, const double* Dhat, int64_t lddh, double* S,
                                      int64_t* status, int* flag) {
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double d = Dhat[i + (int64_t)i * lddh];
    if (!(d > 0.0) || !isfinite(d)) bad = 1;
  }
  __syncthreads();
  const bool ok = !bad;
  if (blockIdx.x == 0 && threadIdx.x == 0) *status = ok ? 0 : -1;
  bool nf = false;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < (int64_t)k * k; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % k), j = (int)(idx / k);
    double v = 0.0;
    if (ok) {
      const double fi = sqrt(Dhat[i + (int64_t)i * lddh]), fj = sqrt(Dhat[j + (int64_t)j * lddh]);
      v = 0.5 * (G[idx] + G[j + (int64_t)i * k]) * (fi * fj);  // exactly symmetric
    }
    S[idx] = v;
    if (!isfinite(v)) nf = true;
  }
  if (nf) atomicOr(flag, 1);
}

__global__ void sym_kernel(int k, const double* G, double* S, int* flag) {
  bool bad = false;
  for (int64_t idx = blockIdx.x * 256 + threadIdx.x; idx < (int64_t)k * k; idx += (int64_t)gridDim.x * 256) {
    const int i = (int)(idx % k), j = (int)(idx / k);
    const double v = 0.5 * (G[idx] + G[j + (int64_t)i * k]);
    S[idx] = v;
    if (!isfinite(v)) bad = true;
  }
  if (bad) atomicOr(flag, 1);
}

// T(:, j) = X(:, j) s_j / sqrt(lam_j) for j < *rank, T(:, j) = 0 for
// rank <= j < r (the columns past the kept rank may hold anything), where X
// is T = F V itself (dh null) or diag(sqrt(dh_ii)) V (a diagonal Dhat, F V
// without a product), and s_j is the sign that makes the largest |V(i, j)|
// (the first on ties) positive; and the columns j < min(r, rank) of
// D = diag(lam) (rank x rank, ld ldd, or the rank when ldd is 0).  256
// threads a block; the grid covers k >= rank rows.
__global__ __launch_bounds__(256) void scale_cols_kernel(int k, int r, const double* lam, const int64_t* rank,
                                                         double* T, double* D, int64_t ldd, const double* V,
                                                         int64_t ldv, const double* dh, int64_t lddh) {
  __shared__ double sbest[4];
  __shared__ int sidx[4];
  const int64_t rk = *rank;
  const int64_t ld = (ldd > 0) ? ldd : rk;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int j = blockIdx.y; j < r; j += gridDim.y) {
    double sgn = 1.0;
    if (j < rk) {  // uniform in the block
      const double* vj = V + (int64_t)j * ldv;
      double best = -1.0;
      int bi = k;
      for (int i = threadIdx.x; i < k; i += 256) {
        const double a = fabs(vj[i]);
        if (a > best) {
          best = a;
          bi = i;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      __syncthreads();  // the previous column's reads of sbest are done
      if (lane == 0) {
        sbest[wv] = best;
        sidx[wv] = bi;
      }
      __syncthreads();
      best = sbest[0];
      bi = sidx[0];
      for (int q = 1; q < 4; ++q)
        if (sbest[q] > best || (sbest[q] == best && sidx[q] < bi)) {
          best = sbest[q];
          bi = sidx[q];
        }
      if (bi < k && vj[bi] < 0.0) sgn = -1.0;
    }
    const double f = (j < rk) ? sgn / sqrt(lam[j]) : 0.0;
    for (int i = blockIdx.x * 256 + threadIdx.x; i < k; i += gridDim.x * 256) {
      double* t = T + i + (int64_t)j * k;
      const double x = dh ? sqrt(dh[i + (int64_t)i * lddh]) * V[i + (int64_t)j * ldv] : *t;
      *t = (j < rk) ? x * f : 0.0;
      if (j < rk && i < rk) D[i + j * ld] = (i == j) ? lam[j] : 0.0;
    }
  }
}

inline unsigned blocks(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(total, 256), 4096));
}

}  // namespace

size_t compress_gram_workspace(int64_t n, int64_t k) {
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(6 * (size_t)k * k * sizeof(double));  // F, G, T1, S, V, T
  add((size_t)k * sizeof(double) + 64);     // lam, status
  add(syev_workspace(k));
  add(std::max({gemm_f64_workspace(k, k, n), gemm_f64_workspace(n, k, k), gemm_f64_workspace(k, k, k)}));
  return b + 4096;
}

bool gram_factor_lowrank(hipStream_t st, int64_t k, const double* Dhat, int64_t lddh, const LowRankD& lr,
                         double* F, int64_t* status) {
  if (!(lr.m >= 1 && lr.m <= kLrMaxM && lr.r <= kLrMaxR && lr.ncopies * lr.r <= k)) return false;
  switch (lr.m) {
#define DME_LRF(MM)                                                                                       \
  case MM:                                                                                                \
    hipLaunchKernelGGL(lowrank_factor_kernel<MM>, dim3(1), dim3(kLrT), 0, st, (int)k, Dhat, lddh, lr.lam, \
                       lr.Z, lr.t, (int)lr.r, lr.ncopies, F, status);                                     \
    break;
    DME_LRF(1) DME_LRF(2) DME_LRF(3) DME_LRF(4) DME_LRF(5) DME_LRF(6) DME_LRF(7) DME_LRF(8)
#undef DME_LRF
    default: return false;
  }
  DME_HIP(hipGetLastError());
  return true;
}

int64_t compress_gram_f64(hipStream_t s, int64_t n, int64_t k, const double* W, int64_t ldw,
                          const double* Dhat, int64_t lddh, bool dhat_diag, const LowRankD* lowrank,
                          double tol, int64_t max_rank, double* L, int64_t ldl, double* Dout, int64_t ldd,
                          int64_t* rank_dev, int* flag_dev, Arena& ws, int64_t rank_hint,
                          const double* F_ready, const int64_t* status_ready, double* T_keep,
                          const std::function<void(hipEvent_t)>* beside) {
  if (k <= 0 || n <= 0) return 0;
  const size_t mark = ws.used;
  double* Fw = ws.get<double>((size_t)k * k);
  double* G = ws.get<double>((size_t)k * k);
  double* T1 = ws.get<double>((size_t)k * k);
  double* S = ws.get<double>((size_t)k * k);
  double* V = ws.get<double>((size_t)k * k);
  double* T = T_keep ? T_keep : ws.get<double>((size_t)k * k);
  double* lam = ws.get<double>(k);
  int64_t* status = ws.get<int64_t>(8);
  const size_t mark_g = ws.used;

  // Dhat = F F^T.  A diagonal Dhat needs no F: its square roots scale the
  // Gram matrix and V in the kernels that read them.  Otherwise F comes ready
  // (formed by the caller on a stream s is already ordered after) or is
  // formed here on the second stream, beside W^T W on s.  A factor that fails
  // (Dhat not positive definite) leaves F = 0 (S = 0 when diagonal), so what
  // follows sees a zero matrix; its status vetoes the rank on its way to the
  // host, which then returns -1 for the caller to compress by Householder QR.
  const bool diag = !F_ready && dhat_diag;
  const double* F = F_ready ? F_ready : Fw;
  const int64_t* fstatus = F_ready ? status_ready : status;
  hipEvent_t f_done = nullptr;
  if (!F_ready && !diag) {
    AuxStream& ax = aux_stream();
    DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
    if (!(lowrank && gram_factor_lowrank(ax.s2, k, Dhat, lddh, *lowrank, Fw, status))) {
      hipLaunchKernelGGL(copy_lower_kernel, dim3(blocks(k * k)), dim3(256), 0, ax.s2, (int)k, Dhat, lddh, Fw);
      DME_HIP(hipGetLastError());
      hipLaunchKernelGGL(chol_lower_kernel, dim3(1), dim3(kCT), 0, ax.s2, (int)k, Fw, k, status);
      DME_HIP(hipGetLastError());
    }
    f_done = ax.record(ax.s2);
  }
  ws.used = mark_g;
  gemm_f64(s, 'T', 'N', k, k, n, 1.0, W, ldw, W, ldw, 0.0, G, k, &ws);
  ws.used = mark_g;
  if (diag) {
    hipLaunchKernelGGL(gram_scale_sym_kernel, dim3(blocks(k * k)), dim3(256), 0, s, (int)k, G, Dhat, lddh, S,
                       status, flag_dev);
  } else {
    if (f_done) DME_HIP(hipStreamWaitEvent(s, f_done, 0));
    // G <- F^T G F, symmetrised
    gemm_f64(s, 'N', 'N', k, k, k, 1.0, G, k, F, k, 0.0, T1, k, &ws);
    ws.used = mark_g;
    gemm_f64(s, 'T', 'N', k, k, k, 1.0, F, k, T1, k, 0.0, G, k, &ws);
    hipLaunchKernelGGL(sym_kernel, dim3(blocks(k * k)), dim3(256), 0, s, (int)k, G, S, flag_dev);
  }
  DME_HIP(hipGetLastError());
  ws.used = mark_g;
  // work the caller runs beside the eigensolver (which keeps one CU busy
  // through the tridiagonal reduction), ordered after the Gram matrix
  if (beside && *beside) (*beside)(aux_stream().record(s));
  // the kept rank travels to the host from the second stream as soon as it is
  // known; the eigenvectors' signs are applied with the column scaling below
  int64_t seq_rank = 0;
  SyevPost post;
  post.signs = false;
  post.rank_veto = fstatus;
  post.rank_seq = &seq_rank;
  syev_trunc_f64(s, k, S, k, tol, std::min(max_rank, k), lam, V, k, rank_dev, flag_dev, ws, post);
  ws.used = mark_g;
  // L = W (F V_I Lam_I^-1/2), D = Lam_I: the products (and D) for a guessed
  // width go ahead of the rank's round trip to the host
  const int64_t kmax = std::min(max_rank, k);
  const int64_t ks = (rank_hint > 0) ? std::min(kmax, rank_hint + 8) : kmax;
  auto form_L = [&](int64_t w) {
    if (!diag) gemm_f64(s, 'N', 'N', k, w, k, 1.0, F, k, V, k, 0.0, T, k, &ws);
    ws.used = mark_g;
    const dim3 sg(cdiv(k, 256), (unsigned)std::min<int64_t>(w, 1024));
    hipLaunchKernelGGL(scale_cols_kernel, sg, dim3(256), 0, s, (int)k, (int)w, lam, rank_dev, T, Dout, ldd, V, k,
                       diag ? Dhat : nullptr, lddh);
    DME_HIP(hipGetLastError());
    gemm_f64(s, 'N', 'N', n, w, k, 1.0, W, ldw, T, k, 0.0, L, ldl, &ws);
    ws.used = mark_g;
  };
  form_L(ks);
  const int64_t rr = value_to_host_wait(aux_stream().s2, seq_rank);
  if (rr <= 0) {
    ws.used = mark;
    return rr < 0 ? -1 : 0;  // -1: Dhat is not positive definite
  }
  if (rr > ks) form_L(rr);  // the guess fell short (D's remaining columns too)
  ws.used = mark;
  return rr;
}

}  // namespace dme
