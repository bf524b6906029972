// Householder QR of a tall-skinny W (n x k) by panels of 32 columns, each
// panel factored as a reduction tree (TSQR) of Householder QRs of 288-row
// leaves:
//
//   level 0: the panel rows [c0, n) are cut into leaves of 288 rows (the last
//            one ragged); one workgroup factors leaf g, B_g = Q_g [R_g; 0],
//            keeps the reflectors V_g in place and the compact-WY factor T_g
//            (Q_g = I - V_g T_g V_g^T), and stacks R_g (32 rows, zero below
//            the diagonal) into the next level's matrix;
//   level l: the stacked R factors are factored the same way, until a single
//            leaf remains; its R is the panel's R.
//
// Q^T is applied to the trailing columns level by level, and Q to the new
// factor at the end in the reverse order.  Row s of level l is row
// (s / 32) * 288 + s % 32 of level l - 1 (the head rows of each leaf), which
// maps every level back to rows of W.
//
// Leaf factorisation (512 threads = 32 columns x 16 row groups): thread
// (c, g) holds rows g + 16 m (m < 18) of column c in registers.  Column step j
// needs one broadcast, the pivot column x_j (LDS, written by its owners at the
// end of step j - 1 together with its alpha and sigma^2), and one reduction
// within each column's 16 lanes: the sum over rows i > j of x_j(i) a_c(i),
// which for c > j is the product that updates column c and for c < j the
// entry v_c^T v_j of the Gram matrix that builds T.  So a step has a single
// barrier.  The pivot column is kept unscaled until the end, so no thread
// rewrites what another still reads.
#include "tsqr.h"

#include <memory>
#include <type_traits>

namespace dme {
namespace {

constexpr int kTB = 32;                   // panel width
constexpr int kTLeaf = 288;               // rows per leaf (9 runs of 32)
constexpr int kTT = 256;                  // block-reflector threads: 32 columns x 8 row groups
constexpr int kTG = kTT / kTB;            // their row groups
constexpr int kTRows = kTLeaf / kTG;      // rows each stages (36)
constexpr int kLT = 512;                  // leaf threads: 32 columns x 16 row groups
constexpr int kLG = kLT / kTB;            // leaf row groups
constexpr int kLRows = kTLeaf / kLG;      // rows per leaf thread (18)
constexpr int kLHq = kTB / kLG;           // of them in the top 32 rows (2)

// Rows of every level of a panel (kernel argument by value).
struct LevelRows {
  int64_t M[kTsqrMaxLevels];
};

// Level-L row s -> row of level 0, or -1 for a padding row (a leaf with fewer
// than 32 rows stacks zero rows that exist on no lower level).
template <int L>
__device__ inline int64_t phys_row(int64_t s, const LevelRows& lr) {
  bool pad = false;
#pragma unroll
  for (int l = L; l > 0; --l) {
    s = (s >> 5) * kTLeaf + (s & (kTB - 1));
    pad = pad || (s >= lr.M[l - 1]);
  }
  return pad ? -1 : s;
}

// r_mode: 0 = R stays in place (single leaf of level 0); 1 = R_g stacked into
// Rdst rows 32 g .. 32 g + 31 (zeros below the diagonal); 2 = R's upper
// triangle written to Rdst (the panel's top rows in W).
__device__ __forceinline__ void leaf_body(int bx, double* mat, int64_t ld, int64_t M, int pb, double* Tout,
                                          double* Rdst, int64_t ld_r, int r_mode) {
  __shared__ double xb[2][kLG][kLRows];  // pivot column, [g][m]: 144-byte rows, 16-byte reads conflict-free
  __shared__ double piv[2][2];               // alpha and sigma^2 of the pivot column
  __shared__ double Zs[kTB][kTB + 1];        // Zs[c][j] = v_c^T v_j for c < j, zero elsewhere
  __shared__ double coef[kTB];               // tau of each reflector
  const int t = threadIdx.x;
  const int c = t / kLG, g = t % kLG;
  const int64_t rbeg = (int64_t)bx * kTLeaf;
  const int rows = (int)min<int64_t>(kTLeaf, M - rbeg);
  const int nv = min(rows, pb);
  double* base = mat + rbeg;
  const bool cin = c < pb;
  // loads are unconditional (clamped to an entry of the block) and masked
  // afterwards, so they are all in flight together
  const int64_t cc0 = (int64_t)min(c, pb - 1) * ld;
  double a[kLRows];
#pragma unroll
  for (int m = 0; m < kLRows; ++m) {
    const int i = g + kLG * m;
    const double v = base[min(i, rows - 1) + cc0];
    a[m] = (i < rows && cin) ? v : 0.0;
  }
  for (int idx = t; idx < kTB * (kTB + 1); idx += kLT) (&Zs[0][0])[idx] = 0.0;
  // pivot data of column p from its owners (all 16 lanes of the column)
  auto publish = [&](int p, int buf) {
    double sq[2] = {0.0, 0.0};  // independent chains
    double al = 0.0;
#pragma unroll
    for (int m = 0; m < kLRows; ++m) {
      const int i = g + kLG * m;
      xb[buf][g][m] = a[m];
      if (m < kLHq) {
        sq[m & 1] += (i > p) ? a[m] * a[m] : 0.0;
        al += (i == p) ? a[m] : 0.0;
      } else {
        sq[m & 1] += a[m] * a[m];
      }
    }
    const double s2 = group16_sum_f64(sq[0] + sq[1]);
    al = group16_sum_f64(al);
    if (g == 0) {
      piv[buf][0] = al;
      piv[buf][1] = s2;
    }
  };
  if (c == 0) publish(0, 0);
  __syncthreads();

  // Column jj of T (upper triangular, Q = I - V T V^T): T(jj, jj) = tau_jj and
  // T(c, jj) = -tau_jj sum_{c <= c2 < jj} T(c, c2) Zs(c2, jj), from the columns
  // before it.  Thread (c, g) sums over c2 = g + 16 q and keeps T(c, c2) for
  // those c2 in registers.  Formed one step after Zs(:, jj), beside the next
  // column step.  (The reads are unconditional; Zs is zero outside c2 < jj.)
  double* To = Tout + (int64_t)bx * kTB * kTB;
  double trow[kTB / kLG] = {0.0, 0.0};
  auto t_column = [&](int jj) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kTB / kLG; ++q) {
      const int c2 = g + kLG * q;
      const double z = Zs[c2][jj];
      s += ((c2 >= c) ? trow[q] : 0.0) * z;
    }
    s = group16_sum_f64(s);
    const double tj = coef[jj];
    const double v = (c == jj) ? tj : ((c < jj) ? -tj * s : 0.0);
#pragma unroll
    for (int q = 0; q < kTB / kLG; ++q) trow[q] = (jj == g + kLG * q) ? v : trow[q];
    if (g == 0) To[c + jj * kTB] = v;
  };

  double my_sc = 0.0, my_beta = 0.0;  // this column's reflector, once it has been the pivot
  for (int j = 0; j < nv; ++j) {
    const int bf = j & 1;
    if (j > 0) t_column(j - 1);
    double xv[kLRows];
#pragma unroll
    for (int m = 0; m < kLRows; ++m) xv[m] = xb[bf][g][m];
    const double alpha = piv[bf][0], s2 = piv[bf][1];
    // reflector j (every thread forms the same values; independent of the
    // products below, so its latency overlaps them)
    double beta = alpha, tau = 0.0, sc = 0.0;
    if (s2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    // sum over rows i > j of x_j(i) a_c(i), and a_c(j)
    double pp[2] = {0.0, 0.0};  // independent chains
    double ah = 0.0;
#pragma unroll
    for (int m = 0; m < kLHq; ++m) {
      const int i = g + kLG * m;
      xv[m] = (i > j) ? xv[m] : 0.0;
      ah += (i == j) ? a[m] : 0.0;
    }
#pragma unroll
    for (int m = 0; m < kLRows; ++m) pp[m & 1] += xv[m] * a[m];
    const double tc = group16_sum_f64(pp[0] + pp[1]);
    const double ahead = group16_sum_f64(ah);
    if (c < j) {
      if (g == 0) Zs[c][j] = my_sc * (ahead + sc * tc);
    } else if (c == j) {
      my_sc = sc;
      my_beta = beta;
      if (g == 0) coef[j] = tau;
    } else {
      // a_c -= tau v (v^T a_c), v = [1; sc x_j(i > j)]
      const double wv = tau * (ahead + sc * tc);
      const double f = wv * sc;
#pragma unroll
      for (int m = 0; m < kLRows; ++m) {
        const int i = g + kLG * m;
        const double u = a[m] - f * xv[m];
        a[m] = (m < kLHq && i == j) ? ahead - wv : u;
      }
      if (c == j + 1 && j + 1 < nv) publish(j + 1, bf ^ 1);
    }
    __syncthreads();
  }

  // reflectors scaled in place, R in the upper part of the head rows
  if (c < nv) {
#pragma unroll
    for (int m = 0; m < kLRows; ++m) {
      const int i = g + kLG * m;
      if (m >= kLHq || i > c) a[m] *= my_sc;
      else if (i == c) a[m] = my_beta;
    }
  }
  if (cin) {
#pragma unroll
    for (int m = 0; m < kLRows; ++m) {
      const int i = g + kLG * m;
      if (i < rows) base[i + (int64_t)c * ld] = a[m];
    }
    if (r_mode == 1) {
#pragma unroll
      for (int m = 0; m < kLHq; ++m) {
        const int i = g + kLG * m;
        Rdst[(int64_t)bx * kTB + i + (int64_t)c * ld_r] = (i <= c && i < rows) ? a[m] : 0.0;
      }
    } else if (r_mode == 2) {
#pragma unroll
      for (int m = 0; m < kLHq; ++m) {
        const int i = g + kLG * m;
        if (i <= c && i < rows) Rdst[i + (int64_t)c * ld_r] = a[m];
      }
    }
  }
  // the last column of T, and zero columns past the reflectors
  t_column(nv - 1);
#pragma unroll
  for (int q = 0; q < kTB / kLG; ++q) {
    const int jj = g + kLG * q;
    if (jj >= nv) To[c + jj * kTB] = 0.0;
  }
}

__global__ __launch_bounds__(kLT) void tsqr_leaf_kernel(double* mat, int64_t ld, int64_t M, int pb,
                                                        double* Tout, double* Rdst, int64_t ld_r,
                                                        int r_mode) {
  leaf_body(blockIdx.x, mat, ld, M, pb, Tout, Rdst, ld_r, r_mode);
}

// C <- (I - V T' V^T) C for every leaf of one level, T' = T^T (trans: applies
// Q^T) or T, on FP64 MFMA.  Block (g, y) handles leaf g (288 rows) and the
// columns [32 y, 32 y + 32); wave w = 2 h + e takes the row half h (144 rows)
// and the column half e (16 columns).  Each lane loads the 36 C entries it
// feeds to the first product, and its result lanes of the last product hold
// exactly those entries, so C is read once and written once:
//   Y_h = V_h^T C_h  (two 16 x 16 tiles per wave, 72 MFMAs over its rows),
//   Z = T' (Y_0 + Y_1)  (one 16 x 16 tile per wave, 8 MFMAs),
//   C_h -= V_h Z  (nine 16-row tiles per wave, 72 MFMAs).
// V of leaf g: level matrix rows [288 g, 288 g + rows), unit diagonal
// implicit, zero above; it is staged in LDS.  C rows are this level's rows
// mapped to rows of level 0: each aligned run of 32 rows of a level is a run
// of 32 rows of level 0, so a block needs 9 base rows.  A run's padding rows
// (a leaf of the level below with fewer than 32 rows) are a suffix of it;
// they read as zero and are not written.  Blocks with no padding rows and a
// full column tile take loads and stores without masks.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTRuns = kTLeaf / kTB;        // 32-row runs per leaf (9)
constexpr int kTHalfSteps = kTLeaf / 8;     // K-steps of 4 rows per row half (36)

template <int LEVEL>
__device__ __forceinline__ void apply_body(int bx, int by, const double* V, int64_t ldv, int64_t M, int pb,
                                           const double* Tin, int trans, const LevelRows& lr, double* C,
                                           int64_t ldc, int64_t ncols) {
  __shared__ double Vs[kTLeaf][kTB + 1];
  __shared__ double Yp[2][kTB][kTB + 1];  // Y of each row half
  __shared__ double Zs[kTB][kTB + 1];
  __shared__ double Ts[kTB][kTB + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int h = w >> 1, e = w & 1;
  const int64_t rbeg = (int64_t)bx * kTLeaf;
  const int rows = (int)min<int64_t>(kTLeaf, M - rbeg);
  const int nv = min(rows, pb);
  const int64_t col = (int64_t)by * kTB + e * 16 + li;
  const bool cok = col < ncols;
  // level-0 base row of each 32-row run (uniform over the block)
  int64_t rb[kTRuns];
  bool full = rows == kTLeaf && (int64_t)by * kTB + kTB <= ncols;
#pragma unroll
  for (int q = 0; q < kTRuns; ++q) {
    rb[q] = phys_row<LEVEL>(rbeg + kTB * q, lr);
    full = full && phys_row<LEVEL>(rbeg + kTB * q + kTB - 1, lr) >= 0;
  }
  const double* Ccol = C + col * ldc;
  // row of level 0 for leaf row i (masked path), -1 for none
  auto crow = [&](int i) -> int64_t {
    return (i < rows && cok) ? phys_row<LEVEL>(rbeg + i, lr) : -1;
  };
  // V staged through registers: thread (a, r0) loads rows r0 + 8 m of column a
  const int va = t >> 3, vr = t & 7;
  double vst[kTRows];
  if (full && pb == kTB) {
    const double* vp = V + rbeg + vr + (int64_t)va * ldv;
#pragma unroll
    for (int m = 0; m < kTRows; ++m) vst[m] = vp[kTG * m];
  } else {
    const double* vp = V + rbeg + (int64_t)min(va, pb - 1) * ldv;
#pragma unroll
    for (int m = 0; m < kTRows; ++m) vst[m] = vp[min(vr + kTG * m, rows - 1)];
  }
  // C entries of this lane: rows 4 s + lk of the leaf, s = 36 h + u
  double cr[kTHalfSteps];
  auto load_c = [&](auto h_tag) {
    constexpr int H = decltype(h_tag)::value;
    if (full) {
#pragma unroll
      for (int u = 0; u < kTHalfSteps; ++u) {
        const int s = kTHalfSteps * H + u;
        cr[u] = Ccol[rb[s >> 3] + 4 * (s & 7) + lk];
      }
    } else {
#pragma unroll
      for (int u = 0; u < kTHalfSteps; ++u) {
        const int64_t pr = crow(4 * (kTHalfSteps * H + u) + lk);
        const double v = Ccol[pr >= 0 ? pr : 0 - col * ldc];
        cr[u] = (pr >= 0) ? v : 0.0;
      }
    }
  };
  if (h == 0) load_c(std::integral_constant<int, 0>{});
  else load_c(std::integral_constant<int, 1>{});
  {
    const double* Tg = Tin + (int64_t)bx * kTB * kTB;
#pragma unroll
    for (int m = 0; m < kTB * kTB / kTT; ++m) {
      const int idx = t + kTT * m;
      const int a = idx % kTB, b = idx / kTB;  // T(a, b)
      const double v = Tg[a + b * kTB];
      if (trans) Ts[b][a] = v;
      else Ts[a][b] = v;
    }
  }
#pragma unroll
  for (int m = 0; m < kTRows; ++m) {
    const int i = vr + kTG * m;
    const double y = (i > va) ? vst[m] : (i == va ? 1.0 : 0.0);
    Vs[i][va] = (i < rows && va < nv) ? y : 0.0;
  }
  __syncthreads();
  // Y_h tiles (reflectors 0-15 and 16-31) x (columns of half e)
  {
    v4d y0 = {0.0, 0.0, 0.0, 0.0}, y1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < kTHalfSteps; ++u) {
      const int i = 4 * (kTHalfSteps * h + u) + lk;
      y0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[i][li], cr[u], y0, 0, 0, 0);
      y1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[i][16 + li], cr[u], y1, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Yp[h][4 * v + lk][e * 16 + li] = y0[v];
      Yp[h][16 + 4 * v + lk][e * 16 + li] = y1[v];
    }
  }
  __syncthreads();
  // Z tile (w / 2, w % 2) = T' Y
  {
    const int zt = w >> 1, zc = w & 1;
    v4d z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < kTB / 4; ++q) {
      const int k = 4 * q + lk;
      const double y = Yp[0][k][zc * 16 + li] + Yp[1][k][zc * 16 + li];
      z = __builtin_amdgcn_mfma_f64_16x16x4f64(Ts[zt * 16 + li][k], y, z, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Zs[zt * 16 + 4 * v + lk][zc * 16 + li] = z[v];
  }
  __syncthreads();
  double zb[kTB / 4];
#pragma unroll
  for (int q = 0; q < kTB / 4; ++q) zb[q] = Zs[4 * q + lk][e * 16 + li];
  // C rows of tiles 9 h .. 9 h + 8, columns of half e
  auto update = [&](auto h_tag) {
    constexpr int H = decltype(h_tag)::value;
#pragma unroll
    for (int r = 0; r < kTRuns; ++r) {
      const int rt = kTRuns * H + r;
      v4d p = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kTB / 4; ++q)
        p = __builtin_amdgcn_mfma_f64_16x16x4f64(Vs[rt * 16 + li][4 * q + lk], zb[q], p, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int u = 4 * r + v;  // s = 4 rt + v = 36 H + u
        const int s = kTHalfSteps * H + u;
        if (full) {
          C[rb[s >> 3] + 4 * (s & 7) + lk + col * ldc] = cr[u] - p[v];
        } else {
          const int64_t pr = crow(4 * s + lk);
          if (pr >= 0) C[pr + col * ldc] = cr[u] - p[v];
        }
      }
    }
  };
  if (h == 0) update(std::integral_constant<int, 0>{});
  else update(std::integral_constant<int, 1>{});
}

template <int LEVEL>
__global__ __launch_bounds__(kTT) void tsqr_apply_kernel(const double* V, int64_t ldv, int64_t M,
                                                         int pb, const double* Tin, int trans,
                                                         LevelRows lr, double* C, int64_t ldc,
                                                         int64_t ncols) {
  apply_body<LEVEL>(blockIdx.x, blockIdx.y, V, ldv, M, pb, Tin, trans, lr, C, ldc, ncols);
}

// Two independent launches in one: blocks [0, nleaf) factor the leaves of one
// tree level, the others apply Q^T of the level below to the next panel's
// columns (block b -> leaf b % agx, column tile b / agx) with the first kTT
// threads (the rest leave before any barrier of that part).
template <int LEVEL>
__global__ __launch_bounds__(kLT) void tsqr_leaf_apply_kernel(double* mat, int64_t ld, int64_t M, int pb,
                                                              double* Tout, double* Rdst, int64_t ld_r,
                                                              int r_mode, int nleaf, const double* V,
                                                              int64_t ldv, int64_t MV, const double* Tin,
                                                              LevelRows lr, double* C, int64_t ldc,
                                                              int64_t ncols, int agx) {
  if ((int)blockIdx.x < nleaf) {
    leaf_body(blockIdx.x, mat, ld, M, pb, Tout, Rdst, ld_r, r_mode);
    return;
  }
  if (threadIdx.x >= kTT) return;
  const int b = (int)blockIdx.x - nleaf;
  apply_body<LEVEL>(b % agx, b / agx, V, ldv, MV, pb, Tin, 1, lr, C, ldc, ncols);
}

void launch_apply(hipStream_t s, const TsqrLevel& L, int level, int pb, int trans, const LevelRows& lr,
                  double* C, int64_t ldc, int64_t ncols) {
  dim3 grid((unsigned)L.G, (unsigned)cdiv(ncols, kTB));
  switch (level) {
#define DME_TSQR_APPLY(LV)                                                                       \
  case LV:                                                                                        \
    hipLaunchKernelGGL(tsqr_apply_kernel<LV>, grid, dim3(kTT), 0, s, L.mat, L.ld, L.M, pb, L.T, \
                       trans, lr, C, ldc, ncols);                                                 \
    break;
    DME_TSQR_APPLY(0) DME_TSQR_APPLY(1) DME_TSQR_APPLY(2) DME_TSQR_APPLY(3)
    DME_TSQR_APPLY(4) DME_TSQR_APPLY(5) DME_TSQR_APPLY(6) DME_TSQR_APPLY(7)
#undef DME_TSQR_APPLY
    default: fail(DME_EINTERNAL, "tsqr: bad level");
  }
  DME_HIP(hipGetLastError());
}

// Leaves of level L (L.G blocks) and Q^T of level A (A.G x column tiles) in one launch.
void launch_leaf_apply(hipStream_t s, const TsqrLevel& L, int pb, double* Rdst, int64_t ld_r, int r_mode,
                       const TsqrLevel& A, int alevel, const LevelRows& lr, double* C, int64_t ldc,
                       int64_t ncols) {
  const int agx = A.G;
  const unsigned nblk = (unsigned)(L.G + (int64_t)agx * cdiv(ncols, kTB));
  switch (alevel) {
#define DME_TSQR_LA(LV)                                                                                        \
  case LV:                                                                                                     \
    hipLaunchKernelGGL(tsqr_leaf_apply_kernel<LV>, dim3(nblk), dim3(kLT), 0, s, L.mat, L.ld, L.M, pb, L.T, Rdst, \
                       ld_r, r_mode, L.G, A.mat, A.ld, A.M, A.T, lr, C, ldc, ncols, agx);                    \
    break;
    DME_TSQR_LA(0) DME_TSQR_LA(1) DME_TSQR_LA(2) DME_TSQR_LA(3) DME_TSQR_LA(4) DME_TSQR_LA(5) DME_TSQR_LA(6)
#undef DME_TSQR_LA
    default: fail(DME_EINTERNAL, "tsqr: bad level");
  }
  DME_HIP(hipGetLastError());
}

LevelRows level_rows(const TsqrPanel& P) {
  LevelRows lr{};
  for (int l = 0; l < P.nlev; ++l) lr.M[l] = P.lev[l].M;
  return lr;
}

}  // namespace

bool tsqr_supported(int64_t n, int64_t k) { return n >= 1 && k >= 1; }

// Workspace for the stacked R factors and T blocks of every panel.
size_t tsqr_workspace(int64_t n, int64_t k) {
  size_t b = 0;
  const int64_t kr = std::min(n, k);
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  for (int64_t c0 = 0; c0 < kr; c0 += kTB) {
    const int pb = (int)std::min<int64_t>(kTB, k - c0);
    int64_t M = n - c0;
    for (int l = 0; l < kTsqrMaxLevels; ++l) {
      const int64_t G = cdiv(M, kTLeaf);
      add((size_t)G * kTB * kTB * sizeof(double));
      if (G == 1) break;
      M = G * kTB;
      add((size_t)M * pb * sizeof(double));
    }
  }
  return b + 4096;
}

namespace {
thread_local AuxStream* g_bound_aux = nullptr;
}  // namespace

void AuxStream::ensure(int dev) {
  if (s2 != nullptr) {
    DME_REQUIRE(dev == device, DME_EINTERNAL, "auxiliary stream used on another device");
    return;
  }
  device = dev;
  DME_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
  ev.assign(64, nullptr);
  for (hipEvent_t& e : ev) DME_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  DME_HIP(hipHostMalloc((void**)&slot, sizeof(Slot), hipHostMallocCoherent));
  slot->value = 0;
  slot->seq = 0;
  seq = 0;
  next = 0;
}

void AuxStream::release() {
  if (s2 == nullptr) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != device) (void)hipSetDevice(device);
  (void)hipStreamSynchronize(s2);
  for (hipEvent_t e : ev)
    if (e) (void)hipEventDestroy(e);
  ev.clear();
  (void)hipStreamDestroy(s2);
  s2 = nullptr;
  if (slot) (void)hipHostFree(slot);
  slot = nullptr;
  if (cur != device) (void)hipSetDevice(cur);
  device = -1;
}

AuxBinding::AuxBinding(AuxStream& a) : prev_(g_bound_aux) { g_bound_aux = &a; }
AuxBinding::~AuxBinding() { g_bound_aux = prev_; }

AuxStream& aux_stream() {
  DME_REQUIRE(g_bound_aux != nullptr, DME_EINTERNAL, "no auxiliary stream bound to this thread");
  int dev = 0;
  DME_HIP(hipGetDevice(&dev));
  g_bound_aux->ensure(dev);
  return *g_bound_aux;
}

// Panels are factored on s.  Q^T of panel p reaches the next panel's columns
// on s (they are what panel p + 1 factors next), level l - 1 in the same
// launch as the leaves of level l, and the columns beyond on a second stream,
// which waits for the panel's tree and runs behind the factorisation of the
// following panels; s waits for that stream before it touches those columns
// (and before returning).
void tsqr_factor(hipStream_t s, int64_t n, int64_t k, double* W, TsqrState& st, Arena& ws) {
  DME_REQUIRE(n < (int64_t(1) << 31), DME_EINVAL, "tsqr: n too large");
  const int64_t ld = n;
  const int64_t kr = std::min(n, k);
  st.n = n;
  st.k = k;
  st.ld = ld;
  st.W = W;
  st.panels.clear();
  AuxStream& ax = aux_stream();
  bool aux_used = false;
  hipEvent_t rest_done = nullptr;  // the second stream finished the previous panel's share
  // (the second stream's first work waits for panel 0's leaves, so for W too)
  for (int64_t c0 = 0; c0 < kr; c0 += kTB) {
    TsqrPanel P;
    P.c0 = c0;
    P.pb = (int)std::min<int64_t>(kTB, k - c0);
    const int pb = P.pb;
    // the tree of this panel: level 0 is the panel itself, in W
    {
      int64_t M = n - c0;
      double* mat = W + c0 + c0 * ld;
      int64_t mld = ld;
      for (int l = 0; l < kTsqrMaxLevels; ++l) {
        TsqrLevel& L = P.lev[l];
        L.M = M;
        L.G = (int)cdiv(M, kTLeaf);
        L.mat = mat;
        L.ld = mld;
        L.T = ws.get<double>((size_t)L.G * kTB * kTB);
        P.nlev = l + 1;
        if (L.G == 1) break;
        if (l + 1 == kTsqrMaxLevels) fail(DME_EINVAL, "tsqr: matrix too tall for the reduction tree");
        const int64_t Mn = (int64_t)L.G * kTB;
        M = Mn;
        mat = ws.get<double>((size_t)Mn * pb);
        mld = Mn;
      }
    }
    const LevelRows lr = level_rows(P);
    const int64_t rest = k - c0 - pb;
    const int64_t near = std::min<int64_t>(rest, kTB);  // the next panel's columns
    const int64_t far = rest - near;
    double* Cnear = W + c0 + (c0 + pb) * ld;
    // leaves level by level on s; Q^T of level l - 1 reaches the next panel's
    // columns in the same launch as the leaves of level l (it needs the
    // previous panel's share of the second stream first)
    for (int l = 0; l < P.nlev; ++l) {
      const TsqrLevel& L = P.lev[l];
      const bool top = (l + 1 == P.nlev);
      double* Rdst = top ? W + c0 + c0 * ld : P.lev[l + 1].mat;
      const int64_t ld_r = top ? ld : P.lev[l + 1].ld;
      const int r_mode = top ? (l > 0 ? 2 : 0) : 1;
      if (l == 0 || near == 0) {
        hipLaunchKernelGGL(tsqr_leaf_kernel, dim3((unsigned)L.G), dim3(kLT), 0, s, L.mat, L.ld, L.M, pb, L.T, Rdst,
                           ld_r, r_mode);
      } else {
        if (l == 1 && rest_done) DME_HIP(hipStreamWaitEvent(s, rest_done, 0));
        launch_leaf_apply(s, L, pb, Rdst, ld_r, r_mode, P.lev[l - 1], l - 1, lr, Cnear, ld, near);
      }
      DME_HIP(hipGetLastError());
    }
    // one event per panel, and only where the second stream needs it (a
    // recorded event costs the stream a few microseconds)
    hipEvent_t leaves_done = (far > 0) ? ax.record(s) : nullptr;
    // Q^T of the top level on the next panel's columns
    if (near > 0) {
      if (P.nlev == 1 && rest_done) DME_HIP(hipStreamWaitEvent(s, rest_done, 0));
      launch_apply(s, P.lev[P.nlev - 1], P.nlev - 1, pb, 1, lr, Cnear, ld, near);
    }
    // Q^T on the columns beyond the next panel: second stream, level by level
    if (far > 0) {
      double* C = W + c0 + (c0 + pb + near) * ld;
      DME_HIP(hipStreamWaitEvent(ax.s2, leaves_done, 0));
      for (int l = 0; l < P.nlev; ++l) launch_apply(ax.s2, P.lev[l], l, pb, 1, lr, C, ld, far);
      aux_used = true;
      rest_done = ax.record(ax.s2);
    }
    st.panels.push_back(P);
  }
  if (aux_used) DME_HIP(hipStreamWaitEvent(s, ax.record(ax.s2), 0));
}

// X (n x ncols, ld ldx) <- Q X.
void tsqr_apply_q(hipStream_t s, const TsqrState& st, double* X, int64_t ldx, int64_t ncols) {
  if (ncols <= 0) return;
  for (int p = (int)st.panels.size() - 1; p >= 0; --p) {
    const TsqrPanel& P = st.panels[p];
    double* C = X + P.c0;
    const LevelRows lr = level_rows(P);
    for (int l = P.nlev - 1; l >= 0; --l) launch_apply(s, P.lev[l], l, P.pb, 0, lr, C, ldx, ncols);
  }
}

}  // namespace dme
