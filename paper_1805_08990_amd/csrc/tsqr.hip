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
// Leaf factorisation (256 threads = 32 columns x 8 row groups): the first 32
// rows of the leaf (where the diagonal of every reflector lies) stay in LDS,
// the other 256 rows in registers, thread (c, g) holding rows 32 + g + 8 r of
// column c.  Column step j makes one reduction: thread (c, g) sums
// x_j(i) a_c(i) over its rows i > j, which for c = j is sigma^2 of the
// reflector, for c > j the product that updates column c and for c < j the
// entry v_c^T v_j of the Gram matrix that builds T (the columns c < j are
// final, so their threads would be idle otherwise).  The column of step j is
// kept unscaled until the end, so no thread rewrites what another still reads.
#include "tsqr.h"

namespace dme {
namespace {

constexpr int kTB = 32;                   // panel width
constexpr int kTT = 256;                  // threads: 32 columns x 8 row groups
constexpr int kTG = kTT / kTB;            // row groups
constexpr int kTHead = kTB;               // head rows of a leaf (LDS)
constexpr int kTPer = 32;                 // body rows per thread (registers)
constexpr int kTLeaf = kTHead + kTG * kTPer;  // 288 rows per leaf
constexpr int kTHq = kTHead / kTG;        // head rows per row group
constexpr int kTAq = kTLeaf / kTG;        // rows per thread in the apply kernel (36)

// Rows of every level of a panel (kernel argument by value).
struct LevelRows {
  int64_t M[kTsqrMaxLevels];
};

// Level-l row s -> row of level 0, or -1 for a padding row (a leaf with fewer
// than 32 rows stacks zero rows that exist on no lower level).
__device__ inline int64_t phys_row(int64_t s, int level, const LevelRows& lr) {
  for (int l = level; l > 0; --l) {
    s = (s >> 5) * kTLeaf + (s & (kTB - 1));
    if (s >= lr.M[l - 1]) return -1;
  }
  return s;
}

// r_mode: 0 = R stays in place (single leaf of level 0); 1 = R_g stacked into
// Rdst rows 32 g .. 32 g + 31 (zeros below the diagonal); 2 = R's upper
// triangle written to Rdst (the panel's top rows in W).
__global__ __launch_bounds__(kTT) void tsqr_leaf_kernel(double* mat, int64_t ld, int64_t M, int pb,
                                                        double* Tout, double* Rdst, int64_t ld_r,
                                                        int r_mode) {
  __shared__ double H[kTHead][kTB + 1];  // head rows
  __shared__ double xb[2][kTPer][kTG];   // body rows of the step's column, [r][g]
  __shared__ double tot[kTB];            // the step's column sums
  __shared__ double Zs[kTB][kTB + 1];    // Zs[c][j] = v_c^T v_j for c < j
  __shared__ double coef[3][kTB];        // beta, tau, scale of each reflector
  const int t = threadIdx.x;
  const int c = t >> 3, g = t & (kTG - 1);
  const int64_t rbeg = (int64_t)blockIdx.x * kTLeaf;
  const int rows = (int)min<int64_t>(kTLeaf, M - rbeg);
  const int nv = min(rows, pb);
  double* base = mat + rbeg;
  const bool cin = c < pb;
#pragma unroll
  for (int q = 0; q < kTHq; ++q) {
    const int i = g + kTG * q;
    H[i][c] = (i < rows && cin) ? base[i + (int64_t)c * ld] : 0.0;
  }
  double vals[kTPer];
#pragma unroll
  for (int r = 0; r < kTPer; ++r) {
    const int i = kTHead + g + kTG * r;
    vals[r] = (i < rows && cin) ? base[i + (int64_t)c * ld] : 0.0;
  }
  if (c == 0) {
#pragma unroll
    for (int r = 0; r < kTPer; ++r) xb[0][r][g] = vals[r];
  }
  if (t < kTB) {
    coef[0][t] = 0.0;
    coef[1][t] = 0.0;
    coef[2][t] = 0.0;
  }
  __syncthreads();

  for (int j = 0; j < nv; ++j) {
    const int bf = j & 1;
    // partial sum over this thread's rows i > j of x_j(i) a_c(i)
    double part = 0.0;
#pragma unroll
    for (int r = 0; r < kTPer; ++r) part += xb[bf][r][g] * vals[r];
#pragma unroll
    for (int q = 0; q < kTHq; ++q) {
      const int i = g + kTG * q;
      if (i > j) part += H[i][j] * H[i][c];
    }
    const double ahead = H[j][c];  // read before row j is updated below
    part = group8_sum_f64(part);
    if (g == 0) tot[c] = part;
    __syncthreads();
    // reflector j (every thread forms the same values)
    const double alpha = H[j][j];
    const double s2 = tot[j];
    double beta = alpha, tau = 0.0, sc = 0.0;
    if (s2 != 0.0) {
      beta = -copysign(sqrt(alpha * alpha + s2), alpha);
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    const double tc = tot[c];
    if (c < j) {
      if (g == 0) Zs[c][j] = coef[2][c] * (ahead + sc * tc);
    } else if (c == j) {
      if (g == 0) {
        coef[0][j] = beta;
        coef[1][j] = tau;
        coef[2][j] = sc;
      }
    } else if (tau != 0.0) {
      // a_c -= tau v (v^T a_c), v = [1; sc x_j(i > j)]
      const double wv = tau * (ahead + sc * tc);
      const double f = wv * sc;
#pragma unroll
      for (int r = 0; r < kTPer; ++r) vals[r] -= f * xb[bf][r][g];
#pragma unroll
      for (int q = 0; q < kTHq; ++q) {
        const int i = g + kTG * q;
        if (i > j) H[i][c] -= f * H[i][j];
        else if (i == j) H[j][c] = ahead - wv;
      }
    }
    if (c == j + 1) {
#pragma unroll
      for (int r = 0; r < kTPer; ++r) xb[bf ^ 1][r][g] = vals[r];
    }
    __syncthreads();
  }

  // reflectors scaled in place, R in the upper part of the head rows
  if (c < nv) {
    const double scc = coef[2][c];
#pragma unroll
    for (int r = 0; r < kTPer; ++r) vals[r] *= scc;
#pragma unroll
    for (int q = 0; q < kTHq; ++q) {
      const int i = g + kTG * q;
      if (i > c) H[i][c] *= scc;
      else if (i == c) H[c][c] = coef[0][c];
    }
  }
  __syncthreads();
  if (cin) {
#pragma unroll
    for (int q = 0; q < kTHq; ++q) {
      const int i = g + kTG * q;
      if (i < rows) base[i + (int64_t)c * ld] = H[i][c];
    }
#pragma unroll
    for (int r = 0; r < kTPer; ++r) {
      const int i = kTHead + g + kTG * r;
      if (i < rows) base[i + (int64_t)c * ld] = vals[r];
    }
    if (r_mode == 1) {
#pragma unroll
      for (int q = 0; q < kTHq; ++q) {
        const int i = g + kTG * q;
        Rdst[(int64_t)blockIdx.x * kTB + i + (int64_t)c * ld_r] = (i <= c && i < rows) ? H[i][c] : 0.0;
      }
    } else if (r_mode == 2) {
#pragma unroll
      for (int q = 0; q < kTHq; ++q) {
        const int i = g + kTG * q;
        if (i <= c && i < rows) Rdst[i + (int64_t)c * ld_r] = H[i][c];
      }
    }
  }
  // T (upper triangular): T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) Zs(0:j, j);
  // lane cc forms row cc, which depends on its own earlier entries only
  if (t < kTB) {
    const int cc = t;
    double Trow[kTB];
#pragma unroll
    for (int j = 0; j < kTB; ++j) {
      double v = 0.0;
      if (j < nv && j >= cc) {
        if (j == cc) {
          v = coef[1][j];
        } else {
          double s = 0.0;
#pragma unroll
          for (int c2 = 0; c2 < j; ++c2)
            if (c2 >= cc) s += Trow[c2] * Zs[c2][j];
          v = -coef[1][j] * s;
        }
      }
      Trow[j] = v;
    }
    double* To = Tout + (int64_t)blockIdx.x * kTB * kTB;
#pragma unroll
    for (int j = 0; j < kTB; ++j) To[cc + j * kTB] = Trow[j];
  }
}

// C <- (I - V T' V^T) C for every leaf of one level, T' = T^T (trans: applies
// Q^T) or T.  Block (g, ct) handles leaf g and columns [32 ct, 32 ct + 32);
// thread (c, q8) holds the leaf rows q8 + 8 m.  V of leaf g: level matrix rows
// [288 g, 288 g + rows), unit diagonal implicit, zero above; C rows are this
// level's rows mapped to rows of level 0.
__global__ __launch_bounds__(kTT) void tsqr_apply_kernel(const double* V, int64_t ldv, int64_t M,
                                                         int pb, const double* Tin, int trans,
                                                         int level, LevelRows lr, double* C,
                                                         int64_t ldc, int64_t ncols) {
  __shared__ double Vs[kTLeaf][kTB + 1];
  __shared__ double Ys[kTB][kTB + 1];
  __shared__ double Zs[kTB][kTB + 1];
  __shared__ double Ts[kTB][kTB + 1];
  const int t = threadIdx.x;
  const int c = t >> 3, g = t & (kTG - 1);
  const int64_t rbeg = (int64_t)blockIdx.x * kTLeaf;
  const int rows = (int)min<int64_t>(kTLeaf, M - rbeg);
  const int nv = min(rows, pb);
  const int64_t col = (int64_t)blockIdx.y * kTB + c;
  const bool cok = col < ncols;
  for (int idx = t; idx < kTLeaf * kTB; idx += kTT) {
    const int i = idx % kTLeaf, a = idx / kTLeaf;
    double v = 0.0;
    if (i < rows && a < nv) v = (i > a) ? V[rbeg + i + (int64_t)a * ldv] : (i == a ? 1.0 : 0.0);
    Vs[i][a] = v;
  }
  {
    const double* Tg = Tin + (int64_t)blockIdx.x * kTB * kTB;
    for (int idx = t; idx < kTB * kTB; idx += kTT) {
      const int a = idx % kTB, b = idx / kTB;  // T(a, b)
      const double v = Tg[a + b * kTB];
      if (trans) Ts[b][a] = v;
      else Ts[a][b] = v;
    }
  }
  // rows of C this thread holds (-1: none); V is zero on padding rows
  double cr[kTAq];
  int64_t pr[kTAq];
#pragma unroll
  for (int m = 0; m < kTAq; ++m) {
    const int i = g + kTG * m;
    pr[m] = (i < rows && cok) ? phys_row(rbeg + i, level, lr) : -1;
    cr[m] = (pr[m] >= 0) ? C[pr[m] + col * ldc] : 0.0;
  }
  __syncthreads();
  // Y = V^T C: partial over this thread's rows, then summed over the 8 lanes
  // of the column
  double y[kTB];
#pragma unroll
  for (int a = 0; a < kTB; ++a) y[a] = 0.0;
#pragma unroll
  for (int m = 0; m < kTAq; ++m) {
    const int i = g + kTG * m;
#pragma unroll
    for (int a = 0; a < kTB; ++a) y[a] += Vs[i][a] * cr[m];
  }
#pragma unroll
  for (int a = 0; a < kTB; ++a) y[a] = group8_sum_f64(y[a]);
#pragma unroll
  for (int m = 0; m < kTB / kTG; ++m) {
    const int a = g + kTG * m;
    Ys[a][c] = y[a];
  }
  __syncthreads();
  // Z = T' Y (rows g + 8 m of column c)
#pragma unroll
  for (int m = 0; m < kTB / kTG; ++m) {
    const int a = g + kTG * m;
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < kTB; ++b) s += Ts[a][b] * Ys[b][c];
    Zs[a][c] = s;
  }
  __syncthreads();
  double z[kTB];
#pragma unroll
  for (int a = 0; a < kTB; ++a) z[a] = Zs[a][c];
  if (!cok) return;
#pragma unroll
  for (int m = 0; m < kTAq; ++m) {
    const int i = g + kTG * m;
    if (pr[m] >= 0) {
      double s = 0.0;
#pragma unroll
      for (int a = 0; a < kTB; ++a) s += Vs[i][a] * z[a];
      C[pr[m] + col * ldc] = cr[m] - s;
    }
  }
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

void tsqr_factor(hipStream_t s, int64_t n, int64_t k, double* W, TsqrState& st, Arena& ws) {
  const int64_t ld = n;
  const int64_t kr = std::min(n, k);
  st.n = n;
  st.k = k;
  st.ld = ld;
  st.W = W;
  st.panels.clear();
  for (int64_t c0 = 0; c0 < kr; c0 += kTB) {
    TsqrPanel P;
    P.c0 = c0;
    P.pb = (int)std::min<int64_t>(kTB, k - c0);
    const int pb = P.pb;
    int64_t M = n - c0;
    double* mat = W + c0 + c0 * ld;  // level 0 is the panel itself, in W
    int64_t mld = ld;
    for (int l = 0; l < kTsqrMaxLevels; ++l) {
      TsqrLevel& L = P.lev[l];
      L.M = M;
      L.G = (int)cdiv(M, kTLeaf);
      L.mat = mat;
      L.ld = mld;
      L.T = ws.get<double>((size_t)L.G * kTB * kTB);
      P.nlev = l + 1;
      if (L.G == 1) {
        // top: R into W rows [c0, c0 + pb) (a single leaf of level 0 holds it in place)
        hipLaunchKernelGGL(tsqr_leaf_kernel, dim3(1), dim3(kTT), 0, s, mat, mld, M, pb, L.T,
                           W + c0 + c0 * ld, ld, l > 0 ? 2 : 0);
        DME_HIP(hipGetLastError());
        break;
      }
      if (l + 1 == kTsqrMaxLevels) fail(DME_EINVAL, "tsqr: matrix too tall for the reduction tree");
      const int64_t Mn = (int64_t)L.G * kTB;
      double* next = ws.get<double>((size_t)Mn * pb);
      hipLaunchKernelGGL(tsqr_leaf_kernel, dim3((unsigned)L.G), dim3(kTT), 0, s, mat, mld, M, pb, L.T,
                         next, Mn, 1);
      DME_HIP(hipGetLastError());
      M = Mn;
      mat = next;
      mld = Mn;
    }
    // Q^T on the trailing columns, level by level
    const int64_t rest = k - c0 - pb;
    if (rest > 0) {
      double* C = W + c0 + (c0 + pb) * ld;
      const LevelRows lr = level_rows(P);
      for (int l = 0; l < P.nlev; ++l) {
        const TsqrLevel& L = P.lev[l];
        dim3 grid((unsigned)L.G, (unsigned)cdiv(rest, kTB));
        hipLaunchKernelGGL(tsqr_apply_kernel, grid, dim3(kTT), 0, s, L.mat, L.ld, L.M, pb, L.T, 1, l,
                           lr, C, ld, rest);
        DME_HIP(hipGetLastError());
      }
    }
    st.panels.push_back(P);
  }
}

// X (n x ncols, ld ldx) <- Q X.
void tsqr_apply_q(hipStream_t s, const TsqrState& st, double* X, int64_t ldx, int64_t ncols) {
  if (ncols <= 0) return;
  for (int p = (int)st.panels.size() - 1; p >= 0; --p) {
    const TsqrPanel& P = st.panels[p];
    double* C = X + P.c0;
    const LevelRows lr = level_rows(P);
    for (int l = P.nlev - 1; l >= 0; --l) {
      const TsqrLevel& L = P.lev[l];
      dim3 grid((unsigned)L.G, (unsigned)cdiv(ncols, kTB));
      hipLaunchKernelGGL(tsqr_apply_kernel, grid, dim3(kTT), 0, s, L.mat, L.ld, L.M, P.pb, L.T, 0, l,
                         lr, C, ldx, ncols);
      DME_HIP(hipGetLastError());
    }
  }
}

}  // namespace dme
