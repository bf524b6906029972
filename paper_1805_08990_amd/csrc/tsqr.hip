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

#include <memory>
#include <type_traits>

namespace dme {
namespace {

constexpr int kTB = 32;                   // panel width
constexpr int kTT = 256;                  // threads: 32 columns x 8 row groups
constexpr int kTG = kTT / kTB;            // row groups
constexpr int kTHead = kTB;               // head rows of a leaf (LDS)
constexpr int kTPer = 32;                 // body rows per thread (registers)
constexpr int kTLeaf = kTHead + kTG * kTPer;  // 288 rows per leaf
constexpr int kTHq = kTHead / kTG;        // head rows per row group

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
__global__ __launch_bounds__(kTT) void tsqr_leaf_kernel(double* mat, int64_t ld, int64_t M, int pb,
                                                        double* Tout, double* Rdst, int64_t ld_r,
                                                        int r_mode) {
  __shared__ double H[kTHead][kTB + 1];  // head rows
  __shared__ double xb[2][kTG][kTPer + 2];  // body rows of the step's column, [g][r] (padded: no bank conflicts)
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
  // loads are unconditional (clamped to an entry of the block) and masked
  // afterwards, so they are all in flight together
  const int64_t cc0 = (int64_t)min(c, pb - 1) * ld;
#pragma unroll
  for (int q = 0; q < kTHq; ++q) {
    const int i = g + kTG * q;
    const bool ok = i < rows && cin;
    const double v = base[min(i, rows - 1) + cc0];
    H[i][c] = ok ? v : 0.0;
  }
  double vals[kTPer];
#pragma unroll
  for (int r = 0; r < kTPer; ++r) {
    const int i = kTHead + g + kTG * r;
    const bool ok = i < rows && cin;
    const double v = base[min(i, rows - 1) + cc0];
    vals[r] = ok ? v : 0.0;
  }
  if (c == 0) {
#pragma unroll
    for (int r = 0; r < kTPer; ++r) xb[0][g][r] = vals[r];
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
    double xv[kTPer];  // body rows of column j, kept for the update below
#pragma unroll
    for (int r = 0; r < kTPer; ++r) xv[r] = xb[bf][g][r];
    double pp[4] = {0.0, 0.0, 0.0, 0.0};  // independent chains
#pragma unroll
    for (int r = 0; r < kTPer; ++r) pp[r & 3] += xv[r] * vals[r];
#pragma unroll
    for (int q = 0; q < kTHq; ++q) {
      const int i = g + kTG * q;
      if (i > j) pp[q] += H[i][j] * H[i][c];
    }
    double part = (pp[0] + pp[1]) + (pp[2] + pp[3]);
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
      for (int r = 0; r < kTPer; ++r) vals[r] -= f * xv[r];
#pragma unroll
      for (int q = 0; q < kTHq; ++q) {
        const int i = g + kTG * q;
        if (i > j) H[i][c] -= f * H[i][j];
        else if (i == j) H[j][c] = ahead - wv;
      }
    }
    if (c == j + 1) {
#pragma unroll
      for (int r = 0; r < kTPer; ++r) xb[bf ^ 1][g][r] = vals[r];
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
  // (branch-free: entries outside the triangle are zero)
  if (t < kTB) {
    const int cc = t;
    double Trow[kTB];
#pragma unroll
    for (int j = 0; j < kTB; ++j) {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int c2 = 0; c2 < j; ++c2) {  // Trow[c2] is zero for c2 < cc
        if (c2 & 1) s1 += Trow[c2] * Zs[c2][j];
        else s0 += Trow[c2] * Zs[c2][j];
      }
      const double tj = coef[1][j];
      const double v = (j == cc) ? tj : -tj * (s0 + s1);
      Trow[j] = (j < nv && j >= cc) ? v : 0.0;
    }
    double* To = Tout + (int64_t)blockIdx.x * kTB * kTB;
#pragma unroll
    for (int j = 0; j < kTB; ++j) To[cc + j * kTB] = Trow[j];
  }
}

// C <- (I - V T' V^T) C for every leaf of one level, T' = T^T (trans: applies
// Q^T) or T, on FP64 MFMA.  Block (g, ct) handles leaf g (288 rows) and the
// columns [32 ct, 32 ct + 32).  The leaf's V (with its implicit unit
// diagonal) is staged in LDS and the block's C entries are loaded into
// registers, all loads issued together.  Wave w takes the 16 x 16 tile
// (w / 2, w % 2) of Y = V^T C (72 MFMAs over the leaf's rows), the block forms
// Z = T' Y in LDS, and wave w then updates rows [144 (w / 2), 144 (w / 2) + 144)
// of column tile w % 2 with 72 more MFMAs.  The C entries a lane feeds to the
// first product are exactly the ones its result lanes hold in the second, so
// C is read once and written once.  V of leaf g: level matrix rows
// [288 g, 288 g + rows), unit diagonal implicit, zero above; C rows are this
// level's rows mapped to rows of level 0 (padding rows read as zero and are
// not written).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTSteps = kTLeaf / 4;  // 72 K-steps of the MFMA over a leaf
constexpr int kTVld = (kTLeaf * kTB) / kTT;  // V entries staged per thread (36)

template <int LEVEL>
__global__ __launch_bounds__(kTT) void tsqr_apply_kernel(const double* V, int64_t ldv, int64_t M,
                                                         int pb, const double* Tin, int trans,
                                                         LevelRows lr, double* C, int64_t ldc,
                                                         int64_t ncols) {
  __shared__ double Vs[kTLeaf][kTB + 1];
  __shared__ double Ys[kTB][kTB + 1];
  __shared__ double Zs[kTB][kTB + 1];
  __shared__ double Ts[kTB][kTB + 1];
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int at = w >> 1, ct = w & 1;
  const int64_t rbeg = (int64_t)blockIdx.x * kTLeaf;
  const int rows = (int)min<int64_t>(kTLeaf, M - rbeg);
  const int nv = min(rows, pb);
  const int64_t col = (int64_t)blockIdx.y * kTB + ct * 16 + li;
  const bool cok = col < ncols;
  // rows of C (n < 2^31), -1 for none
  auto crow = [&](int s) -> int {
    const int i = 4 * s + lk;
    return (i < rows && cok) ? (int)phys_row<LEVEL>(rbeg + i, lr) : -1;
  };
  // every load is unconditional (clamped) and masked afterwards, so all are in flight together
  double vst[kTVld];
#pragma unroll
  for (int m = 0; m < kTVld; ++m) {
    const int idx = t + kTT * m;
    const int i = idx % kTLeaf, a = idx / kTLeaf;
    vst[m] = V[rbeg + min(i, rows - 1) + (int64_t)min(a, pb - 1) * ldv];
  }
  double cr[kTSteps];
#pragma unroll
  for (int s = 0; s < kTSteps; ++s) {
    const int pr = crow(s);
    const double cv = C[(pr >= 0) ? (int64_t)pr + col * ldc : 0];
    cr[s] = (pr >= 0) ? cv : 0.0;
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
#pragma unroll
  for (int m = 0; m < kTVld; ++m) {
    const int idx = t + kTT * m;
    const int i = idx % kTLeaf, a = idx / kTLeaf;
    const double y = (i > a) ? vst[m] : (i == a ? 1.0 : 0.0);
    Vs[i][a] = (i < rows && a < nv) ? y : 0.0;
  }
  __syncthreads();
  // phase 1: Y tile (at, ct) = sum over the leaf rows of V(:, at*16 + .)^T C(:, ct*16 + .)
  // (operands read from LDS 8 steps at a time, ahead of their MFMAs)
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s0 = 0; s0 < kTSteps; s0 += 8) {
    double va[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) va[u] = Vs[4 * (s0 + u) + lk][at * 16 + li];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], cr[s0 + u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) Ys[at * 16 + 4 * v + lk][ct * 16 + li] = acc[v];
  __syncthreads();
  // Z = T' Y: thread (zr, zc) forms rows zr, zr + 8, zr + 16, zr + 24 of column zc
  {
    const int zc = t & 31, zr = t >> 5;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int a = zr + 8 * m;
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < kTB; ++b) s += Ts[a][b] * Ys[b][zc];
      Zs[a][zc] = s;
    }
  }
  __syncthreads();
  double zb[kTB / 4];
#pragma unroll
  for (int q = 0; q < kTB / 4; ++q) zb[q] = Zs[4 * q + lk][ct * 16 + li];
  // phase 3: rows of tiles rt = at * 9 .. at * 9 + 8 of column tile ct
  auto update = [&](auto base_tag) {
    constexpr int R0 = decltype(base_tag)::value;
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      const int rt = R0 + r;
      double va[kTB / 4];
#pragma unroll
      for (int q = 0; q < kTB / 4; ++q) va[q] = Vs[rt * 16 + li][4 * q + lk];
      v4d p = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kTB / 4; ++q) p = __builtin_amdgcn_mfma_f64_16x16x4f64(va[q], zb[q], p, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int s = 4 * rt + v;
        const int pr = crow(s);
        if (pr >= 0) C[(int64_t)pr + col * ldc] = cr[s] - p[v];
      }
    }
  };
  if (at == 0) update(std::integral_constant<int, 0>{});
  else update(std::integral_constant<int, 9>{});
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

// A second stream and a ring of events per host thread and device, for the
// look-ahead of the panel factorisation (default priority, created on first
// use; they are not destroyed, since a thread's end may come after the
// runtime's).
struct AuxStream {
  int device = -1;
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> ev;
  size_t next = 0;
  // A recorded event is only waited on by calls enqueued right after its
  // record, so a ring much longer than the waits in flight can be reused.
  hipEvent_t record(hipStream_t st) {
    hipEvent_t e = ev[next];
    next = (next + 1) % ev.size();
    DME_HIP(hipEventRecord(e, st));
    return e;
  }
};

AuxStream& aux_stream() {
  static thread_local std::vector<std::unique_ptr<AuxStream>> per_device;
  int dev = 0;
  DME_HIP(hipGetDevice(&dev));
  for (auto& a : per_device)
    if (a->device == dev) return *a;
  auto a = std::make_unique<AuxStream>();
  a->device = dev;
  DME_HIP(hipStreamCreateWithFlags(&a->s2, hipStreamNonBlocking));
  a->ev.resize(64);
  for (hipEvent_t& e : a->ev) DME_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  per_device.push_back(std::move(a));
  return *per_device.back();
}

}  // namespace

// Panels are factored on s.  Q^T of panel p reaches the next panel's columns
// on s (they are what panel p + 1 factors next) and the columns beyond on a
// second stream, which waits for each tree level's factor and runs behind
// the factorisation of the following panels; s waits for that stream before
// it touches those columns (and before returning).
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
  // the second stream starts after everything s has queued so far (W is ready)
  DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
  for (int64_t c0 = 0; c0 < kr; c0 += kTB) {
    TsqrPanel P;
    P.c0 = c0;
    P.pb = (int)std::min<int64_t>(kTB, k - c0);
    const int pb = P.pb;
    int64_t M = n - c0;
    double* mat = W + c0 + c0 * ld;  // level 0 is the panel itself, in W
    int64_t mld = ld;
    hipEvent_t lev_done[kTsqrMaxLevels] = {};
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
        lev_done[l] = ax.record(s);
        break;
      }
      if (l + 1 == kTsqrMaxLevels) fail(DME_EINVAL, "tsqr: matrix too tall for the reduction tree");
      const int64_t Mn = (int64_t)L.G * kTB;
      double* next = ws.get<double>((size_t)Mn * pb);
      hipLaunchKernelGGL(tsqr_leaf_kernel, dim3((unsigned)L.G), dim3(kTT), 0, s, mat, mld, M, pb, L.T,
                         next, Mn, 1);
      DME_HIP(hipGetLastError());
      lev_done[l] = ax.record(s);
      M = Mn;
      mat = next;
      mld = Mn;
    }
    const LevelRows lr = level_rows(P);
    const int64_t rest = k - c0 - pb;
    const int64_t near = std::min<int64_t>(rest, kTB);  // the next panel's columns
    const int64_t far = rest - near;
    // Q^T on the columns beyond the next panel: second stream, level by level
    if (far > 0) {
      double* C = W + c0 + (c0 + pb + near) * ld;
      for (int l = 0; l < P.nlev; ++l) {
        DME_HIP(hipStreamWaitEvent(ax.s2, lev_done[l], 0));
        launch_apply(ax.s2, P.lev[l], l, pb, 1, lr, C, ld, far);
      }
      aux_used = true;
    }
    // Q^T on the next panel's columns, on s, after the previous panels' share
    // of the second stream (it updated these columns too)
    if (near > 0) {
      if (rest_done) DME_HIP(hipStreamWaitEvent(s, rest_done, 0));
      double* C = W + c0 + (c0 + pb) * ld;
      for (int l = 0; l < P.nlev; ++l) launch_apply(s, P.lev[l], l, pb, 1, lr, C, ld, near);
    }
    if (far > 0) rest_done = ax.record(ax.s2);
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
