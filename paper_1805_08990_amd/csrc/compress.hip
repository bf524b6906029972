// Column compression of P = W Dhat W^T (the step that follows every
// concatenation in Alg. 1, 2 and 4; method described in Sec. 3 after Alg. 2):
//
//   Householder QR   W = Q R            (blocked, panel width kQB, FP64)
//   small product    M = R Dhat R^T     (FP64 MFMA GEMM)
//   eigenpairs       M = V Lam V^T      (syev.hip), keep |lam| > tol max|lam|
//   new factor       L = Q [V_I; 0],  D = diag(Lam_I)
//
// QR panel: one launch per column; each launch finishes the reflector of the
// previous column from the partial sums the previous launch wrote (every
// block reduces them in the same fixed order), applies it to the rows the
// block owns (one thread per row) and writes the partial sums x^T x and
// x^T a_j of the next column.  The panel's reflectors are then aggregated
// into the compact WY form I - V T V^T and applied to the trailing columns
// with three GEMMs; the same form applies Q to [V_I; 0] at the end.
#include "common.h"

namespace dme {
namespace {

constexpr int kQB = 32;     // QR panel width
constexpr int kQRT = 256;   // rows per block in the panel kernels
constexpr int kQParts = kQB + 1;

// One launch per column c of a panel [c0, c0 + pb):
//  (1) if c > c0, every block reduces (in a fixed order) the partial sums of
//      column p = c - 1 that the previous launch wrote, and forms beta_p, tau_p,
//      the scale of v_p and w_j = tau_p v_p^T a_j for the panel columns j >= c;
//      all blocks get identical values, block 0 stores beta_p, tau_p, scale_p;
//  (2) applies reflector p to the panel rows this block owns;
//  (3) if do_part, writes this block's partial sums over rows i > c of
//      [x^T x, x^T a_{c+1}, ..., x^T a_{c0+pb-1}] (x = column c), and the
//      thread owning row c writes that row's panel entries.
// Partial sums and the row alternate between two buffers (launch c writes
// set c & 1 and reads set (c - 1) & 1), so no launch overwrites what another
// block of the same launch still reads.
__global__ __launch_bounds__(kQRT) void qr_step_kernel(double* W, int64_t ld, int64_t n, int64_t c0,
                                                       int pb, int64_t c, int do_part,
                                                       const double* part_prev, int nparts_prev,
                                                       const double* row_prev, double* part_cur,
                                                       double* row_cur, double* beta, double* tau,
                                                       double* scale) {
  constexpr int kGroups = kQRT / kQB;  // partial-sum groups of the prologue reduction
  __shared__ double red[kQRT / 64][kQParts];
  __shared__ double sred[kGroups][kQB];
  __shared__ double tot[kQParts];
  __shared__ double wcol[kQB];
  __shared__ double bsc[3];  // beta, scale, tau of reflector c - 1
  const int64_t cend = c0 + pb;
  const int ncol = (int)(cend - c);  // panel columns >= c
  if (c > c0) {
    const int64_t p = c - 1;
    const int ncp = ncol + 1;  // panel columns >= p (at most kQB here)
    {
      // thread (g, q) sums the partials b = g, g + kGroups, ... of entry q
      // (independent loads, unrolled), then entry q adds the groups in order
      const int q = threadIdx.x % kQB, g = threadIdx.x / kQB;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      if (q < ncp) {
        int b = g;
        for (; b + 3 * kGroups < nparts_prev; b += 4 * kGroups) {
          a0 += part_prev[(int64_t)b * kQParts + q];
          a1 += part_prev[(int64_t)(b + kGroups) * kQParts + q];
          a2 += part_prev[(int64_t)(b + 2 * kGroups) * kQParts + q];
          a3 += part_prev[(int64_t)(b + 3 * kGroups) * kQParts + q];
        }
        for (; b < nparts_prev; b += kGroups) a0 += part_prev[(int64_t)b * kQParts + q];
      }
      sred[g][q] = (a0 + a1) + (a2 + a3);
    }
    __syncthreads();
    if (threadIdx.x < ncp) {
      double sacc = 0.0;
      for (int g = 0; g < kGroups; ++g) sacc += sred[g][threadIdx.x];
      tot[threadIdx.x] = sacc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double alpha = row_prev[0];
      const double sig2 = tot[0];
      double b, t, sc;
      if (sig2 == 0.0) {
        b = alpha; t = 0.0; sc = 0.0;
      } else {
        b = -copysign(sqrt(alpha * alpha + sig2), alpha);
        t = (b - alpha) / b;
        sc = 1.0 / (alpha - b);
      }
      bsc[0] = b;
      bsc[1] = sc;
      if (blockIdx.x == 0) { beta[p] = b; tau[p] = t; scale[p] = sc; }
      bsc[2] = t;
    }
    __syncthreads();
    const double t = bsc[2];
    const double sc = bsc[1];
    for (int q = threadIdx.x; q < ncol; q += kQRT) wcol[q] = t * (row_prev[q + 1] + sc * tot[q + 1]);
    __syncthreads();
  }
  const int64_t rs = (c > c0) ? c - 1 : c;
  const int64_t i = rs + (int64_t)blockIdx.x * kQRT + threadIdx.x;
  double vals[kQB];
#pragma unroll
  for (int q = 0; q < kQB; ++q) vals[q] = 0.0;
  if (i < n) {
#pragma unroll
    for (int q = 0; q < kQB; ++q)
      if (q < ncol) vals[q] = W[i + (c + q) * ld];
    if (c > c0) {
      const int64_t p = c - 1;
      double vi;
      if (i == p) {
        vi = 1.0;
        W[p + p * ld] = bsc[0];
      } else {
        vi = bsc[1] * W[i + p * ld];
        W[i + p * ld] = vi;
      }
#pragma unroll
      for (int q = 0; q < kQB; ++q) {
        if (q < ncol) {
          vals[q] -= vi * wcol[q];
          W[i + (c + q) * ld] = vals[q];
        }
      }
    }
  }
  if (!do_part) return;
  if (i == c) {
#pragma unroll
    for (int q = 0; q < kQB; ++q)
      if (q < ncol) row_cur[q] = vals[q];
  }
  // partial sums over rows i > c
  const bool use = (i < n) && (i > c);
  const double x = use ? vals[0] : 0.0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < kQB; ++q) {
    if (q < ncol) {
      double v = use ? x * vals[q] : 0.0;
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wv][q] = v;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ncol; q += kQRT) {
    double sacc = 0.0;
    for (int w = 0; w < kQRT / 64; ++w) sacc += red[w][q];
    part_cur[(int64_t)blockIdx.x * kQParts + q] = sacc;
  }
}

// Explicit V of a panel: Vp(i, q) for rows i in [0, n - c0), q in [0, nv).
__global__ void qr_vpanel_kernel(const double* W, int64_t ld, int64_t n, int64_t c0, int nv,
                                 double* Vp, int64_t ldv) {
  const int64_t rows = n - c0;
  const int64_t total = rows * nv;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % rows;
    const int q = (int)(idx / rows);
    double v;
    if (r > q) v = W[(c0 + r) + (c0 + q) * ld];
    else v = (r == q) ? 1.0 : 0.0;
    Vp[r + q * ldv] = v;
  }
}

// Compact WY factor T (nv x nv upper) from G = Vp^T Vp and tau.
__global__ void qr_tmat_kernel(const double* G, int nv, const double* tau, double* T) {
  __shared__ double z[kQB];
  const int r = threadIdx.x;
  for (int idx = r; idx < nv * nv; idx += blockDim.x) T[idx] = 0.0;
  __syncthreads();
  for (int i = 0; i < nv; ++i) {
    const double ti = tau[i];
    if (r < i) z[r] = G[r + i * nv];
    __syncthreads();
    if (r < i) {
      double s = 0.0;
      for (int t = r; t < i; ++t) s += T[r + t * nv] * z[t];
      T[r + i * nv] = -ti * s;
    }
    if (r == i) T[i + i * nv] = ti;
    __syncthreads();
  }
}

// R (kr x k, ld kr) = upper trapezoid of W(0:kr, 0:k).
__global__ void extract_r_kernel(const double* W, int64_t ld, int64_t kr, int64_t k, double* R) {
  const int64_t total = kr * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % kr, c = idx / kr;
    R[r + c * kr] = (r <= c) ? W[r + c * ld] : 0.0;
  }
}

// M <- (M + M^T) / 2, in a separate output.
__global__ void symmetrize_kernel(const double* M, int64_t k, double* S) {
  const int64_t total = k * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = idx % k, c = idx / k;
    S[idx] = 0.5 * (M[r + c * k] + M[c + r * k]);
  }
}

// X (n x r, ld ldx) = [V (kr x r, ld ldv); 0]
__global__ void embed_kernel(const double* V, int64_t ldv, int64_t kr, int64_t n, int64_t r,
                             double* X, int64_t ldx) {
  const int64_t total = n * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % n, c = idx / n;
    X[i + c * ldx] = (i < kr) ? V[i + c * ldv] : 0.0;
  }
}

// D (r x r, ld ldd) = diag(lam[0..r))
__global__ void diag_kernel(const double* lam, int64_t r, double* D, int64_t ldd) {
  const int64_t total = r * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % r, c = idx / r;
    D[i + c * ldd] = (i == c) ? lam[i] : 0.0;
  }
}

inline unsigned blocks_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(total, 256), 8192));
}

}  // namespace

size_t compress_workspace(int64_t n, int64_t k) {
  const int64_t kr = std::min(n, k);
  const int64_t np = cdiv(std::max<int64_t>(kr, 1), kQB);
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add((size_t)n * k * sizeof(double));          // Vp (all panels)
  add((size_t)np * kQB * kQB * sizeof(double)); // T
  add(4 * (size_t)k * sizeof(double));          // beta, tau, scale, lam
  add(2 * (size_t)(cdiv(n, kQRT) + 2) * kQParts * sizeof(double));  // partial sums (two sets)
  add(2 * kQParts * sizeof(double));                                  // pivot rows (two sets)
  add(2 * (size_t)kQB * k * sizeof(double));    // Y, Y2
  add(4 * (size_t)k * k * sizeof(double));      // R, T1, M, S
  add((size_t)k * k * sizeof(double));          // V
  add(syev_workspace(k));
  // largest split-K GEMM issued: Vp^T (n x kQB) times n x k
  size_t g = std::max(gemm_f64_workspace(kQB, k, n), gemm_f64_workspace(kQB, kQB, n));
  g = std::max(g, gemm_f64_workspace(k, k, k));
  g = std::max(g, gemm_f64_workspace(n, k, kQB));
  add(g);
  return b + 4096;
}

int64_t compress_f64(hipStream_t s, int64_t n, int64_t k, double* W, const double* Dhat,
                     double tol, int64_t max_rank, double* L, int64_t ldl, double* Dout,
                     int64_t ldd, int64_t* rank_dev, int* flag_dev, Arena& ws) {
  if (k <= 0 || n <= 0) {
    return 0;
  }
  const int64_t ld = n;
  const int64_t kr = std::min(n, k);
  const int64_t np = cdiv(kr, kQB);
  double* Vp = ws.get<double>((size_t)n * k);
  double* Tm = ws.get<double>((size_t)np * kQB * kQB);
  double* beta = ws.get<double>(k);
  double* tau = ws.get<double>(k);
  double* scale = ws.get<double>(k);
  double* lam = ws.get<double>(k);
  double* part[2];
  double* rowb[2];
  for (int q = 0; q < 2; ++q) {
    part[q] = ws.get<double>((size_t)(cdiv(n, kQRT) + 2) * kQParts);
    rowb[q] = ws.get<double>(kQParts);
  }
  double* Y = ws.get<double>((size_t)kQB * k);
  double* Y2 = ws.get<double>((size_t)kQB * k);
  double* R = ws.get<double>((size_t)k * k);
  double* T1 = ws.get<double>((size_t)k * k);
  double* M = ws.get<double>((size_t)k * k);
  double* S = ws.get<double>((size_t)k * k);
  double* V = ws.get<double>((size_t)k * k);
  const size_t mark = ws.used;

  // ---------------- Householder QR
  for (int64_t p = 0; p < np; ++p) {
    const int64_t c0 = p * kQB;
    const int pb = (int)std::min<int64_t>(kQB, k - c0);       // panel columns (incl. beyond kr)
    const int nv = (int)std::min<int64_t>(kQB, kr - c0);      // reflectors in this panel
    int nparts_prev = 0;
    for (int64_t c = c0; c <= c0 + nv; ++c) {
      const int do_part = (c < c0 + nv) ? 1 : 0;
      const int64_t rs = (c > c0) ? c - 1 : c;
      const int nb = (int)cdiv(n - rs, kQRT);
      const int cur = (int)(c & 1), prev = cur ^ 1;
      hipLaunchKernelGGL(qr_step_kernel, dim3(nb), dim3(kQRT), 0, s, W, ld, n, c0, pb, c, do_part,
                         part[prev], nparts_prev, rowb[prev], part[cur], rowb[cur], beta, tau, scale);
      DME_HIP(hipGetLastError());
      nparts_prev = nb;
    }
    // compact WY of this panel
    double* Vpp = Vp + c0 * n;  // panel p's V, rows [0, n - c0), ld n
    hipLaunchKernelGGL(qr_vpanel_kernel, dim3(blocks_for((n - c0) * nv)), dim3(256), 0, s, W, ld, n,
                       c0, nv, Vpp, n);
    DME_HIP(hipGetLastError());
    double* Tp = Tm + p * kQB * kQB;
    ws.used = mark;
    gemm_f64(s, 'T', 'N', nv, nv, n - c0, 1.0, Vpp, n, Vpp, n, 0.0, Y, nv, &ws);
    hipLaunchKernelGGL(qr_tmat_kernel, dim3(1), dim3(64), 0, s, Y, nv, tau + c0, Tp);
    DME_HIP(hipGetLastError());
    const int64_t rest = k - c0 - pb;
    if (rest > 0) {
      double* Wt = W + c0 + (c0 + pb) * ld;
      ws.used = mark;
      gemm_f64(s, 'T', 'N', nv, rest, n - c0, 1.0, Vpp, n, Wt, ld, 0.0, Y, nv, &ws);
      ws.used = mark;
      gemm_f64(s, 'T', 'N', nv, rest, nv, 1.0, Tp, nv, Y, nv, 0.0, Y2, nv, &ws);
      ws.used = mark;
      gemm_f64(s, 'N', 'N', n - c0, rest, nv, -1.0, Vpp, n, Y2, nv, 1.0, Wt, ld, &ws);
    }
  }

  // ---------------- M = R Dhat R^T, symmetrised
  hipLaunchKernelGGL(extract_r_kernel, dim3(blocks_for(kr * k)), dim3(256), 0, s, W, ld, kr, k, R);
  DME_HIP(hipGetLastError());
  ws.used = mark;
  gemm_f64(s, 'N', 'N', kr, k, k, 1.0, R, kr, Dhat, k, 0.0, T1, kr, &ws);
  ws.used = mark;
  gemm_f64(s, 'N', 'T', kr, kr, k, 1.0, T1, kr, R, kr, 0.0, M, kr, &ws);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for(kr * kr)), dim3(256), 0, s, M, kr, S);
  DME_HIP(hipGetLastError());
  finite_check_f64(s, S, kr, kr, kr, flag_dev);

  // ---------------- eigenpairs with truncation
  ws.used = mark;
  syev_trunc_f64(s, kr, S, kr, tol, std::min(max_rank, kr), lam, V, kr, rank_dev, flag_dev, ws);
  int64_t r = 0;
  DME_HIP(hipMemcpyAsync(&r, rank_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  if (r <= 0) return 0;
  if (ldd <= 0) ldd = r;

  // ---------------- L = Q [V_I; 0], D = diag(lam_I)
  hipLaunchKernelGGL(embed_kernel, dim3(blocks_for(n * r)), dim3(256), 0, s, V, kr, kr, n, r, L, ldl);
  DME_HIP(hipGetLastError());
  for (int64_t p = np - 1; p >= 0; --p) {
    const int64_t c0 = p * kQB;
    const int nv = (int)std::min<int64_t>(kQB, kr - c0);
    double* Vpp = Vp + c0 * n;
    double* Tp = Tm + p * kQB * kQB;
    double* Xp = L + c0;
    ws.used = mark;
    gemm_f64(s, 'T', 'N', nv, r, n - c0, 1.0, Vpp, n, Xp, ldl, 0.0, Y, nv, &ws);
    ws.used = mark;
    gemm_f64(s, 'N', 'N', nv, r, nv, 1.0, Tp, nv, Y, nv, 0.0, Y2, nv, &ws);
    ws.used = mark;
    gemm_f64(s, 'N', 'N', n - c0, r, nv, -1.0, Vpp, n, Y2, nv, 1.0, Xp, ldl, &ws);
  }
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(r * r)), dim3(256), 0, s, lam, r, Dout, ldd);
  DME_HIP(hipGetLastError());
  ws.used = mark;
  return r;
}

}  // namespace dme
