// Riccati subflow on the small factor (Sec. 2.2, exact solution of
// dP/dt = -P B R^-1 B^T P and its low-rank form; Alg. 3 with the B^T of the
// Sec. 2.2 formula):
//
//     D <- (I + t D W R^-1 W^T)^-1 D,    W = L^T B  (r x m)
//
// evaluated through the Woodbury identity as the symmetric m x m form
//
//     Y = D W,  S = R + t W^T Y = Lc Lc^T (Cholesky),  Z = Y Lc^-T,
//     D <- sym(D) - t Z Z^T,
//
// so only an m x m system is factored (m = number of inputs, <= 64 here).
// A non-SPD S (which cannot happen for SPD R and PSD D) raises flag bit 4.
#include "common.h"

namespace dme {
namespace {

constexpr int kRT = 1024;
constexpr int kMaxM = 64;

// One workgroup; every loop keeps several independent loads in flight (the
// step is a latency-bound chain of small products).
__global__ __launch_bounds__(kRT) void riccati_kernel(int r, int m, double* D, int64_t ldd,
                                                      const double* WB, int64_t ldw, const double* R,
                                                      int64_t ldr, double t, double* Y, int* flag) {
  __shared__ double S[kMaxM * kMaxM];
  __shared__ double part[kRT];
  __shared__ int bad;
  const int tid = threadIdx.x;
  // Y = D W  (r x m, ld r): four independent chains over l
  for (int idx = tid; idx < r * m; idx += kRT) {
    const int i = idx % r, a = idx / r;
    const double* dr = D + i;
    const double* wc = WB + (int64_t)a * ldw;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int l = 0;
    for (; l + 4 <= r; l += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += dr[(int64_t)(l + u) * ldd] * wc[l + u];
    }
    for (; l < r; ++l) acc[0] += dr[(int64_t)l * ldd] * wc[l];
    Y[i + (int64_t)a * r] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  __syncthreads();
  // S = R + t W^T Y: with m^2 <= kRT, slice sl of entry o sums rows i = sl mod ns
  // and the slices are added in order; otherwise one thread per entry
  const int mm = m * m;
  if (mm <= kRT) {
    const int ns = kRT / mm;
    const int o = tid % mm, sl = tid / mm;
    double acc = 0.0;
    if (sl < ns) {
      const int a = o % m, b = o / m;
      const double* wa = WB + (int64_t)a * ldw;
      const double* yb = Y + (int64_t)b * r;
      for (int i = sl; i < r; i += ns) acc += wa[i] * yb[i];
    }
    part[tid] = acc;
    __syncthreads();
    if (tid < mm) {
      double tot = 0.0;
      for (int q = 0; q < ns; ++q) tot += part[tid + q * mm];
      const int a = tid % m, b = tid / m;
      S[a + b * kMaxM] = R[a + (int64_t)b * ldr] + t * tot;
    }
  } else {
    for (int idx = tid; idx < mm; idx += kRT) {
      const int a = idx % m, b = idx / m;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      int i = 0;
      for (; i + 4 <= r; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += WB[i + u + (int64_t)a * ldw] * Y[i + u + (int64_t)b * r];
      }
      for (; i < r; ++i) acc[0] += WB[i + (int64_t)a * ldw] * Y[i + (int64_t)b * r];
      S[a + b * kMaxM] = R[a + (int64_t)b * ldr] + t * ((acc[0] + acc[1]) + (acc[2] + acc[3]));
    }
  }
  __syncthreads();
  // Cholesky (lower) of the symmetrised S, serial: m is tiny
  if (tid == 0) {
    bad = 0;
    for (int a = 0; a < m; ++a)
      for (int b = a + 1; b < m; ++b) {
        const double v = 0.5 * (S[a + b * kMaxM] + S[b + a * kMaxM]);
        S[a + b * kMaxM] = v;
        S[b + a * kMaxM] = v;
      }
    for (int j = 0; j < m && !bad; ++j) {
      double dj = S[j + j * kMaxM];
      for (int q = 0; q < j; ++q) dj -= S[j + q * kMaxM] * S[j + q * kMaxM];
      if (!(dj > 0.0)) { bad = 1; break; }
      const double ljj = sqrt(dj);
      S[j + j * kMaxM] = ljj;
      for (int i = j + 1; i < m; ++i) {
        double v = S[i + j * kMaxM];
        for (int q = 0; q < j; ++q) v -= S[i + q * kMaxM] * S[j + q * kMaxM];
        S[i + j * kMaxM] = v / ljj;
      }
    }
    if (bad) atomicOr(flag, 4);
  }
  __syncthreads();
  if (bad) return;
  // Z = Y Lc^-T : row i solves z Lc^T = y (forward substitution), in place in Y
  for (int i = tid; i < r; i += kRT) {
    for (int a = 0; a < m; ++a) {
      double v = Y[i + (int64_t)a * r];
      for (int b = 0; b < a; ++b) v -= Y[i + (int64_t)b * r] * S[a + b * kMaxM];
      Y[i + (int64_t)a * r] = v / S[a + a * kMaxM];
    }
  }
  __syncthreads();
  // D <- sym(D) - t Z Z^T in place: one thread per pair i <= j reads D(i, j)
  // and D(j, i) and writes both (pair p -> column j, row i of the upper triangle)
  const int np = r * (r + 1) / 2;
#pragma unroll 4
  for (int pidx = tid; pidx < np; pidx += kRT) {
    int j = (int)((sqrt(8.0 * pidx + 1.0) - 1.0) * 0.5);
    while (j * (j + 1) / 2 > pidx) --j;
    while ((j + 1) * (j + 2) / 2 <= pidx) ++j;
    const int i = pidx - j * (j + 1) / 2;  // 0 <= i <= j
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += Y[i + (int64_t)a * r] * Y[j + (int64_t)a * r];
    const double v = 0.5 * (D[i + (int64_t)j * ldd] + D[j + (int64_t)i * ldd]) - t * acc;
    D[i + (int64_t)j * ldd] = v;
    D[j + (int64_t)i * ldd] = v;
  }
}

// X (m x r, ld m) = R^-1 Z^T for Z (r x m, ld r): Cholesky of R (m <= kMaxM)
// by one thread, then one thread per column of Z^T (forward and backward
// substitution).  A non-SPD R raises flag bit 4.
__global__ __launch_bounds__(256) void gain_solve_kernel(int m, int r, const double* R, int64_t ldr,
                                                         const double* Z, double* X, int* flag) {
  __shared__ double Lc[kMaxM * kMaxM];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < m * m; idx += blockDim.x) {
    const int a = idx % m, b = idx / m;
    Lc[a + b * kMaxM] = 0.5 * (R[a + (int64_t)b * ldr] + R[b + (int64_t)a * ldr]);
  }
  __syncthreads();
  if (tid == 0) {
    bad = 0;
    for (int j = 0; j < m && !bad; ++j) {
      double dj = Lc[j + j * kMaxM];
      for (int q = 0; q < j; ++q) dj -= Lc[j + q * kMaxM] * Lc[j + q * kMaxM];
      if (!(dj > 0.0)) { bad = 1; break; }
      const double ljj = sqrt(dj);
      Lc[j + j * kMaxM] = ljj;
      for (int i = j + 1; i < m; ++i) {
        double v = Lc[i + j * kMaxM];
        for (int q = 0; q < j; ++q) v -= Lc[i + q * kMaxM] * Lc[j + q * kMaxM];
        Lc[i + j * kMaxM] = v / ljj;
      }
    }
    if (bad) atomicOr(flag, 4);
  }
  __syncthreads();
  if (bad) return;
  for (int c = tid; c < r; c += blockDim.x) {
    double* x = X + (int64_t)c * m;
    for (int a = 0; a < m; ++a) {  // Lc y = z
      double v = Z[c + (int64_t)a * r];
      for (int b = 0; b < a; ++b) v -= Lc[a + b * kMaxM] * x[b];
      x[a] = v / Lc[a + a * kMaxM];
    }
    for (int a = m - 1; a >= 0; --a) {  // Lc^T x = y
      double v = x[a];
      for (int b = a + 1; b < m; ++b) v -= Lc[b + a * kMaxM] * x[b];
      x[a] = v / Lc[a + a * kMaxM];
    }
  }
}

}  // namespace

void riccati_update_f64(hipStream_t s, int64_t r, int64_t m, double* D, int64_t ldd,
                        const double* WB, int64_t ldw, const double* R, int64_t ldr, double t,
                        int* flag_dev, Arena& ws, double* Zout) {
  if (r <= 0 || m <= 0) return;
  DME_REQUIRE(m <= kMaxM, DME_EINVAL, "riccati: m > 64 inputs is not supported");
  double* Y = Zout ? Zout : ws.get<double>((size_t)r * m);
  hipLaunchKernelGGL(riccati_kernel, dim3(1), dim3(kRT), 0, s, (int)r, (int)m, D, ldd, WB, ldw, R,
                     ldr, t, Y, flag_dev);
  DME_HIP(hipGetLastError());
}

// K (m x n, ld ldk) = R^-1 B^T L D L^T: W = L^T B, Z = D W, X = R^-1 Z^T,
// K = X L^T.
void feedback_gain_f64(hipStream_t s, int64_t n, int64_t r, int64_t m, const double* L, int64_t ldl,
                       const double* D, int64_t ldd, const double* B, int64_t ldb, const double* R,
                       int64_t ldr, double* K, int64_t ldk, int* flag_dev, Arena& ws) {
  if (m <= 0 || n <= 0) return;
  DME_REQUIRE(m <= kMaxM, DME_EINVAL, "gain: m > 64 inputs is not supported");
  if (r <= 0) {
    fill_f64(s, K, m, n, ldk, 0.0);
    return;
  }
  double* W = ws.get<double>((size_t)r * m);
  double* Z = ws.get<double>((size_t)r * m);
  double* X = ws.get<double>((size_t)m * r);
  const size_t mark = ws.used;
  gemm_f64(s, 'T', 'N', r, m, n, 1.0, L, ldl, B, ldb, 0.0, W, r, &ws);
  ws.used = mark;
  gemm_f64(s, 'N', 'N', r, m, r, 1.0, D, ldd, W, r, 0.0, Z, r, &ws);
  ws.used = mark;
  hipLaunchKernelGGL(gain_solve_kernel, dim3(1), dim3(256), 0, s, (int)m, (int)r, R, ldr, Z, X, flag_dev);
  DME_HIP(hipGetLastError());
  gemm_f64(s, 'N', 'T', m, n, r, 1.0, X, m, L, ldl, 0.0, K, ldk, &ws);
  ws.used = mark;
}

}  // namespace dme
