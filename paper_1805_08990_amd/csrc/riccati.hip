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

constexpr int kRT = 256;
constexpr int kMaxM = 64;

__global__ __launch_bounds__(kRT) void riccati_kernel(int r, int m, double* D, int64_t ldd,
                                                      const double* WB, int64_t ldw, const double* R,
                                                      int64_t ldr, double t, double* Y, double* Dn,
                                                      int* flag) {
  __shared__ double S[kMaxM * kMaxM];
  __shared__ int bad;
  const int tid = threadIdx.x;
  // Y = D W  (r x m, ld r)
  for (int idx = tid; idx < r * m; idx += kRT) {
    const int i = idx % r, a = idx / r;
    double acc = 0.0;
    for (int l = 0; l < r; ++l) acc += D[i + (int64_t)l * ldd] * WB[l + (int64_t)a * ldw];
    Y[i + (int64_t)a * r] = acc;
  }
  __syncthreads();
  // S = R + t W^T Y
  for (int idx = tid; idx < m * m; idx += kRT) {
    const int a = idx % m, b = idx / m;
    double acc = 0.0;
    for (int i = 0; i < r; ++i) acc += WB[i + (int64_t)a * ldw] * Y[i + (int64_t)b * r];
    S[a + b * kMaxM] = R[a + (int64_t)b * ldr] + t * acc;
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
  // Dn = sym(D) - t Z Z^T
  for (int idx = tid; idx < r * r; idx += kRT) {
    const int i = idx % r, j = idx / r;
    double acc = 0.0;
    for (int a = 0; a < m; ++a) acc += Y[i + (int64_t)a * r] * Y[j + (int64_t)a * r];
    Dn[idx] = 0.5 * (D[i + (int64_t)j * ldd] + D[j + (int64_t)i * ldd]) - t * acc;
  }
  __syncthreads();
  for (int idx = tid; idx < r * r; idx += kRT) {
    const int i = idx % r, j = idx / r;
    D[i + (int64_t)j * ldd] = Dn[idx];
  }
}

}  // namespace

void riccati_update_f64(hipStream_t s, int64_t r, int64_t m, double* D, int64_t ldd,
                        const double* WB, int64_t ldw, const double* R, int64_t ldr, double t,
                        int* flag_dev, Arena& ws) {
  if (r <= 0 || m <= 0) return;
  DME_REQUIRE(m <= kMaxM, DME_EINVAL, "riccati: m > 64 inputs is not supported");
  double* Y = ws.get<double>((size_t)r * m);
  double* Dn = ws.get<double>((size_t)r * r);
  hipLaunchKernelGGL(riccati_kernel, dim3(1), dim3(kRT), 0, s, (int)r, (int)m, D, ldd, WB, ldw, R,
                     ldr, t, Y, Dn, flag_dev);
  DME_HIP(hipGetLastError());
}

}  // namespace dme
