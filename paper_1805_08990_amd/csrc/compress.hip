// Column compression of P = W Dhat W^T (the step that follows every
// concatenation in Alg. 1, 2 and 4; method described in Sec. 3 after Alg. 2):
//
//   Householder QR   W = Q R            (tree QR by 32-column panels, tsqr.hip)
//   small product    M = R Dhat R^T     (FP64 MFMA GEMM)
//   eigenpairs       M = V Lam V^T      (syev.hip), keep |lam| > tol max|lam|
//   new factor       L = Q [V_I; 0],  D = diag(Lam_I)
//
// compress_f64_lead serves W = [Y, U] whose second block U has orthonormal
// columns (the compressed quadrature factor L_I of Alg. 2, the same at every
// step of one step size): U's columns need no Householder panels of their own.
//   C = U^T Y, Y <- Y - U C, twice (classical Gram-Schmidt, repeated once)
//   Y = Q2 R2 (tree QR), so [Y, U] = [Q2, U] Rt with Rt = [[R2, 0], [C, I]]
//   M = Rt Dhat Rt^T, M = V Lam V^T (kept part), as above
//   L = P Q2 [V(0:r, :); 0] + U V(r:k, :), P = I - U U^T
// P removes from Q2's columns the U components that rounding leaves in the
// directions where Y is (numerically) rank-deficient after the projection.
#include "tsqr.h"

namespace dme {
namespace {

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

// Rt (k x k, k = r + q) = [[R2, 0], [C1 + C2, I]], R2 the upper triangle of
// W(0:r, 0:r) (ld ldw), C1, C2 q x r (ld q).
__global__ void build_rt_kernel(const double* W, int64_t ldw, int64_t r, int64_t q, const double* C1,
                                const double* C2, double* Rt) {
  const int64_t k = r + q, total = k * k;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % k, c = idx / k;
    double v;
    if (i < r) v = (c < r && i <= c) ? W[i + c * ldw] : 0.0;
    else if (c < r) v = C1[(i - r) + c * q] + C2[(i - r) + c * q];
    else v = (i == c) ? 1.0 : 0.0;
    Rt[idx] = v;
  }
}

// B (q x r', ld q) = V(r:r+q, 0:r') (ld ldv) - Z (q x r', ld q)
__global__ void lower_minus_kernel(const double* V, int64_t ldv, int64_t r, int64_t q, int64_t rr,
                                   const double* Z, double* B) {
  const int64_t total = q * rr;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % q, c = idx / q;
    B[idx] = V[r + i + c * ldv] - Z[idx];
  }
}

inline unsigned blocks_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(total, 256), 8192));
}

}  // namespace

size_t compress_workspace(int64_t n, int64_t k) {
  size_t b = 0;
  auto add = [&](size_t bytes) { b += (bytes + 255) & ~size_t(255); };
  add(2 * (size_t)k * sizeof(double));          // lam, spare
  add(4 * (size_t)k * k * sizeof(double));      // R, T1, M, S
  add((size_t)k * k * sizeof(double));          // V
  add(syev_workspace(k));
  add(tsqr_workspace(n, k));
  add(gemm_f64_workspace(k, k, k));
  // compress_f64_lead: C1, C2, Z, B (at most k x k each) and its n-deep products
  add(4 * (size_t)k * k * sizeof(double));
  add(std::max(gemm_f64_workspace(k, k, n), gemm_f64_workspace(n, k, k)));
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
  double* lam = ws.get<double>(k);
  double* R = ws.get<double>((size_t)k * k);
  double* T1 = ws.get<double>((size_t)k * k);
  double* M = ws.get<double>((size_t)k * k);
  double* S = ws.get<double>((size_t)k * k);
  double* V = ws.get<double>((size_t)k * k);

  // ---------------- Householder QR; the tree's factors stay reserved until Q is applied
  TsqrState tq;
  tsqr_factor(s, n, k, W, tq, ws);
  const size_t mark_q = ws.used;

  // ---------------- M = R Dhat R^T, symmetrised
  hipLaunchKernelGGL(extract_r_kernel, dim3(blocks_for(kr * k)), dim3(256), 0, s, W, ld, kr, k, R);
  DME_HIP(hipGetLastError());
  ws.used = mark_q;
  gemm_f64(s, 'N', 'N', kr, k, k, 1.0, R, kr, Dhat, k, 0.0, T1, kr, &ws);
  ws.used = mark_q;
  gemm_f64(s, 'N', 'T', kr, kr, k, 1.0, T1, kr, R, kr, 0.0, M, kr, &ws);
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for(kr * kr)), dim3(256), 0, s, M, kr, S);
  DME_HIP(hipGetLastError());
  finite_check_f64(s, S, kr, kr, kr, flag_dev);

  // ---------------- eigenpairs with truncation
  ws.used = mark_q;
  syev_trunc_f64(s, kr, S, kr, tol, std::min(max_rank, kr), lam, V, kr, rank_dev, flag_dev, ws);
  int64_t r = 0;
  DME_HIP(hipMemcpyAsync(&r, rank_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  if (r <= 0) return 0;
  if (ldd <= 0) ldd = r;

  // ---------------- L = Q [V_I; 0], D = diag(lam_I)
  hipLaunchKernelGGL(embed_kernel, dim3(blocks_for(n * r)), dim3(256), 0, s, V, kr, kr, n, r, L, ldl);
  DME_HIP(hipGetLastError());
  tsqr_apply_q(s, tq, L, ldl, r);
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(r * r)), dim3(256), 0, s, lam, r, Dout, ldd);
  DME_HIP(hipGetLastError());
  ws.used = mark_q;
  return r;
}

int64_t compress_f64_lead(hipStream_t s, int64_t n, int64_t r, double* W, const double* U,
                          int64_t ldu, int64_t q, const double* Dhat, double tol, int64_t max_rank,
                          double* L, int64_t ldl, double* Dout, int64_t ldd, int64_t* rank_dev,
                          int* flag_dev, Arena& ws) {
  DME_REQUIRE(r > 0 && q > 0 && n >= r + q, DME_EINVAL, "compress_lead: needs n >= r + q > q > 0");
  const int64_t k = r + q;
  double* lam = ws.get<double>(k);
  double* Rt = ws.get<double>((size_t)k * k);
  double* T1 = ws.get<double>((size_t)k * k);
  double* M = ws.get<double>((size_t)k * k);
  double* S = ws.get<double>((size_t)k * k);
  double* V = ws.get<double>((size_t)k * k);
  double* C1 = ws.get<double>((size_t)q * r);
  double* C2 = ws.get<double>((size_t)q * r);
  double* Z = ws.get<double>((size_t)q * k);
  double* B = ws.get<double>((size_t)q * k);
  const size_t mark0 = ws.used;

  // Y <- P Y twice, C = C1 + C2
  gemm_f64(s, 'T', 'N', q, r, n, 1.0, U, ldu, W, n, 0.0, C1, q, &ws);
  ws.used = mark0;
  gemm_f64(s, 'N', 'N', n, r, q, -1.0, U, ldu, C1, q, 1.0, W, n, &ws);
  ws.used = mark0;
  gemm_f64(s, 'T', 'N', q, r, n, 1.0, U, ldu, W, n, 0.0, C2, q, &ws);
  ws.used = mark0;
  gemm_f64(s, 'N', 'N', n, r, q, -1.0, U, ldu, C2, q, 1.0, W, n, &ws);
  ws.used = mark0;

  // Y = Q2 R2
  TsqrState tq;
  tsqr_factor(s, n, r, W, tq, ws);
  const size_t mark_q = ws.used;

  // M = Rt Dhat Rt^T, symmetrised
  hipLaunchKernelGGL(build_rt_kernel, dim3(blocks_for(k * k)), dim3(256), 0, s, W, n, r, q, C1, C2, Rt);
  DME_HIP(hipGetLastError());
  gemm_f64(s, 'N', 'N', k, k, k, 1.0, Rt, k, Dhat, k, 0.0, T1, k, &ws);
  ws.used = mark_q;
  gemm_f64(s, 'N', 'T', k, k, k, 1.0, T1, k, Rt, k, 0.0, M, k, &ws);
  ws.used = mark_q;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(blocks_for(k * k)), dim3(256), 0, s, M, k, S);
  DME_HIP(hipGetLastError());
  finite_check_f64(s, S, k, k, k, flag_dev);

  syev_trunc_f64(s, k, S, k, tol, std::min(max_rank, k), lam, V, k, rank_dev, flag_dev, ws);
  ws.used = mark_q;
  int64_t rr = 0;
  DME_HIP(hipMemcpyAsync(&rr, rank_dev, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  if (rr <= 0) return 0;
  if (ldd <= 0) ldd = rr;

  // L = P Q2 [V(0:r, :); 0] + U V(r:k, :) = Q2 [...] + U (V(r:k, :) - U^T Q2 [...])
  hipLaunchKernelGGL(embed_kernel, dim3(blocks_for(n * rr)), dim3(256), 0, s, V, k, r, n, rr, L, ldl);
  DME_HIP(hipGetLastError());
  tsqr_apply_q(s, tq, L, ldl, rr);
  gemm_f64(s, 'T', 'N', q, rr, n, 1.0, U, ldu, L, ldl, 0.0, Z, q, &ws);
  ws.used = mark_q;
  hipLaunchKernelGGL(lower_minus_kernel, dim3(blocks_for(q * rr)), dim3(256), 0, s, V, k, r, q, rr, Z, B);
  DME_HIP(hipGetLastError());
  gemm_f64(s, 'N', 'N', n, rr, q, 1.0, U, ldu, B, q, 1.0, L, ldl, &ws);
  ws.used = mark_q;
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(rr * rr)), dim3(256), 0, s, lam, rr, Dout, ldd);
  DME_HIP(hipGetLastError());
  return rr;
}

}  // namespace dme
