// Matrix exponential e^{tX} of a dense n x n operator by scaling and squaring
// with a diagonal Pade approximant (N. J. Higham, "The scaling and squaring
// method for the matrix exponential revisited", SIAM J. Matrix Anal. Appl.
// 26(4), 2005, Algorithm 2.3).  This replaces the Leja-interpolation action
// the paper uses (Sec. 3): the operator is formed once per step size and then
// applied to the low-rank factor with GEMMs.
//
//   1. ||tX||_1 (column sums on the device)  ->  degree m, scaling s
//   2. Y = tX / 2^s; even powers Y^2, Y^4, Y^6 (FP64 MFMA GEMMs)
//   3. U (odd part), V (even part) of the [m/m] numerator; denominator V - U
//   4. (V - U) F = V + U by LU with partial pivoting (lu.hip)
//   5. F <- F^2, s times
#include "common.h"

#include <cmath>

namespace dme {

namespace {

// theta_m of Higham (2005), Table 2.3 (double precision): the largest
// ||X||_1 for which the [m/m] approximant meets the unit-roundoff backward
// error bound.
constexpr int kDegrees[5] = {3, 5, 7, 9, 13};
constexpr double kTheta[5] = {1.495585217958292e-2, 2.539398330063230e-1, 9.504178996162932e-1,
                              2.097847961257068e0, 5.371920351148152e0};

// Numerator coefficients b_j = (2m - j)! m! / ((2m)! j! (m - j)!), from the
// ratio b_{j+1} / b_j = (m - j) / ((j + 1)(2m - j)), evaluated in long double.
void pade_coeffs(int m, double* b) {
  long double c = 1.0L;
  b[0] = 1.0;
  for (int j = 0; j < m; ++j) {
    c = c * (long double)(m - j) / ((long double)(j + 1) * (long double)(2 * m - j));
    b[j + 1] = (double)c;
  }
}

}  // namespace

void expm_params(double nrm1, int* m, int* s) {
  for (int i = 0; i < 4; ++i) {
    if (nrm1 <= kTheta[i]) { *m = kDegrees[i]; *s = 0; return; }
  }
  *m = 13;
  *s = (nrm1 > 0.0) ? std::max(0, (int)std::ceil(std::log2(nrm1 / kTheta[4]))) : 0;
}

size_t expm_workspace(int64_t n) {
  const size_t nn = (size_t)n * n * sizeof(double) + 256;
  return 7 * nn + (size_t)n * sizeof(double) + 512 + lu_solve_workspace(n) +
         gemm_f64_workspace(n, n, n) + 4096;
}

// E = e^{tX}; X, E are n x n device matrices (contiguous), E must not alias X.
void expm_f64(hipStream_t s, int64_t n, const double* X, double t, double* E, Arena& ws, int* m_out,
              int* s_out, int* info_dev) {
  if (n <= 0) return;
  const size_t nn = (size_t)n * n;
  double* Y = ws.get<double>(nn);
  double* Y2 = ws.get<double>(nn);
  double* Y4 = ws.get<double>(nn);
  double* Y6 = ws.get<double>(nn);
  double* T1 = ws.get<double>(nn);
  double* U = ws.get<double>(nn);
  double* V = ws.get<double>(nn);
  double* colsum = ws.get<double>(n);
  double* nrm_dev = ws.get<double>(1);
  const size_t mark = ws.used;

  copy_scaled_f64(s, X, n, Y, n, n, n, t);
  norm1_f64(s, Y, n, n, n, colsum, nrm_dev);
  double nrm = 0.0;
  DME_HIP(hipMemcpyAsync(&nrm, nrm_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  DME_REQUIRE(std::isfinite(nrm), DME_ENUMERIC, "expm: operator has non-finite entries");
  int m = 13, sc = 0;
  expm_params(nrm, &m, &sc);
  if (m_out) *m_out = m;
  if (s_out) *s_out = sc;
  if (sc > 0) scale_f64(s, Y, (int64_t)nn, std::ldexp(1.0, -sc));

  double b[14];
  pade_coeffs(m, b);
  auto mm = [&](const double* P, const double* Q, double beta, double* R) {
    ws.used = mark;
    gemm_f64(s, 'N', 'N', n, n, n, 1.0, P, n, Q, n, beta, R, n, &ws);
  };
  mm(Y, Y, 0.0, Y2);
  if (m == 13) {
    mm(Y2, Y2, 0.0, Y4);
    mm(Y4, Y2, 0.0, Y6);
    // U = Y (Y6 (b13 Y6 + b11 Y4 + b9 Y2) + b7 Y6 + b5 Y4 + b3 Y2 + b1 I)
    lincomb3_f64(s, n, b[13], Y6, b[11], Y4, b[9], Y2, 0.0, T1);
    lincomb3_f64(s, n, b[7], Y6, b[5], Y4, b[3], Y2, b[1], V);
    mm(Y6, T1, 1.0, V);
    mm(Y, V, 0.0, U);
    // V = Y6 (b12 Y6 + b10 Y4 + b8 Y2) + b6 Y6 + b4 Y4 + b2 Y2 + b0 I
    lincomb3_f64(s, n, b[12], Y6, b[10], Y4, b[8], Y2, 0.0, T1);
    lincomb3_f64(s, n, b[6], Y6, b[4], Y4, b[2], Y2, b[0], V);
    mm(Y6, T1, 1.0, V);
  } else {
    // plain even powers Y^2, Y^4 = Y^2 Y^2, Y^6 = Y^4 Y^2, Y^8 = Y^6 Y^2
    const int h = m / 2;  // highest even power index: Y^{2h}
    double* P8 = T1;
    if (h >= 2) mm(Y2, Y2, 0.0, Y4);
    if (h >= 3) mm(Y4, Y2, 0.0, Y6);
    if (h >= 4) mm(Y6, Y2, 0.0, P8);
    // odd = b1 I + b3 Y2 + b5 Y4 + b7 Y6 + b9 Y8 ; even = b0 I + b2 Y2 + ...
    const double* P[5] = {nullptr, Y2, Y4, Y6, P8};
    auto coef = [&](int j) { return (j <= m) ? b[j] : 0.0; };
    // V <- odd part first (stored in V temporarily), then U = Y * odd
    lincomb3_f64(s, n, coef(3), P[1], h >= 2 ? coef(5) : 0.0, h >= 2 ? P[2] : nullptr,
                 h >= 3 ? coef(7) : 0.0, h >= 3 ? P[3] : nullptr, coef(1), V);
    if (h >= 4) lincomb3_f64(s, n, 1.0, V, coef(9), P[4], 0.0, nullptr, 0.0, V);
    mm(Y, V, 0.0, U);
    lincomb3_f64(s, n, coef(2), P[1], h >= 2 ? coef(4) : 0.0, h >= 2 ? P[2] : nullptr,
                 h >= 3 ? coef(6) : 0.0, h >= 3 ? P[3] : nullptr, coef(0), V);
    if (h >= 4) lincomb3_f64(s, n, 1.0, V, coef(8), P[4], 0.0, nullptr, 0.0, V);
  }
  // U <- V - U (denominator q_m), V <- V + U (numerator p_m); solve q F = p
  pade_pm_f64(s, U, V, (int64_t)nn);
  ws.used = mark;
  lu_solve_f64(s, n, U, V, ws, info_dev);
  // squaring phase
  double* cur = V;
  double* other = T1;
  for (int q = 0; q < sc; ++q) {
    double* dst = (q == sc - 1) ? E : other;
    mm(cur, cur, 0.0, dst);
    if (dst != E) std::swap(cur, other);
    else cur = E;
  }
  if (cur != E) copy_f64(s, cur, n, E, n, n, n);
  ws.used = mark;
}

}  // namespace dme
