// Action of the matrix exponential on a block of columns, Y = e^{t A^T} X, by
// Newton interpolation at Leja points (the paper's expleja, Sec. 3 and Sec. 4:
// a one-time spectral estimate from Gershgorin discs, one-time interpolation
// parameters, then a Newton recurrence built from products with A^T).
//
// With [a, b] a real interval holding the spectrum, c = (a + b) / 2 and
// g = (b - a) / 4, As = (A^T - c I) / g has its spectrum in [-2, 2] and
// e^{t A^T} = e^{t c} e^{t g As}.  The time is cut into S substeps; in each,
// e^{rho z} (rho = t g / S) is interpolated at Leja points xi_0 .. xi_m of
// [-2, 2] in Newton form with divided differences d_j:
//     W <- X, P <- d_0 X;  for j < m: W <- (As - xi_j) W, P <- P + d_{j+1} W;
//     X <- e^{t c / S} P.
// The columns form groups (of `group_cols` columns each) with their own time
// t_k: every group shares the recurrence on W (the same As and points) and
// has its own coefficients, substep factor and accumulator columns.  For a
// symmetric operator the error of one substep is at most
// max_{[-2, 2]} |e^{rho z} - p(z)| ||X||, which is what (S, m) are chosen from.
#pragma once

#include <memory>
#include <vector>

#include "common.h"

namespace dme {

// The operator the recurrence multiplies by: a dense A^T (column-major,
// borrowed) or A^T in CSR form (owned, 32-bit column indices).
struct LejaOp {
  int64_t n = 0;
  const double* dense = nullptr;
  int64_t nnz = 0;
  DevBuf rowptr, colind, val;
  // the same rows in fixed-width form when no row has more than kEllWidth
  // entries: row i is a record of kEllRecord doubles at ell + i kEllRecord,
  // its kEllWidth values, then their kEllWidth column indices (int), padded
  // with zeros on the row itself; empty otherwise
  static constexpr int kEllWidth = 8;
  static constexpr int kEllRecord = kEllWidth + kEllWidth / 2;
  DevBuf ell;
  double a = 0.0, b = 0.0;  // Gershgorin interval of the spectrum
  bool symmetric = false;   // CSR: A^T equals A entry for entry
  bool sparse() const { return dense == nullptr; }
};

// Build from a dense A^T on the device (borrowed): Gershgorin interval by the
// column discs of A^T (synchronises `s`).
std::shared_ptr<LejaOp> leja_op_dense(hipStream_t s, int64_t n, const double* AT, Arena& ws);
// Build from A in CSR form on the host (row pointers n + 1, column indices and
// values nnz): transposed on the host, uploaded, Gershgorin interval by rows;
// `symmetric` tells whether A^T = A.
std::shared_ptr<LejaOp> leja_op_csr(hipStream_t s, int64_t n, const int64_t* rowptr,
                                    const int64_t* colind, const double* val, Arena& ws);
// Whether the dense n x n matrix X (device, ld n) is symmetric within
// rel_tol * max|X| (synchronises `s`).
bool dense_symmetric(hipStream_t s, int64_t n, const double* X, double rel_tol, Arena& ws);

// Interpolation parameters for groups of columns with times t_k.
struct LejaPlan {
  double c = 0.0, g = 0.0;
  int S = 1, m = 0;
  int groups = 1;
  int64_t group_cols = 0;
  std::vector<double> xi;     // m + 1 points
  std::vector<double> coef;   // groups x (m + 1): d_j of each group
  std::vector<double> scale;  // groups: e^{t_k c / S}
  DevBuf coef_dev, scale_dev;
};

// Plan for the operator's interval and the group times (t_k >= 0), per-substep
// tolerance `tol` relative to max_{[-2, 2]} e^{rho z}.
std::unique_ptr<LejaPlan> leja_plan(const LejaOp& op, const std::vector<double>& times,
                                    int64_t group_cols, double tol = 1e-14);

// Workspace (bytes) of leja_apply for n x ncols blocks.
size_t leja_workspace(int64_t n, int64_t ncols);
// Y (n x ncols, ld ldy) = e^{t_k A^T} X (ld ldx) per column group; ncols must
// be plan.groups * plan.group_cols (or fewer columns with a single group).
// X and Y may alias.
void leja_apply(hipStream_t s, const LejaOp& op, const LejaPlan& plan, const double* X, int64_t ldx,
                int64_t ncols, double* Y, int64_t ldy, Arena& ws);
// Products with A^T one action makes (S * m), for the flop accounting.
inline int64_t leja_products(const LejaPlan& p) { return (int64_t)p.S * p.m; }
// Updates of the accumulator one action on a CSR operator makes (every second
// term, S * ceil(m / 2)), for the byte accounting.
inline int64_t leja_csr_p_updates(const LejaPlan& p) { return (int64_t)p.S * ((p.m + 1) / 2); }

}  // namespace dme
