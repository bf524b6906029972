// Leja-interpolation action of the matrix exponential (the paper's expleja,
// Sec. 3 and Sec. 4), see leja.h for the recurrence.
//
// Device side: the Gershgorin interval (column discs of a dense A^T, row discs
// of a CSR A^T), a symmetry check, and one launch per Newton term: for a CSR
// operator a fused kernel that forms A^T W for its rows, the next basis block
// W' = (A^T W) / g - (c / g + xi_j) W and the accumulator update
// P += d_{j+1} W' in one pass (W ping-pongs between two buffers); for a dense
// A^T the product runs on the FP64 MFMA GEMM and one elementwise pass does the
// rest.  Host side: Leja points, divided differences and (S, m), in long
// double.
#include "leja.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

namespace dme {
namespace {

constexpr int kT = 256;
constexpr int kMMax = 100;        // largest interpolation degree
constexpr double kRhoMax = 24.0;  // largest t g per substep

inline unsigned grid_for(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(count, kT), 16384));
}

// ---------------------------------------------------------------- intervals
// Column j of A^T: centre A^T(j, j), radius sum_{i != j} |A^T(i, j)|.
__global__ void col_disc_kernel(const double* __restrict__ AT, int64_t n, double* lo, double* hi) {
  __shared__ double red[kT];
  const int64_t j = blockIdx.x;
  const double* col = AT + j * n;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) acc += fabs(col[i]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double c = col[j];
    const double r = red[0] - fabs(c);
    lo[j] = c - r;
    hi[j] = c + r;
  }
}

__global__ void row_disc_kernel(const int64_t* __restrict__ rowptr, const int* __restrict__ colind,
                                const double* __restrict__ val, int64_t n, double* lo, double* hi) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    double c = 0.0, r = 0.0;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      if (colind[k] == i) c += val[k];
      else r += fabs(val[k]);
    }
    lo[i] = c - r;
    hi[i] = c + r;
  }
}

// out[0] = min lo, out[1] = max hi (one workgroup).
__global__ void minmax_kernel(const double* lo, const double* hi, int64_t n, double* out) {
  __shared__ double a[1024], b[1024];
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += 1024) {
    mn = fmin(mn, lo[i]);
    mx = fmax(mx, hi[i]);
  }
  a[threadIdx.x] = mn;
  b[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      a[threadIdx.x] = fmin(a[threadIdx.x], a[threadIdx.x + w]);
      b[threadIdx.x] = fmax(b[threadIdx.x], b[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = a[0];
    out[1] = b[0];
  }
}

// Tile pair (bx, by), bx <= by: max |X(i, j) - X(j, i)| and max |X(i, j)| over
// the two tiles; other blocks write zeros.  32 x 8 threads.
__global__ void symdiff_kernel(const double* __restrict__ X, int64_t n, int64_t nt, double* dpart,
                               double* xpart) {
  __shared__ double t1[32][33], t2[32][33];
  __shared__ double rd[256], rx[256];
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double md = 0.0, mx = 0.0;
  if (bx <= by) {
    for (int k = ty; k < 32; k += 8) {
      const int64_t r1 = bx * 32 + tx, c1 = by * 32 + k;  // tile (bx, by)
      const int64_t r2 = by * 32 + tx, c2 = bx * 32 + k;  // tile (by, bx)
      t1[k][tx] = (r1 < n && c1 < n) ? X[r1 + c1 * n] : 0.0;
      t2[k][tx] = (r2 < n && c2 < n) ? X[r2 + c2 * n] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
      // X(bx*32 + tx, by*32 + k) against X(by*32 + k, bx*32 + tx)
      const double u = t1[k][tx], v = t2[tx][k];
      md = fmax(md, fabs(u - v));
      mx = fmax(mx, fmax(fabs(u), fabs(v)));
    }
  }
  rd[threadIdx.x] = md;
  rx[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + w]);
      rx[threadIdx.x] = fmax(rx[threadIdx.x], rx[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    dpart[by * nt + bx] = rd[0];
    xpart[by * nt + bx] = rx[0];
  }
}

// ------------------------------------------------------------ Newton terms
// Column q belongs to group q / gcols (a single group when gcols >= ncols).
// (column counts are far below 2^31: a 32-bit division)
__device__ __forceinline__ int group_of(int64_t q, int64_t gcols) { return (int)q / (int)gcols; }

// W <- X, P <- d_0 X
__global__ void leja_init_kernel(int64_t n, int64_t ncols, const double* __restrict__ X, int64_t ldx,
                                 double* __restrict__ W, double* __restrict__ P,
                                 const double* __restrict__ coef, int m1, int64_t gcols) {
  const int64_t total = n * ncols;
  for (int64_t idx = blockIdx.x * (int64_t)kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx % n, q = idx / n;
    const double x = X[i + q * ldx];
    W[idx] = x;
    P[idx] = coef[group_of(q, gcols) * m1] * x;
  }
}

// dense operator: Z = A^T W was formed by the GEMM; W <- Z / g - shift W,
// P <- P + d_{j+1} W
__global__ void leja_dense_term_kernel(int64_t n, int64_t ncols, const double* __restrict__ Z,
                                       double* __restrict__ W, double* __restrict__ P, double inv_g,
                                       double shift, const double* __restrict__ coef, int m1, int j1,
                                       int64_t gcols) {
  const int64_t total = n * ncols;
  for (int64_t idx = blockIdx.x * (int64_t)kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t q = idx / n;
    const double w = Z[idx] * inv_g - shift * W[idx];
    W[idx] = w;
    P[idx] += coef[group_of(q, gcols) * m1 + j1] * w;
  }
}

// CSR operator, blocks stored row-major (n x cp, cp = ncols rounded up to
// even): one wave per row, each lane two adjacent columns (and further pairs
// 128 columns apart), so every load and store of a wave is one contiguous run
// of 16-byte pairs; the row's entries are wave-uniform (scalar loads).  Forms
// (A^T W)(i, :) and the next basis row W'(i, :) = (A^T W)(i, :) / g - shift
// W(i, :).  The accumulator is updated every second term: a launch reads the
// basis row W = W_j it starts from anyway, so with pmode 2 it adds
// d_j W + d_{j+1} W' (in that order, the order of one update per term) and the
// launch before it (pmode 0) leaves P alone; pmode 1 adds d_{j+1} W' alone
// (the last term of an odd count).  P is read and written by half the
// launches.
constexpr int kRowsPerBlock = 4;
// Rows with at most this many entries (every row of a 5- or 7-point grid
// operator) take their entries first, as wave-uniform values, and then issue
// the loads of all the W rows they reach together: such a row waits for
// three memory round trips (its extent, its entries, the W rows) instead of
// two per entry.  The padding entries are zeros on the row itself, so the sum
// runs over the same terms in the same order.
constexpr int kFastNnz = 8;

// W'(i, q:q+2) from the sum (A^T W)(i, q:q+2) = acc, and the accumulator update
__device__ __forceinline__ void leja_csr_finish(int64_t o, int64_t q, int64_t ncols, double2 acc, double2 wi,
                                                double* __restrict__ Wout, double* __restrict__ P, double inv_g,
                                                double shift, const double* __restrict__ coef, int m1, int j1,
                                                int64_t gcols, int pmode) {
  double2 wn;
  wn.x = acc.x * inv_g - shift * wi.x;
  wn.y = acc.y * inv_g - shift * wi.y;
  *reinterpret_cast<double2*>(Wout + o) = wn;
  if (pmode != 0) {  // wave-uniform
    double2 pp = *reinterpret_cast<const double2*>(P + o);
    const double* cx = coef + group_of(q, gcols) * m1;
    const double* cy = coef + group_of(q + 1, gcols) * m1;
    if (pmode == 2) {
      pp.x += cx[j1 - 1] * wi.x;
      if (q + 1 < ncols) pp.y += cy[j1 - 1] * wi.y;
    }
    pp.x += cx[j1] * wn.x;
    if (q + 1 < ncols) pp.y += cy[j1] * wn.y;
    *reinterpret_cast<double2*>(P + o) = pp;
  }
}

// The sum over a row's kFastNnz (padded) entries, all W rows loaded at once.
__device__ __forceinline__ void leja_fixed_row(int64_t i, int64_t cp, int64_t ncols, int lane,
                                               const int (&cu)[kFastNnz], const double (&au)[kFastNnz],
                                               const double* __restrict__ Win, double* __restrict__ Wout,
                                               double* __restrict__ P, double inv_g, double shift,
                                               const double* __restrict__ coef, int m1, int j1, int64_t gcols,
                                               int pmode) {
  for (int64_t q = 2 * (int64_t)lane; q < ncols; q += 128) {
    const int64_t o = i * cp + q;
    double2 w[kFastNnz];
#pragma unroll
    for (int u = 0; u < kFastNnz; ++u) w[u] = *reinterpret_cast<const double2*>(Win + (int64_t)cu[u] * cp + q);
    const double2 wi = *reinterpret_cast<const double2*>(Win + o);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < kFastNnz; ++u) {
      acc.x += au[u] * w[u].x;
      acc.y += au[u] * w[u].y;
    }
    leja_csr_finish(o, q, ncols, acc, wi, Wout, P, inv_g, shift, coef, m1, j1, gcols, pmode);
  }
}

// i is the wave's row (the same in every lane)
__device__ __forceinline__ void leja_csr_row(int64_t i, int64_t cp, int64_t ncols, int lane,
                                             const int64_t* __restrict__ rowptr, const int* __restrict__ colind,
                                             const double* __restrict__ val, const double* __restrict__ Win,
                                             double* __restrict__ Wout, double* __restrict__ P, double inv_g,
                                             double shift, const double* __restrict__ coef, int m1, int j1,
                                             int64_t gcols, int pmode) {
  const int64_t k0 = rowptr[i], k1 = rowptr[i + 1];
  const int64_t nnz = k1 - k0;
  if (nnz >= 1 && nnz <= kFastNnz) {  // wave-uniform
    int cu[kFastNnz];
    double au[kFastNnz];
#pragma unroll
    for (int u = 0; u < kFastNnz; ++u) {
      const int64_t kk = k0 + min<int64_t>(u, nnz - 1);  // in [k0, k1)
      cu[u] = (u < nnz) ? colind[kk] : (int)i;
      au[u] = (u < nnz) ? val[kk] : 0.0;
    }
    leja_fixed_row(i, cp, ncols, lane, cu, au, Win, Wout, P, inv_g, shift, coef, m1, j1, gcols, pmode);
    return;
  }
  for (int64_t q = 2 * (int64_t)lane; q < ncols; q += 128) {
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t kk = k0; kk < k1; ++kk) {
      const double a = val[kk];
      const double2 w = *reinterpret_cast<const double2*>(Win + (int64_t)colind[kk] * cp + q);
      acc.x += a * w.x;
      acc.y += a * w.y;
    }
    const int64_t o = i * cp + q;
    const double2 wi = *reinterpret_cast<const double2*>(Win + o);
    leja_csr_finish(o, q, ncols, acc, wi, Wout, P, inv_g, shift, coef, m1, j1, gcols, pmode);
  }
}

// Workgroups go to the XCDs in turn (workgroup b to XCD b % 8, each XCD with
// its own L2).  Workgroup b takes the row block that gives every XCD one
// contiguous range of rows, so the rows a row's entries reach (for a grid
// operator its neighbours one and one grid line away) are mostly in the
// same XCD's range, and each row of W is fetched into about one L2 instead
// of the L2s of both neighbouring blocks.  A bijection on [0, nb) for any
// number of XCDs; 8 sets only the locality.
__device__ __forceinline__ int64_t xcd_row_block(int64_t b, int64_t nb) {
  constexpr int64_t kX = 8;
  const int64_t x = b % kX, q = nb / kX, rem = nb % kX;
  return x * q + min(x, rem) + b / kX;
}

__global__ __launch_bounds__(64 * kRowsPerBlock) void leja_csr_term_kernel(
    int64_t n, int64_t cp, int64_t ncols, const int64_t* __restrict__ rowptr, const int* __restrict__ colind,
    const double* __restrict__ val, const double* __restrict__ ell, const double* __restrict__ Win, double* __restrict__ Wout, double* __restrict__ P, double inv_g,
    double shift, const double* __restrict__ coef, int m1, int j1, int64_t gcols, int pmode) {
  // the wave's row, as a wave-uniform (scalar) value: its extent and entries
  // come by scalar loads
  const int64_t i = xcd_row_block(blockIdx.x, gridDim.x) * kRowsPerBlock +
                    __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (i >= n) return;
  const int lane = threadIdx.x & 63;
  if (ell) {  // fixed-width rows: the entries at a known place, one record
    static_assert(LejaOp::kEllWidth == kFastNnz, "fixed-width rows hold kFastNnz entries");
    const double* rv = ell + i * LejaOp::kEllRecord;
    const int* rc = reinterpret_cast<const int*>(rv + kFastNnz);
    int cu[kFastNnz];
    double au[kFastNnz];
#pragma unroll
    for (int u = 0; u < kFastNnz; ++u) {
      au[u] = rv[u];
      cu[u] = rc[u];
    }
    leja_fixed_row(i, cp, ncols, lane, cu, au, Win, Wout, P, inv_g, shift, coef, m1, j1, gcols, pmode);
    return;
  }
  leja_csr_row(i, cp, ncols, lane, rowptr, colind, val, Win, Wout, P, inv_g, shift, coef, m1, j1, gcols, pmode);
}

// Column-major X (ld ldx) -> row-major W (ld cp) and P = d_0 X, through 32 x 32
// LDS tiles (coalesced on both sides); pad columns [ncols, cp) are zero.
__global__ void leja_init_rm_kernel(int64_t n, int64_t ncols, int64_t cp, const double* __restrict__ X,
                                    int64_t ldx, double* __restrict__ W, double* __restrict__ P,
                                    const double* __restrict__ coef, int m1, int64_t gcols) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    tile[j][tx] = (r < n && c < ncols) ? X[r + c * ldx] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    if (r < n && c < cp) {
      const double x = tile[tx][j];
      W[r * cp + c] = x;
      P[r * cp + c] = (c < ncols) ? coef[group_of(c, gcols) * m1] * x : 0.0;
    }
  }
}

// end of a substep that is not the last, row-major blocks
__global__ void leja_restart_rm_kernel(int64_t n, int64_t ncols, int64_t cp, double* __restrict__ W,
                                       double* __restrict__ P, const double* __restrict__ coef,
                                       const double* __restrict__ scale, int m1, int64_t gcols) {
  const int64_t total = n * cp;
  for (int64_t idx = blockIdx.x * (int64_t)kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t c = idx % cp;
    if (c >= ncols) continue;
    const int g = group_of(c, gcols);
    const double x = scale[g] * P[idx];
    W[idx] = x;
    P[idx] = coef[g * m1] * x;
  }
}

// end of the last substep: Y (column-major, ld ldy) = e^{t c / S} P (row-major)
__global__ void leja_finish_rm_kernel(int64_t n, int64_t ncols, int64_t cp, const double* __restrict__ P,
                                      double* __restrict__ Y, int64_t ldy, const double* __restrict__ scale,
                                      int64_t gcols) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + j, c = c0 + tx;
    tile[j][tx] = (r < n && c < ncols) ? scale[group_of(c, gcols)] * P[r * cp + c] : 0.0;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    if (r < n && c < ncols) Y[r + c * ldy] = tile[tx][j];
  }
}

// end of a substep that is not the last: X' = e^{t c / S} P, W <- X',
// P <- d_0 X'
__global__ void leja_restart_kernel(int64_t n, int64_t ncols, double* __restrict__ W,
                                    double* __restrict__ P, const double* __restrict__ coef,
                                    const double* __restrict__ scale, int m1, int64_t gcols) {
  const int64_t total = n * ncols;
  for (int64_t idx = blockIdx.x * (int64_t)kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int g = group_of(idx / n, gcols);
    const double x = scale[g] * P[idx];
    W[idx] = x;
    P[idx] = coef[g * m1] * x;
  }
}

// end of the last substep: Y = e^{t c / S} P
__global__ void leja_finish_kernel(int64_t n, int64_t ncols, const double* __restrict__ P,
                                   double* __restrict__ Y, int64_t ldy, const double* __restrict__ scale,
                                   int64_t gcols) {
  const int64_t total = n * ncols;
  for (int64_t idx = blockIdx.x * (int64_t)kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx % n, q = idx / n;
    Y[i + q * ldy] = scale[group_of(q, gcols)] * P[idx];
  }
}

// ------------------------------------------------------------------- host
// (Discrete) Leja points of [-2, 2]: xi_0 = 2, then the point of a uniform
// grid where prod_{i<j} |x - xi_i| is largest (sums of logs), kMMax + 1 of them.
const std::vector<long double>& leja_points() {
  static std::vector<long double> pts;
  static std::once_flag once;
  std::call_once(once, [] {
    const int G = 20001;
    std::vector<long double> x(G), lw(G);
    for (int i = 0; i < G; ++i) x[i] = -2.0L + 4.0L * (long double)i / (G - 1);
    pts.push_back(2.0L);
    for (int i = 0; i < G; ++i) lw[i] = std::log(std::fabs(x[i] - 2.0L) + 1e-300L);
    for (int j = 1; j <= kMMax; ++j) {
      int best = 0;
      for (int i = 1; i < G; ++i)
        if (lw[i] > lw[best]) best = i;
      const long double p = x[best];
      pts.push_back(p);
      for (int i = 0; i < G; ++i) lw[i] += std::log(std::fabs(x[i] - p) + 1e-300L);
    }
  });
  return pts;
}

// Divided differences of e^{rho z} at xi_0 .. xi_M by the recursive
// definition (long double).
std::vector<long double> exp_divdiff(long double rho, const std::vector<long double>& xi, int M) {
  std::vector<long double> col(M + 1), d(M + 1);
  for (int i = 0; i <= M; ++i) col[i] = std::exp(rho * xi[i]);
  d[0] = col[0];
  for (int k = 1; k <= M; ++k) {
    for (int i = 0; i + k <= M; ++i) col[i] = (col[i + 1] - col[i]) / (xi[i + k] - xi[i]);
    d[k] = col[0];
  }
  return d;
}

// Smallest degree m whose Newton interpolant of e^{rho z} stays within
// tol * e^{2 rho} on a grid of [-2, 2]; -1 if none up to kMMax.
int degree_for(long double rho, const std::vector<long double>& xi,
               const std::vector<long double>& d, double tol) {
  const int Z = 2001;
  std::vector<long double> z(Z), p(Z, 0.0L), w(Z, 1.0L), f(Z);
  for (int i = 0; i < Z; ++i) {
    z[i] = -2.0L + 4.0L * (long double)i / (Z - 1);
    f[i] = std::exp(rho * z[i]);
  }
  const long double bound = (long double)tol * std::exp(2.0L * rho);
  for (int m = 0; m <= kMMax; ++m) {
    long double err = 0.0L;
    for (int i = 0; i < Z; ++i) {
      p[i] += d[m] * w[i];
      w[i] *= (z[i] - xi[m]);
      err = std::max(err, std::fabs(p[i] - f[i]));
    }
    if (m >= 1 && err <= bound) return m;
  }
  return -1;
}

void interval_from(hipStream_t s, const double* lo, const double* hi, int64_t n, double* out_dev,
                   double* a, double* b) {
  hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, s, lo, hi, n, out_dev);
  DME_HIP(hipGetLastError());
  double h[2];
  DME_HIP(hipMemcpyAsync(h, out_dev, sizeof(h), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  *a = h[0];
  *b = h[1];
  DME_REQUIRE(std::isfinite(*a) && std::isfinite(*b), DME_ENUMERIC,
              "Leja: non-finite entries in the operator");
}

}  // namespace

std::shared_ptr<LejaOp> leja_op_dense(hipStream_t s, int64_t n, const double* AT, Arena& ws) {
  auto op = std::make_shared<LejaOp>();
  op->n = n;
  op->dense = AT;
  const size_t mark = ws.used;
  double* lo = ws.get<double>(n);
  double* hi = ws.get<double>(n);
  double* out = ws.get<double>(2);
  hipLaunchKernelGGL(col_disc_kernel, dim3((unsigned)n), dim3(kT), 0, s, AT, n, lo, hi);
  DME_HIP(hipGetLastError());
  interval_from(s, lo, hi, n, out, &op->a, &op->b);
  ws.used = mark;
  return op;
}

std::shared_ptr<LejaOp> leja_op_csr(hipStream_t s, int64_t n, const int64_t* rowptr,
                                    const int64_t* colind, const double* val, Arena& ws) {
  DME_REQUIRE(n > 0 && n < (int64_t(1) << 31), DME_EINVAL, "sparse A: n out of range");
  DME_REQUIRE(rowptr && rowptr[0] == 0, DME_EINVAL, "sparse A: row pointers must start at 0");
  const int64_t nnz = rowptr[n];
  DME_REQUIRE(nnz >= 0 && (nnz == 0 || (colind && val)), DME_EINVAL, "sparse A: bad nnz or arrays");
  // transpose on the host (counting sort by column): CSR of A^T, each row's
  // entries in ascending column order
  std::vector<int64_t> tp(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    DME_REQUIRE(rowptr[i + 1] >= rowptr[i], DME_EINVAL, "sparse A: row pointers decrease");
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      DME_REQUIRE(colind[k] >= 0 && colind[k] < n, DME_EINVAL, "sparse A: column index out of range");
      tp[colind[k] + 1] += 1;
    }
  }
  for (int64_t j = 0; j < n; ++j) tp[j + 1] += tp[j];
  std::vector<int> tc(nnz);
  std::vector<double> tv(nnz);
  std::vector<int64_t> fill(tp.begin(), tp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const int64_t pos = fill[colind[k]]++;
      tc[pos] = (int)i;
      tv[pos] = val[k];
    }
  auto op = std::make_shared<LejaOp>();
  op->n = n;
  op->nnz = nnz;
  // A^T = A iff every row of A, sorted by column, equals that row of A^T
  // (whose entries the counting sort left in ascending column order)
  op->symmetric = true;
  {
    std::vector<std::pair<int64_t, double>> row;
    for (int64_t i = 0; i < n && op->symmetric; ++i) {
      row.clear();
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) row.push_back({colind[k], val[k]});
      std::sort(row.begin(), row.end());
      if ((int64_t)row.size() != tp[i + 1] - tp[i]) {
        op->symmetric = false;
        break;
      }
      for (size_t q = 0; q < row.size(); ++q) {
        const int64_t k = tp[i] + (int64_t)q;
        if (row[q].first != tc[k] || row[q].second != tv[k]) {
          op->symmetric = false;
          break;
        }
      }
    }
  }
  // fixed-width rows when every row of A^T fits: a row's entries are then at
  // a known place and a term needs no row pointers
  int64_t widest = 0;
  for (int64_t i = 0; i < n; ++i) widest = std::max(widest, tp[i + 1] - tp[i]);
  if (widest <= LejaOp::kEllWidth) {
    constexpr int E = LejaOp::kEllWidth, Rd = LejaOp::kEllRecord;
    static_assert(Rd * sizeof(double) == E * (sizeof(double) + sizeof(int)), "record layout");
    std::vector<double> rec((size_t)n * Rd, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      double* rv = rec.data() + (size_t)i * Rd;
      int cols[E];
      for (int u = 0; u < E; ++u) {
        const int64_t k = tp[i] + u;
        const bool real = k < tp[i + 1];
        rv[u] = real ? tv[k] : 0.0;
        cols[u] = real ? tc[k] : (int)i;
      }
      std::memcpy(rv + E, cols, sizeof(cols));
    }
    op->ell.ensure(rec.size() * sizeof(double));
    DME_HIP(hipMemcpyAsync(op->ell.p, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice, s));
    DME_HIP(hipStreamSynchronize(s));  // the host vector goes out of scope
  }
  op->rowptr.ensure((size_t)(n + 1) * sizeof(int64_t));
  op->colind.ensure((size_t)std::max<int64_t>(nnz, 1) * sizeof(int));
  op->val.ensure((size_t)std::max<int64_t>(nnz, 1) * sizeof(double));
  DME_HIP(hipMemcpyAsync(op->rowptr.p, tp.data(), (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  if (nnz) {
    DME_HIP(hipMemcpyAsync(op->colind.p, tc.data(), (size_t)nnz * sizeof(int), hipMemcpyHostToDevice, s));
    DME_HIP(hipMemcpyAsync(op->val.p, tv.data(), (size_t)nnz * sizeof(double), hipMemcpyHostToDevice, s));
  }
  const size_t mark = ws.used;
  double* lo = ws.get<double>(n);
  double* hi = ws.get<double>(n);
  double* out = ws.get<double>(2);
  hipLaunchKernelGGL(row_disc_kernel, dim3(grid_for(n)), dim3(kT), 0, s, op->rowptr.as<int64_t>(),
                     op->colind.as<int>(), op->val.as<double>(), n, lo, hi);
  DME_HIP(hipGetLastError());
  interval_from(s, lo, hi, n, out, &op->a, &op->b);  // also waits for the uploads
  ws.used = mark;
  return op;
}

bool dense_symmetric(hipStream_t s, int64_t n, const double* X, double rel_tol, Arena& ws) {
  if (n <= 1) return true;
  const int64_t nt = cdiv(n, 32);
  const size_t mark = ws.used;
  double* dp = ws.get<double>((size_t)nt * nt);
  double* xp = ws.get<double>((size_t)nt * nt);
  double* out = ws.get<double>(2);
  hipLaunchKernelGGL(symdiff_kernel, dim3((unsigned)nt, (unsigned)nt), dim3(256), 0, s, X, n, nt, dp, xp);
  DME_HIP(hipGetLastError());
  // max of both partial sets: minmax over (-dp, xp) would mix them, so two passes
  double hd[2], hx[2];
  hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, s, dp, dp, nt * nt, out);
  DME_HIP(hipGetLastError());
  DME_HIP(hipMemcpyAsync(hd, out, sizeof(hd), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, s, xp, xp, nt * nt, out);
  DME_HIP(hipGetLastError());
  DME_HIP(hipMemcpyAsync(hx, out, sizeof(hx), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  ws.used = mark;
  return hd[1] <= rel_tol * hx[1];
}

std::unique_ptr<LejaPlan> leja_plan(const LejaOp& op, const std::vector<double>& times,
                                    int64_t group_cols, double tol) {
  DME_REQUIRE(!times.empty() && group_cols > 0, DME_EINVAL, "Leja plan: no column groups");
  auto p = std::make_unique<LejaPlan>();
  p->c = 0.5 * (op.a + op.b);
  p->g = 0.25 * (op.b - op.a);
  p->groups = (int)times.size();
  p->group_cols = group_cols;
  double tmax = 0.0;
  for (double t : times) {
    DME_REQUIRE(t >= 0.0 && std::isfinite(t), DME_EINVAL, "Leja plan: times must be >= 0");
    tmax = std::max(tmax, t);
  }
  const std::vector<long double>& xi = leja_points();
  std::vector<std::vector<long double>> dd(p->groups);
  if (p->g <= 0.0) {
    // A^T = c I on its discs: e^{t A^T} X = e^{t c} X, one term of degree 0
    p->S = 1;
    p->m = 0;
    for (int k = 0; k < p->groups; ++k) dd[k] = {1.0L};
  } else {
    const double rho_total = tmax * p->g;
    int S = std::max(1, (int)std::ceil(rho_total / kRhoMax));
    int m = -1;
    for (; S <= 1 << 20; S *= 2) {
      m = 0;
      bool ok = true;
      for (int k = 0; k < p->groups && ok; ++k) {
        const long double rho = (long double)times[k] * p->g / S;
        dd[k] = exp_divdiff(rho, xi, kMMax);
        const int mk = degree_for(rho, xi, dd[k], tol);
        if (mk < 0) ok = false;
        m = std::max(m, mk);
      }
      if (ok) break;
    }
    DME_REQUIRE(m >= 1, DME_ENUMERIC, "Leja plan: no interpolation degree meets the tolerance");
    p->S = S;
    p->m = m;
  }
  const int m1 = p->m + 1;
  p->xi.resize(m1);
  for (int j = 0; j < m1; ++j) p->xi[j] = (double)xi[j];
  p->coef.resize((size_t)p->groups * m1);
  p->scale.resize(p->groups);
  for (int k = 0; k < p->groups; ++k) {
    for (int j = 0; j < m1; ++j) p->coef[(size_t)k * m1 + j] = (double)dd[k][j];
    p->scale[k] = std::exp(times[k] * p->c / p->S);
  }
  p->coef_dev.ensure(p->coef.size() * sizeof(double));
  p->scale_dev.ensure(p->scale.size() * sizeof(double));
  DME_HIP(hipMemcpy(p->coef_dev.p, p->coef.data(), p->coef.size() * sizeof(double), hipMemcpyHostToDevice));
  DME_HIP(hipMemcpy(p->scale_dev.p, p->scale.data(), p->scale.size() * sizeof(double), hipMemcpyHostToDevice));
  return p;
}

size_t leja_workspace(int64_t n, int64_t ncols) {
  const size_t blk = ((size_t)n * ((ncols + 1) & ~int64_t(1)) * sizeof(double) + 255) & ~size_t(255);
  return 3 * blk + gemm_f64_workspace(n, ncols, n) + 1024;
}

void leja_apply(hipStream_t s, const LejaOp& op, const LejaPlan& plan, const double* X, int64_t ldx,
                int64_t ncols, double* Y, int64_t ldy, Arena& ws) {
  const int64_t n = op.n;
  if (n <= 0 || ncols <= 0) return;
  DME_REQUIRE(plan.groups == 1 || ncols == (int64_t)plan.groups * plan.group_cols, DME_EINTERNAL,
              "Leja: columns do not match the plan's groups");
  const int64_t gcols = plan.groups == 1 ? std::max<int64_t>(ncols, plan.group_cols) : plan.group_cols;
  const int m1 = plan.m + 1;
  const double* coef = plan.coef_dev.as<double>();
  const double* scale = plan.scale_dev.as<double>();
  const size_t mark = ws.used;
  const size_t blk = (size_t)n * ((ncols + 1) & ~int64_t(1));
  double* W = ws.get<double>(blk);
  double* W2 = ws.get<double>(blk);  // CSR: the other half of the ping-pong; dense: A^T W
  double* P = ws.get<double>(blk);
  const size_t mark_gemm = ws.used;
  const unsigned gb = grid_for(n * ncols);
  const double inv_g = plan.g > 0.0 ? 1.0 / plan.g : 0.0;
  if (op.sparse()) {
    // row-major blocks, n x cp
    const int64_t cp = (ncols + 1) & ~int64_t(1);
    const dim3 tgrid((unsigned)cdiv(n, 32), (unsigned)cdiv(cp, 32));
    hipLaunchKernelGGL(leja_init_rm_kernel, tgrid, dim3(256), 0, s, n, ncols, cp, X, ldx, W, P, coef, m1, gcols);
    DME_HIP(hipGetLastError());
    const unsigned rgrid = (unsigned)cdiv(n, kRowsPerBlock);
    for (int sub = 0; sub < plan.S; ++sub) {
      for (int j = 0; j < plan.m; ++j) {
        const double shift = plan.c * inv_g + plan.xi[j];
        // P takes d_j W_j + d_{j+1} W_{j+1} at odd j, d_m W_m at the last
        // term of an odd count, nothing otherwise: every term of the substep
        // is in P when the substep ends
        const int pmode = (j & 1) ? 2 : (j + 1 == plan.m ? 1 : 0);
        hipLaunchKernelGGL(leja_csr_term_kernel, dim3(rgrid), dim3(64 * kRowsPerBlock), 0, s, n, cp, ncols,
                           op.rowptr.as<int64_t>(), op.colind.as<int>(), op.val.as<double>(),
                           op.ell.bytes ? op.ell.as<double>() : nullptr, W, W2, P, inv_g, shift, coef, m1,
                           j + 1, gcols, pmode);
        DME_HIP(hipGetLastError());
        std::swap(W, W2);
      }
      if (sub + 1 < plan.S) {
        hipLaunchKernelGGL(leja_restart_rm_kernel, dim3(grid_for(n * cp)), dim3(kT), 0, s, n, ncols, cp, W, P,
                           coef, scale, m1, gcols);
        DME_HIP(hipGetLastError());
      }
    }
    hipLaunchKernelGGL(leja_finish_rm_kernel, tgrid, dim3(256), 0, s, n, ncols, cp, P, Y, ldy, scale, gcols);
    DME_HIP(hipGetLastError());
    ws.used = mark;
    return;
  }
  hipLaunchKernelGGL(leja_init_kernel, dim3(gb), dim3(kT), 0, s, n, ncols, X, ldx, W, P, coef, m1, gcols);
  DME_HIP(hipGetLastError());
  for (int sub = 0; sub < plan.S; ++sub) {
    for (int j = 0; j < plan.m; ++j) {
      const double shift = plan.c * inv_g + plan.xi[j];
      ws.used = mark_gemm;
      gemm_f64(s, 'N', 'N', n, ncols, n, 1.0, op.dense, n, W, n, 0.0, W2, n, &ws);
      hipLaunchKernelGGL(leja_dense_term_kernel, dim3(gb), dim3(kT), 0, s, n, ncols, W2, W, P, inv_g,
                         shift, coef, m1, j + 1, gcols);
      DME_HIP(hipGetLastError());
    }
    if (sub + 1 < plan.S) {
      hipLaunchKernelGGL(leja_restart_kernel, dim3(gb), dim3(kT), 0, s, n, ncols, W, P, coef, scale, m1, gcols);
      DME_HIP(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(leja_finish_kernel, dim3(gb), dim3(kT), 0, s, n, ncols, P, Y, ldy, scale, gcols);
  DME_HIP(hipGetLastError());
  ws.used = mark;
}

}  // namespace dme
