// Bandwidth-bound helpers: fills, copies, the Pade linear combinations, the
// 1-norm of the scaled operator, block-diagonal assembly, finiteness scan.
// Each thread walks contiguous column segments so that loads and stores are
// coalesced 64-lane runs of a column-major matrix.
#include "common.h"

namespace dme {
namespace {

constexpr int kT = 256;

inline unsigned grid_for(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(count, kT), 8192));
}

__global__ void fill_kernel(double* X, int64_t rows, int64_t cols, int64_t ld, double v) {
  const int64_t total = rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i % rows, c = i / rows;
    X[r + c * ld] = v;
  }
}

__global__ void copy_scaled_kernel(const double* X, int64_t ldx, double* Y, int64_t ldy,
                                   int64_t rows, int64_t cols, double alpha) {
  const int64_t total = rows * cols;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i % rows, c = i / rows;
    Y[r + c * ldy] = alpha * X[r + c * ldx];
  }
}

// 32 x 32 tiles through LDS so that both the read and the write are coalesced.
__global__ void transpose_kernel(const double* X, int64_t ldx, double* Y, int64_t ldy,
                                 int64_t rows, int64_t cols, double alpha) {
  __shared__ double tile[32][33];
  const int64_t r0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int64_t r = r0 + tx, c = c0 + j;
    if (r < rows && c < cols) tile[j][tx] = X[r + c * ldx];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t yr = c0 + tx, yc = r0 + j;  // Y(c, r) = X(r, c)
    if (yr < cols && yc < rows) Y[yr + yc * ldy] = alpha * tile[tx][j];
  }
}

__global__ void lincomb3_kernel(int64_t n, double a, const double* X1, double b, const double* X2,
                                double c, const double* X3, double d, double* Y) {
  const int64_t total = n * n;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    double v = 0.0;
    if (X1) v += a * X1[i];
    if (X2) v += b * X2[i];
    if (X3) v += c * X3[i];
    if ((i % n) == (i / n)) v += d;
    Y[i] = v;
  }
}

__global__ void scale_kernel(double* X, int64_t count, double alpha) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < count; i += (int64_t)gridDim.x * kT)
    X[i] *= alpha;
}

__global__ void pade_pm_kernel(double* U, double* V, int64_t count) {
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < count; i += (int64_t)gridDim.x * kT) {
    const double u = U[i], v = V[i];
    U[i] = v - u;
    V[i] = v + u;
  }
}

// One wave per column: sum |X(:, c)| in a fixed order (lane-strided then a
// butterfly), so the result is reproducible.
__global__ void colabs_kernel(const double* X, int64_t rows, int64_t cols, int64_t ld,
                              double* colsum) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
  if (c >= cols) return;
  double s = 0.0;
  const double* col = X + c * ld;
  for (int64_t r = lane; r < rows; r += 64) s += fabs(col[r]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) colsum[c] = s;
}

__global__ void max_kernel(const double* v, int64_t count, double* out) {
  __shared__ double sm[kT];
  double m = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += kT) m = fmax(m, v[i]);
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sm[0];
}

// out (k1+k2 square) = blkdiag(D1, scale2 * D2); D2 == nullptr means identity.
__global__ void blkdiag2_kernel(const double* D1, int64_t k1, int64_t ld1, const double* D2,
                                int64_t k2, int64_t ld2, double scale2, double* out, int64_t ldo) {
  const int64_t k = k1 + k2, total = k * k;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i % k, c = i / k;
    double v = 0.0;
    if (r < k1 && c < k1) v = D1[r + c * ld1];
    else if (r >= k1 && c >= k1) {
      const int64_t rr = r - k1, cc = c - k1;
      v = D2 ? scale2 * D2[rr + cc * ld2] : (rr == cc ? scale2 : 0.0);
    }
    out[r + c * ldo] = v;
  }
}

__global__ void finite_kernel(const double* X, int64_t rows, int64_t cols, int64_t ld, int* flag) {
  const int64_t total = rows * cols;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i % rows, c = i / rows;
    if (!isfinite(X[r + c * ld])) bad = true;
  }
  if (bad) atomicOr(flag, 1);
}

// Sums of (A - B)^2 and B^2 over a rows x cols block: one pair of partial
// sums per workgroup (grid-stride over the entries, tree reduction in LDS),
// then one workgroup adds the partials in a fixed order.
constexpr int kDiffBlocks = 256;

__global__ void sqdiff_partial_kernel(const double* A, int64_t lda, const double* B, int64_t ldb,
                                      int64_t rows, int64_t cols, double* part) {
  __shared__ double sd[kT], sb[kT];
  const int64_t total = rows * cols;
  double d2 = 0.0, b2 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kT + threadIdx.x; i < total; i += (int64_t)gridDim.x * kT) {
    const int64_t r = i % rows, c = i / rows;
    const double b = B[r + c * ldb];
    const double d = A[r + c * lda] - b;
    d2 += d * d;
    b2 += b * b;
  }
  sd[threadIdx.x] = d2;
  sb[threadIdx.x] = b2;
  __syncthreads();
  for (int w = kT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sd[threadIdx.x] += sd[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sd[0];
    part[2 * blockIdx.x + 1] = sb[0];
  }
}

__global__ void sum_pairs_kernel(const double* part, int count, double* out) {
  if (threadIdx.x == 0) {
    double d2 = 0.0, b2 = 0.0;
    for (int i = 0; i < count; ++i) {
      d2 += part[2 * i];
      b2 += part[2 * i + 1];
    }
    out[0] = d2;
    out[1] = b2;
  }
}

}  // namespace

void fill_f64(hipStream_t s, double* X, int64_t rows, int64_t cols, int64_t ld, double v) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(rows * cols)), dim3(kT), 0, s, X, rows, cols, ld, v);
  DME_HIP(hipGetLastError());
}

void copy_scaled_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     int64_t rows, int64_t cols, double alpha) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(copy_scaled_kernel, dim3(grid_for(rows * cols)), dim3(kT), 0, s, X, ldx, Y,
                     ldy, rows, cols, alpha);
  DME_HIP(hipGetLastError());
}

void copy_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t rows,
              int64_t cols) {
  copy_scaled_f64(s, X, ldx, Y, ldy, rows, cols, 1.0);
}

void transpose_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy,
                   int64_t rows, int64_t cols, double alpha) {
  if (rows <= 0 || cols <= 0) return;
  dim3 grid((unsigned)cdiv(rows, 32), (unsigned)cdiv(cols, 32));
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(kT), 0, s, X, ldx, Y, ldy, rows, cols, alpha);
  DME_HIP(hipGetLastError());
}

void lincomb3_f64(hipStream_t s, int64_t n, double a, const double* X1, double b, const double* X2,
                  double c, const double* X3, double d, double* Y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(lincomb3_kernel, dim3(grid_for(n * n)), dim3(kT), 0, s, n, a, X1, b, X2, c,
                     X3, d, Y);
  DME_HIP(hipGetLastError());
}

void scale_f64(hipStream_t s, double* X, int64_t count, double alpha) {
  if (count <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(count)), dim3(kT), 0, s, X, count, alpha);
  DME_HIP(hipGetLastError());
}

void pade_pm_f64(hipStream_t s, double* U, double* V, int64_t count) {
  if (count <= 0) return;
  hipLaunchKernelGGL(pade_pm_kernel, dim3(grid_for(count)), dim3(kT), 0, s, U, V, count);
  DME_HIP(hipGetLastError());
}

void norm1_f64(hipStream_t s, const double* X, int64_t rows, int64_t cols, int64_t ld,
               double* colsum, double* out) {
  if (cols <= 0) {
    fill_f64(s, out, 1, 1, 1, 0.0);
    return;
  }
  hipLaunchKernelGGL(colabs_kernel, dim3((unsigned)cdiv(cols, kT / 64)), dim3(kT), 0, s, X, rows,
                     cols, ld, colsum);
  DME_HIP(hipGetLastError());
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(kT), 0, s, colsum, cols, out);
  DME_HIP(hipGetLastError());
}

void blkdiag2_f64(hipStream_t s, const double* D1, int64_t k1, int64_t ld1, const double* D2,
                  int64_t k2, int64_t ld2, double scale2, double* out, int64_t ldo) {
  const int64_t k = k1 + k2;
  if (k <= 0) return;
  hipLaunchKernelGGL(blkdiag2_kernel, dim3(grid_for(k * k)), dim3(kT), 0, s, D1, k1, ld1, D2, k2,
                     ld2, scale2, out, ldo);
  DME_HIP(hipGetLastError());
}

void finite_check_f64(hipStream_t s, const double* X, int64_t rows, int64_t cols, int64_t ld,
                      int* flag) {
  if (rows <= 0 || cols <= 0) return;
  hipLaunchKernelGGL(finite_kernel, dim3(grid_for(rows * cols)), dim3(kT), 0, s, X, rows, cols, ld,
                     flag);
  DME_HIP(hipGetLastError());
}

}  // namespace dme

namespace dme {

size_t diff_norms_workspace() { return 2 * kDiffBlocks * sizeof(double); }

void diff_norms_f64(hipStream_t s, const double* A, int64_t lda, const double* B, int64_t ldb,
                    int64_t rows, int64_t cols, double* part, double* out) {
  const int64_t total = rows * cols;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kDiffBlocks, cdiv(total, kT)));
  hipLaunchKernelGGL(sqdiff_partial_kernel, dim3(blocks), dim3(kT), 0, s, A, lda, B, ldb, rows, cols, part);
  DME_HIP(hipGetLastError());
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(64), 0, s, part, blocks, out);
  DME_HIP(hipGetLastError());
}

}  // namespace dme
