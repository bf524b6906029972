// Dense LU with partial pivoting and the multi-right-hand-side solve used for
// the Pade denominator of the matrix exponential: (V - U) F = V + U.
//
// Blocked right-looking factorisation with panel width kNB:
//   panel   : per column, one launch eliminates the previous pivot row from the
//             panel rows (each thread one row) and writes per-workgroup argmax
//             partials of the next column; a one-workgroup launch picks the
//             pivot (largest |a|, first index on ties) and stages the two rows
//             that swap.
//   swaps   : applied to the columns outside the panel and to the right-hand
//             sides (one thread per column, swaps in order).
//   U12     : inv(L11) * A12 (inverted unit-lower diagonal block, FP64 GEMM).
//   A22     : A22 - L21 * U12 (FP64 MFMA GEMM).
// The solve then runs blocked forward and backward substitution with inverted
// diagonal blocks, so all O(n^3) work is in the GEMM.
#include "common.h"

namespace dme {
namespace {

constexpr int kNB = 64;       // panel / triangular block width
constexpr int kRowsT = 256;   // threads (rows) per workgroup in panel kernels

struct ArgMax {
  double v;
  int64_t i;
};

__device__ inline void argmax_merge(double& v, int64_t& i, double v2, int64_t i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

// Block-level argmax of |val| over the rows this block owns; writes one partial.
__device__ void block_argmax(double v, int64_t i, ArgMax* part) {
  __shared__ double sv[kRowsT];
  __shared__ int64_t si[kRowsT];
  sv[threadIdx.x] = v;
  si[threadIdx.x] = i;
  __syncthreads();
  for (int s = kRowsT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double a = sv[threadIdx.x];
      int64_t ai = si[threadIdx.x];
      argmax_merge(a, ai, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = a;
      si[threadIdx.x] = ai;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = ArgMax{sv[0], si[0]};
}

// Partial argmax of |A(i, j)| for rows i >= j.
__global__ void argmax_partial_kernel(const double* A, int64_t lda, int64_t n, int64_t j,
                                      ArgMax* part) {
  const int64_t i = j + (int64_t)blockIdx.x * kRowsT + threadIdx.x;
  double v = -1.0;
  int64_t idx = INT64_MAX;
  if (i < n) { v = fabs(A[i + j * lda]); idx = i; }
  block_argmax(v, idx, part);
}

// Pick the pivot of column j from `nparts` partials, stage rows j and p of the
// panel columns [j0, j0 + jb) into rowj / rowp.
__global__ void pivot_final_kernel(double* A, int64_t lda, int64_t j, int64_t j0, int jb,
                                   const ArgMax* part, int nparts, int64_t* piv, double* rowj,
                                   double* rowp, int* info) {
  __shared__ double sv[kRowsT];
  __shared__ int64_t si[kRowsT];
  double v = -1.0;
  int64_t idx = INT64_MAX;
  for (int t = threadIdx.x; t < nparts; t += kRowsT) argmax_merge(v, idx, part[t].v, part[t].i);
  sv[threadIdx.x] = v;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int s = kRowsT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      double a = sv[threadIdx.x];
      int64_t ai = si[threadIdx.x];
      argmax_merge(a, ai, sv[threadIdx.x + s], si[threadIdx.x + s]);
      sv[threadIdx.x] = a;
      si[threadIdx.x] = ai;
    }
    __syncthreads();
  }
  int64_t p = si[0];
  // every candidate was NaN: keep the diagonal row (the NaN reaches the result
  // and is reported by the finiteness checks)
  if (p < j || p >= (int64_t)INT64_MAX / 2) p = j;
  if (threadIdx.x == 0) {
    piv[j] = p;
    if (!(sv[0] > 0.0) && *info == 0) *info = (int)(j + 1);  // zero (or NaN) pivot column
  }
  for (int c = threadIdx.x; c < jb; c += kRowsT) {
    rowj[c] = A[j + (j0 + c) * lda];
    rowp[c] = A[p + (j0 + c) * lda];
  }
}

// Swap rows j <-> p inside the panel and eliminate column j from rows > j of
// the panel columns; then write argmax partials of column j + 1.
__global__ void elim_kernel(double* A, int64_t lda, int64_t n, int64_t j, int64_t j0, int jb,
                            const int64_t* piv, const double* rowj_g, const double* rowp_g,
                            ArgMax* part) {
  __shared__ double rowj[kNB], rowp[kNB];
  for (int c = threadIdx.x; c < jb; c += kRowsT) {
    rowj[c] = rowj_g[c];
    rowp[c] = rowp_g[c];
  }
  __syncthreads();
  const int64_t p = piv[j];
  const int jl = (int)(j - j0);
  const double pv = rowp[jl];
  const int64_t i = j + (int64_t)blockIdx.x * kRowsT + threadIdx.x;
  double next = -1.0;
  int64_t nidx = INT64_MAX;
  if (i < n) {
    if (i == j) {
      for (int c = 0; c < jb; ++c) A[j + (j0 + c) * lda] = rowp[c];
    } else {
      // source row values: row p now holds the old row j
      const bool isp = (i == p);
      for (int c = 0; c < jl; ++c)
        if (isp) A[i + (j0 + c) * lda] = rowj[c];
      const double aij = isp ? rowj[jl] : A[i + (j0 + jl) * lda];
      const double l = (pv != 0.0) ? aij / pv : 0.0;
      A[i + (j0 + jl) * lda] = l;
      for (int c = jl + 1; c < jb; ++c) {
        const double a = isp ? rowj[c] : A[i + (j0 + c) * lda];
        const double v = a - l * rowp[c];
        A[i + (j0 + c) * lda] = v;
        if (c == jl + 1) { next = fabs(v); nidx = i; }
      }
    }
  }
  if (jl + 1 < jb) {
    // rows >= j + 1 only; block 0 thread 0 is row j (excluded above by i == j path)
    block_argmax(next, nidx, part);
  }
}

// Apply the panel's row swaps piv[j0 .. j0+jb) to columns [c0, c1) of X.
__global__ void swap_rows_kernel(double* X, int64_t ldx, int64_t c0, int64_t c1, int64_t j0, int jb,
                                 const int64_t* piv) {
  const int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  double* col = X + c * ldx;
  for (int t = 0; t < jb; ++t) {
    const int64_t j = j0 + t, p = piv[j];
    if (p != j) {
      const double a = col[j];
      col[j] = col[p];
      col[p] = a;
    }
  }
}

// Invert a b x b triangular diagonal block at T (ld ldt) into X (ld b).
// lower != 0: unit lower triangular; else non-unit upper triangular.
// One thread per column of the inverse; block and inverse are staged in LDS.
__global__ void tri_inv_kernel(const double* T, int64_t ldt, int b, int lower, double* X) {
  __shared__ double s[kNB * kNB];
  __shared__ double x[kNB * (kNB + 1)];
  for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
    const int r = idx % b, c = idx / b;
    s[r + c * kNB] = T[r + c * ldt];
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < b) {
    double* xc = x + c * (kNB + 1);
    for (int r = 0; r < b; ++r) xc[r] = 0.0;
    if (lower) {
      xc[c] = 1.0;
      for (int r = c + 1; r < b; ++r) {
        double acc = 0.0;
        for (int t = c; t < r; ++t) acc += s[r + t * kNB] * xc[t];
        xc[r] = -acc;
      }
    } else {
      xc[c] = 1.0 / s[c + c * kNB];
      for (int r = c - 1; r >= 0; --r) {
        double acc = 0.0;
        for (int t = r + 1; t <= c; ++t) acc += s[r + t * kNB] * xc[t];
        xc[r] = -acc / s[r + r * kNB];
      }
    }
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
    const int r = idx % b, cc = idx / b;
    X[r + (int64_t)cc * b] = x[r + cc * (kNB + 1)];
  }
}

}  // namespace

size_t lu_solve_workspace(int64_t n) { return lu_solve_workspace(n, n); }

size_t lu_solve_workspace(int64_t n, int64_t nrhs) {
  const int64_t nparts = cdiv(n, kRowsT) + 1;
  const int64_t w = std::max(n, nrhs);
  size_t b = 0;
  b += (size_t)n * sizeof(int64_t) + 256;             // piv
  b += (size_t)nparts * sizeof(ArgMax) + 256;          // partials
  b += 2 * (kNB * sizeof(double) + 256);               // rowj, rowp
  b += (size_t)kNB * kNB * sizeof(double) + 256;       // inverse block
  b += (size_t)kNB * w * sizeof(double) + 256;         // row-block temp
  // split-K workspace of the largest GEMM issued (skinny ones)
  b += std::max({gemm_f64_workspace(kNB, w, kNB), gemm_f64_workspace(n, n, kNB),
                 gemm_f64_workspace(n, nrhs, kNB)}) + 256;
  return b;
}

void lu_solve_f64(hipStream_t s, int64_t n, double* A, double* Q, Arena& ws, int* info_dev) {
  lu_solve_f64(s, n, A, Q, n, n, ws, info_dev);
}

void lu_solve_f64(hipStream_t s, int64_t n, double* A, double* Q, int64_t ldq, int64_t nrhs, Arena& ws,
                  int* info_dev) {
  if (n <= 0) return;
  const int64_t lda = n;
  int64_t* piv = ws.get<int64_t>(n);
  ArgMax* part = ws.get<ArgMax>(cdiv(n, kRowsT) + 1);
  double* rowj = ws.get<double>(kNB);
  double* rowp = ws.get<double>(kNB);
  double* inv = ws.get<double>(kNB * kNB);
  double* tmp = ws.get<double>((size_t)kNB * std::max(n, nrhs));
  const size_t mark = ws.used;

  // ---------------- factorisation
  for (int64_t j0 = 0; j0 < n; j0 += kNB) {
    const int jb = (int)std::min<int64_t>(kNB, n - j0);
    // nparts: number of partials written by the previous launch (it covered
    // rows >= the previous column, so it may have one more block than the
    // rows below the current column need).
    int nparts = (int)cdiv(n - j0, kRowsT);
    hipLaunchKernelGGL(argmax_partial_kernel, dim3(nparts), dim3(kRowsT), 0, s, A, lda, n, j0, part);
    DME_HIP(hipGetLastError());
    for (int64_t j = j0; j < j0 + jb; ++j) {
      hipLaunchKernelGGL(pivot_final_kernel, dim3(1), dim3(kRowsT), 0, s, A, lda, j, j0, jb, part,
                         nparts, piv, rowj, rowp, info_dev);
      DME_HIP(hipGetLastError());
      const int nb = (int)cdiv(n - j, kRowsT);
      nparts = nb;
      // Partials written here are for column j + 1 and cover rows >= j; row j
      // itself contributes nothing (it takes the pivot row), so the next
      // pivot search over rows >= j + 1 is exact.
      hipLaunchKernelGGL(elim_kernel, dim3(nb), dim3(kRowsT), 0, s, A, lda, n, j, j0, jb, piv, rowj,
                         rowp, part);
      DME_HIP(hipGetLastError());
    }
    // swaps outside the panel and on the right-hand sides
    if (j0 > 0) {
      hipLaunchKernelGGL(swap_rows_kernel, dim3((unsigned)cdiv(j0, 256)), dim3(256), 0, s, A, lda,
                         (int64_t)0, j0, j0, jb, piv);
      DME_HIP(hipGetLastError());
    }
    if (j0 + jb < n) {
      hipLaunchKernelGGL(swap_rows_kernel, dim3((unsigned)cdiv(n - j0 - jb, 256)), dim3(256), 0, s,
                         A, lda, j0 + jb, n, j0, jb, piv);
      DME_HIP(hipGetLastError());
    }
    if (nrhs > 0)
      hipLaunchKernelGGL(swap_rows_kernel, dim3((unsigned)cdiv(nrhs, 256)), dim3(256), 0, s, Q, ldq,
                         (int64_t)0, nrhs, j0, jb, piv);
    DME_HIP(hipGetLastError());
    const int64_t rest = n - j0 - jb;
    if (rest > 0) {
      // U12 = inv(L11) A12
      hipLaunchKernelGGL(tri_inv_kernel, dim3(1), dim3(kNB), 0, s, A + j0 + j0 * lda, lda, jb, 1, inv);
      DME_HIP(hipGetLastError());
      double* A12 = A + j0 + (j0 + jb) * lda;
      copy_f64(s, A12, lda, tmp, jb, jb, rest);
      ws.used = mark;
      gemm_f64(s, 'N', 'N', jb, rest, jb, 1.0, inv, jb, tmp, jb, 0.0, A12, lda, &ws);
      // A22 -= L21 U12
      ws.used = mark;
      gemm_f64(s, 'N', 'N', rest, rest, jb, -1.0, A + (j0 + jb) + j0 * lda, lda, A12, lda, 1.0,
               A + (j0 + jb) + (j0 + jb) * lda, lda, &ws);
    }
  }

  if (nrhs <= 0) {
    ws.used = mark;
    return;
  }
  // ---------------- forward substitution L Y = Q (unit lower)
  for (int64_t i0 = 0; i0 < n; i0 += kNB) {
    const int ib = (int)std::min<int64_t>(kNB, n - i0);
    hipLaunchKernelGGL(tri_inv_kernel, dim3(1), dim3(kNB), 0, s, A + i0 + i0 * lda, lda, ib, 1, inv);
    DME_HIP(hipGetLastError());
    copy_f64(s, Q + i0, ldq, tmp, ib, ib, nrhs);
    ws.used = mark;
    gemm_f64(s, 'N', 'N', ib, nrhs, ib, 1.0, inv, ib, tmp, ib, 0.0, Q + i0, ldq, &ws);
    const int64_t below = n - i0 - ib;
    if (below > 0) {
      ws.used = mark;
      gemm_f64(s, 'N', 'N', below, nrhs, ib, -1.0, A + (i0 + ib) + i0 * lda, lda, Q + i0, ldq, 1.0,
               Q + i0 + ib, ldq, &ws);
    }
  }
  // ---------------- backward substitution U X = Y
  const int64_t nblk = cdiv(n, kNB);
  for (int64_t bi = nblk - 1; bi >= 0; --bi) {
    const int64_t i0 = bi * kNB;
    const int ib = (int)std::min<int64_t>(kNB, n - i0);
    hipLaunchKernelGGL(tri_inv_kernel, dim3(1), dim3(kNB), 0, s, A + i0 + i0 * lda, lda, ib, 0, inv);
    DME_HIP(hipGetLastError());
    copy_f64(s, Q + i0, ldq, tmp, ib, ib, nrhs);
    ws.used = mark;
    gemm_f64(s, 'N', 'N', ib, nrhs, ib, 1.0, inv, ib, tmp, ib, 0.0, Q + i0, ldq, &ws);
    if (i0 > 0) {
      ws.used = mark;
      gemm_f64(s, 'N', 'N', i0, nrhs, ib, -1.0, A + i0 * lda, lda, Q + i0, ldq, 1.0, Q, ldq, &ws);
    }
  }
  ws.used = mark;
}

}  // namespace dme
