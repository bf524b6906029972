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
//   L = P Q2 [V(0:r, :); 0] + U V(r:k, :), P = I - U U^T, with Q2 [I_r; 0] formed
//   on a second stream while the k x k eigenproblem runs
// P removes from Q2's columns the U components that rounding leaves in the
// directions where Y is (numerically) rank-deficient after the projection.
#include "tsqr.h"

#include <thread>
#include <vector>

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

// X (n x r, ld ldx) = [I_r; 0]
__global__ void eye_kernel(int64_t n, int64_t r, double* X, int64_t ldx) {
  const int64_t total = n * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx % n, c = idx / n;
    X[i + c * ldx] = (i == c) ? 1.0 : 0.0;
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

// Products with the tall orthonormal block U (n x q, q <= 64) on FP64 MFMA 16x16x4.
//   ts_partial_kernel: P_b = U_b^T Y_b for the row block b of nsub * 32 rows
//     (blockIdx.x) and 128 columns of Y (blockIdx.y). Stages of 32 rows of
//     U and Y go through LDS (coalesced column loads, prefetched one stage
//     ahead into registers); wave w forms the result rows 16 w .. 16 w + 15
//     for all 8 column tiles, lane group lk feeding K-steps 2 p, 2 p + 1 with
//     the stage rows 8 lk + 2 p, 8 lk + 2 p + 1 (one 16-byte LDS read each).
//   ts_reduce_kernel: sums the block partials in a fixed order.
//   ts_update_kernel: Y += sign U C, computed as tiles of Y^T = C^T U^T so
//     that the 16 lanes of one accumulator row hold 16 consecutive rows of
//     one column of Y (coalesced read-modify-write); C^T's operand stays in
//     registers and U streams through.
typedef double v4d_c __attribute__((ext_vector_type(4)));
constexpr int kTsMaxQ = 64;
constexpr int kTsSub = 32;                 // rows per LDS stage
constexpr int kTsLd = kTsSub + 2;          // LDS column stride in doubles (16-byte aligned)
constexpr int kTsSlots = kTsMaxQ + 128;    // U columns, then 128 columns of Y
constexpr int kTsLoads = kTsSlots / 4 / 4; // column quads per wave and stage
constexpr int kTsUpRowTiles = 2;           // 16-row tiles per wave in the update
constexpr int kTsUpRows = 16 * kTsUpRowTiles;

// V2: n, ldu, ldy even and U, Y 16-byte aligned, so a lane's row pair is one
// 16-byte load.
template <bool V2>
__global__ __launch_bounds__(256) void ts_partial_kernel(int64_t n, int q, int r, int nsub,
                                                         const double* __restrict__ U, int64_t ldu,
                                                         const double* __restrict__ Y, int64_t ldy,
                                                         double* __restrict__ P) {
  __shared__ __align__(16) double sm[2][kTsSlots * kTsLd];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int c0 = blockIdx.y * 128;
  const int rc = min(r - c0, 128);  // columns of Y in this block
  const int64_t rbase = (int64_t)blockIdx.x * nsub * kTsSub;
  const int rp = 2 * li;  // this lane's row pair within a stage (loads)

  double pre[kTsLoads][2];
  const auto load_stage = [&](int st) {
    const int64_t r0 = rbase + (int64_t)st * kTsSub + rp;
#pragma unroll
    for (int it = 0; it < kTsLoads; ++it) {
      const int slot = 4 * (w + 4 * it) + lk;
      const double* src = nullptr;
      if (slot < kTsMaxQ) {
        if (slot < q) src = U + (int64_t)slot * ldu;
      } else if (slot - kTsMaxQ < rc) {
        src = Y + (int64_t)(c0 + slot - kTsMaxQ) * ldy;
      }
      if (V2) {
        double2 v = make_double2(0.0, 0.0);
        if (src && r0 < n) v = *reinterpret_cast<const double2*>(src + r0);
        pre[it][0] = v.x;
        pre[it][1] = v.y;
      } else {
        pre[it][0] = (src && r0 < n) ? src[r0] : 0.0;
        pre[it][1] = (src && r0 + 1 < n) ? src[r0 + 1] : 0.0;
      }
    }
  };
  const auto store_stage = [&](int buf) {
#pragma unroll
    for (int it = 0; it < kTsLoads; ++it) {
      const int slot = 4 * (w + 4 * it) + lk;
      *reinterpret_cast<double2*>(&sm[buf][slot * kTsLd + rp]) = make_double2(pre[it][0], pre[it][1]);
    }
  };

  v4d_c acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = v4d_c{0.0, 0.0, 0.0, 0.0};
  const bool wq = 16 * w < q;  // wave-uniform

  load_stage(0);
  store_stage(0);
  __syncthreads();
  for (int st = 0; st < nsub; ++st) {
    if (st + 1 < nsub) load_stage(st + 1);
    if (wq) {
      const double* b = sm[st & 1];
#pragma unroll
      for (int p = 0; p < kTsSub / 8; ++p) {
        const int row = 8 * lk + 2 * p;
        const double2 a2 = *reinterpret_cast<const double2*>(&b[(16 * w + li) * kTsLd + row]);
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          if (16 * t < rc) {
            const double2 b2 = *reinterpret_cast<const double2*>(&b[(kTsMaxQ + 16 * t + li) * kTsLd + row]);
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.x, b2.x, acc[t], 0, 0, 0);
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a2.y, b2.y, acc[t], 0, 0, 0);
          }
        }
      }
    }
    if (st + 1 < nsub) store_stage((st + 1) & 1);
    __syncthreads();
  }
  if (!wq) return;
  double* Pb = P + (int64_t)blockIdx.x * q * r;
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + 4 * v + lk, j = 16 * t + li;
      if (i < q && j < rc) Pb[i + (int64_t)(c0 + j) * q] = acc[t][v];
    }
}

// out (q x r, ld q) = base + sign * sum_b P_b (base may be null: 0). A block of
// 256 threads serves 32 entries, eight threads each: thread slice z sums the
// blocks b = z mod 8 in a fixed grouping, and the eight slice sums are added in
// slice order.
constexpr int kTsRedCols = 32;
__global__ __launch_bounds__(256) void ts_reduce_kernel(int nb, int q, int r, const double* __restrict__ P,
                                                        const double* base, int64_t ldb, double sign,
                                                        double* out) {
  __shared__ double part[8][kTsRedCols];
  const int64_t total = (int64_t)q * r;
  const int e = threadIdx.x % kTsRedCols, z = threadIdx.x / kTsRedCols;
  const int64_t idx = (int64_t)blockIdx.x * kTsRedCols + e;
  double s0 = 0.0, s1 = 0.0;
  if (idx < total) {
    // blocks z, z + 8, ...: eight loads in flight per group
    int b = z;
    for (; b + 56 < nb; b += 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = P[(int64_t)(b + 8 * u) * total + idx];
      s0 += ((v[0] + v[1]) + (v[2] + v[3]));
      s1 += ((v[4] + v[5]) + (v[6] + v[7]));
    }
    for (; b < nb; b += 8) s0 += P[(int64_t)b * total + idx];
  }
  part[z][e] = s0 + s1;
  __syncthreads();
  if (z == 0 && idx < total) {
    double sum = 0.0;
#pragma unroll
    for (int t = 0; t < 8; ++t) sum += part[t][e];
    const int i = (int)(idx % q), j = (int)(idx / q);
    out[idx] = (base ? base[i + (int64_t)j * ldb] : 0.0) + sign * sum;
  }
}

// Block (x, y): rows x * kTsUpRows .. + kTsUpRows, columns y * 128 .. + 128;
// wave w takes the two 16-column tiles y * 128 + 32 w + 16 e (e = 0, 1) and
// the block's row tiles.
__global__ __launch_bounds__(256) void ts_update_kernel(int64_t n, int q, int r, const double* __restrict__ U,
                                                        int64_t ldu, const double* __restrict__ C, double sign,
                                                        double* __restrict__ Y, int64_t ldy) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int ctile = (int)blockIdx.y * 128 + 32 * w;
  if (ctile >= r) return;  // no barriers in this kernel
  const bool two = ctile + 16 < r;  // wave-uniform
  const int nks = (q + 3) / 4;
  // A = sign C^T: lane (li, lk) holds sign * C(4 kk + lk, ctile + 16 e + li)
  double a[2][kTsMaxQ / 4];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int col = ctile + 16 * e + li;
#pragma unroll
    for (int kk = 0; kk < kTsMaxQ / 4; ++kk) {
      const int kq = 4 * kk + lk;
      const double cv = C[min(kq, q - 1) + (int64_t)min(col, r - 1) * q];
      a[e][kk] = (kq < q && col < r) ? sign * cv : 0.0;
    }
  }
#pragma unroll
  for (int rt = 0; rt < kTsUpRowTiles; ++rt) {
    const int64_t r0 = (int64_t)blockIdx.x * kTsUpRows + 16 * rt;
    const int64_t row = r0 + li;
    const bool rok = row < n;
    const int64_t rc = rok ? row : n - 1;
    double bu[kTsMaxQ / 4];  // all loads issued before the products
#pragma unroll
    for (int kk = 0; kk < kTsMaxQ / 4; ++kk) bu[kk] = U[rc + (int64_t)min(4 * kk + lk, q - 1) * ldu];
    v4d_c acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < kTsMaxQ / 4; ++kk)
      if (kk < nks) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0][kk], bu[kk], acc0, 0, 0, 0);
        if (two) acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[1][kk], bu[kk], acc1, 0, 0, 0);
      }
    // acc_e[v] = (sign C^T U^T)(ctile + 16 e + 4 v + lk, row)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int col0 = ctile + 4 * v + lk, col1 = col0 + 16;
      if (rok && col0 < r) Y[row + (int64_t)col0 * ldy] += acc0[v];
      if (rok && col1 < r) Y[row + (int64_t)col1 * ldy] += acc1[v];
    }
  }
}

// The compression's rank goes to the host through the pinned, coherent slot
// of the bound auxiliary stream: one thread copies it and then bumps the
// slot's sequence number, and the host polls that number (a stream
// synchronisation sleeps, which costs tens of microseconds of idle device time
// per compression).
__global__ void rank_to_host_kernel(const int64_t* __restrict__ src, AuxStream::Slot* slot, int64_t seq) {
  if (threadIdx.x == 0) {
    const int64_t v = *(volatile const int64_t*)src;
    __hip_atomic_store(&slot->value, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&slot->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace

int64_t value_to_host_launch(hipStream_t s, const int64_t* src) {
  AuxStream& ax = aux_stream();
  const int64_t seq = ++ax.seq;
  hipLaunchKernelGGL(rank_to_host_kernel, dim3(1), dim3(64), 0, s, src, ax.slot, seq);
  DME_HIP(hipGetLastError());
  return seq;
}

int64_t value_to_host_wait(hipStream_t s, int64_t seq) {
  AuxStream::Slot* slot = aux_stream().slot;
  // poll for up to ~50 ms, then fall back to a synchronisation (which also
  // reports an error of the stream)
  for (int it = 0; it < 1000000; ++it) {
    if (__atomic_load_n(&slot->seq, __ATOMIC_ACQUIRE) == seq) return __atomic_load_n(&slot->value, __ATOMIC_RELAXED);
    if (it >= 1000) std::this_thread::yield();
    if (it >= 20000) break;
  }
  DME_HIP(hipStreamSynchronize(s));
  DME_REQUIRE(__atomic_load_n(&slot->seq, __ATOMIC_ACQUIRE) == seq, DME_EINTERNAL,
              "a device value did not reach the host");
  return __atomic_load_n(&slot->value, __ATOMIC_RELAXED);
}

namespace {

inline unsigned blocks_for(int64_t total) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(total, 256), 8192));
}

// Stages per row block of ts_partial_kernel (at most 256 row blocks).
inline int ts_nsub(int64_t n) { return (int)std::max<int64_t>(1, cdiv(n, 256 * kTsSub)); }
inline int ts_blocks(int64_t n) { return (int)cdiv(n, (int64_t)ts_nsub(n) * kTsSub); }

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
  // compress_f64_lead: C1, C2, Z, B (at most k x k each), the per-row-block
  // partial products of U^T Y, and its n-deep products
  add(4 * (size_t)k * k * sizeof(double));
  add((size_t)ts_blocks(n) * kTsMaxQ * k * sizeof(double));
  add((size_t)n * k * sizeof(double));  // Qe = Q2 [I; 0]
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
  // Qe = Q [I_kr; 0] on the second stream, beside the eigenproblem below
  double* Qe = ws.get<double>((size_t)n * kr);
  const size_t mark_q = ws.used;
  AuxStream& ax = aux_stream();
  DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
  hipLaunchKernelGGL(eye_kernel, dim3(blocks_for(n * kr)), dim3(256), 0, ax.s2, n, kr, Qe, n);
  DME_HIP(hipGetLastError());
  tsqr_apply_q(ax.s2, tq, Qe, n, kr);
  hipEvent_t qe_done = ax.record(ax.s2);

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
  const int64_t r = rank_to_host(s, rank_dev);
  if (r <= 0) {
    DME_HIP(hipStreamWaitEvent(s, qe_done, 0));  // the second stream still reads W
    return 0;
  }
  if (ldd <= 0) ldd = r;

  // ---------------- L = Q [V_I; 0] = Qe V_I, D = diag(lam_I)
  DME_HIP(hipStreamWaitEvent(s, qe_done, 0));
  gemm_f64(s, 'N', 'N', n, r, kr, 1.0, Qe, n, V, kr, 0.0, L, ldl, &ws);
  ws.used = mark_q;
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

  // Y <- P Y twice, C = C1 + C2
  const bool ts = q <= kTsMaxQ;
  const int nsub = ts_nsub(n), nch = ts_blocks(n);
  double* Pt = ts ? ws.get<double>((size_t)nch * q * k) : nullptr;
  const size_t mark0 = ws.used;
  const auto ts_project = [&](const double* Yp, int64_t ldy, int64_t cols, const double* base, int64_t ldb,
                              double sign, double* out) {
    const dim3 grid(nch, (unsigned)cdiv(cols, 128));
    const bool v2 = n % 2 == 0 && ldu % 2 == 0 && ldy % 2 == 0 && ((uintptr_t)U & 15) == 0 && ((uintptr_t)Yp & 15) == 0;
    if (v2)
      hipLaunchKernelGGL(ts_partial_kernel<true>, grid, dim3(256), 0, s, n, (int)q, (int)cols, nsub, U, ldu, Yp, ldy,
                         Pt);
    else
      hipLaunchKernelGGL(ts_partial_kernel<false>, grid, dim3(256), 0, s, n, (int)q, (int)cols, nsub, U, ldu, Yp,
                         ldy, Pt);
    DME_HIP(hipGetLastError());
    hipLaunchKernelGGL(ts_reduce_kernel, dim3((unsigned)cdiv(q * cols, kTsRedCols)), dim3(256), 0, s, nch, (int)q,
                       (int)cols, Pt, base, ldb, sign, out);
    DME_HIP(hipGetLastError());
  };
  const auto ts_update = [&](const double* Cm, int64_t cols, double sign, double* Yp, int64_t ldy) {
    const dim3 grid((unsigned)cdiv(n, kTsUpRows), (unsigned)cdiv(cols, 128));
    hipLaunchKernelGGL(ts_update_kernel, grid, dim3(256), 0, s, n, (int)q, (int)cols, U, ldu, Cm, sign, Yp, ldy);
    DME_HIP(hipGetLastError());
  };
  if (ts) {
    ts_project(W, n, r, nullptr, 0, 1.0, C1);
    ts_update(C1, r, -1.0, W, n);
    ts_project(W, n, r, nullptr, 0, 1.0, C2);
    ts_update(C2, r, -1.0, W, n);
  } else {
    gemm_f64(s, 'T', 'N', q, r, n, 1.0, U, ldu, W, n, 0.0, C1, q, &ws);
    ws.used = mark0;
    gemm_f64(s, 'N', 'N', n, r, q, -1.0, U, ldu, C1, q, 1.0, W, n, &ws);
    ws.used = mark0;
    gemm_f64(s, 'T', 'N', q, r, n, 1.0, U, ldu, W, n, 0.0, C2, q, &ws);
    ws.used = mark0;
    gemm_f64(s, 'N', 'N', n, r, q, -1.0, U, ldu, C2, q, 1.0, W, n, &ws);
    ws.used = mark0;
  }

  // Y = Q2 R2
  TsqrState tq;
  tsqr_factor(s, n, r, W, tq, ws);
  // Qe = Q2 [I_r; 0] on the second stream, beside the k x k eigenproblem
  // below (which needs none of it); L's Q2 part is then one product Qe V_top
  double* Qe = ws.get<double>((size_t)n * r);
  const size_t mark_q = ws.used;
  AuxStream& ax = aux_stream();
  DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
  hipLaunchKernelGGL(eye_kernel, dim3(blocks_for(n * r)), dim3(256), 0, ax.s2, n, r, Qe, n);
  DME_HIP(hipGetLastError());
  tsqr_apply_q(ax.s2, tq, Qe, n, r);
  hipEvent_t qe_done = ax.record(ax.s2);

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
  const int64_t rr = rank_to_host(s, rank_dev);
  if (rr <= 0) {
    DME_HIP(hipStreamWaitEvent(s, qe_done, 0));  // the second stream still reads W
    return 0;
  }
  if (ldd <= 0) ldd = rr;

  // L = P Q2 [V(0:r, :); 0] + U V(r:k, :) = Q2 [...] + U (V(r:k, :) - U^T Q2 [...])
  DME_HIP(hipStreamWaitEvent(s, qe_done, 0));
  gemm_f64(s, 'N', 'N', n, rr, r, 1.0, Qe, n, V, k, 0.0, L, ldl, &ws);
  ws.used = mark_q;
  if (ts) {
    ts_project(L, ldl, rr, V + r, k, -1.0, B);
    ts_update(B, rr, 1.0, L, ldl);
  } else {
    gemm_f64(s, 'T', 'N', q, rr, n, 1.0, U, ldu, L, ldl, 0.0, Z, q, &ws);
    ws.used = mark_q;
    hipLaunchKernelGGL(lower_minus_kernel, dim3(blocks_for(q * rr)), dim3(256), 0, s, V, k, r, q, rr, Z, B);
    DME_HIP(hipGetLastError());
    gemm_f64(s, 'N', 'N', n, rr, q, 1.0, U, ldu, B, q, 1.0, L, ldl, &ws);
    ws.used = mark_q;
  }
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(rr * rr)), dim3(256), 0, s, lam, rr, Dout, ldd);
  DME_HIP(hipGetLastError());
  return rr;
}

}  // namespace dme
