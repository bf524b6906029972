// Column compression of P = W Dhat W^T (the step that follows every
// concatenation in Alg. 1, 2 and 4; method described in Sec. 3 after Alg. 2):
//
//   Householder QR   W = Q R            (tree QR by 32-column panels, tsqr.hip)
//   small product    M = R Dhat R^T     (FP64 MFMA GEMM)
//   eigenpairs       M = V Lam V^T      (syev.hip), keep |lam| > tol max|lam|
//   new factor       L = Q [V_I; 0],  D = diag(Lam_I)
//
// This is the oracle's formulation; it serves the step-level dme_compress, the
// quadrature factor of the setup, and the solver's compressions whose Dhat is
// not positive definite (the others go through the Gram matrix, gram.hip).
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

// A device int64 reaches the host through the pinned, coherent slot of the
// bound auxiliary stream: one thread copies it and then bumps the slot's
// sequence number, and the host polls that number (a stream synchronisation
// sleeps, which costs tens of microseconds of idle device time per call).
__global__ void rank_to_host_kernel(const int64_t* __restrict__ src, const int64_t* __restrict__ veto,
                                    AuxStream::Slot* slot, int64_t seq) {
  if (threadIdx.x == 0) {
    int64_t v = *(volatile const int64_t*)src;
    if (veto && *(volatile const int64_t*)veto != 0) v = -1;
    __hip_atomic_store(&slot->value, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&slot->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}

}  // namespace

int64_t value_to_host_launch(hipStream_t s, const int64_t* src, const int64_t* veto) {
  AuxStream& ax = aux_stream();
  const int64_t seq = ++ax.seq;
  hipLaunchKernelGGL(rank_to_host_kernel, dim3(1), dim3(64), 0, s, src, veto, ax.slot, seq);
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
  add((size_t)n * k * sizeof(double));  // Qe = Q [I; 0]
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

}  // namespace dme
