// Shared host/device helpers for the differential-matrix-equation library.
// All matrices are FP64 (or BF16 pieces of FP64 values) in column-major order.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/dme.h"

namespace dme {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string& msg);

#define DME_HIP(expr)                                                          \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess)                                                      \
      ::dme::fail(DME_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define DME_REQUIRE(cond, code, msg)                                           \
  do {                                                                         \
    if (!(cond)) ::dme::fail((code), (msg));                                   \
  } while (0)

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device buffer owned by the library (hipMalloc / hipFree).
// A buffer attached with attach() is borrowed: release() forgets it.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  bool own = true;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), own(o.own) { o.p = nullptr; o.bytes = 0; o.own = true; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; own = o.own;
      o.p = nullptr; o.bytes = 0; o.own = true;
    }
    return *this;
  }
  void attach(void* q, size_t b) { release(); p = q; bytes = b; own = false; }
  ~DevBuf() { release(); }
  void alloc(size_t b);
  void ensure(size_t b) { if (b > bytes) { release(); alloc(b); } }
  void release();
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Scratch arena that grows on demand; the pointers it hands out are valid
// until the next reset().  Used for per-call temporaries of the step-level
// entry points.
struct Arena {
  DevBuf buf;
  size_t used = 0;
  void reset() { used = 0; }
  // Reserve `bytes` of capacity up front (invalidates earlier pointers).
  void reserve(size_t bytes) { buf.ensure(bytes); used = 0; }
  // Hand out caller-provided device memory instead (borrowed: never freed,
  // never grown; get() beyond it fails with DME_EINTERNAL).
  void attach(void* p, size_t bytes) { buf.attach(p, bytes); used = 0; }
  template <class T> T* get(size_t count) {
    size_t b = (count * sizeof(T) + 255) & ~size_t(255);
    DME_REQUIRE(used + b <= buf.bytes, DME_EINTERNAL, "arena overflow");
    T* out = reinterpret_cast<T*>(static_cast<char*>(buf.p) + used);
    used += b;
    return out;
  }
};

// Optional hook around the main kernel of the step product (the skinny FP64
// kernel or the split-BF16 kernel): a caller that wants that one kernel's
// device time installs it for the current host thread; the launcher calls
// before() and after() on the launch stream with the product's shape
// (Y = E X, E m x k, X k x ncols) and the bytes per entry of E.
struct KernelTimer {
  virtual ~KernelTimer() = default;
  virtual void before(hipStream_t s) = 0;
  virtual void after(hipStream_t s, int64_t m, int64_t ncols, int64_t k, int e_bytes) = 0;
};
KernelTimer*& kernel_timer();

// ---------------------------------------------------------------------------
// Wave reductions on the DPP / permlane paths (register-to-register lane
// moves, no LDS round trip).  Every lane of a group ends with the group's sum,
// bitwise the same in every lane (each step adds a pair in both orders, and
// addition commutes).  Groups: 8 lanes (xor 1, 2, then the 8-lane mirror),
// 16 (the 16-lane mirror), 32 (swap of adjacent 16-lane rows) and the whole
// wave (swap of the two 32-lane halves).
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ inline double dpp_mov_f64(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  // every pattern used reads a valid lane, so no old value is kept (bound_ctrl)
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, true);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, true);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
#else
  return v;
#endif
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within 8
constexpr int kDppMirror = 0x140;     // lane i <-> 15 - i within 16
constexpr int kDppRor8 = 0x128;       // lane i <- lane i ^ 8 within 16 (rotate by 8)

// v + (v of the lane 16 (S = 16) or 32 (S = 32) away), by a permlane swap
template <int S>
__device__ inline double swap_sum_f64(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t l = (uint32_t)b, h = (uint32_t)(b >> 32);
  uint32_t l0, l1, h0, h1;
  if constexpr (S == 16) {
    const auto lo = __builtin_amdgcn_permlane16_swap(l, l, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(h, h, false, false);
    l0 = lo[0]; l1 = lo[1]; h0 = hi[0]; h1 = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane32_swap(l, l, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(h, h, false, false);
    l0 = lo[0]; l1 = lo[1]; h0 = hi[0]; h1 = hi[1];
  }
  const double a = __longlong_as_double((long long)(((uint64_t)h0 << 32) | l0));
  const double c = __longlong_as_double((long long)(((uint64_t)h1 << 32) | l1));
  return a + c;
#else
  return v;
#endif
}
// sum over aligned groups of 8 lanes
__device__ inline double group8_sum_f64(double v) {
  v += dpp_mov_f64<kDppXor1>(v);
  v += dpp_mov_f64<kDppXor2>(v);
  v += dpp_mov_f64<kDppHalfMirror>(v);
  return v;
}
// sum over aligned groups of 16 lanes
__device__ inline double group16_sum_f64(double v) {
  v = group8_sum_f64(v);
  return v + dpp_mov_f64<kDppMirror>(v);
}
// sum over aligned halves of the wave (32 lanes)
__device__ inline double half_wave_sum_f64(double v) { return swap_sum_f64<16>(group16_sum_f64(v)); }
// sum over the whole wave
__device__ inline double wave_sum_f64(double v) { return swap_sum_f64<32>(half_wave_sum_f64(v)); }

// ---------------------------------------------------------------------------
// Kernel launchers (each in its own .hip file)
// ---------------------------------------------------------------------------

// C = alpha * op(A) * op(B) + beta * C, FP64 MFMA.  op(X) = X ('N') or X^T ('T').
// M x N result, inner dimension K.  beta == 0 never reads C.
void gemm_f64(hipStream_t s, char ta, char tb, int64_t M, int64_t N, int64_t K,
              double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
              double beta, double* C, int64_t ldc, Arena* ws = nullptr);

// Workspace (bytes) gemm_f64 may need for a split-K launch of this shape.
size_t gemm_f64_workspace(int64_t M, int64_t N, int64_t K);

// Rows a workgroup of the step-product kernels takes (the FP64 skinny path
// and the split-BF16 product), the unit a row range of a product is cut in.
constexpr int kRowBlock = 128;
// C (m x N) = A (m x K, ld lda) B (K x N, ld ldb) by the FP64 step-product
// kernel with the inner dimension cut into ns chunks (a workgroup per
// kRowBlock rows and chunk); N <= 256, K >= 16.  ws provides ns m N doubles
// (+256 bytes).  A row range of a larger product is (A + row0, m).
void gemm_f64_rows(hipStream_t s, int64_t m, int64_t N, int64_t K, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc, int ns, Arena& ws);

// Elementwise / small helpers (elementwise.hip)
void fill_f64(hipStream_t s, double* X, int64_t rows, int64_t cols, int64_t ld, double v);
void copy_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy,
              int64_t rows, int64_t cols);
// Y = alpha * X^T (X rows x cols -> Y cols x rows)
void transpose_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy,
                   int64_t rows, int64_t cols, double alpha);
// Y = a*X1 + b*X2 + c*X3 + d*I   (any of X1..X3 may be null when its coefficient is 0)
void lincomb3_f64(hipStream_t s, int64_t n, double a, const double* X1, double b,
                  const double* X2, double c, const double* X3, double d, double* Y);
// X *= alpha (n x n, contiguous)
void scale_f64(hipStream_t s, double* X, int64_t count, double alpha);
// (U, V) -> (V - U, V + U) in place: U <- V - U, V <- V + U
void pade_pm_f64(hipStream_t s, double* U, double* V, int64_t count);
// column absolute sums -> colsum[n]; then device max -> out (1 double)
void norm1_f64(hipStream_t s, const double* X, int64_t rows, int64_t cols, int64_t ld,
               double* colsum, double* out);
// D <- blkdiag(D1 (k1 x k1, ld1), w * I_p) style assembly into a k x k matrix
void blkdiag2_f64(hipStream_t s, const double* D1, int64_t k1, int64_t ld1, const double* D2,
                  int64_t k2, int64_t ld2, double scale2, double* out, int64_t ldo);
// Scaled column block copy: Y[:, j] = alpha * X[:, j]
void copy_scaled_f64(hipStream_t s, const double* X, int64_t ldx, double* Y, int64_t ldy,
                     int64_t rows, int64_t cols, double alpha);
// out[0] = sum (A - B)^2, out[1] = sum B^2 over a rows x cols block (device
// doubles); `part` is a device scratch of diff_norms_workspace() bytes.
size_t diff_norms_workspace();
void diff_norms_f64(hipStream_t s, const double* A, int64_t lda, const double* B, int64_t ldb,
                    int64_t rows, int64_t cols, double* part, double* out);
// NaN/Inf scan: sets *flag = 1 if any entry of X is not finite.
void finite_check_f64(hipStream_t s, const double* X, int64_t rows, int64_t cols, int64_t ld,
                      int* flag);

// LU with partial pivoting and the Pade solve (lu.hip)
struct LuWork;
// Solve P X = Q in place (Q <- P^-1 Q); P is destroyed.  n x n contiguous.
// Returns through *info_dev (device int): 0 ok, j+1 if pivot j is exactly zero.
void lu_solve_f64(hipStream_t s, int64_t n, double* P, double* Q, Arena& ws, int* info_dev);
size_t lu_solve_workspace(int64_t n);
// The same with an n x nrhs right-hand side Q (ld ldq).
void lu_solve_f64(hipStream_t s, int64_t n, double* P, double* Q, int64_t ldq, int64_t nrhs, Arena& ws,
                  int* info_dev);
size_t lu_solve_workspace(int64_t n, int64_t nrhs);

// A second stream beside the caller's, a ring of events for the waits
// between the two, and a pinned, coherent host slot through which a one-thread
// kernel hands a scalar (a compression's rank) to the host without a stream
// synchronisation.  Every solver and every context owns one: it is created on
// first use (on the current device) and destroyed with its owner, after the
// owner's stream and the second stream are synchronised, so no event or slot
// outlives the work that uses it.  The owner binds it to the calling host
// thread (AuxBinding) while it enqueues work; the tree QR, the compressions
// and the eigensolver use the bound one.
struct AuxStream {
  struct Slot {
    int64_t value;
    int64_t seq;
  };
  int device = -1;
  hipStream_t s2 = nullptr;
  std::vector<hipEvent_t> ev;
  size_t next = 0;
  Slot* slot = nullptr;  // pinned, coherent host memory
  int64_t seq = 0;       // last sequence number handed to the slot
  AuxStream() = default;
  AuxStream(const AuxStream&) = delete;
  AuxStream& operator=(const AuxStream&) = delete;
  ~AuxStream() { release(); }
  // Create the stream, events and slot on device `dev` (the current device).
  void ensure(int dev);
  // Synchronise the second stream and destroy what ensure() created.
  void release();
  // A recorded event is only waited on by calls enqueued right after its
  // record, so a ring much longer than the waits in flight can be reused.
  hipEvent_t record(hipStream_t st) {
    hipEvent_t e = ev[next];
    next = (next + 1) % ev.size();
    DME_HIP(hipEventRecord(e, st));
    return e;
  }
};
// The AuxStream bound to the calling thread (created on first use); fails
// with DME_EINTERNAL when none is bound.
AuxStream& aux_stream();
// Binds `a` to the calling thread for the lifetime of the binding (nestable).
class AuxBinding {
 public:
  explicit AuxBinding(AuxStream& a);
  ~AuxBinding();
  AuxBinding(const AuxBinding&) = delete;
  AuxBinding& operator=(const AuxBinding&) = delete;

 private:
  AuxStream* prev_;
};

// Householder QR + eigen compression (compress.hip)
size_t compress_workspace(int64_t n, int64_t k);
// W (n x k, ld n) is destroyed.  Dhat k x k (ld k).  Output L (n x r, ld ldl), Dout (r x r, ld ldd).
// rank_dev: device int64 receiving r; flag_dev: device int receiving error flags
// (1: non-finite, 2: rank capped at max_rank).  Waits on the host until the rank is
// known (the stream's earlier work is done) and returns r.
int64_t compress_f64(hipStream_t s, int64_t n, int64_t k, double* W, const double* Dhat, double tol,
                  int64_t max_rank, double* L, int64_t ldl, double* Dout, int64_t ldd,
                  int64_t* rank_dev, int* flag_dev, Arena& ws);
// The same compression through the Gram matrix (gram.hip) for a symmetric
// positive definite Dhat (ld lddh; dhat_diag: Dhat is diagonal): Dhat = F F^T,
// G = F^T W^T W F, G = V Lam V^T truncated, L = W F V_I Lam_I^-1/2.  W (n x k,
// ld ldw) is read only.  Returns the kept rank, or -1 (nothing written) when
// Dhat is not numerically positive definite.  L must hold min(max_rank, k)
// columns: the products forming L are queued for a guessed width (rank_hint +
// 8 columns, rank_hint <= 0: every column) before the rank reaches the host,
// so that the round trip overlaps them; columns from the rank on come out zero,
// and a rank above the guess is served by a second product.
//
// lowrank (optional): the D blocks of Dhat (rows and columns [c r, (c + 1) r)
// for c < ncopies; the rest of Dhat is diagonal) are diag(lam) - t Z Z^T, the
// Riccati update of a diagonal D (lam r, Z r x m with m <= 8, device).  Their
// factor is then formed directly, F_D = Lam^1/2 (I - Zh K Zh^T) with
// Zh = sqrt(t) Lam^-1/2 Z and K = (I + (I - Zh^T Zh)^1/2)^-1 (an m x m matrix
// function): F_D F_D^T = Lam^1/2 (I - Zh Zh^T) Lam^1/2, with no Cholesky.
struct LowRankD {
  const double* lam;
  const double* Z;
  double t;
  int64_t r, m;
  int ncopies;
};
size_t compress_gram_workspace(int64_t n, int64_t k);
//
// F_ready (optional, k x k, ld k): the factor of Dhat already formed on the
// device by gram_factor_lowrank, ordered before the work s holds; its status
// (0, or -1 when Dhat is not positive definite) in *status_ready.
// T_keep (optional, k x min(max_rank, k), ld k): receives T = F V_I
// Lam_I^-1/2, so that L = W T (columns from the rank on zero).
// beside (optional): called once, after the Gram matrix and before the
// eigensolver are enqueued, with an event recorded on s there; work the
// caller enqueues on another stream after that event runs beside the
// eigensolver's one-workgroup tridiagonal reduction.
int64_t compress_gram_f64(hipStream_t s, int64_t n, int64_t k, const double* W, int64_t ldw,
                          const double* Dhat, int64_t lddh, bool dhat_diag, const LowRankD* lowrank,
                          double tol, int64_t max_rank, double* L, int64_t ldl, double* Dout, int64_t ldd,
                          int64_t* rank_dev, int* flag_dev, Arena& ws, int64_t rank_hint = 0,
                          const double* F_ready = nullptr, const int64_t* status_ready = nullptr,
                          double* T_keep = nullptr, const std::function<void(hipEvent_t)>* beside = nullptr);
// Launches the closed-form factor F (k x k, ld k) of a Dhat in the LowRankD
// form on st, with its status in *status; returns false, launching nothing,
// when the form's limits (m <= 8, r <= 256) do not hold.
bool gram_factor_lowrank(hipStream_t st, int64_t k, const double* Dhat, int64_t lddh, const LowRankD& lr,
                         double* F, int64_t* status);
// A device int64 to the host through the bound auxiliary stream's pinned slot:
// launch() enqueues the copy on s and returns its sequence number (the value
// sent is -1 instead when *veto is nonzero), wait() polls for it (falling back
// to a stream synchronisation), rank_to_host() does both.
int64_t value_to_host_launch(hipStream_t s, const int64_t* src, const int64_t* veto = nullptr);
int64_t value_to_host_wait(hipStream_t s, int64_t seq);
inline int64_t rank_to_host(hipStream_t s, const int64_t* rank_dev) {
  return value_to_host_wait(s, value_to_host_launch(s, rank_dev));
}

// Symmetric eigen-decomposition of a k x k matrix (syev.hip).
// Eigenvalues sorted by |lambda| descending; only those with |lambda| > tol*max|lambda|
// (at most max_keep) get eigenvectors.  Writes kept count to *keep_dev.
// A caller that finishes the vectors itself can leave the sign convention
// (largest |entry| of each column positive, the first on ties) to its own
// kernels (signs = false), and have the kept count sent to the host through
// the bound auxiliary stream as soon as it is known (rank_seq set: the
// sequence number for value_to_host_wait on the second stream; the value is
// -1 when *rank_veto is nonzero).
struct SyevPost {
  bool signs = true;
  const int64_t* rank_veto = nullptr;
  int64_t* rank_seq = nullptr;
};
size_t syev_workspace(int64_t k);
void syev_trunc_f64(hipStream_t s, int64_t k, const double* M, int64_t ldm, double tol,
                    int64_t max_keep, double* lam_out, double* V_out, int64_t ldv,
                    int64_t* keep_dev, int* flag_dev, Arena& ws, const SyevPost& post = SyevPost());

// Riccati subflow (riccati.hip): D (r x r) <- D - t D W (R + t W^T D W)^-1 W^T D, W = L^T B.
// LQR feedback gain K (m x n, ld ldk) = R^-1 B^T L D L^T (riccati.hip).
void feedback_gain_f64(hipStream_t s, int64_t n, int64_t r, int64_t m, const double* L, int64_t ldl,
                       const double* D, int64_t ldd, const double* B, int64_t ldb, const double* R,
                       int64_t ldr, double* K, int64_t ldk, int* flag_dev, Arena& ws);
// Zout (optional, r x m, ld r): receives Z with D_new = sym(D) - t Z Z^T.
void riccati_update_f64(hipStream_t s, int64_t r, int64_t m, double* D, int64_t ldd,
                        const double* WB, int64_t ldw, const double* R, int64_t ldr, double t,
                        int* flag_dev, Arena& ws, double* Zout = nullptr);

}  // namespace dme
