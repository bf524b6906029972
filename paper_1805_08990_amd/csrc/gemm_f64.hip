// FP64 MFMA GEMM for gfx950: C = alpha * op(A) op(B) + beta * C, column-major.
//
// Used for every dense product of the method: the Pade powers and the
// squaring phase of e^{tX} (n x n x n), the LU trailing update and the
// triangular solves, the step product e^{tA^T} L (n x n x r) and the
// tall-skinny products of the Householder compression (split-K).
//
// Tile structure: a 256-thread workgroup (4 wave64s as 2 x 2) owns a BM x BN
// block of C; op(A) and op(B) slabs of depth BK are staged through LDS with
// the next slab prefetched into registers while the current one feeds
// v_mfma_f64_16x16x4_f64.  The MFMA is fed with op(B) as its first operand
// and op(A) as its second so that the accumulator lanes hold 16 consecutive
// rows of C: the epilogue stores are then contiguous 128-byte runs of a C
// column.  Split-K writes partial tiles to a workspace and a second kernel
// adds them in fixed order, so results are deterministic.
#include "common.h"

namespace dme {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kPad = 16;  // LDS row padding in doubles (staggers the 4 k-rows of a fragment read)

template <int BM, int BN, int BK, bool TA, bool TB>
__global__ __launch_bounds__(kThreads) void gemm_f64_kernel(
    int M, int N, int K, int kchunk, double alpha, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    double* __restrict__ partial) {
  constexpr int WTM = BM / 2, WTN = BN / 2;  // wave tile
  constexpr int TM = WTM / 16, TN = WTN / 16;
  constexpr int LA = BM * BK / kThreads;  // A elements per thread per slab
  constexpr int LB = BN * BK / kThreads;
  static_assert(LA * kThreads == BM * BK && LB * kThreads == BN * BK, "tile/thread mismatch");

  __shared__ double sA[BK][BM + kPad];
  __shared__ double sB[BK][BN + kPad];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int m0 = blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);

  v4d acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[LA], rb[LB];

  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int idx = tid + i * kThreads;
      int ml, kl;
      if (!TA) { ml = idx % BM; kl = idx / BM; }
      else     { kl = idx % BK; ml = idx / BK; }
      const int m = m0 + ml, k = k0 + kl;
      double v = 0.0;
      if (m < M && k < kend) v = TA ? A[k + (int64_t)m * lda] : A[m + (int64_t)k * lda];
      ra[i] = v;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + i * kThreads;
      int nl, kl;
      if (!TB) { kl = idx % BK; nl = idx / BK; }
      else     { nl = idx % BN; kl = idx / BN; }
      const int n = n0 + nl, k = k0 + kl;
      double v = 0.0;
      if (n < N && k < kend) v = TB ? B[n + (int64_t)k * ldb] : B[k + (int64_t)n * ldb];
      rb[i] = v;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int idx = tid + i * kThreads;
      int ml, kl;
      if (!TA) { ml = idx % BM; kl = idx / BM; }
      else     { kl = idx % BK; ml = idx / BK; }
      sA[kl][ml] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + i * kThreads;
      int nl, kl;
      if (!TB) { kl = idx % BK; nl = idx / BK; }
      else     { nl = idx % BN; kl = idx / BN; }
      sB[kl][nl] = rb[i];
    }
  };

  const int r16 = lane & 15;
  const int kq = lane >> 4;

  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();
    store();
    __syncthreads();
    if (k0 + BK < kend) load(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      double fa[TN], fb[TM];
#pragma unroll
      for (int j = 0; j < TN; ++j) fa[j] = sB[kk * 4 + kq][wn * WTN + j * 16 + r16];
#pragma unroll
      for (int i = 0; i < TM; ++i) fb[i] = sA[kk * 4 + kq][wm * WTM + i * 16 + r16];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[j], fb[i], acc[i][j], 0, 0, 0);
    }
  }

  // Epilogue.  The FP64 16x16x4 MFMA leaves element v of lane l at row
  // 4 v + l / 16, column l % 16 of its 16 x 16 result (rows of the result are
  // columns of C here): lane holds C(m = base_m + r16, n = base_n + 4*v + kq).
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int m = m0 + wm * WTM + i * 16 + r16;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int n = n0 + wn * WTN + j * 16 + v * 4 + kq;
        if (m < M && n < N) {
          if (partial) {
            partial[(int64_t)blockIdx.z * M * N + m + (int64_t)n * M] = acc[i][j][v];
          } else {
            double* c = C + m + (int64_t)n * ldc;
            const double out = alpha * acc[i][j][v];
            *c = (beta == 0.0) ? out : out + beta * (*c);
          }
        }
      }
    }
  }
}

// C = alpha * sum_z partial[z] + beta * C, summed in z order.
__global__ void splitk_reduce_kernel(int M, int N, int nsplit, double alpha,
                                     const double* __restrict__ partial, double beta,
                                     double* __restrict__ C, int64_t ldc) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    // eight loads in flight, four chains (the loop is latency-bound otherwise)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int z = 0;
    for (; z + 8 <= nsplit; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(z + u) * total + idx];
      s0 += v[0] + v[4];
      s1 += v[1] + v[5];
      s2 += v[2] + v[6];
      s3 += v[3] + v[7];
    }
    for (; z < nsplit; ++z) s0 += partial[(int64_t)z * total + idx];
    const double s = (s0 + s1) + (s2 + s3);
    const int64_t m = idx % M, n = idx / M;
    double* c = C + m + n * ldc;
    const double out = alpha * s;
    *c = (beta == 0.0) ? out : out + beta * (*c);
  }
}

// Small products (M, N <= kSmallMaxMN, K <= kSmallMaxK: the k x k products of
// the compression and the eigensolver).  The tiled kernel gives them only a
// few 64 x 64 tiles, each a long chain of slabs; here a 4-wave workgroup owns
// a 16 x 16 tile of C and its waves take every fourth 4-deep step of K, with
// operands loaded straight from global memory (they are L2-resident) four
// steps ahead, and the four partial tiles are added in wave order through LDS
// (deterministic).  Same lane layout and epilogue as gemm_f64_kernel.
// Longer K with at most kSmallSplitTiles tiles of C (the r x m product L^T B
// of the Riccati step): the grid also splits K into chunks of about
// kSmallChunk, whose partial tiles splitk_reduce_kernel adds in chunk order.
constexpr int kSmallMaxMN = 256;
constexpr int kSmallMaxK = 2048;
constexpr int kSmallUnroll = 4;
constexpr int kSmallSplitTiles = 16;
constexpr int kSmallChunk = 512;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f64_small_kernel(int M, int N, int K, int kchunk, double alpha,
                                                             const double* __restrict__ A, int64_t lda,
                                                             const double* __restrict__ B, int64_t ldb,
                                                             double beta, double* __restrict__ C, int64_t ldc,
                                                             double* __restrict__ partial) {
  __shared__ v4d red[3][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  const int m = blockIdx.x * 16 + r16, n = blockIdx.y * 16 + r16;
  const bool min_ = m < M, nin = n < N;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  auto opA = [&](int k) -> double {
    return (min_ && k < kend) ? (TA ? A[k + (int64_t)m * lda] : A[m + (int64_t)k * lda]) : 0.0;
  };
  auto opB = [&](int k) -> double {
    return (nin && k < kend) ? (TB ? B[n + (int64_t)k * ldb] : B[k + (int64_t)n * ldb]) : 0.0;
  };
  v4d acc = v4d{0.0, 0.0, 0.0, 0.0};
  // wave w: steps k0 = kbeg + 4 (w + 4 s); kSmallUnroll steps loaded before they are used
  for (int k0 = kbeg + 4 * wave; k0 < kend; k0 += 16 * kSmallUnroll) {
    double fa[kSmallUnroll], fb[kSmallUnroll];
#pragma unroll
    for (int u = 0; u < kSmallUnroll; ++u) {
      const int k = k0 + 16 * u + kq;
      fa[u] = opB(k);
      fb[u] = opA(k);
    }
#pragma unroll
    for (int u = 0; u < kSmallUnroll; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[u], fb[u], acc, 0, 0, 0);
  }
  if (wave > 0) red[wave - 1][lane] = acc;
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int w = 0; w < 3; ++w) acc += red[w][lane];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int nn = blockIdx.y * 16 + v * 4 + kq;
      if (min_ && nn < N) {
        if (partial) {
          partial[(int64_t)blockIdx.z * M * N + m + (int64_t)nn * M] = acc[v];
        } else {
          double* c = C + m + (int64_t)nn * ldc;
          const double out = alpha * acc[v];
          *c = (beta == 0.0) ? out : out + beta * (*c);
        }
      }
    }
  }
}

// Gram products C = alpha W^T W + beta C of a tall W (n x k, k <= 192, n >=
// kSyMinK): the compression's W^T W.  A workgroup (eight waves) stages 64-row
// blocks of W in LDS (each row block read from HBM once, every load of a
// thread issued before its first LDS store) and accumulates the upper 16 x 16
// tiles of W_b^T W_b on FP64 MFMA, a wave taking every eighth tile pair, so
// that a tile's accumulator is updated once per 4-deep step with the other
// pairs' MFMAs between (no dependent issue), two waves per SIMD.  Workgroup b
// adds row blocks b, b + grid, ... and writes its upper tiles to partial[b];
// a second kernel sums the partials and writes both triangles from the upper
// one (C is exactly symmetric).
constexpr int kSyMaxT = 12;     // k <= 192
constexpr int kSyRows = 64;     // rows of W per LDS stage
constexpr int kSyMinK = 2048;   // rows of W from which this path is taken
constexpr int kSyMaxGrid = 256;
constexpr int kSyWaves = 8;

template <int T>
__global__ __launch_bounds__(64 * kSyWaves) void syrk_tn_kernel(int n, int k, const double* __restrict__ W,
                                                                int64_t ldw, double* __restrict__ partial) {
  constexpr int NP = T * (T + 1) / 2;                     // upper tile pairs
  constexpr int PW = (NP + kSyWaves - 1) / kSyWaves;      // pairs per wave
  constexpr int LD = 16 * T + 1;                          // LDS row stride (doubles)
  constexpr int NL = kSyRows * 16 * T / (64 * kSyWaves);  // entries a thread stages per block
  extern __shared__ double sW[];                          // kSyRows x LD
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  int ta[PW], tb[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) {
    int p = wave + kSyWaves * q, b = 0;
    while (p >= b + 1) {  // pair p = b (b + 1) / 2 + a, a <= b
      p -= b + 1;
      ++b;
    }
    ta[q] = p;
    tb[q] = b;
  }
  v4d acc[PW];
#pragma unroll
  for (int q = 0; q < PW; ++q) acc[q] = v4d{0.0, 0.0, 0.0, 0.0};
  for (int blk = blockIdx.x; (int64_t)blk * kSyRows < n; blk += gridDim.x) {
    const int64_t r0 = (int64_t)blk * kSyRows;
    // row lane of the block, columns wave + 8 u (an entry out of range reads
    // entry 0 and is zeroed, so that the loads need no branch)
    const bool rok = r0 + lane < n;
    double st[NL];
#pragma unroll
    for (int u = 0; u < NL; ++u) {
      const int col = wave + kSyWaves * u;
      const bool ok = rok && col < k;
      st[u] = W[ok ? r0 + lane + (int64_t)col * ldw : 0];
      st[u] = ok ? st[u] : 0.0;
    }
    __syncthreads();  // the previous stage is consumed
#pragma unroll
    for (int u = 0; u < NL; ++u) sW[lane * LD + wave + kSyWaves * u] = st[u];
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < kSyRows / 4; ++kk) {
      const double* rowp = sW + (4 * kk + kq) * LD + r16;
#pragma unroll
      for (int q = 0; q < PW; ++q)
        if (wave + kSyWaves * q < NP)
          acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(rowp[16 * tb[q]], rowp[16 * ta[q]], acc[q], 0, 0, 0);
    }
  }
  // lane holds C(m = 16 ta + r16, n = 16 tb + 4 v + kq) of each of its tiles
  double* out = partial + (int64_t)blockIdx.x * k * k;
#pragma unroll
  for (int q = 0; q < PW; ++q)
    if (wave + kSyWaves * q < NP) {
      const int m = 16 * ta[q] + r16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int nn = 16 * tb[q] + 4 * v + kq;
        if (m < k && nn < k) out[m + (int64_t)nn * k] = acc[q][v];
      }
    }
}

// C(i, j) = C(j, i) = alpha sum_b partial[b](i, j) (+ beta C) over the upper
// triangle i <= j: a block takes 32 entries and its eight 32-thread groups
// the partials b = g mod 8 (eight loads in flight each); the group sums are
// added in a fixed order (deterministic).
__global__ __launch_bounds__(256) void syrk_reduce_kernel(int k, int nb, double alpha,
                                                          const double* __restrict__ partial, double beta,
                                                          double* __restrict__ C, int64_t ldc) {
  __shared__ double red[8][33];
  const int64_t kk = (int64_t)k * k, nup = (int64_t)k * (k + 1) / 2;
  const int e = threadIdx.x & 31, g = threadIdx.x >> 5;
  for (int64_t base = (int64_t)blockIdx.x * 32; base < nup; base += (int64_t)gridDim.x * 32) {
    const int64_t u = base + e;
    int i = 0, j = 0;
    if (u < nup) {  // u = j (j + 1) / 2 + i, i <= j
      j = (int)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
      while ((int64_t)j * (j + 1) / 2 > u) --j;
      while ((int64_t)(j + 1) * (j + 2) / 2 <= u) ++j;
      i = (int)(u - (int64_t)j * (j + 1) / 2);
    }
    const double* pp = partial + i + (int64_t)j * k;
    double sc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (u < nup) {
      int b = g;
      for (; b + 56 < nb; b += 64) {
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = pp[(int64_t)(b + 8 * q) * kk];
#pragma unroll
        for (int q = 0; q < 8; ++q) sc[q] += v[q];
      }
      for (; b < nb; b += 8) sc[0] += pp[(int64_t)b * kk];
    }
    red[g][e] = ((sc[0] + sc[1]) + (sc[2] + sc[3])) + ((sc[4] + sc[5]) + (sc[6] + sc[7]));
    __syncthreads();
    if (g == 0 && u < nup) {
      const double sum = ((red[0][e] + red[1][e]) + (red[2][e] + red[3][e])) +
                         ((red[4][e] + red[5][e]) + (red[6][e] + red[7][e]));
      const double out = alpha * sum;
      double* c1 = C + i + (int64_t)j * ldc;
      double* c2 = C + j + (int64_t)i * ldc;
      if (beta == 0.0) {
        *c1 = out;
        *c2 = out;
      } else {
        const double v1 = out + beta * (*c1);
        const double v2 = (i == j) ? v1 : out + beta * (*c2);
        *c1 = v1;
        *c2 = v2;
      }
    }
    __syncthreads();  // red is reused
  }
}

int syrk_grid(int64_t n) { return (int)std::min<int64_t>(cdiv(n, kSyRows), kSyMaxGrid); }

bool use_syrk(char ta, char tb, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
              const double* B, int64_t ldb) {
  return (ta == 'T' || ta == 't') && (tb == 'N' || tb == 'n') && A == B && lda == ldb && M == N &&
         M <= 16 * kSyMaxT && K >= kSyMinK;
}

template <int BM, int BN, int BK, bool TA, bool TB>
void launch_tile(hipStream_t s, int M, int N, int K, int nsplit, int kchunk, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc, double* partial) {
  dim3 grid((unsigned)cdiv(M, BM), (unsigned)cdiv(N, BN), (unsigned)nsplit);
  hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, BK, TA, TB>), grid, dim3(kThreads), 0, s, M, N, K,
                     kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
}

template <int BM, int BN, int BK>
void dispatch_trans(hipStream_t s, char ta, char tb, int M, int N, int K, int nsplit, int kchunk,
                    double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                    double beta, double* C, int64_t ldc, double* partial) {
  const bool TA = (ta == 'T' || ta == 't');
  const bool TB = (tb == 'T' || tb == 't');
  if (!TA && !TB)
    launch_tile<BM, BN, BK, false, false>(s, M, N, K, nsplit, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  else if (TA && !TB)
    launch_tile<BM, BN, BK, true, false>(s, M, N, K, nsplit, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  else if (!TA && TB)
    launch_tile<BM, BN, BK, false, true>(s, M, N, K, nsplit, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  else
    launch_tile<BM, BN, BK, true, true>(s, M, N, K, nsplit, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
}

// Skinny product Y = E X for a tall square operator E (M x K, M, K large)
// and a narrow X (K x N, N <= 256): the step product e^{tA^T} L.  A 512-thread
// workgroup owns 128 rows of Y and every column (TN 16-column tiles); wave w
// owns rows w*16 .. w*16+15, so each entry of E is read from HBM by exactly one
// wave, straight into registers (a lane reads 16 consecutive rows of one
// column per load).  The X slab of a K step (16 x 16 TN) is staged in LDS,
// double-buffered, and shared by the eight waves (measured at n = 16384,
// r = 122: 1.39 ms against 1.59 ms with four waves and 64 rows; two row tiles
// per wave, a 32-deep slab or other K splits did not do better).  K is split into nsplit
// chunks and workgroup b takes chunk b % nsplit: with nsplit = 8 each chunk
// (and its slice of X, K/8 x N doubles) belongs to one XCD and its L2.  Every
// column's arithmetic is the same whatever N is, so batching columns of
// several problems does not change any result.
constexpr int kSkBK = 16;
constexpr int kSkThreads = 512;
constexpr int kSkRows = 16 * (kSkThreads / 64);

template <int TN>
__global__ __launch_bounds__(kSkThreads) void gemm_f64_skinny_kernel(
    int M, int N, int K, int nsplit, int kchunk, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double* __restrict__ partial) {
  constexpr int NC = TN * 16;
  constexpr int LB = (kSkBK * NC + kSkThreads - 1) / kSkThreads;  // X entries per thread per slab
  __shared__ double sB[2][kSkBK][NC + 8];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int split = blockIdx.x % nsplit;
  const int rb = blockIdx.x / nsplit;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int r16 = lane & 15;
  const int kq = lane >> 4;
  const int row = rb * kSkRows + wave * 16 + r16;
  const bool row_ok = row < M;

  v4d acc[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) acc[j] = v4d{0.0, 0.0, 0.0, 0.0};

  // A (the n x n operator, streamed from HBM) passes through a two-slab ring:
  // a slab's fragments are loaded two slabs ahead, about 3 us at this shape,
  // beyond the loaded HBM latency
  double ra[2][4], rb_[LB];
  auto load_a = [&](int k0, double (&dst)[4]) {
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int k = k0 + s4 * 4 + kq;
      dst[s4] = (row_ok && k < kend) ? A[row + (int64_t)k * lda] : 0.0;
    }
  };
  auto load_b = [&](int k0) {
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + i * kSkThreads;
      const int kl = idx % kSkBK, c = idx / kSkBK;
      const int k = k0 + kl;
      rb_[i] = (c < N && k < kend && idx < kSkBK * NC) ? B[k + (int64_t)c * ldb] : 0.0;
    }
  };
  auto store_b = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int idx = tid + i * kSkThreads;
      if (idx < kSkBK * NC) {
        const int kl = idx % kSkBK, c = idx / kSkBK;
        sB[buf][kl][c] = rb_[i];
      }
    }
  };

  if (kbeg < kend) {
    load_b(kbeg);
    store_b(0);
    load_a(kbeg, ra[0]);
    load_a(kbeg + kSkBK, ra[1]);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += 2 * kSkBK) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int kc = k0 + u * kSkBK;
      if (kc < kend) {  // uniform
        const bool more = (kc + kSkBK) < kend;
        if (more) load_b(kc + kSkBK);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            const double bv = sB[buf][s4 * 4 + kq][j * 16 + r16];
            acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ra[u][s4], bv, acc[j], 0, 0, 0);
          }
        }
        if (kc + 2 * kSkBK < kend) load_a(kc + 2 * kSkBK, ra[u]);
        if (more) store_b(buf ^ 1);
        __syncthreads();
        buf ^= 1;
      }
    }
  }

  // element v of lane l holds row 4 v + l / 16 (of the wave's 16) of column
  // l % 16 of each tile (FP64 16x16x4 MFMA result layout)
  const int rowb = rb * kSkRows + wave * 16 + kq;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int col = j * 16 + r16;
    if (col < N) {
      double* dst = partial + ((int64_t)split * N + col) * M;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        if (rowb + 4 * v < M) dst[rowb + 4 * v] = acc[j][v];
    }
  }
}

// C(i, j) = alpha * sum_z partial[z][j][i] + beta * C(i, j), FP64, fixed order.
__global__ void skinny_reduce_kernel(int M, int N, int nsplit, double alpha,
                                     const double* __restrict__ partial, double beta,
                                     double* __restrict__ C, int64_t ldc) {
  const int64_t total = (int64_t)M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    // eight loads in flight, four chains (the loop is latency-bound otherwise)
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int z = 0;
    for (; z + 8 <= nsplit; z += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(int64_t)(z + u) * total + idx];
      s0 += v[0] + v[4];
      s1 += v[1] + v[5];
      s2 += v[2] + v[6];
      s3 += v[3] + v[7];
    }
    for (; z < nsplit; ++z) s0 += partial[(int64_t)z * total + idx];
    const double s = (s0 + s1) + (s2 + s3);
    const int64_t m = idx % M, n = idx / M;
    double* c = C + m + n * ldc;
    const double out = alpha * s;
    *c = (beta == 0.0) ? out : out + beta * (*c);
  }
}

constexpr int kSkMaxN = 256;

bool use_skinny(char ta, char tb, int64_t M, int64_t N, int64_t K) {
  return ta == 'N' && tb == 'N' && M >= 1024 && K >= 1024 && N >= 1 && N <= kSkMaxN;
}

int skinny_nsplit(int64_t M, int64_t K) {
  const int64_t rowblocks = cdiv(M, kSkRows);
  int64_t ns = 4;  // two workgroups per CU at n = 16384; fewer partials to write and sum
  while (rowblocks * ns < 512 && K / (ns * 2) >= 256) ns *= 2;
  while (ns > 1 && K / ns < kSkBK) ns /= 2;
  return (int)ns;
}

template <int TN>
void launch_skinny(hipStream_t s, int M, int N, int K, int ns, int kchunk, const double* A,
                   int64_t lda, const double* B, int64_t ldb, double* partial) {
  const int64_t rowblocks = cdiv(M, kSkRows);
  hipLaunchKernelGGL((gemm_f64_skinny_kernel<TN>), dim3((unsigned)(rowblocks * ns)), dim3(kSkThreads),
                     0, s, M, N, K, ns, kchunk, A, lda, B, ldb, partial);
}

void gemm_f64_skinny(hipStream_t s, int M, int N, int K, double alpha, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                     double* partial, int ns_force = 0) {
  const int ns0 = ns_force > 0 ? ns_force : skinny_nsplit(M, K);
  const int kchunk = (int)(cdiv(cdiv(K, ns0), kSkBK) * kSkBK);
  const int ns = (int)cdiv(K, kchunk);  // no empty chunk
  const int tn = (int)cdiv(N, 16);
  KernelTimer* kt = kernel_timer();
  if (kt) kt->before(s);
  switch (tn) {
#define DME_SKINNY_CASE(T) \
  case T: launch_skinny<T>(s, M, N, K, ns, kchunk, A, lda, B, ldb, partial); break;
    DME_SKINNY_CASE(1) DME_SKINNY_CASE(2) DME_SKINNY_CASE(3) DME_SKINNY_CASE(4)
    DME_SKINNY_CASE(5) DME_SKINNY_CASE(6) DME_SKINNY_CASE(7) DME_SKINNY_CASE(8)
    DME_SKINNY_CASE(9) DME_SKINNY_CASE(10) DME_SKINNY_CASE(11) DME_SKINNY_CASE(12)
    DME_SKINNY_CASE(13) DME_SKINNY_CASE(14) DME_SKINNY_CASE(15) DME_SKINNY_CASE(16)
#undef DME_SKINNY_CASE
    default: fail(DME_EINTERNAL, "skinny gemm: bad tile count");
  }
  DME_HIP(hipGetLastError());
  if (kt) kt->after(s, M, N, K, (int)sizeof(double));
  const int64_t total = (int64_t)M * N;
  const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 8192);
  hipLaunchKernelGGL(skinny_reduce_kernel, dim3(blocks), dim3(256), 0, s, M, N, ns, alpha, partial,
                     beta, C, ldc);
  DME_HIP(hipGetLastError());
}

struct Plan {
  int bm, bn, nsplit, kchunk;
};

constexpr int kBK = 16;
constexpr int kTargetBlocks = 1024;  // ~4 workgroups per CU on 256 CUs
constexpr int kMinKChunk = 256;
constexpr int64_t kMinTiles = 256;      // one tile per CU

Plan plan_for(int64_t M, int64_t N, int64_t K) {
  Plan p;
  // the largest tile that still gives every CU a tile (small products are
  // latency-bound: more, smaller tiles finish sooner)
  if (N <= 256 && K <= 512)                                              { p.bm = 64;  p.bn = 64; }  // tall x narrow, short K: latency-bound tiles
  else if (M >= 128 && N >= 128 && cdiv(M, 128) * cdiv(N, 128) >= kMinTiles) { p.bm = 128; p.bn = 128; }
  else if (M >= 128 && cdiv(M, 128) * cdiv(N, 64) >= kMinTiles)         { p.bm = 128; p.bn = 64; }
  else                                                                   { p.bm = 64;  p.bn = 64; }
  const int64_t tiles = cdiv(M, p.bm) * cdiv(N, p.bn);
  int64_t nsplit = 1;
  if (tiles < kTargetBlocks && K >= 2 * kMinKChunk) {
    nsplit = std::min<int64_t>(cdiv(kTargetBlocks, tiles), K / kMinKChunk);
    nsplit = std::max<int64_t>(1, std::min<int64_t>(nsplit, 256));
  }
  int64_t kchunk = cdiv(cdiv(K, nsplit), kBK) * kBK;
  if (kchunk <= 0) kchunk = kBK;
  nsplit = std::max<int64_t>(1, cdiv(K, kchunk));
  p.nsplit = (int)nsplit;
  p.kchunk = (int)kchunk;
  return p;
}

}  // namespace

size_t gemm_f64_workspace_tiled(int64_t M, int64_t N, int64_t K);

// Largest workspace any product of at most N columns may take (the skinny
// path serves every width up to kSkMaxN).
size_t gemm_f64_workspace(int64_t M, int64_t N, int64_t K) {
  size_t w = gemm_f64_workspace_tiled(M, N, K);
  if (K > kSmallMaxK)  // the small path's K chunks: at most kSmallSplitTiles 16 x 16 tiles of C
    w = std::max(w, (size_t)std::min<int64_t>(cdiv(K, kSmallChunk), 256) * (size_t)(kSmallSplitTiles * 256) *
                        sizeof(double) + 256);
  if (M == N && K >= kSyMinK) {  // a Gram product W^T W of up to M columns may take the syrk path
    const size_t ms = (size_t)std::min<int64_t>(M, 16 * kSyMaxT);
    w = std::max(w, (size_t)syrk_grid(K) * ms * ms * sizeof(double) + 256);
  }
  const int64_t nn = std::min<int64_t>(N, kSkMaxN);
  if (use_skinny('N', 'N', M, nn, K))
    w = std::max(w, (size_t)skinny_nsplit(M, K) * (size_t)M * (size_t)nn * sizeof(double) + 256);
  return w;
}

size_t gemm_f64_workspace_tiled(int64_t M, int64_t N, int64_t K) {
  Plan p = plan_for(M, N, K);
  if (p.nsplit <= 1) return 0;
  return (size_t)p.nsplit * (size_t)M * (size_t)N * sizeof(double) + 256;
}

static_assert(kSkRows == kRowBlock, "row block of the skinny path");

void gemm_f64_rows(hipStream_t s, int64_t m, int64_t N, int64_t K, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double* C, int64_t ldc, int ns, Arena& ws) {
  if (m <= 0 || N <= 0) return;
  DME_REQUIRE(m < (1ll << 31) && K >= kSkBK && K < (1ll << 31) && N <= kSkMaxN && ns >= 1, DME_EINVAL,
              "row-range product: shape outside the skinny path");
  const size_t mark = ws.used;
  double* partial = ws.get<double>((size_t)ns * m * N);
  gemm_f64_skinny(s, (int)m, (int)N, (int)K, 1.0, A, lda, B, ldb, 0.0, C, ldc, partial, ns);
  ws.used = mark;
}

void gemm_f64(hipStream_t s, char ta, char tb, int64_t M, int64_t N, int64_t K, double alpha,
              const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
              int64_t ldc, Arena* ws) {
  if (M <= 0 || N <= 0) return;
  DME_REQUIRE(M < (1ll << 31) && N < (1ll << 31) && K < (1ll << 31), DME_EINVAL, "gemm dims too large");
  if (K <= 0) {
    // C = beta * C
    if (beta == 0.0) fill_f64(s, C, M, N, ldc, 0.0);
    else if (beta != 1.0) copy_scaled_f64(s, C, ldc, C, ldc, M, N, beta);
    return;
  }
  if (use_skinny(ta, tb, M, N, K) && ws != nullptr) {
    const int ns = skinny_nsplit(M, K);
    double* partial = ws->get<double>((size_t)ns * M * N);
    gemm_f64_skinny(s, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta, C, ldc, partial);
    return;
  }
  if (use_syrk(ta, tb, M, N, K, A, lda, B, ldb) && ws != nullptr) {
    const int T = (int)cdiv(M, 16), grid = syrk_grid(K);
    double* partial = ws->get<double>((size_t)grid * M * M);
    const size_t lds = (size_t)kSyRows * (16 * T + 1) * sizeof(double);
    switch (T) {
#define DME_SYRK(TT)                                                                                    \
  case TT:                                                                                              \
    hipLaunchKernelGGL((syrk_tn_kernel<TT>), dim3(grid), dim3(64 * kSyWaves), lds, s, (int)K, (int)M, A, lda, \
                       partial);                                                                      \
    break;
      DME_SYRK(1) DME_SYRK(2) DME_SYRK(3) DME_SYRK(4) DME_SYRK(5) DME_SYRK(6)
      DME_SYRK(7) DME_SYRK(8) DME_SYRK(9) DME_SYRK(10) DME_SYRK(11) DME_SYRK(12)
#undef DME_SYRK
      default: fail(DME_EINTERNAL, "syrk: bad tile count");
    }
    DME_HIP(hipGetLastError());
    hipLaunchKernelGGL(syrk_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(M * (M + 1) / 2, 32), 4096)),
                       dim3(256), 0, s, (int)M, grid, alpha, partial, beta, C, ldc);
    DME_HIP(hipGetLastError());
    return;
  }
  const int64_t small_tiles = cdiv(M, 16) * cdiv(N, 16);
  if (M <= kSmallMaxMN && N <= kSmallMaxMN &&
      (K <= kSmallMaxK || (small_tiles <= kSmallSplitTiles && ws != nullptr))) {
    int nsplit = 1, kchunk = (int)K;
    double* partial = nullptr;
    if (K > kSmallMaxK) {
      nsplit = (int)std::min<int64_t>(cdiv(K, kSmallChunk), 256);
      kchunk = (int)(cdiv(cdiv(K, nsplit), 64) * 64);
      nsplit = (int)cdiv(K, kchunk);
      partial = ws->get<double>((size_t)nsplit * M * N);
    }
    const dim3 grid((unsigned)cdiv(M, 16), (unsigned)cdiv(N, 16), (unsigned)nsplit);
    const bool TA = (ta == 'T' || ta == 't'), TB = (tb == 'T' || tb == 't');
    const int iM = (int)M, iN = (int)N, iK = (int)K;
    if (!TA && !TB)
      hipLaunchKernelGGL((gemm_f64_small_kernel<false, false>), grid, dim3(256), 0, s, iM, iN, iK, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
    else if (TA && !TB)
      hipLaunchKernelGGL((gemm_f64_small_kernel<true, false>), grid, dim3(256), 0, s, iM, iN, iK, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
    else if (!TA && TB)
      hipLaunchKernelGGL((gemm_f64_small_kernel<false, true>), grid, dim3(256), 0, s, iM, iN, iK, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
    else
      hipLaunchKernelGGL((gemm_f64_small_kernel<true, true>), grid, dim3(256), 0, s, iM, iN, iK, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
    DME_HIP(hipGetLastError());
    if (partial) {
      hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(M * N, 256), 4096)), dim3(256),
                         0, s, iM, iN, nsplit, alpha, partial, beta, C, ldc);
      DME_HIP(hipGetLastError());
    }
    return;
  }
  Plan p = plan_for(M, N, K);
  double* partial = nullptr;
  if (p.nsplit > 1) {
    if (ws == nullptr) {
      p.nsplit = 1;
      p.kchunk = (int)(cdiv(K, kBK) * kBK);
    } else {
      partial = ws->get<double>((size_t)p.nsplit * M * N);
    }
  }
  const int iM = (int)M, iN = (int)N, iK = (int)K;
  if (p.bm == 128 && p.bn == 128)
    dispatch_trans<128, 128, kBK>(s, ta, tb, iM, iN, iK, p.nsplit, p.kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  else if (p.bm == 128)
    dispatch_trans<128, 64, kBK>(s, ta, tb, iM, iN, iK, p.nsplit, p.kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  else
    dispatch_trans<64, 64, kBK>(s, ta, tb, iM, iN, iK, p.nsplit, p.kchunk, alpha, A, lda, B, ldb, beta, C, ldc, partial);
  DME_HIP(hipGetLastError());
  if (partial) {
    const int64_t total = M * N;
    const int blocks = (int)std::min<int64_t>(cdiv(total, 256), 4096);
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(blocks), dim3(256), 0, s, iM, iN, p.nsplit, alpha,
                       partial, beta, C, ldc);
    DME_HIP(hipGetLastError());
  }
}

}  // namespace dme
