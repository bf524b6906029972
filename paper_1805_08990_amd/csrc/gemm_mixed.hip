// Split-precision step product Y = E X on BF16 MFMA (gfx950), for the
// mixed-precision mode of the solver.
//
// E (n x n, the operator e^{tA^T}) is kept as FP32; every FP32 value is the
// exact sum of three BF16 pieces x = x1 + x2 + x3 (each piece takes the next
// 8 significant bits).  X (n x r, FP64) is rounded to FP32 and split the same
// way (directly from FP64).  The product keeps the six piece products whose order is at most
// 2^-16 of the leading one,
//
//     E X ~ E1 X1 + (E1 X2 + E2 X1) + (E1 X3 + E2 X2 + E3 X1),
//
// so the result carries the FP32 representation error of E and X (relative
// 2^-24 per entry) and the dropped terms (E2 X3, E3 X2, E3 X3: below 2^-24
// relative).  For each 32-wide K step the six products are summed by
// v_mfma_f32_16x16x32_bf16 into a fresh FP32 accumulator, and the step sums
// are added in FP64; the chunks of the split K range are summed in FP64 in a
// fixed order, so results are deterministic.
//
// Layout:
//   Et     FP32, row-major E (Et[i * lde + k] = E(i, k)), lde = n rounded up to
//          a multiple of 64, zero padding: a lane's 8 consecutive k of one row
//          are one 32-byte load.
//   Xs     BF16, three planes, column-major with ld = lde and rpad = 16 TN
//          columns, zero padded.
//   partial FP64, [split][col][row].
//
// Work decomposition: a 256-thread workgroup (4 wave64s, 32 rows each) owns
// 128 rows of Y and every column (TN 16-column tiles).  The FP64 accumulators
// of a wave's 32 x 16 TN tile keep it at one wave per SIMD; splitting the
// columns over two waves per SIMD doubles the E loads and splits and measured
// slower.
// The K range is split into nsplit chunks; workgroup b takes chunk b % nsplit,
// so every chunk is handled by the same one or two XCDs and the chunk's slice
// of Xs (lde/nsplit x rpad x 3 pieces) stays in their L2.  The Xs tile of a K
// step is staged once in LDS (double-buffered) and read by all 4 waves; E
// fragments go straight from HBM to registers and are split into pieces in
// registers.
#include "solver.h"

namespace dme {

struct MixedOp {
  DevBuf Et;          // n x lde FP32, row-major E
  int64_t n = 0, lde = 0;
};

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kMT = 256;        // threads per workgroup (4 waves)
constexpr int kMRowsWave = 32;  // two 16-row MFMA tiles per wave
constexpr int kMRows = (kMT / 64) * kMRowsWave;  // 128 rows per workgroup
constexpr int kMBK = 32;        // K per step (one MFMA K)
constexpr int kMPD = 4;         // E register stages (steps loaded ahead)
constexpr int kMFl = 4;         // steps per FP32 accumulation span (128 K)
static_assert(kMFl % kMPD == 0, "the E ring must cycle within an accumulation span");

// FP32 -> BF16 bits with round-to-nearest-even (finite inputs).
__device__ __forceinline__ u16 bf16_rne(float x) {
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (u16)(b >> 16);
}
__device__ __forceinline__ float bf16_to_f32(u16 h) { return __uint_as_float(((uint32_t)h) << 16); }

// Exact three-piece split of an FP32 value.
__device__ __forceinline__ void split3(float x, u16& a, u16& b, u16& c) {
  a = bf16_rne(x);
  const float r1 = x - bf16_to_f32(a);
  b = bf16_rne(r1);
  const float r2 = r1 - bf16_to_f32(b);
  c = bf16_rne(r2);
}

// Three-piece split of two FP32 values at once, packed two BF16 per word
// (low half: x0's piece).  The first piece rounds to nearest even, the
// remainder r = x - x1 is exact and has at most 16 significant bits; the
// second piece truncates r to 8 significant bits and the third is the exact
// rest (at most 8 significant bits, so it is a BF16 value as it stands).
// |x2| <= 2^-8 |x|, |x3| < 2^-15 |x|; x = x1 + x2 + x3 exactly.
__device__ __forceinline__ void split3x2(float x0, float x1, uint32_t& a, uint32_t& b, uint32_t& c) {
  const uint32_t u0 = __float_as_uint(x0), u1 = __float_as_uint(x1);
  const uint32_t a0 = (u0 + 0x7FFFu + ((u0 >> 16) & 1u)) & 0xFFFF0000u;
  const uint32_t a1 = (u1 + 0x7FFFu + ((u1 >> 16) & 1u)) & 0xFFFF0000u;
  const float r0 = x0 - __uint_as_float(a0), r1 = x1 - __uint_as_float(a1);
  const uint32_t b0 = __float_as_uint(r0) & 0xFFFF0000u, b1 = __float_as_uint(r1) & 0xFFFF0000u;
  const float q0 = r0 - __uint_as_float(b0), q1 = r1 - __uint_as_float(b1);
  a = (a0 >> 16) | a1;
  b = (b0 >> 16) | b1;
  c = (__float_as_uint(q0) >> 16) | (__float_as_uint(q1) & 0xFFFF0000u);
}

// Three-piece split of an FP64 value (each piece rounds what the earlier
// ones left; the residual is below 2^-24 of |x|).
__device__ __forceinline__ void split3_d(double x, u16& a, u16& b, u16& c) {
  a = bf16_rne((float)x);
  const double r1 = x - (double)bf16_to_f32(a);
  b = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f32(b);
  c = bf16_rne((float)r2);
}

typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

union Frag {
  bf16x8 v;
  u16 h[8];
  u32x4 q;
};

// E (FP64, column-major, ld n) -> Et (FP32 row-major, ld lde), zero padding in
// columns [n, lde).  32 x 32 tiles through LDS: coalesced on both sides.
__global__ void mixed_prep_e_kernel(const double* __restrict__ E, int64_t n, float* __restrict__ Et,
                                    int64_t lde) {
  __shared__ float tile[32][33];
  const int64_t i0 = (int64_t)blockIdx.y * 32;  // row block of E (= row of Et)
  const int64_t k0 = (int64_t)blockIdx.x * 32;  // column block of E
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int j = ty; j < 32; j += 8) {
    const int64_t i = i0 + tx, k = k0 + j;
    tile[j][tx] = (i < n && k < n) ? (float)E[i + k * n] : 0.0f;
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int64_t i = i0 + j, k = k0 + tx;
    if (i < n && k < lde) Et[i * lde + k] = tile[tx][j];
  }
}

// X (FP64, n x r, ld ldx) -> three BF16 planes (ld lde, rpad columns, zero
// padded).  One thread per (k, col) entry.
__global__ void mixed_split_x_kernel(const double* __restrict__ X, int64_t ldx, int64_t n, int64_t r,
                                     int64_t lde, int64_t rpad, u16* __restrict__ Xs) {
  const int64_t total = lde * rpad;
  const int64_t plane = lde * rpad;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx % lde, c = idx / lde;
    const double x = (k < n && c < r) ? X[k + c * ldx] : 0.0;
    u16 a, b, d;
    split3_d(x, a, b, d);
    Xs[idx] = a;
    Xs[plane + idx] = b;
    Xs[2 * plane + idx] = d;
  }
}

// One workgroup = 4 waves = 128 rows of Y and every column (TN 16-column
// tiles); wave w owns rows 32 w .. 32 w + 31 (two 16-row MFMA tiles).  The K
// range is split into nsplit chunks; workgroup b takes chunk b % nsplit.  Per
// 32-wide K step the Xs tile (three pieces) is staged in LDS (double-buffered,
// one barrier per step) and shared by the four waves; every wave reads its E
// fragments straight from HBM into a ring of kMPD register stages (loads
// issued kMPD steps ahead, addresses clamped so no load sits behind a
// branch), splits them into BF16 pieces in registers and runs the six piece
// products of its 2 x TN tiles.  The products accumulate in FP32 over kMFl
// steps (128 K) and are then added to FP64 accumulators.
template <int TN>
__global__ __launch_bounds__(kMT) void gemm_mixed_kernel(int n, int lde, int rpad, int nsplit,
                                                         int kchunk, const float* __restrict__ Et,
                                                         const u16* __restrict__ Xs, int r,
                                                         double* __restrict__ partial) {
  constexpr int NC = TN * 16;          // columns covered
  constexpr int QPC = kMBK / 8;        // 16-byte chunks per column of a step's tile
  constexpr int CHUNKS = 3 * NC * QPC; // 16-byte chunks of one Xs tile
  constexpr int CPT = (CHUNKS + kMT - 1) / kMT;
  __shared__ u32x4 sX[2][3][NC][QPC + 1];
  __shared__ u32x4 sSink;  // target of the stores of threads past the tile (no branch)

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int split = blockIdx.x % nsplit;
  const int rb = blockIdx.x / nsplit;
  const int kbeg = split * kchunk;
  const int kend = min(lde, kbeg + kchunk);
  const int nsteps = (kend - kbeg) / kMBK;  // a multiple of kMFl
  const int row_l = lane & 15;
  const int kg = lane >> 4;  // k group: k = 8 kg .. 8 kg + 7 of a step
  const int64_t plane = (int64_t)lde * rpad;

  double acc[2][TN][4];
  f32x4 fa[2][TN];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][j][v] = 0.0;
      fa[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

  // E rows of this lane (clamped: rows past n compute values nobody stores)
  const float* erow[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int row = min(rb * kMRows + wave * kMRowsWave + t * 16 + row_l, n - 1);
    erow[t] = Et + (int64_t)row * lde + kg * 8;
  }
  float4 ering[kMPD][2][2];
  auto load_e = [&](int step, float4 (&dst)[2][2]) {
    const int k0 = kbeg + min(step, nsteps - 1) * kMBK;  // clamped: the tail re-reads the last step
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const float4* src = reinterpret_cast<const float4*>(erow[t] + k0);
      dst[t][0] = src[0];
      dst[t][1] = src[1];
    }
  };
  // Xs tiles pass through a ring of register stages (u32x4: promotable to
  // VGPRs), loaded as far ahead as the E fragments
  u32x4 xring[kMPD][CPT];
#define DME_LOAD_X(step, dst)                                                                    \
  do {                                                                                           \
    const int k0_ = kbeg + min((step), nsteps - 1) * kMBK;                                       \
    _Pragma("unroll") for (int c = 0; c < CPT; ++c) {                                            \
      const int idx = min(tid + c * kMT, CHUNKS - 1);                                            \
      const int q = idx % QPC, col = (idx / QPC) % NC, pc = (idx / QPC) / NC;                    \
      (dst)[c] = *reinterpret_cast<const u32x4*>(Xs + pc * plane + (int64_t)col * lde + k0_ + q * 8); \
    }                                                                                            \
  } while (0)
#define DME_STORE_X(buf, src)                                                                    \
  do {                                                                                           \
    _Pragma("unroll") for (int c = 0; c < CPT; ++c) {                                            \
      const int idx = tid + c * kMT;                                                             \
      const int ic = min(idx, CHUNKS - 1);                                                       \
      const int q = ic % QPC, col = (ic / QPC) % NC, pc = (ic / QPC) / NC;                       \
      u32x4* dst = (idx < CHUNKS) ? &sX[(buf)][pc][col][q] : &sSink;                             \
      *dst = (src)[c];                                                                           \
    }                                                                                            \
  } while (0)

  // Loads are issued in the order X(s), E(s) (prologue) and E(s + kMPD),
  // X(s + 1 + kMPD) (step s); waiting for the tile or fragments a step needs
  // then leaves the loads of the next kMPD - 1 steps in flight.
  if (nsteps > 0) {
#pragma unroll
    for (int u = 0; u < kMPD; ++u) {
      DME_LOAD_X(u, xring[u]);
      load_e(u, ering[u]);
    }
    DME_STORE_X(0, xring[0]);
    DME_LOAD_X(kMPD, xring[0]);
  }
  __syncthreads();
  for (int s0 = 0; s0 < nsteps; s0 += kMFl) {
#pragma unroll
    for (int u = 0; u < kMFl; ++u) {
      const int s = s0 + u;
      const int slot = u % kMPD;  // kMFl is a multiple of kMPD
      const int buf = u & 1;      // s0 is even
      // split this step's E fragments into three BF16 pieces, then refill the slot
      Frag ef[2][3];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const float4 lo = ering[slot][t][0], hi = ering[slot][t][1];
        uint32_t w[3][4];
        split3x2(lo.x, lo.y, w[0][0], w[1][0], w[2][0]);
        split3x2(lo.z, lo.w, w[0][1], w[1][1], w[2][1]);
        split3x2(hi.x, hi.y, w[0][2], w[1][2], w[2][2]);
        split3x2(hi.z, hi.w, w[0][3], w[1][3], w[2][3]);
#pragma unroll
        for (int pc = 0; pc < 3; ++pc) ef[t][pc].q = u32x4{w[pc][0], w[pc][1], w[pc][2], w[pc][3]};
      }
      load_e(s + kMPD, ering[slot]);
      // column tiles in pairs: four independent accumulation chains between
      // dependent MFMAs (each accumulator still takes its six products in
      // the order below: smallest first)
#pragma unroll
      for (int j = 0; j < TN; j += 2) {
        constexpr int pe[6] = {2, 1, 0, 1, 0, 0}, px[6] = {0, 1, 2, 0, 1, 0};  // pieces of E and X
        const int nj = (j + 1 < TN) ? 2 : 1;
        Frag xf[2][3];
#pragma unroll
        for (int jj = 0; jj < 2; ++jj)
          if (jj < nj) {
#pragma unroll
            for (int pc = 0; pc < 3; ++pc) xf[jj][pc].q = sX[buf][pc][(j + jj) * 16 + row_l][kg];
          }
#pragma unroll
        for (int p = 0; p < 6; ++p)
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
            if (jj < nj) {
#pragma unroll
              for (int t = 0; t < 2; ++t)
                fa[t][j + jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][pe[p]].v, xf[jj][px[p]].v,
                                                                        fa[t][j + jj], 0, 0, 0);
            }
      }
      if (u == kMFl - 1) {
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][j][v] += (double)fa[t][j][v];
            fa[t][j] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
      }
      // the next step's tile goes to LDS, and its ring stage takes the tile
      // kMPD steps later
      DME_STORE_X(buf ^ 1, xring[(u + 1) % kMPD]);
      DME_LOAD_X(s + 1 + kMPD, xring[(u + 1) % kMPD]);
      __syncthreads();
    }
  }

#undef DME_LOAD_X
#undef DME_STORE_X
  // lane holds rows 4 kg .. 4 kg + 3 of column row_l of each 16 x 16 tile
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int row0 = rb * kMRows + wave * kMRowsWave + t * 16 + kg * 4;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = j * 16 + row_l;
      if (col < r) {
        double* dst = partial + ((int64_t)split * r + col) * n;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row0 + v < n) dst[row0 + v] = acc[t][j][v];
      }
    }
  }
}

// Y(i, j) = sum over splits of partial, in FP64 and split order.
__global__ void mixed_reduce_kernel(const double* __restrict__ partial, int64_t n, int64_t r,
                                    int nsplit, double* __restrict__ Y, int64_t ldy) {
  const int64_t total = n * r;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += partial[(int64_t)z * total + idx];
    const int64_t i = idx % n, j = idx / n;
    Y[i + j * ldy] = s;
  }
}

constexpr int kMaxTN = 8;
constexpr int kMinChunk = 1024;

// K granularity: one FP32 accumulation span, so every span is full
constexpr int kMKGran = kMFl * kMBK;

int64_t lde_for(int64_t n) { return cdiv(n, kMKGran) * kMKGran; }

// K chunks: enough workgroups to cover every CU, chunks of at least kMinChunk
int nsplit_for(int64_t n) {
  const int64_t lde = lde_for(n);
  const int64_t rowblocks = cdiv(n, kMRows);
  int64_t ns = 1;
  while (rowblocks * ns < 256 && lde / (ns * 2) >= kMinChunk) ns *= 2;
  return (int)ns;
}

template <int TN>
void launch_mixed(hipStream_t s, int64_t n, int64_t lde, int64_t rpad, int nsplit, int kchunk,
                  const float* Et, const u16* Xs, int64_t r, double* partial) {
  const int64_t rowblocks = cdiv(n, kMRows);
  hipLaunchKernelGGL((gemm_mixed_kernel<TN>), dim3((unsigned)(rowblocks * nsplit)), dim3(kMT), 0, s,
                     (int)n, (int)lde, (int)rpad, nsplit, kchunk, Et, Xs, (int)r, partial);
}

}  // namespace

std::shared_ptr<MixedOp> mixed_op_new() { return std::make_shared<MixedOp>(); }

void mixed_op_build(hipStream_t s, int64_t n, const double* E, MixedOp& op) {
  op.n = n;
  op.lde = lde_for(n);
  op.Et.ensure((size_t)n * op.lde * sizeof(float));
  dim3 grid((unsigned)cdiv(op.lde, 32), (unsigned)cdiv(n, 32));
  hipLaunchKernelGGL(mixed_prep_e_kernel, grid, dim3(256), 0, s, E, n, op.Et.as<float>(), op.lde);
  DME_HIP(hipGetLastError());
}

size_t gemm_mixed_workspace(int64_t n, int64_t r) {
  const int64_t lde = lde_for(n);
  const int64_t rpad = cdiv(std::min<int64_t>(r, 16 * kMaxTN), 16) * 16;
  const int ns = nsplit_for(n);
  return (size_t)3 * lde * rpad * sizeof(u16) + 256 +
         (size_t)ns * n * std::min<int64_t>(r, 16 * kMaxTN) * sizeof(double) + 256;
}

static_assert(kMRows == kRowBlock, "row block of the split-BF16 product");

int gemm_mixed_nsplit(int64_t n) { return nsplit_for(n); }

// Rows [row0, row0 + rows) of Y (n x r, ld ldy, FP64) = E X with X (n x r,
// ld ldx, FP64); rows < 0: all of them.  ns_force > 0 cuts the inner
// dimension into that many chunks instead of the default.
void gemm_mixed(hipStream_t s, const MixedOp& op, const double* X, int64_t ldx, int64_t r, double* Y,
                int64_t ldy, Arena& ws, int64_t row0, int64_t rows, int ns_force) {
  const int64_t nk = op.n;  // inner dimension
  if (rows < 0) rows = nk - row0;
  if (nk <= 0 || r <= 0 || rows <= 0) return;
  DME_REQUIRE(nk < (1ll << 30) && row0 >= 0 && row0 + rows <= nk, DME_EINVAL, "mixed gemm: bad rows");
  const int64_t n = rows;  // rows of the result this call forms
  const int ns0 = ns_force > 0 ? ns_force : nsplit_for(nk);
  const int kchunk = (int)(cdiv(cdiv(op.lde, ns0), kMKGran) * kMKGran);
  const int ns = (int)cdiv(op.lde, kchunk);  // no empty chunk
  Y += row0;
  const size_t mark = ws.used;
  for (int64_t c0 = 0; c0 < r; c0 += 16 * kMaxTN) {
    const int64_t rc = std::min<int64_t>(r - c0, 16 * kMaxTN);
    const int tn = (int)cdiv(rc, 16);
    const int64_t rpad = 16 * tn;
    ws.used = mark;
    u16* Xs = ws.get<u16>((size_t)3 * op.lde * rpad);
    double* partial = ws.get<double>((size_t)ns * n * rc);
    hipLaunchKernelGGL(mixed_split_x_kernel, dim3((unsigned)std::min<int64_t>(cdiv(op.lde * rpad, 256), 8192)),
                       dim3(256), 0, s, X + c0 * ldx, ldx, nk, rc, op.lde, rpad, Xs);
    DME_HIP(hipGetLastError());
    const float* Et = op.Et.as<float>() + row0 * op.lde;
    KernelTimer* kt = kernel_timer();
    if (kt) kt->before(s);
    switch (tn) {
#define DME_MIXED_CASE(T) \
  case T: launch_mixed<T>(s, n, op.lde, rpad, ns, kchunk, Et, Xs, rc, partial); break;
      DME_MIXED_CASE(1) DME_MIXED_CASE(2) DME_MIXED_CASE(3) DME_MIXED_CASE(4)
      DME_MIXED_CASE(5) DME_MIXED_CASE(6) DME_MIXED_CASE(7) DME_MIXED_CASE(8)
#undef DME_MIXED_CASE
      default: fail(DME_EINTERNAL, "mixed gemm: bad tile count");
    }
    DME_HIP(hipGetLastError());
    if (kt) kt->after(s, n, rc, nk, (int)sizeof(float));
    hipLaunchKernelGGL(mixed_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n * rc, 256), 8192)),
                       dim3(256), 0, s, partial, n, rc, ns, Y + c0 * ldy, ldy);
    DME_HIP(hipGetLastError());
  }
  ws.used = mark;
}

}  // namespace dme
