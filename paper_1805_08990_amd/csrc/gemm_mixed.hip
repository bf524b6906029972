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
// Work decomposition: a 512-thread workgroup (8 wave64s, 4 row groups x 2
// column halves) owns 128 rows of Y and every column (TN 16-column tiles).
// The K range is split into nsplit chunks; workgroup b takes chunk b % nsplit,
// so every chunk is handled by the same one or two XCDs and the chunk's slice
// of Xs (lde/nsplit x rpad x 3 pieces) stays in their L2.  The Xs tile of a K
// step is staged once in LDS (double-buffered) and read by all 8 waves; E
// fragments go straight from HBM to registers (the two waves of a row group
// read the same rows, the second from cache) and are split into pieces in
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

constexpr int kMT = 512;       // threads per workgroup
constexpr int kMWaves = kMT / 64;
constexpr int kMRowsWave = 32;  // two 16-row MFMA tiles per wave
constexpr int kMRows = 4 * kMRowsWave;  // 128 rows per workgroup (4 row groups)
constexpr int kMBK = 32;        // K per step (one MFMA K)
constexpr int kMLdsK = kMBK + 8;  // padded k extent of an LDS column (bf16)

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

// Three-piece split of an FP64 value (each piece rounds what the earlier
// ones left; the residual is below 2^-24 of |x|).
__device__ __forceinline__ void split3_d(double x, u16& a, u16& b, u16& c) {
  a = bf16_rne((float)x);
  const double r1 = x - (double)bf16_to_f32(a);
  b = bf16_rne((float)r1);
  const double r2 = r1 - (double)bf16_to_f32(b);
  c = bf16_rne((float)r2);
}

union Frag {
  bf16x8 v;
  u16 h[8];
  uint4 q;
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

// KS = MFMA K-steps (of 32) per main-loop iteration: 2 when the double-
// buffered X tile fits in LDS (TN <= 8), else 1.
//
// Wave layout: 8 waves = 4 row groups x 2 column halves.  Wave (g, hc) owns
// rows g*32 .. g*32+31 of the workgroup's 128 (two 16-row MFMA tiles) and the
// column tiles [hc*TW, min(TN, (hc+1)*TW)).  For every 32-wide K step the six
// piece products of a tile are summed by the MFMA into a fresh FP32
// accumulator (the five small ones first) and that step's sum is added to an
// FP64 accumulator: FP32 rounding then acts on one step's partial only.
template <int TN, int KS>
__global__ __launch_bounds__(kMT) void gemm_mixed_kernel(int n, int lde, int rpad, int nsplit,
                                                         int kchunk, const float* __restrict__ Et,
                                                         const u16* __restrict__ Xs, int r,
                                                         double* __restrict__ partial) {
  constexpr int NC = TN * 16;             // columns covered
  constexpr int TW = (TN + 1) / 2;        // column tiles per wave
  constexpr int BK = kMBK * KS;           // K per iteration
  constexpr int QPC = BK / 8;             // 16-byte chunks per column of the tile
  constexpr int CHUNKS = 3 * NC * QPC;    // 16-byte chunks of one Xs tile
  constexpr int CPT = (CHUNKS + kMT - 1) / kMT;
  __shared__ uint4 sX[2][3][NC][QPC + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int rg = wave & 3, hc = wave >> 2;
  const int jbeg = hc * TW;
  const int split = blockIdx.x % nsplit;
  const int rb = blockIdx.x / nsplit;
  const int kbeg = split * kchunk;
  const int kend = min(lde, kbeg + kchunk);
  const int row_l = lane & 15;
  const int kg = lane >> 4;  // k group: k = 8 kg .. 8 kg + 7 of a 32-wide step
  const int64_t plane = (int64_t)lde * rpad;

  double acc[2][TW][4];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int j = 0; j < TW; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[t][j][v] = 0.0;

  int rows[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) rows[t] = rb * kMRows + rg * kMRowsWave + t * 16 + row_l;

  // E fragments of an iteration: [substep][tile][8 consecutive k]
  float ecur[KS][2][8];
  auto load_e = [&](int k0, float (&dst)[KS][2][8]) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        if (rows[t] < n) {
          const float4* src =
              reinterpret_cast<const float4*>(Et + (int64_t)rows[t] * lde + k0 + ks * kMBK + kg * 8);
          const float4 a = src[0], b = src[1];
          dst[ks][t][0] = a.x; dst[ks][t][1] = a.y; dst[ks][t][2] = a.z; dst[ks][t][3] = a.w;
          dst[ks][t][4] = b.x; dst[ks][t][5] = b.y; dst[ks][t][6] = b.z; dst[ks][t][7] = b.w;
        } else {
#pragma unroll
          for (int q = 0; q < 8; ++q) dst[ks][t][q] = 0.f;
        }
      }
  };

  uint4 stage[CPT];
  auto load_x = [&](int k0) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int idx = tid + c * kMT;
      if (idx < CHUNKS) {
        const int q = idx % QPC;
        const int col = (idx / QPC) % NC;
        const int pc = (idx / QPC) / NC;
        stage[c] = *reinterpret_cast<const uint4*>(Xs + pc * plane + (int64_t)col * lde + k0 + q * 8);
      }
    }
  };
  auto store_x = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
      const int idx = tid + c * kMT;
      if (idx < CHUNKS) {
        const int q = idx % QPC;
        const int col = (idx / QPC) % NC;
        const int pc = (idx / QPC) / NC;
        sX[buf][pc][col][q] = stage[c];
      }
    }
  };

  if (kbeg < kend) {
    load_x(kbeg);
    store_x(0);
    load_e(kbeg, ecur);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = (k0 + BK) < kend;
    float enext[KS][2][8];
    if (more) {
      load_x(k0 + BK);
      load_e(k0 + BK, enext);
    }
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      // split this substep's E fragments into three BF16 pieces
      Frag ef[2][3];
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          split3(ecur[ks][t][q], ef[t][0].h[q], ef[t][1].h[q], ef[t][2].h[q]);
#pragma unroll
      for (int jj = 0; jj < TW; ++jj) {
        const int j = jbeg + jj;
        if (j < TN) {
          Frag xf[3];
#pragma unroll
          for (int pc = 0; pc < 3; ++pc) xf[pc].q = sX[buf][pc][j * 16 + row_l][ks * 4 + kg];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][2].v, xf[0].v, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][1].v, xf[1].v, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][0].v, xf[2].v, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][1].v, xf[0].v, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][0].v, xf[1].v, a, 0, 0, 0);
            a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ef[t][0].v, xf[0].v, a, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[t][jj][v] += (double)a[v];
          }
        }
      }
    }
    if (more) {
      store_x(buf ^ 1);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int q = 0; q < 8; ++q) ecur[ks][t][q] = enext[ks][t][q];
    }
    __syncthreads();
    buf ^= 1;
  }

  // lane holds rows 4 kg .. 4 kg + 3 of column row_l of each 16 x 16 tile
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int row0 = rb * kMRows + rg * kMRowsWave + t * 16 + kg * 4;
#pragma unroll
    for (int jj = 0; jj < TW; ++jj) {
      const int col = (jbeg + jj) * 16 + row_l;
      if (jbeg + jj < TN && col < r) {
        double* dst = partial + ((int64_t)split * r + col) * n;
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (row0 + v < n) dst[row0 + v] = acc[t][jj][v];
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

constexpr int kMaxTN = 16;
constexpr int kMinChunk = 256;

// K granularity: two MFMA K-steps, so every main-loop iteration is full
constexpr int kMKGran = 2 * kMBK;

int64_t lde_for(int64_t n) { return cdiv(n, kMKGran) * kMKGran; }

int nsplit_for(int64_t n) {
  const int64_t lde = lde_for(n);
  const int64_t rowblocks = cdiv(n, kMRows);
  int64_t ns = 4;
  while (rowblocks * ns < 512 && lde / (ns * 2) >= kMinChunk) ns *= 2;
  while (ns > 1 && lde / ns < kMKGran) ns /= 2;
  return (int)ns;
}

template <int TN>
void launch_mixed(hipStream_t s, int64_t n, int64_t lde, int64_t rpad, int nsplit, int kchunk,
                  const float* Et, const u16* Xs, int64_t r, double* partial) {
  const int64_t rowblocks = cdiv(n, kMRows);
  constexpr int KS = (TN <= 8) ? 2 : 1;
  hipLaunchKernelGGL((gemm_mixed_kernel<TN, KS>), dim3((unsigned)(rowblocks * nsplit)), dim3(kMT), 0,
                     s, (int)n, (int)lde, (int)rpad, nsplit, kchunk, Et, Xs, (int)r, partial);
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

// Y (n x r, ld ldy, FP64) = E X with X (n x r, ld ldx, FP64).
void gemm_mixed(hipStream_t s, const MixedOp& op, const double* X, int64_t ldx, int64_t r, double* Y,
                int64_t ldy, Arena& ws) {
  const int64_t n = op.n;
  if (n <= 0 || r <= 0) return;
  DME_REQUIRE(n < (1ll << 30), DME_EINVAL, "mixed gemm: n too large");
  const int ns = nsplit_for(n);
  const int kchunk = (int)(cdiv(cdiv(op.lde, ns), kMKGran) * kMKGran);
  const size_t mark = ws.used;
  for (int64_t c0 = 0; c0 < r; c0 += 16 * kMaxTN) {
    const int64_t rc = std::min<int64_t>(r - c0, 16 * kMaxTN);
    const int tn = (int)cdiv(rc, 16);
    const int64_t rpad = 16 * tn;
    ws.used = mark;
    u16* Xs = ws.get<u16>((size_t)3 * op.lde * rpad);
    double* partial = ws.get<double>((size_t)ns * n * rc);
    hipLaunchKernelGGL(mixed_split_x_kernel, dim3((unsigned)std::min<int64_t>(cdiv(op.lde * rpad, 256), 8192)),
                       dim3(256), 0, s, X + c0 * ldx, ldx, n, rc, op.lde, rpad, Xs);
    DME_HIP(hipGetLastError());
    const float* Et = op.Et.as<float>();
    KernelTimer* kt = kernel_timer();
    if (kt) kt->before(s);
    switch (tn) {
#define DME_MIXED_CASE(T) \
  case T: launch_mixed<T>(s, n, op.lde, rpad, ns, kchunk, Et, Xs, rc, partial); break;
      DME_MIXED_CASE(1) DME_MIXED_CASE(2) DME_MIXED_CASE(3) DME_MIXED_CASE(4)
      DME_MIXED_CASE(5) DME_MIXED_CASE(6) DME_MIXED_CASE(7) DME_MIXED_CASE(8)
      DME_MIXED_CASE(9) DME_MIXED_CASE(10) DME_MIXED_CASE(11) DME_MIXED_CASE(12)
      DME_MIXED_CASE(13) DME_MIXED_CASE(14) DME_MIXED_CASE(15) DME_MIXED_CASE(16)
#undef DME_MIXED_CASE
      default: fail(DME_EINTERNAL, "mixed gemm: bad tile count");
    }
    DME_HIP(hipGetLastError());
    if (kt) kt->after(s, n, rc, n, (int)sizeof(float));
    hipLaunchKernelGGL(mixed_reduce_kernel, dim3((unsigned)std::min<int64_t>(cdiv(n * rc, 256), 8192)),
                       dim3(256), 0, s, partial, n, rc, ns, Y + c0 * ldy, ldy);
    DME_HIP(hipGetLastError());
  }
  ws.used = mark;
}

}  // namespace dme
