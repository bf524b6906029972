// Allocation-free variant of the Riccati subflow entry point (dme_riccati) for
// callers that cannot allocate device memory during the call (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// Its temporaries (W_B = L^T B, the split-K partial sums of that product and
// the m-column staging of the m x m update) live in one file-scope device
// array, `scratch`, of kScratchBytes.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in symbol): the device address
// is looked up once per device with hipGetSymbolAddress while the device is
// current (at context creation) and that address is what the kernels get.
// Every call on a device shares the device's copy, so calls that overlap on
// one device race; nothing in it needs to start at zero (every product writes
// the whole of its partial sums, the flags live in the context).
#include <map>
#include <mutex>

#include "ctx.h"

namespace dme {
namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;  // 8 MiB per device

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of that device's `scratch`

void* scratch_address(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  int cur = -1;
  DME_HIP(hipGetDevice(&cur));
  DME_REQUIRE(cur == device, DME_EINTERNAL, "scratch lookup needs its device current");
  void* ptr = nullptr;
  DME_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  DME_REQUIRE(ptr != nullptr, DME_EHIP, "hipGetSymbolAddress returned no address for the scratch");
  g_scratch_ptr[device] = ptr;
  return ptr;
}

size_t aligned(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

void noalloc_scratch_init(int device) { (void)scratch_address(device); }

}  // namespace dme

extern "C" int dme_riccati_noalloc(dme_ctx* ctx, int64_t n, int64_t r, int64_t m, const double* L,
                                   const double* B, const double* R, double t, double* D) {
  return dme::guarded_call([&] {
    DME_REQUIRE(ctx != nullptr, DME_EINVAL, "null context");
    DME_REQUIRE(n >= 0 && r >= 0 && m >= 0, DME_EINVAL, "riccati_noalloc: negative size");
    DME_HIP(hipSetDevice(ctx->device));
    if (r == 0 || m == 0) return;
    DME_REQUIRE(L && B && R && D, DME_EINVAL, "riccati_noalloc: null pointer");
    // the same temporaries dme_riccati takes from the context's arena
    const size_t need = dme::aligned((size_t)r * m * sizeof(double)) +
                        dme::aligned(dme::gemm_f64_workspace(r, m, n)) +
                        dme::aligned((size_t)r * m * sizeof(double));
    DME_REQUIRE(need <= dme::kScratchBytes, DME_EINVAL,
                "riccati_noalloc: r = " + std::to_string(r) + ", m = " + std::to_string(m) +
                    ", n = " + std::to_string(n) + " need " + std::to_string(need) +
                    " bytes of scratch, more than the static " + std::to_string(dme::kScratchBytes));
    dme::Arena ws;
    ws.attach(dme::scratch_address(ctx->device), dme::kScratchBytes);
    int* flags = ctx->flags.as<int>();
    dme::fill_f64(ctx->stream, ctx->flags.as<double>(), 8, 1, 8, 0.0);
    double* WB = ws.get<double>((size_t)r * m);
    dme::gemm_f64(ctx->stream, 'T', 'N', r, m, n, 1.0, L, n, B, n, 0.0, WB, r, &ws);
    dme::riccati_update_f64(ctx->stream, r, m, D, r, WB, r, R, m, t, flags, ws);
    int h[4];
    DME_HIP(hipMemcpyAsync(h, flags, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    DME_HIP(hipStreamSynchronize(ctx->stream));
    DME_REQUIRE((h[0] & 4) == 0, DME_ENUMERIC, "riccati_noalloc: R + t W^T D W is not SPD");
  });
}
