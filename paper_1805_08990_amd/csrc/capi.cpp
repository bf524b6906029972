// C ABI (include/dme.h): argument checking, error codes, ownership.
#include <algorithm>
#include <cstring>
#include <functional>
#include <memory>
#include <new>

#include "ctx.h"

namespace dme {

thread_local std::string g_last_error;

void fail(int code, const std::string& msg) { throw Error{code, msg}; }

void DevBuf::alloc(size_t b) {
  if (b == 0) b = 256;
  hipError_t e = hipMalloc(&p, b);
  if (e != hipSuccess) {
    p = nullptr;
    bytes = 0;
    (void)hipGetLastError();
    fail(DME_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed: " + hipGetErrorString(e));
  }
  bytes = b;
}

void DevBuf::release() {
  if (p && own) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  own = true;
}

KernelTimer*& kernel_timer() {
  thread_local KernelTimer* t = nullptr;
  return t;
}

dme_result* result_from_solver(Solver& sv) {
  auto res = std::make_unique<dme_result>();
  res->n = sv.n;
  res->r = sv.r;
  res->steps = sv.step;
  res->precision = sv.opts.precision;
  res->err_est = sv.err_estimate();
  res->L.resize((size_t)sv.n * sv.r);
  res->D.resize((size_t)sv.r * sv.r);
  if (sv.r > 0) {
    DME_HIP(hipMemcpyAsync(res->L.data(), sv.Lc(), res->L.size() * sizeof(double),
                           hipMemcpyDeviceToHost, sv.s));
    DME_HIP(hipMemcpyAsync(res->D.data(), sv.Dc(), res->D.size() * sizeof(double),
                           hipMemcpyDeviceToHost, sv.s));
  }
  DME_HIP(hipStreamSynchronize(sv.s));
  return res.release();
}

}  // namespace dme


struct dme_solver {
  dme_ctx* ctx = nullptr;
  dme::Solver sv;
};

namespace {

template <class F>
int guarded(F&& f) {
  try {
    f();
    return DME_OK;
  } catch (const dme::Error& e) {
    dme::g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    dme::g_last_error = "host allocation failed";
    return DME_ENOMEM;
  } catch (const std::exception& e) {
    dme::g_last_error = e.what();
    return DME_EINTERNAL;
  } catch (...) {
    dme::g_last_error = "unknown exception";
    return DME_EINTERNAL;
  }
}

}  // namespace

namespace dme {
int guarded_call(const std::function<void()>& f) { return guarded(f); }
}  // namespace dme

namespace {

int* ctx_flags(dme_ctx* c) { return c->flags.as<int>(); }
int64_t* ctx_rank(dme_ctx* c) { return reinterpret_cast<int64_t*>(c->flags.as<char>() + 16); }

void ctx_reset_flags(dme_ctx* c) { dme::fill_f64(c->stream, c->flags.as<double>(), 8, 1, 8, 0.0); }

void ctx_read_flags(dme_ctx* c, int* h) {
  DME_HIP(hipMemcpyAsync(h, c->flags.p, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
  DME_HIP(hipStreamSynchronize(c->stream));
}

void require_ctx(dme_ctx* c) { DME_REQUIRE(c != nullptr, DME_EINVAL, "null context"); }

void make_result(dme::Solver& sv, dme_result** out) { *out = dme::result_from_solver(sv); }

int solve_impl(dme_ctx* ctx, const dme_problem* prob, const dme_opts* opts, int is_dre,
               dme_result** out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(prob && opts && out, DME_EINVAL, "null argument");
    *out = nullptr;
    DME_HIP(hipSetDevice(ctx->device));
    dme::Solver sv;
    sv.s = ctx->stream;
    sv.device = ctx->device;
    sv.setup(*prob, *opts, is_dre != 0);
    sv.advance(sv.N);
    make_result(sv, out);
  });
}

}  // namespace

extern "C" {

const char* dme_strerror(int code) {
  switch (code) {
    case DME_OK: return "ok";
    case DME_EINVAL: return "invalid argument";
    case DME_ENOMEM: return "out of memory";
    case DME_ERANK: return "rank exceeds max_rank";
    case DME_ENUMERIC: return "numerical failure";
    case DME_EAGAIN: return "not ready";
    case DME_EHIP: return "HIP runtime error";
    case DME_EINTERNAL: return "internal error";
    default: return "unknown error";
  }
}

const char* dme_last_error(void) { return dme::g_last_error.c_str(); }

int dme_create(dme_ctx** ctx, int device, void* stream) {
  return guarded([&] {
    DME_REQUIRE(ctx != nullptr, DME_EINVAL, "null ctx pointer");
    *ctx = nullptr;
    int ndev = 0;
    DME_HIP(hipGetDeviceCount(&ndev));
    DME_REQUIRE(device >= 0 && device < ndev, DME_EINVAL, "no such HIP device");
    DME_HIP(hipSetDevice(device));
    auto c = std::make_unique<dme_ctx>();
    c->device = device;
    // NULL is the null (default) stream, which is what PyTorch's current
    // stream usually is: the library then orders with the caller's work
    c->stream = static_cast<hipStream_t>(stream);
    c->flags.ensure(64);
    dme::noalloc_scratch_init(device);
    *ctx = c.release();
  });
}

void dme_destroy(dme_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->aux.release();
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

int dle_solve(dme_ctx* ctx, const dme_problem* prob, const dme_opts* opts, dme_result** out) {
  return solve_impl(ctx, prob, opts, 0, out);
}

int dre_solve(dme_ctx* ctx, const dme_problem* prob, const dme_opts* opts, dme_result** out) {
  return solve_impl(ctx, prob, opts, 1, out);
}

int dme_solver_create(dme_ctx* ctx, const dme_problem* prob, const dme_opts* opts, int is_dre,
                      dme_solver** out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(prob && opts && out, DME_EINVAL, "null argument");
    *out = nullptr;
    DME_HIP(hipSetDevice(ctx->device));
    auto sv = std::make_unique<dme_solver>();
    sv->ctx = ctx;
    sv->sv.s = ctx->stream;
    sv->sv.device = ctx->device;
    sv->sv.setup(*prob, *opts, is_dre != 0);
    *out = sv.release();
  });
}

int dme_solver_step(dme_solver* sv, int64_t nsteps) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr && nsteps >= 0, DME_EINVAL, "bad solver or step count");
    DME_HIP(hipSetDevice(sv->sv.device));
    sv->sv.advance(nsteps);
  });
}

int dme_solver_state(const dme_solver* sv, int64_t* step, int64_t* nsteps_total, int64_t* rank) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr, DME_EINVAL, "null solver");
    if (step) *step = sv->sv.step;
    if (nsteps_total) *nsteps_total = sv->sv.N;
    if (rank) *rank = sv->sv.r;
  });
}

int dme_solver_setup_info(const dme_solver* sv, double* expm_ms, double* quad_ms, int64_t* rank_quad) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr, DME_EINVAL, "null solver");
    if (expm_ms) *expm_ms = sv->sv.expm_ms;
    if (quad_ms) *quad_ms = sv->sv.quad_ms;
    if (rank_quad) *rank_quad = sv->sv.rank_quad;
  });
}

int dme_solver_result(dme_solver* sv, dme_result** out) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr && out != nullptr, DME_EINVAL, "null argument");
    DME_HIP(hipSetDevice(sv->sv.device));
    make_result(sv->sv, out);
  });
}

int dme_solver_gain(dme_solver* sv, double* K, int64_t ldk) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr && K != nullptr, DME_EINVAL, "null argument");
    dme::Solver& S = sv->sv;
    DME_REQUIRE(S.is_dre, DME_EINVAL, "gain: the solver has no B and R (not a DRE)");
    DME_REQUIRE(ldk >= S.m, DME_EINVAL, "gain: ldk < m");
    DME_HIP(hipSetDevice(S.device));
    S.ws.reset();
    double* Kd = S.ws.get<double>((size_t)S.m * S.n);
    dme::feedback_gain_f64(S.s, S.n, S.r, S.m, S.Lc(), S.n, S.Dc(), S.r, S.B.as<double>(), S.n,
                           S.R.as<double>(), S.m, Kd, S.m, S.flag_dev(), S.ws);
    std::vector<double> h((size_t)S.m * S.n);
    DME_HIP(hipMemcpyAsync(h.data(), Kd, h.size() * sizeof(double), hipMemcpyDeviceToHost, S.s));
    DME_HIP(hipStreamSynchronize(S.s));
    S.check_flags("gain");
    for (int64_t j = 0; j < S.n; ++j)
      for (int64_t i = 0; i < S.m; ++i) K[i + j * ldk] = h[(size_t)i + (size_t)j * S.m];
  });
}

int dme_solver_profile(dme_solver* sv, int enable) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr, DME_EINVAL, "null solver");
    DME_HIP(hipSetDevice(sv->sv.device));
    sv->sv.flush_timings();
    DME_REQUIRE(enable >= 0 && enable <= 2, DME_EINVAL, "profile: enable is 0, 1 or 2");
    sv->sv.profiling = enable;
    for (auto& a : sv->sv.phase) a = dme::PhaseAcc{};
  });
}

int dme_solver_profile_get(dme_solver* sv, int phase, int64_t* count, double* ms, double* flops,
                           double* bytes) {
  return guarded([&] {
    DME_REQUIRE(sv != nullptr && phase >= 0 && phase < 5, DME_EINVAL, "bad solver or phase");
    DME_HIP(hipSetDevice(sv->sv.device));
    sv->sv.flush_timings();
    const dme::PhaseAcc& a = sv->sv.phase[phase];
    if (count) *count = a.count;
    if (ms) *ms = a.ms;
    if (flops) *flops = a.flops;
    if (bytes) *bytes = a.bytes;
  });
}

void dme_solver_free(dme_solver* sv) {
  if (!sv) return;
  (void)hipSetDevice(sv->sv.device);
  (void)hipStreamSynchronize(sv->sv.s);
  delete sv;
}

int dme_result_info(const dme_result* res, int64_t* n, int64_t* r, int64_t* steps, double* err_est) {
  return guarded([&] {
    DME_REQUIRE(res != nullptr, DME_EINVAL, "null result");
    if (n) *n = res->n;
    if (r) *r = res->r;
    if (steps) *steps = res->steps;
    if (err_est) *err_est = res->err_est;
  });
}

int dme_result_copy(const dme_result* res, double* L, double* D) {
  return guarded([&] {
    DME_REQUIRE(res != nullptr, DME_EINVAL, "null result");
    if (L && !res->L.empty()) std::memcpy(L, res->L.data(), res->L.size() * sizeof(double));
    if (D && !res->D.empty()) std::memcpy(D, res->D.data(), res->D.size() * sizeof(double));
  });
}

void dme_result_free(dme_result* res) { delete res; }

int dme_expm(dme_ctx* ctx, int64_t n, const double* X, double t, double* E, int* m_out, int* s_out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(n >= 0 && (n == 0 || (X && E)), DME_EINVAL, "bad expm arguments");
    DME_REQUIRE(X != E || n == 0, DME_EINVAL, "expm: X and E must not alias");
    DME_REQUIRE(std::isfinite(t), DME_EINVAL, "expm: t must be finite");
    DME_HIP(hipSetDevice(ctx->device));
    if (n == 0) return;
    ctx->ws.reserve(dme::expm_workspace(n));
    ctx_reset_flags(ctx);
    dme::expm_f64(ctx->stream, n, X, t, E, ctx->ws, m_out, s_out, ctx_flags(ctx) + 1);
    int h[4];
    ctx_read_flags(ctx, h);
    DME_REQUIRE(h[1] == 0, DME_ENUMERIC, "expm: singular Pade denominator");
  });
}

int dme_gemm_f64(dme_ctx* ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                 double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double beta, double* C, int64_t ldc) {
  return guarded([&] {
    require_ctx(ctx);
    const bool ta = (transa == 'T' || transa == 't'), tb = (transb == 'T' || transb == 't');
    DME_REQUIRE((transa == 'N' || transa == 'n' || ta) && (transb == 'N' || transb == 'n' || tb),
                DME_EINVAL, "gemm: trans must be 'N' or 'T'");
    DME_REQUIRE(M >= 0 && N >= 0 && K >= 0, DME_EINVAL, "gemm: negative dimension");
    DME_REQUIRE(ldc >= std::max<int64_t>(1, M), DME_EINVAL, "gemm: ldc < M");
    DME_REQUIRE(lda >= std::max<int64_t>(1, ta ? K : M), DME_EINVAL, "gemm: lda too small");
    DME_REQUIRE(ldb >= std::max<int64_t>(1, tb ? N : K), DME_EINVAL, "gemm: ldb too small");
    DME_HIP(hipSetDevice(ctx->device));
    ctx->ws.reserve(dme::gemm_f64_workspace(M, N, K) + 1024);
    dme::gemm_f64(ctx->stream, ta ? 'T' : 'N', tb ? 'T' : 'N', M, N, K, alpha, A, lda, B, ldb, beta,
                  C, ldc, &ctx->ws);
  });
}

int dme_gemm_mixed(dme_ctx* ctx, int64_t n, int64_t r, const double* E, const double* X,
                   int64_t ldx, double* Y, int64_t ldy) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(n >= 0 && r >= 0, DME_EINVAL, "gemm_mixed: negative size");
    DME_REQUIRE(n == 0 || r == 0 || (E && X && Y), DME_EINVAL, "gemm_mixed: null pointer");
    DME_REQUIRE(ldx >= std::max<int64_t>(1, n) && ldy >= std::max<int64_t>(1, n), DME_EINVAL,
                "gemm_mixed: leading dimension < n");
    DME_HIP(hipSetDevice(ctx->device));
    if (n == 0 || r == 0) return;
    std::shared_ptr<dme::MixedOp> op = dme::mixed_op_new();
    dme::mixed_op_build(ctx->stream, n, E, *op);
    ctx->ws.reserve(dme::gemm_mixed_workspace(n, r) + 4096);
    dme::gemm_mixed(ctx->stream, *op, X, ldx, r, Y, ldy, ctx->ws);
    // the operator copy is released when this call returns
    DME_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int dme_expmv_leja(dme_ctx* ctx, int64_t n, const double* A_dev, const int64_t* A_rowptr,
                   const int64_t* A_colind, const double* A_val, double t, int64_t ncols,
                   const double* X, double* Y, int* S_out, int* m_out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(n >= 0 && ncols >= 0, DME_EINVAL, "expmv_leja: negative size");
    DME_REQUIRE(std::isfinite(t) && t >= 0, DME_EINVAL, "expmv_leja: t must be finite and >= 0");
    DME_REQUIRE((A_dev != nullptr) != (A_rowptr != nullptr), DME_EINVAL,
                "expmv_leja: give A either dense (device) or in CSR form (host)");
    DME_HIP(hipSetDevice(ctx->device));
    if (n == 0) return;
    DME_REQUIRE(ncols == 0 || (X && Y), DME_EINVAL, "expmv_leja: null X or Y");
    std::shared_ptr<dme::LejaOp> op;
    dme::DevBuf AT;
    ctx->ws.reserve((size_t)dme::cdiv(n, 32) * dme::cdiv(n, 32) * 2 * sizeof(double) +
                    2 * n * sizeof(double) + 4096);
    if (A_dev) {
      AT.ensure((size_t)n * n * sizeof(double));
      dme::transpose_f64(ctx->stream, A_dev, n, AT.as<double>(), n, n, n, 1.0);
      DME_REQUIRE(dme::dense_symmetric(ctx->stream, n, AT.as<double>(), 1e-14, ctx->ws), DME_EINVAL,
                  "expmv_leja: A is not symmetric");
      op = dme::leja_op_dense(ctx->stream, n, AT.as<double>(), ctx->ws);
    } else {
      op = dme::leja_op_csr(ctx->stream, n, A_rowptr, A_colind, A_val, ctx->ws);
      const bool sym = op->symmetric;
      DME_REQUIRE(sym, DME_EINVAL, "expmv_leja: A is not symmetric");
    }
    std::unique_ptr<dme::LejaPlan> plan = dme::leja_plan(*op, {t}, 1);
    if (S_out) *S_out = plan->S;
    if (m_out) *m_out = plan->m;
    if (ncols > 0) {
      ctx->ws.reserve(dme::leja_workspace(n, ncols));
      dme::leja_apply(ctx->stream, *op, *plan, X, n, ncols, Y, n, ctx->ws);
    }
    DME_HIP(hipStreamSynchronize(ctx->stream));
  });
}

int dme_compress(dme_ctx* ctx, int64_t n, int64_t k, double* W, const double* Dhat, double tol,
                 int64_t max_rank, double* L, double* D, int64_t* r_out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(n >= 0 && k >= 0 && max_rank >= 0, DME_EINVAL, "compress: negative size");
    DME_REQUIRE(tol > 0, DME_EINVAL, "compress: tol must be positive");
    DME_REQUIRE(k == 0 || (W && Dhat && L && D), DME_EINVAL, "compress: null pointer");
    DME_HIP(hipSetDevice(ctx->device));
    int64_t r = 0;
    if (k > 0 && n > 0) {
      ctx->ws.reserve(dme::compress_workspace(n, k));
      dme::AuxBinding bind(ctx->aux);
      ctx_reset_flags(ctx);
      r = dme::compress_f64(ctx->stream, n, k, W, Dhat, tol, std::min(max_rank, std::min(n, k)), L,
                            n, D, max_rank, ctx_rank(ctx), ctx_flags(ctx), ctx->ws);
      int h[4];
      ctx_read_flags(ctx, h);
      DME_REQUIRE((h[0] & 1) == 0, DME_ENUMERIC, "compress: non-finite values");
      if (r_out) *r_out = r;
      DME_REQUIRE((h[0] & 2) == 0, DME_ERANK, "compress: rank exceeds max_rank");
    }
    if (r_out) *r_out = r;
  });
}

int dme_riccati(dme_ctx* ctx, int64_t n, int64_t r, int64_t m, const double* L, const double* B,
                const double* R, double t, double* D) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(n >= 0 && r >= 0 && m >= 0, DME_EINVAL, "riccati: negative size");
    DME_HIP(hipSetDevice(ctx->device));
    if (r == 0 || m == 0) return;
    DME_REQUIRE(L && B && R && D, DME_EINVAL, "riccati: null pointer");
    ctx->ws.reserve(dme::gemm_f64_workspace(r, m, n) + (size_t)r * (r + 2 * m) * sizeof(double) + 8192);
    ctx_reset_flags(ctx);
    double* WB = ctx->ws.get<double>((size_t)r * m);
    dme::gemm_f64(ctx->stream, 'T', 'N', r, m, n, 1.0, L, n, B, n, 0.0, WB, r, &ctx->ws);
    dme::riccati_update_f64(ctx->stream, r, m, D, r, WB, r, R, m, t, ctx_flags(ctx), ctx->ws);
    int h[4];
    ctx_read_flags(ctx, h);
    DME_REQUIRE((h[0] & 4) == 0, DME_ENUMERIC, "riccati: R + t W^T D W is not SPD");
  });
}

int dme_syev(dme_ctx* ctx, int64_t k, const double* M, double tol, int64_t max_keep, double* lam,
             double* V, int64_t* keep_out) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(k >= 0 && max_keep >= 0, DME_EINVAL, "syev: negative size");
    DME_REQUIRE(tol >= 0, DME_EINVAL, "syev: tol must be >= 0");
    DME_HIP(hipSetDevice(ctx->device));
    int64_t keep = 0;
    if (k > 0) {
      DME_REQUIRE(M && lam && V, DME_EINVAL, "syev: null pointer");
      ctx->ws.reserve(dme::syev_workspace(k));
      dme::AuxBinding bind(ctx->aux);
      ctx_reset_flags(ctx);
      dme::syev_trunc_f64(ctx->stream, k, M, k, tol, std::min(max_keep, k), lam, V, k,
                          ctx_rank(ctx), ctx_flags(ctx), ctx->ws);
      DME_HIP(hipMemcpyAsync(&keep, ctx_rank(ctx), sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
      DME_HIP(hipStreamSynchronize(ctx->stream));
    }
    if (keep_out) *keep_out = keep;
  });
}

int dme_register_operator(dme_ctx* ctx, const double* A, int64_t n, uint64_t* op_id) {
  return guarded([&] {
    require_ctx(ctx);
    DME_REQUIRE(A != nullptr && n > 0 && op_id != nullptr, DME_EINVAL, "bad operator arguments");
    DME_HIP(hipSetDevice(ctx->device));
    auto op = std::make_shared<dme::RegisteredOp>();
    op->n = n;
    dme::DevBuf tmp((size_t)n * n * sizeof(double));
    DME_HIP(hipMemcpyAsync(tmp.p, A, (size_t)n * n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    op->AT.ensure((size_t)n * n * sizeof(double));
    dme::transpose_f64(ctx->stream, tmp.as<double>(), n, op->AT.as<double>(), n, n, n, 1.0);
    DME_HIP(hipStreamSynchronize(ctx->stream));
    {
      dme::Arena lws;
      lws.reserve((size_t)dme::cdiv(n, 32) * dme::cdiv(n, 32) * 2 * sizeof(double) + 2 * n * sizeof(double) + 4096);
      if (dme::dense_symmetric(ctx->stream, n, op->AT.as<double>(), 1e-14, lws))
        op->lop = dme::leja_op_dense(ctx->stream, n, op->AT.as<double>(), lws);
    }
    std::lock_guard<std::mutex> g(ctx->ops_mu);
    op->id = ctx->next_op++;
    ctx->ops[op->id] = op;
    *op_id = op->id;
  });
}

int dme_server_start(dme_ctx* ctx, size_t hbm_budget_bytes, int max_slots, dme_server** srv) {
  return guarded([&] {
    DME_REQUIRE(srv != nullptr, DME_EINVAL, "null server pointer");
    *srv = nullptr;
    *srv = dme::server_start(ctx, hbm_budget_bytes, max_slots);
  });
}

int dme_server_warm(dme_server* srv, uint64_t op_id, double t, int precision, int quad_nodes) {
  return guarded([&] {
    DME_REQUIRE(std::isfinite(t) && t > 0, DME_EINVAL, "t must be positive");
    dme::server_warm(srv, op_id, t, precision, quad_nodes);
  });
}

int dme_submit(dme_server* srv, uint64_t op_id, const dme_problem* prob, const dme_opts* opts,
               int is_dre, uint64_t* ticket) {
  return guarded([&] {
    DME_REQUIRE(prob && opts && ticket, DME_EINVAL, "null argument");
    *ticket = dme::server_submit(srv, op_id, *prob, *opts, is_dre);
  });
}

int dme_poll(dme_server* srv, uint64_t ticket, dme_result** out) {
  int code = DME_OK;
  std::string msg;
  const int rc = guarded([&] {
    DME_REQUIRE(out != nullptr, DME_EINVAL, "null result pointer");
    *out = nullptr;
    code = dme::server_poll(srv, ticket, out, &msg);
  });
  if (rc != DME_OK) return rc;
  if (code != DME_OK && code != DME_EAGAIN) dme::g_last_error = msg;
  return code;
}

int dme_server_stats_get(dme_server* srv, dme_server_stats* out) {
  return guarded([&] { dme::server_stats(srv, out); });
}

int dme_server_stop(dme_server* srv) {
  return guarded([&] {
    DME_REQUIRE(srv != nullptr, DME_EINVAL, "null server");
    dme::server_stop(srv);
  });
}

int dme_result_serving(const dme_result* res, int* precision, int* fell_back, double* latency_s,
                       double* queue_s) {
  return guarded([&] {
    DME_REQUIRE(res != nullptr, DME_EINVAL, "null result");
    if (precision) *precision = res->precision;
    if (fell_back) *fell_back = res->fell_back;
    if (latency_s) *latency_s = res->latency_s;
    if (queue_s) *queue_s = res->queue_s;
  });
}

}  // extern "C"
