// Splitting-scheme driver: operator setup and the step loop.
//
// Subflows on P = L D L^T (Sec. 2.1 - 2.4, Alg. 1 - 4):
//   T1(t)  L <- e^{tA^T} L                                      (Sec. 2.1)
//   T2(t)  L <- [L, C^T], D <- blkdiag(D, t I), compress         (Sec. 2.1, Alg. 1)
//   T12(t) L <- [e^{tA^T} L, L_I], D <- blkdiag(D, D_I), compress (Alg. 2)
//          with (L_I, D_I) the compressed Gauss-Legendre factor of
//          int_0^t e^{sA^T} C^T C e^{sA} ds                          (Sec. 2.1 eq. for P(t))
//   T3(t)  D <- (I + t D L^T B R^-1 B^T L)^-1 D                    (Sec. 2.2, Alg. 3)
//   T4(t)  L <- [L, sqrt(t) S L, t/sqrt(2) S^2 L], D <- blkdiag(D, D, D),
//          compress                                                (Sec. 2.3, Alg. 4)
// composed as Lie or Strang steps in the orders listed in Sec. 3.  Every
// product runs on the device; the host only sequences launches and reads back
// the rank after each compression.
#include "solver.h"

#include <cmath>

namespace dme {

void gauss_legendre(int K, double t, std::vector<double>& nodes, std::vector<double>& weights) {
  // Newton iteration on the Legendre polynomial P_K (three-term recurrence),
  // starting from the standard cosine guesses; weights 2 / ((1 - x^2) P_K'(x)^2).
  nodes.assign(K, 0.0);
  weights.assign(K, 0.0);
  for (int i = 0; i < K; ++i) {
    long double x = std::cos(M_PI * (i + 0.75) / (K + 0.5));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = x;
      for (int j = 2; j <= K; ++j) {
        const long double p2 = ((2.0L * j - 1.0L) * x * p1 - (j - 1.0L) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      long double pk = (K == 0) ? 1.0L : p1;
      long double pkm1 = (K == 1) ? 1.0L : p0;
      if (K == 1) { pk = x; pkm1 = 1.0L; }
      dp = K * (x * pk - pkm1) / (x * x - 1.0L);
      const long double dx = pk / dp;
      x -= dx;
      if (std::fabs((double)dx) < 1e-19) break;
    }
    const long double w = 2.0L / ((1.0L - x * x) * dp * dp);
    // ascending order: i = 0 gives the largest root
    nodes[K - 1 - i] = (double)(0.5L * t * (x + 1.0L));
    weights[K - 1 - i] = (double)(0.5L * t * w);
  }
}

std::vector<Stage> step_sequence(bool is_dre, bool has_S, int split, int scheme) {
  const bool strang = (scheme == DME_STRANG);
  DME_REQUIRE(scheme == DME_LIE || scheme == DME_STRANG, DME_EINVAL, "unknown scheme");
  std::vector<Sub> inner;
  if (is_dre) inner.push_back(Sub::T3);
  if (has_S) inner.push_back(Sub::T4);
  std::vector<Stage> seq;
  if (split == DME_SPLIT_F12) {
    if (inner.empty()) return {{Sub::T12, 1.0}};
    if (!strang) {
      seq.push_back({Sub::T12, 1.0});
      for (Sub x : inner) seq.push_back({x, 1.0});
      return seq;
    }
    if (inner.size() == 1) return {{Sub::T12, 0.5}, {inner[0], 1.0}, {Sub::T12, 0.5}};
    return {{Sub::T12, 0.5}, {Sub::T3, 0.5}, {Sub::T4, 1.0}, {Sub::T3, 0.5}, {Sub::T12, 0.5}};
  }
  if (split == DME_SPLIT_F1F2) {
    DME_REQUIRE(inner.size() <= 1, DME_EINVAL, "four-term splitting is not part of the method");
    if (inner.empty()) {
      if (!strang) return {{Sub::T1, 1.0}, {Sub::T2, 1.0}};
      return {{Sub::T1, 0.5}, {Sub::T2, 1.0}, {Sub::T1, 0.5}};
    }
    const Sub x = inner[0];
    if (!strang) return {{Sub::T1, 1.0}, {Sub::T2, 1.0}, {x, 1.0}};
    return {{Sub::T1, 0.5}, {Sub::T2, 0.5}, {x, 1.0}, {Sub::T2, 0.5}, {Sub::T1, 0.5}};
  }
  if (split == DME_SPLIT_F1F3F2) {
    DME_REQUIRE(inner.size() == 1, DME_EINVAL, "F1F3F2 needs exactly one of B (DRE) or S");
    const Sub x = inner[0];
    if (!strang) return {{Sub::T1, 1.0}, {x, 1.0}, {Sub::T2, 1.0}};
    return {{Sub::T1, 0.5}, {x, 0.5}, {Sub::T2, 1.0}, {x, 0.5}, {Sub::T1, 0.5}};
  }
  fail(DME_EINVAL, "unknown split");
}

namespace {

struct EventTimer {
  hipEvent_t a, b;
  hipStream_t s;
  explicit EventTimer(hipStream_t st) : s(st) {
    DME_HIP(hipEventCreate(&a));
    DME_HIP(hipEventCreate(&b));
    DME_HIP(hipEventRecord(a, s));
  }
  double stop_ms() {
    DME_HIP(hipEventRecord(b, s));
    DME_HIP(hipEventSynchronize(b));
    float ms = 0.f;
    DME_HIP(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
  ~EventTimer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

void upload(hipStream_t s, DevBuf& dst, const double* src, size_t count) {
  dst.ensure(std::max<size_t>(count, 1) * sizeof(double));
  if (count) DME_HIP(hipMemcpyAsync(dst.p, src, count * sizeof(double), hipMemcpyHostToDevice, s));
}

}  // namespace

hipEvent_t Solver::mark_begin(hipStream_t st) {
  if (!profiling) return nullptr;
  hipEvent_t e;
  if (!event_pool.empty()) {
    e = event_pool.back();
    event_pool.pop_back();
  } else {
    DME_HIP(hipEventCreate(&e));
  }
  DME_HIP(hipEventRecord(e, st ? st : s));
  return e;
}

void Solver::mark_end(int ph, hipEvent_t a, double flops, double bytes, int64_t launches, hipStream_t st) {
  if (!profiling || a == nullptr) return;
  hipEvent_t b = mark_begin(st);
  pending.push_back({ph, a, b, flops, bytes, launches});
}

void Solver::flush_timings() {
  if (pending.empty()) return;
  DME_HIP(hipStreamSynchronize(s));
  if (s3) DME_HIP(hipStreamSynchronize(s3));
  for (const PendingTiming& t : pending) {
    float ms = 0.f;
    DME_HIP(hipEventElapsedTime(&ms, t.a, t.b));
    PhaseAcc& acc = phase[t.phase];
    acc.count += t.launches;
    acc.ms += ms;
    acc.flops += t.flops;
    acc.bytes += t.bytes;
    event_pool.push_back(t.a);
    event_pool.push_back(t.b);
  }
  pending.clear();
}

Solver::~Solver() {
  // the solve's work on both of its streams ends before its events, rank slot
  // and device buffers go
  (void)hipStreamSynchronize(s);
  if (s3) {
    (void)hipStreamSynchronize(s3);
    (void)hipStreamDestroy(s3);
  }
  if (ey_done) (void)hipEventDestroy(ey_done);
  aux.release();
  for (const PendingTiming& t : pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
}

void Solver::check_flags(const char* where) {
  int h[4] = {0, 0, 0, 0};
  DME_HIP(hipMemcpyAsync(h, flags.p, sizeof(h), hipMemcpyDeviceToHost, s));
  DME_HIP(hipStreamSynchronize(s));
  if (h[0] == 0 && h[1] == 0) return;
  std::string w(where);
  if (h[1] != 0) fail(DME_ENUMERIC, w + ": singular Pade denominator (zero pivot)");
  if (h[0] & 1) fail(DME_ENUMERIC, w + ": non-finite values in the factor");
  if (h[0] & 4) fail(DME_ENUMERIC, w + ": Riccati block R + t W^T D W is not SPD");
  if (h[0] & 2) fail(DME_ERANK, w + ": compressed rank exceeds max_rank");
  fail(DME_EINTERNAL, w + ": unknown device flag");
}

void Solver::setup(const dme_problem& prob, const dme_opts& o, bool dre,
                   const OperatorProvider* provider) {
  const bool sparse_in = prob.A_val != nullptr;
  DME_REQUIRE(prob.n > 0 && (prob.A || sparse_in || provider), DME_EINVAL, "need n > 0 and A");
  DME_REQUIRE(prob.p > 0 && prob.C, DME_EINVAL, "need p > 0 and C (Q = C^T C)");
  DME_REQUIRE(o.h > 0 && o.T > 0, DME_EINVAL, "T and h must be positive");
  DME_REQUIRE(o.tol > 0, DME_EINVAL, "tol must be positive");
  DME_REQUIRE(prob.r0 >= 0, DME_EINVAL, "r0 must be >= 0");
  DME_REQUIRE(prob.r0 == 0 || (prob.L0 && prob.D0), DME_EINVAL, "r0 > 0 needs L0 and D0");
  AuxBinding bind(aux);
  n = prob.n;
  p = prob.p;
  is_dre = dre;
  has_S = prob.S != nullptr;
  opts = o;
  if (opts.quad_nodes <= 0) opts.quad_nodes = 7;
  DME_REQUIRE(opts.quad_nodes <= 64, DME_EINVAL, "quad_nodes must be <= 64");
  DME_REQUIRE(opts.precision == DME_FP64 || opts.precision == DME_MIXED, DME_EINVAL,
              "unknown precision");
  DME_REQUIRE(opts.action == DME_ACTION_DENSE || opts.action == DME_ACTION_LEJA, DME_EINVAL,
              "unknown action");
  DME_REQUIRE(!(opts.action == DME_ACTION_LEJA && opts.precision == DME_MIXED), DME_EINVAL,
              "the Leja action runs in FP64 (precision must be DME_FP64)");
  DME_REQUIRE(opts.action == DME_ACTION_LEJA || prob.A || provider, DME_EINVAL,
              "the dense exponential needs the dense A (a CSR A needs DME_ACTION_LEJA)");
  DME_REQUIRE(prob.M == nullptr || (prob.A != nullptr && provider == nullptr), DME_EINVAL,
              "the mass matrix form needs the dense A");
  const double Nf = std::round(o.T / o.h);
  DME_REQUIRE(Nf >= 1 && std::fabs(Nf * o.h - o.T) <= 1e-12 * o.T, DME_EINVAL, "T/h is not an integer");
  N = (int64_t)Nf;
  if (dre) {
    m = prob.m;
    DME_REQUIRE(m > 0 && prob.B && prob.R, DME_EINVAL, "DRE needs m > 0, B and R");
    // R must be SPD: host Cholesky of the m x m input (validation only)
    std::vector<double> Rc(prob.R, prob.R + m * m);
    for (int64_t j = 0; j < m; ++j) {
      double dj = Rc[j + j * m];
      for (int64_t q = 0; q < j; ++q) dj -= Rc[j + q * m] * Rc[j + q * m];
      DME_REQUIRE(dj > 0, DME_EINVAL, "R is not symmetric positive definite");
      const double l = std::sqrt(dj);
      Rc[j + j * m] = l;
      for (int64_t i = j + 1; i < m; ++i) {
        double v = Rc[i + j * m];
        for (int64_t q = 0; q < j; ++q) v -= Rc[i + q * m] * Rc[j + q * m];
        Rc[i + j * m] = v / l;
      }
    }
  } else {
    m = 0;
  }
  seq = step_sequence(dre, has_S, opts.split, opts.scheme);
  {
    double t12 = -1.0;
    ahead_same_t = true;
    for (const Stage& st : seq)
      if (st.sub == Sub::T12) {
        if (t12 >= 0.0 && st.frac != t12) ahead_same_t = false;
        t12 = st.frac;
      }
    if (t12 < 0.0) ahead_same_t = false;
  }
  sizes_for(n, p, opts, &max_rank, &kmax);
  DME_REQUIRE(prob.r0 <= max_rank, DME_EINVAL, "r0 exceeds max_rank");

  DME_HIP(hipSetDevice(device));
  DME_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
  if (hipDeviceGetAttribute(&xccs, hipDeviceAttributeNumberOfXccs, device) != hipSuccess || xccs < 1) xccs = 1;
  flags.ensure(64);
  fill_f64(s, flags.as<double>(), 8, 1, 8, 0.0);

  {
    DevBuf Cd;
    upload(s, Cd, prob.C, (size_t)p * n);
    CT.ensure((size_t)n * p * sizeof(double));
    transpose_f64(s, Cd.as<double>(), p, CT.as<double>(), n, p, n, 1.0);
    DME_HIP(hipStreamSynchronize(s));
  }
  if (provider == nullptr && prob.A) {
    DevBuf A;
    upload(s, A, prob.A, (size_t)n * n);
    AT.ensure((size_t)n * n * sizeof(double));
    transpose_f64(s, A.as<double>(), n, AT.as<double>(), n, n, n, 1.0);
    DME_HIP(hipStreamSynchronize(s));
    ATp = AT.as<double>();
  }
  if (prob.M) apply_mass_matrix(prob.M);
  if (!lop) {
    if (sparse_in) {
      ws.reserve((size_t)2 * n * sizeof(double) + 4096);
      lop = leja_op_csr(s, n, prob.A_rowptr, prob.A_colind, prob.A_val, ws);
      if (!lop->symmetric) lop.reset();
    } else if (ATp) {
      ws.reserve((size_t)cdiv(n, 32) * cdiv(n, 32) * 2 * sizeof(double) + 2 * n * sizeof(double) + 4096);
      if (dense_symmetric(s, n, ATp, 1e-14, ws)) lop = leja_op_dense(s, n, ATp, ws);
    }
  }
  DME_REQUIRE(opts.action != DME_ACTION_LEJA || lop, DME_EINVAL,
              "the Leja action needs a symmetric A (real spectrum)");
  if (dre) {
    upload(s, B, prob.B, (size_t)n * m);
    upload(s, R, prob.R, (size_t)m * m);
  }
  if (has_S) upload(s, S, prob.S, (size_t)n * n);

  for (int q = 0; q < 2; ++q) {
    L[q].ensure((size_t)n * max_rank * sizeof(double));
    D[q].ensure((size_t)max_rank * max_rank * sizeof(double));
  }
  W.ensure((size_t)n * kmax * sizeof(double));
  Dhat.ensure((size_t)kmax * kmax * sizeof(double));
  WB.ensure((size_t)max_rank * std::max<int64_t>(m, 1) * sizeof(double));
  lamT3.ensure((size_t)max_rank * sizeof(double));
  ZT3.ensure((size_t)max_rank * std::max<int64_t>(m, 1) * sizeof(double));
  if (m >= 1 && m <= 8) Fpre.ensure((size_t)kmax * kmax * sizeof(double) + 64);
  if (has_S) SL.ensure((size_t)n * max_rank * sizeof(double));
  ws.reserve(workspace_bytes(n, m, max_rank, kmax, opts.precision) +
             leja_workspace(n, std::max<int64_t>(max_rank, (int64_t)opts.quad_nodes * p)));

  cur = 0;
  r = prob.r0;
  d_diag = (r == 0);
  d_lowrank = false;
  if (r > 0) {
    DME_HIP(hipMemcpyAsync(L[0].p, prob.L0, (size_t)n * r * sizeof(double), hipMemcpyHostToDevice, s));
    DME_HIP(hipMemcpyAsync(D[0].p, prob.D0, (size_t)r * r * sizeof(double), hipMemcpyHostToDevice, s));
  }

  for (const Stage& st : seq) {
    const double t = st.frac * o.h;
    if (st.sub == Sub::T1 || st.sub == Sub::T12) {
      if (!ops.count(t)) {
        EventTimer tm(s);
        if (opts.action == DME_ACTION_LEJA) {
          auto set = std::make_shared<OperatorSet>();
          set->n = n;
          set->t = t;
          set->precision = DME_FP64;
          set->lop = lop;
          set->plan = leja_plan(*lop, {t}, 1);
          ops[t] = set;
        } else {
          ops[t] = provider ? (*provider)(t)
                            : build_operator_set(s, n, ATp, t, opts.precision, 0, false, flag_dev() + 1);
        }
        DME_REQUIRE(ops[t] && ops[t]->n == n && ops[t]->precision == opts.precision, DME_EINTERNAL,
                    "operator set does not match the problem");
        expm_ms += tm.stop_ms();
      }
    }
    if (st.sub == Sub::T12 && !Q.count(t)) {
      EventTimer tm(s);
      build_quadrature(t);
      quad_ms += tm.stop_ms();
    }
  }
  check_flags("setup");
  step = 0;
}

size_t operator_set_bytes(int64_t n, int precision, int K, bool keep_nodes) {
  const size_t nn = (size_t)n * n;
  size_t b = nn * sizeof(double);
  if (precision == DME_MIXED) b += (size_t)n * cdiv(n, 64) * 64 * sizeof(float);
  if (keep_nodes) b += (size_t)K * nn * sizeof(double);
  return b;
}

std::shared_ptr<OperatorSet> build_operator_set(hipStream_t s, int64_t n, const double* AT, double t,
                                                int precision, int K, bool keep_nodes, int* info_dev) {
  hipEvent_t a, b;
  DME_HIP(hipEventCreate(&a));
  DME_HIP(hipEventCreate(&b));
  DME_HIP(hipEventRecord(a, s));
  auto op = std::make_shared<OperatorSet>();
  op->n = n;
  op->t = t;
  op->precision = precision;
  op->K = keep_nodes ? K : 0;
  Arena ews;
  ews.reserve(expm_workspace(n));
  op->E.ensure((size_t)n * n * sizeof(double));
  expm_f64(s, n, AT, t, op->E.as<double>(), ews, nullptr, nullptr, info_dev);
  if (precision == DME_MIXED) {
    op->mix = mixed_op_new();
    mixed_op_build(s, n, op->E.as<double>(), *op->mix);
  }
  if (keep_nodes) {
    std::vector<double> nodes, weights;
    gauss_legendre(K, t, nodes, weights);
    op->nodes.resize(K);
    for (int q = 0; q < K; ++q) {
      ews.reset();
      op->nodes[q].ensure((size_t)n * n * sizeof(double));
      expm_f64(s, n, AT, nodes[q], op->nodes[q].as<double>(), ews, nullptr, nullptr, info_dev);
    }
  }
  DME_HIP(hipEventRecord(b, s));
  DME_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  DME_HIP(hipEventElapsedTime(&ms, a, b));
  op->build_ms = ms;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return op;
}

size_t Solver::workspace_bytes(int64_t n, int64_t m, int64_t max_rank, int64_t kmax, int precision) {
  size_t wsb = compress_workspace(n, kmax);
  wsb += gemm_f64_workspace(max_rank, std::max<int64_t>(m, 1), n) + 4096;
  wsb += gemm_f64_workspace(n, max_rank, n) + 4096;
  if (precision == DME_MIXED) wsb += gemm_mixed_workspace(n, max_rank) + 4096;
  wsb += (size_t)max_rank * (max_rank + 64) * sizeof(double) + 4096;  // riccati scratch
  wsb += compress_gram_workspace(n, kmax);
  return wsb;
}

void Solver::sizes_for(int64_t n, int64_t p, const dme_opts& o, int64_t* max_rank_out,
                       int64_t* kmax_out) {
  const int K = o.quad_nodes > 0 ? o.quad_nodes : 7;
  const int64_t mr = (o.max_rank > 0) ? std::min<int64_t>(o.max_rank, n) : std::min<int64_t>(n, 512);
  const int64_t Kp = (int64_t)K * p;
  *max_rank_out = mr;
  *kmax_out = std::max({mr + p, mr + Kp, 3 * mr, Kp});
}

size_t Solver::state_bytes(int64_t n, int64_t m, int64_t p, bool has_S, const dme_opts& o) {
  int64_t mr = 0, km = 0;
  sizes_for(n, p, o, &mr, &km);
  const int K = o.quad_nodes > 0 ? o.quad_nodes : 7;
  const int64_t Kp = (int64_t)K * p;
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) & ~size_t(255); };
  add((size_t)n * p * 8);                                     // C^T
  add((size_t)n * std::max<int64_t>(m, 1) * 8);                // B
  add((size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(m, 1) * 8);
  if (has_S) add((size_t)n * n * 8 + (size_t)n * mr * 8);
  add(2 * ((size_t)n * mr * 8 + (size_t)mr * mr * 8));          // L, D ping-pong
  add((size_t)n * km * 8 + (size_t)km * km * 8);                // W, Dhat
  add((size_t)mr * std::max<int64_t>(m, 1) * 8);                // W_B
  add((size_t)mr * (std::max<int64_t>(m, 1) + 1) * 8);          // lam and Z of a T3 update
  if (m >= 1 && m <= 8) add((size_t)km * km * 8 + 64);          // its factor, formed ahead
  add(2 * ((size_t)n * Kp * 8 + (size_t)Kp * Kp * 8));          // quadrature factors (h and h/2)
  add(workspace_bytes(n, m, mr, km, o.precision));
  add(leja_workspace(n, std::max<int64_t>(mr, Kp)));
  return b + 64;
}

// Mass-matrix form (Sec. 5.1, Ex. 4): M^T dP/dt M = A^T P M + M^T P A + Q + ...
// becomes the standard form with A M^-1 in place of A and C M^-1 in place of C
// (Q = C^T C -> M^-T Q M^-1); B, R and S are unchanged.  On the device:
// A^T <- M^-T A^T and C^T <- M^-T C^T by one LU factorisation of M^T with
// partial pivoting and a solve with the n + p right-hand sides [A^T, C^T].
void Solver::apply_mass_matrix(const double* Mh) {
  DME_REQUIRE(ATp == AT.as<double>() && ATp != nullptr, DME_EINTERNAL, "mass matrix without A^T");
  const int64_t nr = n + p;
  DevBuf Mt((size_t)n * n * sizeof(double));
  DevBuf rhs((size_t)n * nr * sizeof(double));
  {
    DevBuf Md;
    upload(s, Md, Mh, (size_t)n * n);
    transpose_f64(s, Md.as<double>(), n, Mt.as<double>(), n, n, n, 1.0);
    copy_f64(s, AT.as<double>(), n, rhs.as<double>(), n, n, n);
    copy_f64(s, CT.as<double>(), n, rhs.as<double>() + (size_t)n * n, n, n, p);
    DME_HIP(hipStreamSynchronize(s));
  }
  Arena lws;
  lws.reserve(lu_solve_workspace(n, nr));
  lu_solve_f64(s, n, Mt.as<double>(), rhs.as<double>(), n, nr, lws, flag_dev() + 1);
  copy_f64(s, rhs.as<double>(), n, AT.as<double>(), n, n, n);
  copy_f64(s, rhs.as<double>() + (size_t)n * n, n, CT.as<double>(), n, n, p);
  DME_HIP(hipStreamSynchronize(s));
  int h[4] = {0, 0, 0, 0};
  DME_HIP(hipMemcpy(h, flags.p, sizeof(h), hipMemcpyDeviceToHost));
  DME_REQUIRE(h[1] == 0, DME_ENUMERIC, "mass matrix: M is singular (zero pivot)");
}

void Solver::build_quadrature(double t) {
  const int K = opts.quad_nodes;
  std::vector<double> nodes, weights;
  gauss_legendre(K, t, nodes, weights);
  const int64_t kq = (int64_t)K * p;
  const OperatorSet& op = *ops.at(t);
  // columns [e^{s_k A^T} C^T]_k directly into W, weights into Dhat
  double* Wd = W.as<double>();
  if (lop && (int)op.nodes.size() != K) {
    // the K node actions by Leja interpolation (Alg. 2 with expleja): one
    // block of K copies of C^T, group k advanced to time s_k
    for (int q = 0; q < K; ++q) copy_f64(s, CT.as<double>(), n, Wd + (int64_t)q * p * n, n, n, p);
    std::unique_ptr<LejaPlan> plan = leja_plan(*lop, nodes, p);
    ws.reset();
    leja_apply(s, *lop, *plan, Wd, n, kq, Wd, n, ws);
    DME_HIP(hipStreamSynchronize(s));  // the plan's device coefficients go with it
  } else {
    // dense node operators e^{s_k A^T}: the products e^{s_k A^T} C^T in FP64,
    // or in DME_MIXED through the split-BF16 product (an FP32 copy of each
    // node operator); the first node's product is also formed in FP64 there,
    // and its relative distance enters the error estimate
    const bool mixedq = opts.precision == DME_MIXED;
    std::shared_ptr<MixedOp> mq = mixedq ? mixed_op_new() : nullptr;
    Arena qa;  // the node products (and, in DME_MIXED, the first one's FP64 twin)
    qa.reserve(gemm_f64_workspace(n, p, n) + (mixedq ? gemm_mixed_workspace(n, p) : 0) +
               (size_t)n * p * sizeof(double) + diff_norms_workspace() + 16384);
    auto node_product = [&](const double* Ek, int q) {
      double* dst = Wd + (int64_t)q * p * n;
      qa.reset();
      if (!mixedq) {
        gemm_f64(s, 'N', 'N', n, p, n, 1.0, Ek, n, CT.as<double>(), n, 0.0, dst, n, &qa);
        return;
      }
      mixed_op_build(s, n, Ek, *mq);
      gemm_mixed(s, *mq, CT.as<double>(), n, p, dst, n, qa);
      if (q == 0) {
        qa.reset();
        double* y64 = qa.get<double>((size_t)n * p);
        const size_t mark = qa.used;
        gemm_f64(s, 'N', 'N', n, p, n, 1.0, Ek, n, CT.as<double>(), n, 0.0, y64, n, &qa);
        qa.used = mark;
        double* part = qa.get<double>(diff_norms_workspace() / sizeof(double));
        double* out = qa.get<double>(2);
        diff_norms_f64(s, dst, n, y64, n, n, p, part, out);
        double h2[2] = {0.0, 0.0};
        DME_HIP(hipMemcpyAsync(h2, out, sizeof(h2), hipMemcpyDeviceToHost, s));
        DME_HIP(hipStreamSynchronize(s));
        quad_delta = std::max(quad_delta, h2[1] > 0.0 ? std::sqrt(h2[0] / h2[1]) : 0.0);
      }
    };
    if ((int)op.nodes.size() == K) {
      for (int q = 0; q < K; ++q) node_product(op.nodes[q].as<double>(), q);
    } else {
      DME_REQUIRE(ATp != nullptr, DME_EINTERNAL, "quadrature factor needs the operator or its nodes");
      DevBuf Ek((size_t)n * n * sizeof(double));
      Arena ews;
      ews.reserve(expm_workspace(n));
      for (int q = 0; q < K; ++q) {
        ews.reset();
        expm_f64(s, n, ATp, nodes[q], Ek.as<double>(), ews, nullptr, nullptr, flag_dev() + 1);
        node_product(Ek.as<double>(), q);
      }
    }
  }
  double* Dh = Dhat.as<double>();
  fill_f64(s, Dh, kq, kq, kq, 0.0);
  for (int q = 0; q < K; ++q)
    blkdiag2_f64(s, nullptr, 0, 1, nullptr, p, 1, weights[q], Dh + (int64_t)q * p * (kq + 1), kq);
  DME_HIP(hipStreamSynchronize(s));
  QuadFactor& f = Q[t];
  f.L.ensure((size_t)n * kq * sizeof(double));
  f.D.ensure((size_t)kq * kq * sizeof(double));
  ws.reset();
  f.r = compress_f64(s, n, kq, Wd, Dh, opts.tol, std::min<int64_t>(kq, n), f.L.as<double>(), n,
                     f.D.as<double>(), 0, rank_dev(), flag_dev(), ws);
  rank_quad = std::max(rank_quad, f.r);
  check_flags("quadrature factor");
}

namespace {
// Times the main kernel of each step product into phase DME_PHASE_STEP_KERNEL
// with the method's algorithmic work of that launch: 2 m k ncols flops; E
// read once plus X read and Y written in FP64.
struct StepKernelTimer : KernelTimer {
  Solver* sv = nullptr;
  hipEvent_t a = nullptr;
  void before(hipStream_t st) override { a = sv->mark_begin(st); }
  void after(hipStream_t st, int64_t m, int64_t ncols, int64_t k, int e_bytes) override {
    sv->mark_end(DME_PHASE_STEP_KERNEL, a, 2.0 * m * k * ncols,
                 (double)e_bytes * m * k + 8.0 * ((double)k * ncols + (double)m * ncols), 1, st);
    a = nullptr;
  }
};
// Workgroups of a step-product kernel one CU holds at a time: two of the
// FP64 kernel, one of the split-BF16 kernel.
int per_cu(int precision) { return precision == DME_MIXED ? 1 : 2; }
// Longest split of the inner dimension n (chunks of at least 1024 or 256).
int64_t split_cap(int precision, int64_t n) {
  return std::max<int64_t>(1, n / (precision == DME_MIXED ? 1024 : 256));
}

// The split of the inner dimension that gives `rows` rows of a step product
// one wave of workgroups on `slots` workgroup slots (a workgroup per
// kRowBlock rows and chunk): the wave's time falls with the chunk length.
int fill_split_for(int64_t rows, int64_t slots, int64_t cap) {
  const int64_t rb = cdiv(rows, kRowBlock);
  return (int)std::max<int64_t>(1, std::min<int64_t>(slots / std::max<int64_t>(rb, 1), cap));
}

}  // namespace

int Solver::fill_split(int64_t rows) const {
  return fill_split_for(rows, (int64_t)per_cu(opts.precision) * cus, split_cap(opts.precision, n));
}

void Solver::product_rows(double t, const double* X, int64_t cols, int64_t row0, int64_t rows, int ns,
                          hipStream_t st, Arena& a) {
  double* Y = EW.as<double>() + (max_rank - cols) * n;
  const OperatorSet& set = *ops.at(t);
  if (set.lop) {
    // the Leja action is formed for every row at once (its terms are short
    // launches that leave room between them for the compression's kernels);
    // profiling level 2 times it as its Newton-term launches
    DME_REQUIRE(row0 == 0 && rows == n, DME_EINTERNAL, "Leja action ahead: all rows at once");
    hipEvent_t ev = profiling == 2 ? mark_begin(st) : nullptr;
    leja_apply(st, *set.lop, *set.plan, X, n, cols, Y, n, a);
    const int64_t prods = leja_products(*set.plan);
    // per term the operator and the basis block read and written; the
    // accumulator read and written every second term
    mark_end(DME_PHASE_STEP_KERNEL, ev, (double)prods * 2.0 * set.lop->nnz * cols,
             (double)prods * (12.0 * set.lop->nnz + 8.0 * n + 16.0 * n * cols) +
                 (double)leja_csr_p_updates(*set.plan) * 16.0 * n * cols,
             prods, st);
    return;
  }
  if (opts.precision == DME_MIXED)
    gemm_mixed(st, *set.mix, X, n, cols, Y, n, a, row0, rows, ns);
  else
    gemm_f64_rows(st, rows, cols, n, set.E.as<double>() + row0, n, X, n, Y + row0, n, ns, a);
}

void Solver::apply_E(double t, const double* X, int64_t rr, double* Y, int64_t ldy) {
  ws.reset();
  const OperatorSet& set = *ops.at(t);
  if (set.lop) {
    // profiling level 1 times the action as the step-product phase, level 2
    // as its Newton-term launches (the events bracket the whole action, so
    // the block transposes at its ends count against the terms)
    hipEvent_t ev = profiling ? mark_begin() : nullptr;
    leja_apply(s, *set.lop, *set.plan, X, n, rr, Y, ldy, ws);
    // S m products with A^T (2 nnz r flops each for CSR, 2 n^2 r dense); per
    // term the basis block is read and written, and the accumulator is
    // updated (every second term on a CSR operator)
    const int64_t prods = leja_products(*set.plan);
    const bool csr = set.lop->sparse();
    const double opf = csr ? 2.0 * set.lop->nnz : 2.0 * (double)n * n;
    const double opb = csr ? 12.0 * set.lop->nnz + 8.0 * n : 8.0 * (double)n * n;
    const double pupd = csr ? (double)leja_csr_p_updates(*set.plan) : (double)prods;
    mark_end(profiling == 2 ? DME_PHASE_STEP_KERNEL : DME_PHASE_STEP_GEMM, ev, (double)prods * opf * rr,
             (double)prods * (opb + 16.0 * n * rr) + pupd * 16.0 * n * rr, prods);
    return;
  }
  StepKernelTimer kt;
  kt.sv = this;
  KernelTimer* prev = kernel_timer();
  if (profiling) kernel_timer() = &kt;
  hipEvent_t ev = mark_phase();
  if (opts.precision == DME_MIXED) {
    gemm_mixed(s, *ops.at(t)->mix, X, n, rr, Y, ldy, ws);
    // algorithmic work of Y = E X: 2 n^2 r flops; the FP32 operator read once
    mark_end(0, ev, 2.0 * n * n * rr, 4.0 * (double)n * n + 16.0 * n * rr);
  } else {
    gemm_f64(s, 'N', 'N', n, rr, n, 1.0, ops.at(t)->E.as<double>(), n, X, n, 0.0, Y, ldy, &ws);
    // algorithmic work of Y = E X: 2 n^2 r flops; E read once, X read, Y written
    mark_end(0, ev, 2.0 * n * n * rr, 8.0 * ((double)n * n + 2.0 * n * rr));
  }
  kernel_timer() = prev;
}

void Solver::plan_beside(int64_t k, int64_t* rows_out, int* ns_out) const {
  *rows_out = 0;
  *ns_out = 0;
  if (r <= 0 || n < kRowBlock || cus <= xccs) return;
  const bool mixed = opts.precision == DME_MIXED;
  // Measured on gfx950 (n = 16384, k ~ 178): the tridiagonal reduction takes
  // about 1.9 us a step; the whole product one wave of workgroups, the FP64
  // kernel at ~50 TFLOP/s and the split-BF16 kernel reading the FP32
  // operator at ~2.8 TB/s; beside the reduction the FP64 kernel's workgroups
  // run ~1.6x slower than in a whole product (the split-BF16 ones at full
  // speed); rows still running when the reduction ends hold the CUs the rest
  // of the eigensolver needs, which waits about as long as they overrun.
  const double tau = 1.9e-6 * (double)k;
  const double t_full = mixed ? 4.0 * (double)n * n / 2.8e12 : 2.0 * (double)n * n * r / 50e12;
  const double slow = mixed ? 1.0 : 1.6;
  const int64_t cap = split_cap(opts.precision, n), rb_all = cdiv(n, kRowBlock);
  const int64_t slots = (int64_t)per_cu(opts.precision) * cus;
  // workgroups go to the XCDs in turn: one CU left free in every XCD keeps
  // the reduction's CU, wherever it is, from costing a workgroup a second turn
  const int64_t slots_b = (int64_t)per_cu(opts.precision) * (cus - xccs);
  const double t_wg = t_full * fill_split_for(n, slots, cap);  // a workgroup's time at split 1
  // c row blocks beside (the longest split that fits the slots): the
  // shortest critical path, the remainder's wave plus the overrun's delay;
  // the smallest c on ties
  double best = t_full;
  for (int64_t c = 1; c <= std::min(rb_all, slots_b); ++c) {
    const int64_t ns_c = std::min<int64_t>(cap, slots_b / c);
    if (ns_c < 1) break;
    const double t_c = slow * t_wg / ns_c;
    const int64_t rb_r = rb_all - c;
    const double t_r = rb_r > 0 ? t_wg / fill_split_for(rb_r * kRowBlock, slots, cap) : 0.0;
    const double path = t_r + std::max(0.0, t_c - tau);
    if (path < best * (1.0 - 1e-3)) {
      best = path;
      *rows_out = std::min<int64_t>(n, c * kRowBlock);
      *ns_out = (int)ns_c;
    }
  }
}

void Solver::compress_into(int64_t k, int ncopies, double ahead_t) {
  ws.reset();
  hipEvent_t ev = mark_phase();
  // through the Gram matrix while Dhat is positive definite (every DLE / DRE
  // compression from a positive semidefinite P0), by Householder QR otherwise
  LowRankD lr{lamT3.as<double>(), ZT3.as<double>(), t3, r, m, ncopies};
  const double* Fr = f_ready ? Fpre.as<double>() : nullptr;
  const int64_t* Fs = f_ready ? reinterpret_cast<const int64_t*>(Fr + k * k) : nullptr;
  f_ready = false;
  // the next T12's product ahead: e^{tA^T} Y for Y = W[:, 0:r] on s3, its
  // first rows beside the tridiagonal reduction (a Leja action: all of it)
  drop_ahead();
  int64_t rows_b = 0;
  int ns_b = 0;
  const bool leja_ahead = ahead_t > 0.0 && ops.at(ahead_t)->lop != nullptr;
  if (leja_ahead) {
    if (r > 0) rows_b = n;  // the whole action beside the compression
  } else if (ahead_t > 0.0) {
    plan_beside(k, &rows_b, &ns_b);
  }
  std::function<void(hipEvent_t)> beside;
  bool launched = false;
  if (rows_b > 0) {
    if (!s3) DME_HIP(hipStreamCreateWithFlags(&s3, hipStreamNonBlocking));
    if (!ey_done) DME_HIP(hipEventCreateWithFlags(&ey_done, hipEventDisableTiming));
    // e^{tA^T} Y (at most max_rank columns) and e^{tA^T} L_I (at most K p)
    const int64_t kq = std::max<int64_t>(1, (int64_t)opts.quad_nodes * p);
    EW.ensure((size_t)n * (max_rank + kq) * sizeof(double));
    Tk.ensure((size_t)(max_rank + kq) * max_rank * sizeof(double));
    const size_t need = leja_ahead ? leja_workspace(n, r) + 4096
                                   : (size_t)ns_b * rows_b * std::max<int64_t>(r + 16, kRowBlock) * sizeof(double) +
                                         (size_t)3 * (n + kRowBlock) * kRowBlock * sizeof(uint16_t) +
                                         4096;  // partials, X pieces
    if (ws3.buf.bytes < need) ws3.reserve(need);
    const int64_t rY = r;
    beside = [this, ahead_t, rows_b, ns_b, rY, &launched](hipEvent_t e) {
      DME_HIP(hipStreamWaitEvent(s3, e, 0));
      StepKernelTimer kt;
      kt.sv = this;
      KernelTimer* prev = kernel_timer();
      if (profiling) kernel_timer() = &kt;
      ws3.reset();
      product_rows(ahead_t, W.as<double>(), rY, 0, rows_b, ns_b, s3, ws3);
      kernel_timer() = prev;
      DME_HIP(hipEventRecord(ey_done, s3));
      launched = true;
      beside_live = true;
    };
  }
  int64_t rn = compress_gram_f64(s, n, k, W.as<double>(), n, Dhat.as<double>(), k, d_diag,
                                 d_lowrank ? &lr : nullptr, opts.tol, max_rank, Ln(), n, Dn(), 0, rank_dev(),
                                 flag_dev(), ws, r, Fr, Fs,  // the rank before: the guess for the new one
                                 rows_b > 0 ? Tk.as<double>() : nullptr, rows_b > 0 ? &beside : nullptr);
  const double kk = (double)k;
  if (rn >= 0) {
    // W^T W 2 n k^2, L = W T 2 n k r', the k x k products and eigenproblem ~ 14 k^3
    mark_end(1, ev, 2.0 * n * kk * kk + 2.0 * n * kk * rn + 14.0 * kk * kk * kk,
             8.0 * (2.0 * n * kk + n * rn));
    if (launched && rn > 0) {  // L = W T: the next T12 takes [e^{tA^T} Y, e^{tA^T} L_I] T
      ey_ok = tk_ok = true;
      ey_t = ahead_t;
      ey_cols = r;
      ey_rows = rows_b;
      tk_k = k;
    }
  } else {
    ws.reset();
    rn = compress_f64(s, n, k, W.as<double>(), Dhat.as<double>(), opts.tol, max_rank, Ln(), n, Dn(), 0,
                      rank_dev(), flag_dev(), ws);
    // Householder QR 2 n k^2 - 2/3 k^3, Q application 4 n k r', small eigenproblem ~ 10 k^3
    mark_end(1, ev, 2.0 * n * kk * kk + 4.0 * n * kk * rn + 10.0 * kk * kk * kk,
             8.0 * (2.0 * n * kk + 2.0 * n * rn));
  }
  cur ^= 1;
  r = rn;
  d_diag = true;
  d_lowrank = false;
}

void Solver::apply_T1(double t) {
  settle_beside();
  drop_ahead();
  if (r == 0) return;
  apply_E(t, Lc(), r, Ln(), n);
  ++nprod;
  copy_f64(s, Dc(), r, Dn(), r, r, r);
  cur ^= 1;
}

void Solver::apply_T2(double t) {
  settle_beside();
  drop_ahead();
  double* Wd = W.as<double>();
  if (r > 0) copy_f64(s, Lc(), n, Wd, n, n, r);
  copy_f64(s, CT.as<double>(), n, Wd + r * n, n, n, p);
  const int64_t k = r + p;
  blkdiag2_f64(s, Dc(), r, r, nullptr, p, 1, t, Dhat.as<double>(), k);
  compress_into(k);
}

void Solver::apply_T12(double t, bool ext_product) {
  const QuadFactor& f = Q.at(t);
  double* Wd = W.as<double>();
  const int64_t k = r + f.r;
  const OperatorSet& set = *ops.at(t);
  // dense products (FP64 up to 256 columns), or the Leja action on a CSR operator
  const bool leja = set.lop && set.lop->sparse();
  const bool can_ahead = ahead && ahead_same_t && !ext_product && (!set.lop || leja) &&
                         (leja || opts.precision == DME_MIXED || r <= 256);
  // e^{tA^T} L = [e^{tA^T} Y, e^{tA^T} L_I] T from the product formed ahead
  const bool from_ahead = can_ahead && r > 0 && ey_ok && tk_ok && ey_t == t && tk_k == ey_cols + f.r;
  settle_beside();  // (the rows formed beside are complete before W changes)
  // D-hat (and after a T3 update its factor; the quadrature columns of W too
  // unless W still holds the Y of the product formed ahead) on the second
  // stream, beside the product
  hipEvent_t w_ready = nullptr;
  if (k > 0) {
    AuxStream& ax = aux_stream();
    DME_HIP(hipStreamWaitEvent(ax.s2, ax.record(s), 0));
    blkdiag2_f64(ax.s2, Dc(), r, r, f.D.as<double>(), f.r, f.r, 1.0, Dhat.as<double>(), k);
    if (f.r > 0 && !from_ahead) copy_f64(ax.s2, f.L.as<double>(), n, Wd + r * n, n, n, f.r);
    if (d_lowrank && Fpre.bytes > 0) {
      const LowRankD lr{lamT3.as<double>(), ZT3.as<double>(), t3, r, m, 1};
      double* F = Fpre.as<double>();
      f_ready = gram_factor_lowrank(ax.s2, k, Dhat.as<double>(), k, lr, F, reinterpret_cast<int64_t*>(F + k * k));
    }
    w_ready = ax.record(ax.s2);
  }
  if (from_ahead) {
    hipEvent_t ev = mark_phase();
    StepKernelTimer kt;
    kt.sv = this;
    KernelTimer* prev = kernel_timer();
    if (profiling) kernel_timer() = &kt;
    // the rows not formed beside the last compression (W[:, 0:ey_cols] is
    // still the Y they multiply)
    const int64_t rest = n - ey_rows;
    ws.reset();
    if (rest > 0) product_rows(t, Wd, ey_cols, ey_rows, rest, fill_split(rest), s, ws);
    kernel_timer() = prev;
    if (eli_t != t) {  // e^{tA^T} L_I beside it, in FP64 (formed once per t)
      DevBuf& e = ELI[t];
      if (e.bytes == 0) {
        e.ensure((size_t)n * std::max<int64_t>(f.r, 1) * sizeof(double));
        ws.reset();
        if (f.r > 0 && leja)
          leja_apply(s, *set.lop, *set.plan, f.L.as<double>(), n, f.r, e.as<double>(), n, ws);
        else if (f.r > 0)
          gemm_f64(s, 'N', 'N', n, f.r, n, 1.0, set.E.as<double>(), n, f.L.as<double>(), n, 0.0,
                   e.as<double>(), n, &ws);
      }
      if (f.r > 0) copy_f64(s, e.as<double>(), n, EW.as<double>() + max_rank * n, n, n, f.r);
      eli_t = t;
    }
    ws.reset();
    gemm_f64(s, 'N', 'N', n, r, tk_k, 1.0, EW.as<double>() + (max_rank - ey_cols) * n, n, Tk.as<double>(),
             tk_k, 0.0, Wd, n, &ws);
    if (f.r > 0) copy_f64(s, f.L.as<double>(), n, Wd + r * n, n, n, f.r);
    ++nprod;
    mark_end(0, ev, 2.0 * rest * n * ey_cols + 2.0 * n * tk_k * r,
             8.0 * ((double)rest * n + (double)n * (tk_k + r)));
    drop_ahead();  // consumed
  } else {
    drop_ahead();
    if (r > 0 && !ext_product) apply_E(t, Lc(), r, Wd, n);
    if (r > 0) ++nprod;  // (a grouped product of the server counts the same)
  }
  if (k == 0) return;
  DME_HIP(hipStreamWaitEvent(s, w_ready, 0));
  compress_into(k, 1, (can_ahead && r > 0) ? t : 0.0);
}

void Solver::apply_T3(double t) {
  if (r == 0) return;
  hipEvent_t ev = mark_phase();
  ws.reset();
  gemm_f64(s, 'T', 'N', r, m, n, 1.0, Lc(), n, B.as<double>(), n, 0.0, WB.as<double>(), r, &ws);
  ws.reset();
  // T3 on a diagonal D keeps D = diag(lam) - t Z Z^T in factored form for the
  // next compression (its factor then needs no Cholesky)
  const bool lowrank = d_diag && m <= 8;
  if (lowrank) copy_f64(s, Dc(), r + 1, lamT3.as<double>(), 1, 1, r);  // the diagonal of D
  riccati_update_f64(s, r, m, Dc(), r, WB.as<double>(), r, R.as<double>(), m, t, flag_dev(), ws,
                     lowrank ? ZT3.as<double>() : nullptr);
  d_diag = false;
  d_lowrank = lowrank;
  t3 = t;
  mark_end(2, ev, 2.0 * n * r * m + 2.0 * r * r * m, 8.0 * ((double)n * r + (double)n * m));
}

void Solver::apply_T4(double t) {
  settle_beside();
  drop_ahead();
  if (r == 0) return;
  double* Wd = W.as<double>();
  hipEvent_t ev = mark_phase();
  ws.reset();
  gemm_f64(s, 'N', 'N', n, r, n, 1.0, S.as<double>(), n, Lc(), n, 0.0, SL.as<double>(), n, &ws);
  copy_f64(s, Lc(), n, Wd, n, n, r);
  copy_scaled_f64(s, SL.as<double>(), n, Wd + r * n, n, n, r, std::sqrt(t));
  ws.reset();
  gemm_f64(s, 'N', 'N', n, r, n, t / std::sqrt(2.0), S.as<double>(), n, SL.as<double>(), n, 0.0,
           Wd + 2 * r * n, n, &ws);
  mark_end(3, ev, 4.0 * n * n * r, 8.0 * (2.0 * n * n + 4.0 * n * r));
  const int64_t k = 3 * r;
  double* Dh = Dhat.as<double>();
  fill_f64(s, Dh, k, k, k, 0.0);
  for (int q = 0; q < 3; ++q) copy_f64(s, Dc(), r, Dh + q * r * (k + 1), k, r, r);
  compress_into(k, 3);
}

double Solver::err_estimate() {
  settle_beside();
  drop_ahead();  // W is scratch below
  const double u = std::ldexp(1.0, -53);
  double delta = 0.0;
  if (opts.precision == DME_MIXED && r > 0 && !ops.empty()) {
    AuxBinding bind(aux);
    const OperatorSet& op = *ops.rbegin()->second;
    DME_REQUIRE(op.mix != nullptr, DME_EINTERNAL, "mixed operator set without its FP32 copy");
    double* Ym = W.as<double>();  // W and the spare factor are free between steps
    double* Y64 = Ln();
    ws.reset();
    gemm_mixed(s, *op.mix, Lc(), n, r, Ym, n, ws);
    ws.reset();
    gemm_f64(s, 'N', 'N', n, r, n, 1.0, op.E.as<double>(), n, Lc(), n, 0.0, Y64, n, &ws);
    ws.reset();
    double* part = ws.get<double>(diff_norms_workspace() / sizeof(double));
    double* out = ws.get<double>(2);
    diff_norms_f64(s, Ym, n, Y64, n, n, r, part, out);
    double h[2] = {0.0, 0.0};
    DME_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
    DME_HIP(hipStreamSynchronize(s));
    delta = h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
  }
  // the Leja action's interpolation error: at most 1e-14 per substep
  double action = 0.0;
  for (const auto& kv : ops)
    if (kv.second->plan) action = std::max(action, 1e-14 * kv.second->plan->S);
  const double per_product = std::max({delta, action, std::sqrt((double)n) * u});
  // a quadrature factor formed by split-BF16 products adds its relative error
  // with every application of the quadrature term (at most one per product)
  return 2.0 * (double)nprod * per_product + (double)nprod * quad_delta;
}

void Solver::run_stage(size_t i, bool ext_product) {
  AuxBinding bind(aux);
  const Stage& st = seq.at(i);
  const double t = st.frac * opts.h;
  switch (st.sub) {
    case Sub::T1: apply_T1(t); break;
    case Sub::T2: apply_T2(t); break;
    case Sub::T12: apply_T12(t, ext_product); break;
    case Sub::T3: apply_T3(t); break;
    case Sub::T4: apply_T4(t); break;
  }
}

void Solver::advance(int64_t nsteps) {
  AuxBinding bind(aux);
  ahead = true;
  try {
    for (int64_t it = 0; it < nsteps; ++it) {
      for (size_t i = 0; i < seq.size(); ++i) run_stage(i);
      end_step();
    }
  } catch (...) {
    ahead = false;
    drop_ahead();
    throw;
  }
  ahead = false;
  flush_timings();
  check_flags("step");
}

}  // namespace dme
