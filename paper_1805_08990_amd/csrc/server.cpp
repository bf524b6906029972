// Request server: continuous batching of DLE / DRE solves on one GPU.
//
// Clients submit solves (host data copied on submit) against operators
// registered once on the context.  A scheduler thread runs "ticks": it admits
// waiting requests in arrival order while a slot is free and the HBM ledger
// (operator cache + per-solve state) stays within the budget, then advances
// every admitted solve by one time step, and retires the finished ones.
//
// Inside a tick the stages of the step sequences run in lockstep.  For a T12
// stage, the solves that use the same cached operator e^{tA^T} are served by
// one product over their column-concatenated factors ([L_1 ... L_g] gathered
// into one block, one skinny FP64 or split-BF16 product, results scattered to
// each solve's workspace), so the operator is streamed from HBM once for the
// group.  Every column's arithmetic in those products is independent of the
// other columns, so a solve's result does not depend on what it was batched
// with.  The rest of each stage (concatenation, compression, Riccati update)
// runs per solve on the solve's own stream, the solves in parallel on worker
// threads, so their kernels overlap on the device.
//
// A mixed-precision request that trips a numerical guard (non-finite values,
// rank above max_rank) is re-run from the start in FP64.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>

#include "ctx.h"

namespace dme {
namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  static const clk::time_point t0 = clk::now();
  return std::chrono::duration<double>(clk::now() - t0).count();
}

// Fixed-size worker pool running one batch of tasks at a time.
class Pool {
 public:
  Pool(int n, int device) : device_(device) {
    for (int i = 0; i < n; ++i) th_.emplace_back([this] { loop(); });
  }
  ~Pool() {
    {
      std::lock_guard<std::mutex> g(mu_);
      quit_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }
  // Run every task, return when all have finished.
  void run(std::vector<std::function<void()>>& tasks) {
    if (tasks.empty()) return;
    if (tasks.size() == 1 || th_.empty()) {
      for (auto& f : tasks) f();
      return;
    }
    {
      std::lock_guard<std::mutex> g(mu_);
      tasks_ = &tasks;
      next_ = 0;
      left_ = tasks.size();
      ++gen_;
    }
    cv_.notify_all();
    std::unique_lock<std::mutex> g(mu_);
    done_.wait(g, [this] { return left_ == 0; });
    tasks_ = nullptr;
  }

 private:
  void loop() {
    (void)hipSetDevice(device_);  // the current device is per host thread
    uint64_t seen = 0;
    for (;;) {
      std::function<void()>* f = nullptr;
      {
        std::unique_lock<std::mutex> g(mu_);
        cv_.wait(g, [&] { return quit_ || (tasks_ && next_ < tasks_->size()) || gen_ != seen; });
        if (quit_) return;
        seen = gen_;
        if (!tasks_ || next_ >= tasks_->size()) continue;
        f = &(*tasks_)[next_++];
      }
      (*f)();
      std::lock_guard<std::mutex> g(mu_);
      if (--left_ == 0) done_.notify_all();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  std::vector<std::function<void()>>* tasks_ = nullptr;
  size_t next_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool quit_ = false;
  int device_ = 0;
};

struct OpKey {
  uint64_t op;
  double t;
  int precision, K;
  bool operator<(const OpKey& o) const {
    if (op != o.op) return op < o.op;
    if (t != o.t) return t < o.t;
    if (precision != o.precision) return precision < o.precision;
    return K < o.K;
  }
};

struct CacheEntry {
  std::shared_ptr<OperatorSet> set;
  size_t bytes = 0;
  int users = 0;
  uint64_t last_tick = 0;
};

enum ReqStatus { kPending = 0, kActive = 1, kDone = 2, kFailed = 3 };

struct Request {
  uint64_t ticket = 0, op_id = 0;
  int is_dre = 0;
  dme_opts opts{};
  int precision = DME_FP64;  // precision in use
  bool fell_back = false;
  int64_t n = 0, m = 0, p = 0, r0 = 0;
  std::vector<double> B, C, R, S, L0, D0;
  double t_arrival = 0.0, t_admit = -1.0, t_done = -1.0;
  size_t state_bytes = 0;
  std::vector<OpKey> keys;
  std::unique_ptr<Solver> sv;
  hipStream_t stream = nullptr;
  std::atomic<int> status{kPending};
  int err = 0;
  std::string msg;
  dme_result* result = nullptr;
  bool failed_in_tick = false;
  int fail_code = 0;
  std::string fail_msg;
};

}  // namespace
}  // namespace dme

struct dme_server {
  dme_ctx* ctx = nullptr;
  size_t budget = 0;
  int max_slots = 1;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<dme::Request>> incoming;
  std::map<uint64_t, std::shared_ptr<dme::Request>> tickets;
  uint64_t next_ticket = 1;
  // scheduler-thread state
  std::deque<std::shared_ptr<dme::Request>> pending;
  std::vector<std::shared_ptr<dme::Request>> active;
  std::map<dme::OpKey, dme::CacheEntry> cache;
  size_t used = 0, peak = 0;
  uint64_t tick = 0;
  hipStream_t gstream = nullptr, bstream = nullptr;
  dme::DevBuf gX, gY, bflags;
  dme::Arena gws;
  std::unique_ptr<dme::Pool> pool;
  std::thread sched;
  std::atomic<bool> stop{false};
  // statistics (guarded by mu)
  std::vector<double> latencies, queue_times;
  int64_t completed = 0, failed = 0, fallbacks = 0, steps_done = 0, cold_builds = 0;
  double cold_build_s = 0.0, t_first_arrival = -1.0, t_last_done = -1.0;
  std::string fatal;
};

namespace dme {
namespace {

std::vector<double> host_copy(const double* p, size_t count) {
  return p && count ? std::vector<double>(p, p + count) : std::vector<double>();
}

// Step fractions t for which a request needs e^{tA^T}.
std::vector<double> operator_times(const Request& q) {
  std::vector<Stage> seq = step_sequence(q.is_dre != 0, !q.S.empty(), q.opts.split, q.opts.scheme);
  std::vector<double> ts;
  for (const Stage& st : seq)
    if (st.sub == Sub::T1 || st.sub == Sub::T12) {
      const double t = st.frac * q.opts.h;
      if (std::find(ts.begin(), ts.end(), t) == ts.end()) ts.push_back(t);
    }
  return ts;
}

int quad_nodes(const dme_opts& o) { return o.quad_nodes > 0 ? o.quad_nodes : 7; }

void set_keys(Request& q) {
  q.keys.clear();
  for (double t : operator_times(q)) q.keys.push_back({q.op_id, t, q.precision, quad_nodes(q.opts)});
}

size_t request_state_bytes(const Request& q) {
  dme_opts o = q.opts;
  o.precision = q.precision;
  return Solver::state_bytes(q.n, q.is_dre ? q.m : 0, q.p, !q.S.empty(), o);
}

std::shared_ptr<RegisteredOp> find_op(dme_ctx* ctx, uint64_t id) {
  std::lock_guard<std::mutex> g(ctx->ops_mu);
  auto it = ctx->ops.find(id);
  return it == ctx->ops.end() ? nullptr : it->second;
}

// Bytes still to be added to the ledger to admit q (missing operator sets
// plus the solve state).
// Served operator sets keep the quadrature node exponentials only for a
// nonsymmetric A; for a symmetric one each request forms its quadrature factor
// with the Leja action on the registered A^T.
bool keeps_nodes(dme_server* S, uint64_t op_id) {
  std::shared_ptr<RegisteredOp> op = find_op(S->ctx, op_id);
  return !(op && op->lop);
}

size_t admission_bytes(dme_server* S, const Request& q) {
  size_t b = q.state_bytes;
  for (const OpKey& k : q.keys)
    if (!S->cache.count(k)) b += operator_set_bytes(q.n, k.precision, k.K, keeps_nodes(S, k.op));
  return b;
}

// Drop cached operator sets no admitted solve uses, least recently used
// first, until `need` more bytes fit.  Returns whether they fit.
bool make_room(dme_server* S, size_t need) {
  while (S->used + need > S->budget) {
    auto victim = S->cache.end();
    for (auto it = S->cache.begin(); it != S->cache.end(); ++it)
      if (it->second.users == 0 && (victim == S->cache.end() || it->second.last_tick < victim->second.last_tick))
        victim = it;
    if (victim == S->cache.end()) return false;
    S->used -= victim->second.bytes;
    S->cache.erase(victim);
  }
  return true;
}

CacheEntry& get_operator(dme_server* S, const OpKey& k, int64_t n, bool cold) {
  auto it = S->cache.find(k);
  if (it != S->cache.end()) return it->second;
  std::shared_ptr<RegisteredOp> op = find_op(S->ctx, k.op);
  DME_REQUIRE(op != nullptr, DME_EINVAL, "unknown operator id");
  DME_REQUIRE(op->n == n, DME_EINVAL, "operator size differs from the problem size");
  const double t0 = now_s();
  CacheEntry e;
  const bool nodes = !op->lop;
  e.set = build_operator_set(S->bstream, n, op->AT.as<double>(), k.t, k.precision, k.K, nodes,
                             S->bflags.as<int>());
  int info = 0;
  DME_HIP(hipMemcpy(&info, S->bflags.as<int>(), sizeof(int), hipMemcpyDeviceToHost));
  DME_REQUIRE(info == 0, DME_ENUMERIC, "operator: singular Pade denominator");
  e.bytes = operator_set_bytes(n, k.precision, k.K, nodes);
  S->used += e.bytes;
  S->peak = std::max(S->peak, S->used);
  if (cold) {
    std::lock_guard<std::mutex> g(S->mu);
    S->cold_builds += 1;
    S->cold_build_s += now_s() - t0;
  }
  return S->cache.emplace(k, std::move(e)).first->second;
}

// The request's stream is synchronised first, then its solver goes (which
// synchronises and destroys the solver's second stream, events and rank slot),
// and the request's stream last, so nothing of the solve refers to a
// destroyed stream.
void release_request_state(dme_server* S, Request& q) {
  for (const OpKey& k : q.keys) {
    auto it = S->cache.find(k);
    if (it != S->cache.end()) it->second.users -= 1;
  }
  if (q.stream) (void)hipStreamSynchronize(q.stream);
  if (q.sv) {
    q.sv.reset();
    S->used -= q.state_bytes;
  }
  if (q.stream) {
    (void)hipStreamDestroy(q.stream);
    q.stream = nullptr;
  }
}

void finish(dme_server* S, Request& q, int code, const std::string& msg) {
  const double t = now_s();
  std::lock_guard<std::mutex> g(S->mu);
  q.t_done = t;
  if (code == DME_OK) {
    q.status = kDone;
    S->completed += 1;
    S->latencies.push_back(q.t_done - q.t_arrival);
    S->queue_times.push_back(q.t_admit - q.t_arrival);
    if (q.fell_back) S->fallbacks += 1;
  } else {
    q.status = kFailed;
    q.err = code;
    q.msg = msg;
    S->failed += 1;
  }
  S->t_last_done = t;
}

// Try to admit q; returns false when it has to wait for room.
bool admit(dme_server* S, const std::shared_ptr<Request>& qp) {
  Request& q = *qp;
  if ((int)S->active.size() >= S->max_slots) return false;
  const size_t need = admission_bytes(S, q);
  if (need > S->budget) {
    finish(S, q, DME_ENOMEM, "request needs more device memory than the server budget");
    return true;
  }
  // operators q will use must not be evicted to make room for q
  for (const OpKey& k : q.keys) {
    auto it = S->cache.find(k);
    if (it != S->cache.end()) it->second.users += 1;
  }
  const bool fits = make_room(S, need);
  for (const OpKey& k : q.keys) {
    auto it = S->cache.find(k);
    if (it != S->cache.end()) it->second.users -= 1;
  }
  if (!fits) return false;
  try {
    std::map<double, std::shared_ptr<OperatorSet>> sets;
    for (const OpKey& k : q.keys) {
      CacheEntry& e = get_operator(S, k, q.n, true);
      e.users += 1;
      e.last_tick = S->tick;
      sets[k.t] = e.set;
    }
    if (!q.stream) DME_HIP(hipStreamCreateWithFlags(&q.stream, hipStreamNonBlocking));
    q.sv = std::make_unique<Solver>();
    q.sv->s = q.stream;
    q.sv->device = S->ctx->device;
    {
      std::shared_ptr<RegisteredOp> op = find_op(S->ctx, q.op_id);
      DME_REQUIRE(op != nullptr, DME_EINVAL, "unknown operator id");
      q.sv->ATp = op->AT.as<double>();
      q.sv->lop = op->lop;
    }
    S->used += q.state_bytes;
    S->peak = std::max(S->peak, S->used);
    dme_problem prob{};
    prob.n = q.n;
    prob.m = q.is_dre ? q.m : 0;
    prob.p = q.p;
    prob.r0 = q.r0;
    prob.A = nullptr;
    prob.B = q.B.empty() ? nullptr : q.B.data();
    prob.C = q.C.data();
    prob.R = q.R.empty() ? nullptr : q.R.data();
    prob.S = q.S.empty() ? nullptr : q.S.data();
    prob.L0 = q.L0.empty() ? nullptr : q.L0.data();
    prob.D0 = q.D0.empty() ? nullptr : q.D0.data();
    dme_opts o = q.opts;
    o.precision = q.precision;
    OperatorProvider provider = [&sets](double t) { return sets.at(t); };
    q.sv->setup(prob, o, q.is_dre != 0, &provider);
    q.status = kActive;
    if (q.t_admit < 0) q.t_admit = now_s();
    S->active.push_back(qp);
  } catch (const Error& e) {
    release_request_state(S, q);
    finish(S, q, e.code, e.msg);
  }
  return true;
}

// Re-run a failed mixed-precision request in FP64 from the start.
bool fall_back(dme_server* S, const std::shared_ptr<Request>& qp) {
  Request& q = *qp;
  if (q.precision != DME_MIXED) return false;
  if (q.fail_code != DME_ENUMERIC && q.fail_code != DME_ERANK) return false;
  release_request_state(S, q);
  q.precision = DME_FP64;
  q.fell_back = true;
  q.failed_in_tick = false;
  q.status = kPending;
  set_keys(q);
  q.state_bytes = request_state_bytes(q);
  S->pending.push_front(qp);
  return true;
}

void run_guarded(Request& q, const std::function<void()>& f) {
  if (q.failed_in_tick) return;
  try {
    f();
  } catch (const Error& e) {
    q.failed_in_tick = true;
    q.fail_code = e.code;
    q.fail_msg = e.msg;
  } catch (const std::exception& e) {
    q.failed_in_tick = true;
    q.fail_code = DME_EINTERNAL;
    q.fail_msg = e.what();
  }
}

// One product e^{tA^T} [L_1 ... L_g] for the group, results into each W.
void grouped_product(dme_server* S, const OperatorSet& set, std::vector<Request*>& grp) {
  const int64_t n = set.n;
  int64_t cols = 0;
  for (Request* q : grp) cols += q->sv->r;
  if (cols == 0) return;
  hipEvent_t ev;
  DME_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  for (Request* q : grp) {
    DME_HIP(hipEventRecord(ev, q->stream));
    DME_HIP(hipStreamWaitEvent(S->gstream, ev, 0));
  }
  S->gX.ensure((size_t)n * cols * sizeof(double));
  S->gY.ensure((size_t)n * cols * sizeof(double));
  double* X = S->gX.as<double>();
  double* Y = S->gY.as<double>();
  int64_t off = 0;
  for (Request* q : grp) {
    if (q->sv->r > 0) copy_f64(S->gstream, q->sv->Lc(), n, X + off * n, n, n, q->sv->r);
    off += q->sv->r;
  }
  size_t wsb = (set.precision == DME_MIXED) ? gemm_mixed_workspace(n, cols) : gemm_f64_workspace(n, cols, n);
  S->gws.reserve(wsb + 4096);
  if (set.precision == DME_MIXED) {
    gemm_mixed(S->gstream, *set.mix, X, n, cols, Y, n, S->gws);
  } else {
    gemm_f64(S->gstream, 'N', 'N', n, cols, n, 1.0, set.E.as<double>(), n, X, n, 0.0, Y, n, &S->gws);
  }
  off = 0;
  for (Request* q : grp) {
    if (q->sv->r > 0) copy_f64(S->gstream, Y + off * n, n, q->sv->W.as<double>(), n, n, q->sv->r);
    off += q->sv->r;
  }
  DME_HIP(hipEventRecord(ev, S->gstream));
  for (Request* q : grp) DME_HIP(hipStreamWaitEvent(q->stream, ev, 0));
  DME_HIP(hipEventDestroy(ev));
}

void run_tick(dme_server* S) {
  S->tick += 1;
  size_t nstages = 0;
  for (auto& q : S->active) {
    q->failed_in_tick = false;
    nstages = std::max(nstages, q->sv->seq.size());
  }
  for (size_t st = 0; st < nstages; ++st) {
    // group the T12 stages by operator set
    std::map<const OperatorSet*, std::vector<Request*>> groups;
    std::vector<std::function<void()>> tasks;
    for (auto& qp : S->active) {
      Request* q = qp.get();
      if (q->failed_in_tick || st >= q->sv->seq.size()) continue;
      const Stage& sg = q->sv->seq[st];
      if (sg.sub == Sub::T12 && q->sv->r > 0) {
        groups[q->sv->ops.at(sg.frac * q->opts.h).get()].push_back(q);
      } else {
        tasks.push_back([q, st] { run_guarded(*q, [&] { q->sv->run_stage(st, false); }); });
      }
    }
    for (auto& g : groups) {
      std::vector<Request*>& grp = g.second;
      if (grp.size() == 1) {
        Request* q = grp[0];
        tasks.push_back([q, st] { run_guarded(*q, [&] { q->sv->run_stage(st, false); }); });
        continue;
      }
      grouped_product(S, *g.first, grp);
      for (Request* q : grp)
        tasks.push_back([q, st] { run_guarded(*q, [&] { q->sv->run_stage(st, true); }); });
    }
    S->pool->run(tasks);
  }
  // end of step: flags, step counters
  std::vector<std::function<void()>> tasks;
  for (auto& qp : S->active) {
    Request* q = qp.get();
    tasks.push_back([q] {
      run_guarded(*q, [&] {
        q->sv->end_step();
        q->sv->check_flags("served step");
      });
    });
  }
  S->pool->run(tasks);
  int64_t stepped = 0;
  for (auto& q : S->active)
    if (!q->failed_in_tick) stepped += 1;
  std::lock_guard<std::mutex> g(S->mu);
  S->steps_done += stepped;
}

void retire(dme_server* S) {
  std::vector<std::shared_ptr<Request>> keep;
  for (auto& qp : S->active) {
    Request& q = *qp;
    if (q.failed_in_tick) {
      if (!fall_back(S, qp)) {
        release_request_state(S, q);
        finish(S, q, q.fail_code, q.fail_msg);
      }
      continue;
    }
    if (q.sv->step < q.sv->N) {
      keep.push_back(qp);
      continue;
    }
    int code = DME_OK;
    std::string msg;
    dme_result* res = nullptr;
    try {
      res = result_from_solver(*q.sv);
    } catch (const Error& e) {
      code = e.code;
      msg = e.msg;
    }
    release_request_state(S, q);
    if (res) {
      res->fell_back = q.fell_back ? 1 : 0;
      res->precision = q.precision;
      res->latency_s = now_s() - q.t_arrival;
      res->queue_s = q.t_admit - q.t_arrival;
      q.result = res;
    }
    finish(S, q, code, msg);
  }
  S->active.swap(keep);
}

void scheduler(dme_server* S) {
  try {
    DME_HIP(hipSetDevice(S->ctx->device));
    while (true) {
      {
        std::unique_lock<std::mutex> g(S->mu);
        if (S->active.empty() && S->pending.empty() && S->incoming.empty()) {
          if (S->stop) break;
          S->cv.wait_for(g, std::chrono::milliseconds(2));
        }
        while (!S->incoming.empty()) {
          S->pending.push_back(S->incoming.front());
          S->incoming.pop_front();
        }
        if (S->stop && S->active.empty() && S->pending.empty()) break;
      }
      while (!S->pending.empty()) {
        std::shared_ptr<Request> q = S->pending.front();
        if (!admit(S, q)) break;
        S->pending.pop_front();
      }
      if (!S->active.empty()) {
        run_tick(S);
        retire(S);
      }
    }
  } catch (const Error& e) {
    std::lock_guard<std::mutex> g(S->mu);
    S->fatal = e.msg;
  }
}

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t lo = (size_t)pos;
  const size_t hi = std::min(lo + 1, v.size() - 1);
  const double f = pos - (double)lo;
  return v[lo] * (1.0 - f) + v[hi] * f;
}

}  // namespace
}  // namespace dme

// The C entry points of the server live in capi.cpp's error-handling scope;
// these helpers are called from there.
namespace dme {

dme_server* server_start(dme_ctx* ctx, size_t budget, int max_slots) {
  DME_REQUIRE(ctx != nullptr, DME_EINVAL, "null context");
  DME_REQUIRE(max_slots >= 1 && max_slots <= 256, DME_EINVAL, "max_slots must be in 1..256");
  DME_REQUIRE(budget > 0, DME_EINVAL, "zero memory budget");
  DME_HIP(hipSetDevice(ctx->device));
  auto S = std::make_unique<dme_server>();
  S->ctx = ctx;
  S->budget = budget;
  S->max_slots = max_slots;
  DME_HIP(hipStreamCreateWithFlags(&S->gstream, hipStreamNonBlocking));
  DME_HIP(hipStreamCreateWithFlags(&S->bstream, hipStreamNonBlocking));
  S->bflags.ensure(64);
  DME_HIP(hipMemset(S->bflags.p, 0, 64));
  const int workers = std::max(1, std::min(max_slots, 16));
  S->pool = std::make_unique<Pool>(workers, ctx->device);
  dme_server* raw = S.release();
  raw->sched = std::thread([raw] { scheduler(raw); });
  return raw;
}

void server_warm(dme_server* S, uint64_t op_id, double t, int precision, int K) {
  DME_REQUIRE(S != nullptr, DME_EINVAL, "null server");
  DME_REQUIRE(precision == DME_FP64 || precision == DME_MIXED, DME_EINVAL, "unknown precision");
  std::shared_ptr<RegisteredOp> op = find_op(S->ctx, op_id);
  DME_REQUIRE(op != nullptr, DME_EINVAL, "unknown operator id");
  // warm-up runs before requests arrive: the scheduler is idle, but take the
  // cache under the same thread discipline by pausing it
  std::unique_lock<std::mutex> g(S->mu);
  DME_REQUIRE(S->active.empty() && S->pending.empty() && S->incoming.empty(), DME_EINVAL,
              "warm the server before submitting requests");
  g.unlock();
  const OpKey k{op_id, t, precision, K > 0 ? K : 7};
  if (S->cache.count(k)) return;
  const size_t b = operator_set_bytes(op->n, precision, k.K, !op->lop);
  DME_REQUIRE(make_room(S, b), DME_ENOMEM, "operator does not fit the server budget");
  CacheEntry& e = get_operator(S, k, op->n, false);
  e.last_tick = S->tick;
}

uint64_t server_submit(dme_server* S, uint64_t op_id, const dme_problem& prob, const dme_opts& opts,
                       int is_dre) {
  DME_REQUIRE(S != nullptr, DME_EINVAL, "null server");
  std::shared_ptr<RegisteredOp> op = find_op(S->ctx, op_id);
  DME_REQUIRE(op != nullptr, DME_EINVAL, "unknown operator id");
  DME_REQUIRE(prob.n == op->n, DME_EINVAL, "problem size differs from the operator");
  DME_REQUIRE(prob.p > 0 && prob.C, DME_EINVAL, "need p > 0 and C");
  DME_REQUIRE(!is_dre || (prob.m > 0 && prob.B && prob.R), DME_EINVAL, "DRE needs m > 0, B and R");
  DME_REQUIRE(prob.r0 == 0 || (prob.L0 && prob.D0), DME_EINVAL, "r0 > 0 needs L0 and D0");
  DME_REQUIRE(opts.h > 0 && opts.T > 0 && opts.tol > 0, DME_EINVAL, "T, h and tol must be positive");
  DME_REQUIRE(opts.precision == DME_FP64 || opts.precision == DME_MIXED, DME_EINVAL,
              "unknown precision");
  auto q = std::make_shared<Request>();
  q->op_id = op_id;
  q->is_dre = is_dre ? 1 : 0;
  q->opts = opts;
  q->precision = opts.precision;
  q->n = prob.n;
  q->m = is_dre ? prob.m : 0;
  q->p = prob.p;
  q->r0 = prob.r0;
  const size_t n = (size_t)prob.n;
  if (is_dre) {
    q->B = host_copy(prob.B, n * prob.m);
    q->R = host_copy(prob.R, (size_t)prob.m * prob.m);
  }
  q->C = host_copy(prob.C, (size_t)prob.p * n);
  if (prob.S) q->S = host_copy(prob.S, n * n);
  if (prob.r0 > 0) {
    q->L0 = host_copy(prob.L0, n * prob.r0);
    q->D0 = host_copy(prob.D0, (size_t)prob.r0 * prob.r0);
  }
  // validate the step sequence and T/h here so errors come back from submit
  (void)step_sequence(is_dre != 0, prob.S != nullptr, opts.split, opts.scheme);
  const double Nf = std::round(opts.T / opts.h);
  DME_REQUIRE(Nf >= 1 && std::fabs(Nf * opts.h - opts.T) <= 1e-12 * opts.T, DME_EINVAL,
              "T/h is not an integer");
  set_keys(*q);
  q->state_bytes = request_state_bytes(*q);
  q->t_arrival = now_s();
  std::lock_guard<std::mutex> g(S->mu);
  DME_REQUIRE(!S->stop, DME_EINVAL, "server is stopping");
  q->ticket = S->next_ticket++;
  if (S->t_first_arrival < 0) S->t_first_arrival = q->t_arrival;
  S->tickets[q->ticket] = q;
  S->incoming.push_back(q);
  S->cv.notify_all();
  return q->ticket;
}

// DME_EAGAIN while the request is in flight; its error code if it failed.
int server_poll(dme_server* S, uint64_t ticket, dme_result** out, std::string* msg) {
  DME_REQUIRE(S != nullptr && out != nullptr, DME_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->tickets.find(ticket);
  DME_REQUIRE(it != S->tickets.end(), DME_EINVAL, "unknown ticket");
  Request& q = *it->second;
  if (q.status == kDone) {
    *out = q.result;
    q.result = nullptr;
    S->tickets.erase(it);
    return DME_OK;
  }
  if (q.status == kFailed) {
    const int code = q.err;
    *msg = q.msg;
    S->tickets.erase(it);
    return code;
  }
  if (!S->fatal.empty()) {
    *msg = "server stopped: " + S->fatal;
    return DME_EINTERNAL;
  }
  return DME_EAGAIN;
}

void server_stats(dme_server* S, dme_server_stats* st) {
  DME_REQUIRE(S != nullptr && st != nullptr, DME_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(S->mu);
  std::memset(st, 0, sizeof(*st));
  st->completed = S->completed;
  st->failed = S->failed;
  st->fallbacks = S->fallbacks;
  st->steps = S->steps_done;
  st->cold_builds = S->cold_builds;
  st->cold_build_s = S->cold_build_s;
  st->p50_s = percentile(S->latencies, 0.50);
  st->p99_s = percentile(S->latencies, 0.99);
  st->queue_p50_s = percentile(S->queue_times, 0.50);
  st->queue_p99_s = percentile(S->queue_times, 0.99);
  const double span = (S->t_last_done > S->t_first_arrival && S->t_first_arrival >= 0)
                          ? S->t_last_done - S->t_first_arrival
                          : 0.0;
  st->req_per_s = span > 0 ? (double)S->completed / span : 0.0;
  st->steps_per_s = span > 0 ? (double)S->steps_done / span : 0.0;
  st->peak_bytes = (int64_t)S->peak;
  int64_t inflight = 0;
  for (auto& kv : S->tickets)
    if (kv.second->status == kPending || kv.second->status == kActive) inflight += 1;
  st->in_flight = inflight;
}

void server_stop(dme_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
  }
  S->cv.notify_all();
  if (S->sched.joinable()) S->sched.join();
  (void)hipSetDevice(S->ctx->device);
  (void)hipDeviceSynchronize();
  for (auto& kv : S->tickets) {
    Request& q = *kv.second;
    if (q.result) dme_result_free(q.result);
    q.result = nullptr;
    q.sv.reset();
    if (q.stream) (void)hipStreamDestroy(q.stream);
    q.stream = nullptr;
  }
  S->pool.reset();
  S->cache.clear();
  if (S->gstream) (void)hipStreamDestroy(S->gstream);
  if (S->bstream) (void)hipStreamDestroy(S->bstream);
  delete S;
}

}  // namespace dme
