// Library-side definitions of the opaque C ABI handles shared by the entry
// points (capi.cpp) and the request server (server.cpp).
#pragma once

#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "solver.h"

namespace dme {

// An operator A registered once and kept on the device as A^T, so that served
// requests name it instead of re-sending n^2 values.
struct RegisteredOp {
  uint64_t id = 0;
  int64_t n = 0;
  DevBuf AT;
  // the Leja operator on AT when A is symmetric (served quadrature factors
  // then need no node exponentials); null otherwise
  std::shared_ptr<LejaOp> lop;
};

}  // namespace dme

struct dme_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  dme::Arena ws;
  dme::DevBuf flags;
  dme::AuxStream aux;  // second stream, event ring and rank slot of the step-level calls
  std::mutex ops_mu;
  std::map<uint64_t, std::shared_ptr<dme::RegisteredOp>> ops;
  uint64_t next_op = 1;
};

struct dme_result {
  int64_t n = 0, r = 0, steps = 0;
  double err_est = 0.0;  // Solver::err_estimate() when the result was taken
  std::vector<double> L, D;
  // served requests: precision used (dme_precision), 1 if it fell back to FP64,
  // arrival-to-completion and arrival-to-admission times (seconds)
  int precision = 0, fell_back = 0;
  double latency_s = 0.0, queue_s = 0.0;
};

namespace dme {
// Copy the solver's current (L, D) into a new host result.
dme_result* result_from_solver(Solver& sv);

extern thread_local std::string g_last_error;

// Runs f, turning a dme::Error (or another exception) into its return code and
// the thread's last error message (the C entry points' error handling).
int guarded_call(const std::function<void()>& f);

// The static device scratch of the allocation-free entry points (noalloc.hip):
// its address on `device` is looked up once, with that device current.
void noalloc_scratch_init(int device);

// Request server (server.cpp); errors are thrown as dme::Error.
dme_server* server_start(dme_ctx* ctx, size_t budget, int max_slots);
void server_warm(dme_server* S, uint64_t op_id, double t, int precision, int K);
uint64_t server_submit(dme_server* S, uint64_t op_id, const dme_problem& prob, const dme_opts& opts,
                       int is_dre);
int server_poll(dme_server* S, uint64_t ticket, dme_result** out, std::string* msg);
void server_stats(dme_server* S, dme_server_stats* st);
void server_stop(dme_server* S);
}  // namespace dme
