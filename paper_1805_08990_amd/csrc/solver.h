// Solver state for one differential Lyapunov / Riccati solve: operators and
// factors resident in HBM, stepped by the splitting schemes of Sec. 2 / Sec. 3.
#pragma once

#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "common.h"
#include "leja.h"

namespace dme {

// Host helpers shared by the driver (defined in expm.hip / solver.hip).
void expm_params(double nrm1, int* m, int* s);
size_t expm_workspace(int64_t n);
void expm_f64(hipStream_t s, int64_t n, const double* X, double t, double* E, Arena& ws, int* m_out,
              int* s_out, int* info_dev);
// K-point Gauss-Legendre nodes and weights on [0, t] (ascending nodes).
void gauss_legendre(int K, double t, std::vector<double>& nodes, std::vector<double>& weights);

enum class Sub { T1, T2, T12, T3, T4 };

struct Stage {
  Sub sub;
  double frac;  // fraction of h
};

// Subflows of one step in application order (operators act right to left).
std::vector<Stage> step_sequence(bool is_dre, bool has_S, int split, int scheme);

struct MixedOp;  // FP32 copy of an operator for the split-BF16 product (gemm_mixed.hip)

// Operators derived from A for one step fraction t: e^{tA^T} in FP64 and, in
// the mixed mode, its FP32 copy; optionally the K Gauss-Legendre node
// exponentials e^{s_k A^T} on [0, t], kept when many right-hand sides C are
// served from one operator (a single solve forms them one at a time while it
// builds its quadrature factor and keeps none).
//
// With the Leja action (DME_ACTION_LEJA) the set holds no E: e^{tA^T} X is
// applied by Newton interpolation at Leja points with products by A^T (`lop`,
// dense or CSR) under the interpolation parameters `plan`.
struct OperatorSet {
  int64_t n = 0;
  double t = 0.0;
  int precision = DME_FP64;
  int K = 0;
  DevBuf E;                      // n x n, e^{tA^T}
  std::shared_ptr<MixedOp> mix;  // FP32 copy of E (mixed mode)
  std::vector<DevBuf> nodes;     // e^{s_k A^T}, k = 0 .. K-1 (when kept)
  std::shared_ptr<LejaOp> lop;   // Leja action: the operator A^T
  std::shared_ptr<LejaPlan> plan;
  double build_ms = 0.0;
};

// Device bytes an operator set holds.
size_t operator_set_bytes(int64_t n, int precision, int K, bool keep_nodes);
// Form the operator set of AT = A^T (device, n x n) on stream s (synchronous).
// info_dev: device int receiving a nonzero LU pivot failure flag.
std::shared_ptr<OperatorSet> build_operator_set(hipStream_t s, int64_t n, const double* AT, double t,
                                                int precision, int K, bool keep_nodes, int* info_dev);

// Supplies the operator set for a step fraction t (a cache shared by
// several solves); null means the solve builds its own.
using OperatorProvider = std::function<std::shared_ptr<OperatorSet>(double t)>;

struct QuadFactor {
  DevBuf L;  // n x r
  DevBuf D;  // r x r
  int64_t r = 0;
};

// Build the FP32 row-major copy of E (n x n, FP64 column-major).
void mixed_op_build(hipStream_t s, int64_t n, const double* E, MixedOp& op);
std::shared_ptr<MixedOp> mixed_op_new();
// Y (n x r, ld ldy) = E X on BF16 MFMA with three-piece splits, FP32 chunk
// accumulation and an FP64 sum over chunks; or only the rows [row0, row0 +
// rows) of Y, with the inner dimension cut into ns_force chunks (0: the
// default split, gemm_mixed_nsplit).  One workgroup per kRowBlock rows and
// chunk.
void gemm_mixed(hipStream_t s, const MixedOp& op, const double* X, int64_t ldx, int64_t r, double* Y,
                int64_t ldy, Arena& ws, int64_t row0 = 0, int64_t rows = -1, int ns_force = 0);
int gemm_mixed_nsplit(int64_t n);
size_t gemm_mixed_workspace(int64_t n, int64_t r);

struct PhaseAcc {
  int64_t count = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};

struct PendingTiming {
  int phase;
  hipEvent_t a, b;
  double flops, bytes;
  int64_t launches;
};

struct Solver {
  hipStream_t s = nullptr;
  int device = 0;
  int64_t n = 0, m = 0, p = 0;
  bool is_dre = false, has_S = false;
  dme_opts opts{};
  int64_t N = 0, step = 0;
  std::vector<Stage> seq;
  int64_t max_rank = 0, kmax = 0;

  DevBuf AT;   // n x n, A^T (only when the solve builds its own operators)
  // Dense A^T on the device (AT, or a registered operator's copy); null when A
  // is given in CSR form only.
  const double* ATp = nullptr;
  // A^T for the Leja action (the quadrature nodes and, with DME_ACTION_LEJA,
  // the steps): CSR when A came in that form, else the dense A^T when it is
  // symmetric (the interpolation needs a real spectrum); null otherwise.
  std::shared_ptr<LejaOp> lop;
  DevBuf B;    // n x m
  DevBuf CT;   // n x p, C^T
  DevBuf R;    // m x m
  DevBuf S;    // n x n
  std::map<double, std::shared_ptr<OperatorSet>> ops;  // t -> e^{tA^T} (+ FP32 copy, nodes)
  std::map<double, QuadFactor> Q;                       // t -> (L_I, D_I)

  DevBuf L[2], D[2];
  int cur = 0;
  int64_t r = 0;
  bool d_diag = true;  // D is diagonal (a compression's output; T3 fills it)
  // D = diag(lamT3) - t3 Z Z^T with Z in ZT3 (T3 applied to a diagonal D)
  bool d_lowrank = false;
  double t3 = 0.0;
  DevBuf lamT3, ZT3;
  DevBuf W, Dhat, WB, SL;
  // the factor of a Dhat in that form, formed on the second stream beside
  // the step product (kmax x kmax doubles, then its int64 status)
  DevBuf Fpre;
  bool f_ready = false;

  // Step products ahead of need (dense operators, FP64 up to 256 columns,
  // or the Leja action on a CSR operator; every T12 of the step with the same
  // t, driven by advance()).  A compression through the Gram matrix
  // gives L = W T with W = [Y, L_I], so the next T12 needs
  // e^{tA^T} L = [e^{tA^T} Y, e^{tA^T} L_I] T: the product e^{tA^T} Y can
  // start before the compression ends.  A dense product's first rows run on
  // s3 beside the compression's one-workgroup tridiagonal reduction, the rest
  // when the next T12 needs them; the Leja action (a chain of short launches
  // that leave room for the compression's kernels) runs whole on s3 beside
  // the compression.  e^{tA^T} L_I is formed once per t.
  //   EW (n x (max_rank + K p)): e^{tA^T} Y in the columns [max_rank - ey_cols,
  //   max_rank), e^{tA^T} L_I from column max_rank on (so the two are one
  //   n x k operand); Tk: T of the last such compression (tk_k x rank, ld tk_k).
  DevBuf EW, Tk;
  std::map<double, DevBuf> ELI;  // t -> e^{tA^T} L_I (n x its rank), FP64
  double eli_t = -1.0;           // the t whose e^{tA^T} L_I is in EW
  bool ahead = false;            // set by advance() (a server groups its products instead)
  bool ahead_same_t = false;     // every T12 stage of the step has the same t
  bool ey_ok = false;            // EW holds (rows [0, ey_rows) of) e^{ey_t A^T} W[:, 0:ey_cols]
  double ey_t = 0.0;
  int64_t ey_cols = 0, ey_rows = 0;
  bool tk_ok = false;
  int64_t tk_k = 0;
  int cus = 0;                   // compute units of the device
  int xccs = 1;                  // its compute dies (XCDs)
  hipStream_t s3 = nullptr;
  hipEvent_t ey_done = nullptr;  // the rows formed on s3
  Arena ws3;
  DevBuf flags;  // int flags[4]; int64 rank at offset 16
  Arena ws;
  AuxStream aux;  // second stream, event ring and rank slot of this solve

  double expm_ms = 0.0, quad_ms = 0.0;
  int64_t rank_quad = 0;
  int64_t nprod = 0;  // products e^{tA^T} L applied so far
  double quad_delta = 0.0;  // relative error of split-BF16 quadrature node products (DME_MIXED)

  int profiling = 0;  // 0 off, 1 every phase, 2 the step product kernel alone
  hipEvent_t mark_phase() { return profiling == 1 ? mark_begin() : nullptr; }
  PhaseAcc phase[5];
  std::vector<PendingTiming> pending;
  std::vector<hipEvent_t> event_pool;
  // events on st (the solve's stream when null)
  hipEvent_t mark_begin(hipStream_t st = nullptr);
  // launches: how many launches of the phase's kernel the interval holds
  void mark_end(int ph, hipEvent_t a, double flops, double bytes, int64_t launches = 1,
                hipStream_t st = nullptr);
  void flush_timings();
  ~Solver();

  double* Lc() { return L[cur].as<double>(); }
  double* Dc() { return D[cur].as<double>(); }
  double* Ln() { return L[cur ^ 1].as<double>(); }
  double* Dn() { return D[cur ^ 1].as<double>(); }
  int* flag_dev() { return flags.as<int>(); }
  int64_t* rank_dev() { return reinterpret_cast<int64_t*>(flags.as<char>() + 16); }

  // Upload the problem and build (or take from `provider`) its operators.
  // With a provider, prob.A is not read.
  void setup(const dme_problem& prob, const dme_opts& o, bool dre,
             const OperatorProvider* provider = nullptr);
  void advance(int64_t nsteps);
  void check_flags(const char* where);
  // Device bytes setup() allocates for this solve (operators excluded).
  static size_t state_bytes(int64_t n, int64_t m, int64_t p, bool has_S, const dme_opts& o);
  static size_t workspace_bytes(int64_t n, int64_t m, int64_t max_rank, int64_t kmax, int precision);
  static void sizes_for(int64_t n, int64_t p, const dme_opts& o, int64_t* max_rank, int64_t* kmax);

  // Finer-grained stepping (used when several solves share one product):
  // run stage `i` of the step sequence; for a T12 stage, `ext_product` says
  // that W[:, 0:r] already holds e^{tA^T} L.
  void run_stage(size_t i, bool ext_product = false);
  // Called after the last stage of a step.
  void end_step() { ++step; }
  // Estimated relative Frobenius distance between the current P = L D L^T and
  // the same scheme run in FP64 throughout: 2 N_p max(delta, sqrt(n) u), with
  // N_p the products e^{tA^T} L applied so far, u = 2^-53 and, in the mixed
  // mode, delta the relative error of one split-BF16 product measured on the
  // current factor against an FP64 product of the same operator (delta = 0 in
  // FP64).  Each product perturbs P = Y D Y^T by at most about 2 delta
  // relative, and the later flows do not amplify it (the heat semigroup and
  // the compressions are contractions), so the sum over products bounds the
  // drift to first order.  Enqueues two products and synchronises.
  double err_estimate();

 private:
  void apply_T1(double t);
  void apply_T2(double t);
  void apply_T12(double t, bool ext_product);
  void apply_T3(double t);
  void apply_T4(double t);
  // W (n x k), Dhat (k x k) -> new (L, D); Dhat holds ncopies copies of D
  // (from row 0), the rest of it is diagonal
  // ahead_t > 0: W[:, 0:r] is Y of a T12 with that t, and the next T12's
  // product goes ahead beside this compression
  void compress_into(int64_t k, int ncopies = 1, double ahead_t = 0.0);
  // rows [row0, row0 + rows) of e^{tA^T} X (X n x cols) into EW's product
  // columns, ns chunks of the inner dimension, on st with arena a
  void product_rows(double t, const double* X, int64_t cols, int64_t row0, int64_t rows, int ns,
                    hipStream_t st, Arena& a);
  void drop_ahead() { ey_ok = false; tk_ok = false; }
  // the solve's stream waits for rows still forming on s3 (they read
  // W[:, 0:ey_cols]) before anything writes W again
  bool beside_live = false;
  void settle_beside() {
    if (beside_live) DME_HIP(hipStreamWaitEvent(s, ey_done, 0));
    beside_live = false;
  }
  // split of the inner dimension for `rows` rows of a step product in one
  // wave of workgroups
  int fill_split(int64_t rows) const;
  // rows of the next product to form beside a compression of width k (a
  // multiple of kRowBlock, or n; 0: none) and their split
  void plan_beside(int64_t k, int64_t* rows, int* ns) const;
  void apply_E(double t, const double* X, int64_t r, double* Y, int64_t ldy);
  void build_quadrature(double t);
  void apply_mass_matrix(const double* M);
};

}  // namespace dme
