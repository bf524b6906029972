/*
 * dme.h -- C ABI of the MI355X (gfx950) low-rank splitting solver for
 * differential Lyapunov and Riccati equations.
 *
 * Problem (Mena, Pfurtscheller, Stillfjord 2018, Sec. 1 and Sec. 2):
 *
 *     dP/dt = A^T P + P A + Q + G(P),   P(0) = P0 = L0 D0 L0^T,   Q = C^T C,
 *     G = 0                      differential Lyapunov equation (Sec. 2.1)
 *     G = -P B R^-1 B^T P        differential Riccati equation (Sec. 2.2)
 *     plus S P S^T when S is given  (generalized equations, Sec. 2.3 / 2.4)
 *
 * The solution is carried as P = L D L^T (Sec. 2, low-rank paragraph) and
 * advanced by Lie or Strang compositions of the subflows T1, T2, T12, T3, T4
 * (Sec. 2 and the scheme list of Sec. 3), with column compression after every
 * concatenation (Alg. 1, 2, 4).  The dense operator e^{tA^T} is formed once by
 * scaling and squaring with a diagonal Pade approximant (Higham 2005, Alg. 2.3)
 * and applied to L by FP64 (or split-BF16) MFMA GEMMs.
 *
 * Conventions for every entry point:
 *   - All matrices are FP64 and column-major; leading dimension = row count
 *     unless an ld argument says otherwise.
 *   - "host" pointers are read during the call only and stay owned by the
 *     caller; "device" pointers are HBM addresses on the context's device,
 *     also caller-owned; results (dme_result) are owned by the library until
 *     dme_result_free.
 *   - Return value: DME_OK (0) or a negative error code; dme_last_error()
 *     returns a message for the calling thread's most recent failure.
 *   - A context is used by one host thread at a time.  Step-level calls are
 *     enqueued on the context's stream; solve-level calls synchronise it.
 */
#ifndef DME_H
#define DME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
#define DME_OK 0
#define DME_EINVAL (-1)    /* bad dimensions, T/h not an integer, tol <= 0, R not SPD */
#define DME_ENOMEM (-2)    /* device allocation failed or memory budget exceeded */
#define DME_ERANK (-3)     /* compressed rank exceeds max_rank */
#define DME_ENUMERIC (-4)  /* NaN/Inf, singular Pade denominator, non-SPD Riccati block */
#define DME_EAGAIN (-5)    /* result not ready yet (serving) */
#define DME_EHIP (-6)      /* HIP runtime error */
#define DME_EINTERNAL (-7) /* internal invariant violated */

typedef struct dme_ctx dme_ctx;
typedef struct dme_result dme_result;
typedef struct dme_solver dme_solver;

/* Problem data (Sec. 1 equation; Sec. 2.2 Riccati term; Sec. 2.3 S term;
 * Sec. 5.1 Ex. 4 mass matrix).  All pointers are host pointers,
 * n x n / n x m / p x n / m x m / n x r0 / r0 x r0.  The fields after D0 are
 * optional: zero-initialise the struct and set what is used.
 *
 * Mass-matrix form (Sec. 5.1, Ex. 4): with M given the equation is
 *     M^T dP/dt M = A^T P M + M^T P A + Q + (Riccati / S terms in M^T P M),
 * solved as the standard form with A M^-1 in place of A and C M^-1 in place
 * of C (the library factors M^T once by LU with partial pivoting on the
 * device); B, R, S keep their meaning.  Needs the dense A.
 *
 * Sparse A (for DME_ACTION_LEJA, the paper's operator-action method):
 * A_rowptr (n + 1 entries, A_rowptr[0] = 0), A_colind and A_val (nnz
 * entries each, column indices in [0, n)) hold A in CSR form; A may then be
 * NULL.  The library transposes it on the host once and keeps A^T in CSR form
 * on the device. */
typedef struct {
  int64_t n, m, p, r0;
  const double *A;  /* n x n, required unless A is given in CSR form        */
  const double *B;  /* n x m, NULL iff m == 0                             */
  const double *C;  /* p x n, Q = C^T C, required (p >= 1)                */
  const double *R;  /* m x m SPD, NULL iff m == 0                         */
  const double *S;  /* n x n or NULL (adds S P S^T)                       */
  const double *L0; /* n x r0 (NULL iff r0 == 0, i.e. P0 = 0)             */
  const double *D0; /* r0 x r0 symmetric                                  */
  const double *M;  /* n x n mass matrix or NULL (M = I)                   */
  const int64_t *A_rowptr; /* CSR of A: n + 1 row pointers, or NULL         */
  const int64_t *A_colind; /* nnz column indices                            */
  const double *A_val;     /* nnz values (NULL: no CSR form)                */
} dme_problem;

/* Composition order (operators act right to left, Sec. 2):
 *   DME_LIE:    one step = T_last(h) ... T_first(h)
 *   DME_STRANG: palindromic, outer subflows over h/2, the middle over h.   */
typedef enum { DME_LIE = 0, DME_STRANG = 1 } dme_scheme;

/* Which subflows:
 *   DME_SPLIT_F12:    linear part A^T P + P A + Q solved with the quadrature
 *                     formula (Alg. 2); DRE adds T3 (Sec. 3, first scheme);
 *                     with S the generalized DRE scheme T12 T3 T4 T3 T12.
 *   DME_SPLIT_F1F2:   T1 / T2 split of Alg. 1; with B (or S) the three-term
 *                     scheme T1 T2 T3 T2 T1 (Sec. 3, second scheme).
 *   DME_SPLIT_F1F3F2: reversed three-term scheme T1 T3 T2 T3 T1 (Sec. 3). */
typedef enum { DME_SPLIT_F12 = 0, DME_SPLIT_F1F2 = 1, DME_SPLIT_F1F3F2 = 2 } dme_split;

/* DME_FP64: every product in FP64 MFMA.
 * DME_MIXED: the step products e^{tA^T} L (the T1 / T12 products of every
 *            step, the bulk of a step's flops and HBM traffic) and, where the
 *            quadrature nodes are dense operators (a nonsymmetric A), the node
 *            products e^{s_k A^T} C^T of the quadrature factor in split BF16
 *            MFMA with FP32 accumulation flushed to FP64.  The operator setup
 *            (Pade, LU, squaring), the Leja node actions of a symmetric A, the
 *            compression, T3 and T4 stay FP64.  Each result states its
 *            estimated distance to the FP64 computation (dme_result_info). */
typedef enum { DME_FP64 = 0, DME_MIXED = 1 } dme_precision;

/* How e^{tA^T} L is applied in the T1 / T12 products:
 * DME_ACTION_DENSE: the dense operator e^{tA^T}, formed once per step fraction
 *            by Pade scaling and squaring (Higham 2005), applied by GEMM.
 * DME_ACTION_LEJA: the paper's expleja (Sec. 3, Sec. 4): Newton interpolation
 *            of e^{t A^T} at Leja points of the Gershgorin interval, applied
 *            by products with A^T (CSR when A is given in CSR form, else the
 *            dense A); no n x n exponential is formed.  FP64 only; needs a
 *            symmetric A (real spectrum) and no mass matrix.
 * Either way the quadrature nodes of T12 use the Leja action when A is
 * symmetric (or in CSR form) and node exponentials otherwise.              */
typedef enum { DME_ACTION_DENSE = 0, DME_ACTION_LEJA = 1 } dme_action;

typedef struct {
  double T;        /* final time                                            */
  double h;        /* step; N = round(T/h) with |N h - T| <= 1e-12 T          */
  double tol;      /* compression: keep |lambda_i| > tol * max |lambda|      */
  int scheme;      /* dme_scheme                                            */
  int split;       /* dme_split                                             */
  int precision;   /* dme_precision                                         */
  int quad_nodes;  /* Gauss-Legendre nodes K for T12 (0 -> 7)               */
  int64_t max_rank;/* rank cap (0 -> min(n, 512))                           */
  int action;      /* dme_action (0: dense exponential)                     */
} dme_opts;

/* ------------------------------------------------------------- context */
/* Create a context on HIP device `device`.  `stream` is the hipStream_t the
 * context enqueues on (NULL: the null stream); it stays owned by the caller
 * and must outlive the context. */
int dme_create(dme_ctx **ctx, int device, void *stream);
void dme_destroy(dme_ctx *ctx);
const char *dme_strerror(int code);
const char *dme_last_error(void);

/* --------------------------------------------------------- whole solves */
/* G = 0 (Sec. 2.1; Alg. 1 and Alg. 2). B, R are ignored. */
int dle_solve(dme_ctx *ctx, const dme_problem *prob, const dme_opts *opts, dme_result **out);
/* G = -P B R^-1 B^T P (Sec. 2.2; Alg. 3 inside the Sec. 3 schemes). */
int dre_solve(dme_ctx *ctx, const dme_problem *prob, const dme_opts *opts, dme_result **out);

/* Stepwise form of the same solves: create = upload + operator setup
 * (e^{tA^T}, quadrature factor), step = advance `nsteps` time steps with all
 * data resident in HBM, result = copy of the current (L, D).
 * is_dre: 0 -> DLE, 1 -> DRE.  A solver owns its device memory.
 * Stepping with the dense operators, or with the Leja action on a CSR
 * operator, forms each step product ahead of need:
 * after a compression L = W T with W = [Y, L_I], and e^{tA^T} L is taken as
 * [e^{tA^T} Y, e^{tA^T} L_I] T, most of it beside the compression.  Stepping in
 * pieces repeats one call's arithmetic exactly; a server's grouped products
 * (and a step after an error estimate, which drops what was formed ahead)
 * agree with it to FP64 roundoff, or to the split-BF16 product error. */
int dme_solver_create(dme_ctx *ctx, const dme_problem *prob, const dme_opts *opts, int is_dre,
                      dme_solver **out);
int dme_solver_step(dme_solver *sv, int64_t nsteps);
/* steps taken, total steps N, current rank r. */
int dme_solver_state(const dme_solver *sv, int64_t *step, int64_t *nsteps_total, int64_t *rank);
/* Setup timing (ms): e^{tA^T} formation, quadrature factor; rank of the
 * quadrature factor. */
int dme_solver_setup_info(const dme_solver *sv, double *expm_ms, double *quad_ms, int64_t *rank_quad);
int dme_solver_result(dme_solver *sv, dme_result **out);

/* LQR feedback gain at the solver's current step (Sec. 1, the LQR setting):
 * K = R^-1 B^T P with P = L D L^T, written to K (host, m x n, column-major,
 * ld ldk >= m).  Computed on the device (L^T B, D W, an m x m Cholesky solve
 * with R, X L^T) and copied out; synchronises the solver's stream.  Errors:
 * DME_EINVAL for a solver without B and R (DLE), ldk < m, m > 64 or null
 * pointers; flag bit 4 (R not SPD) is reported like the solver's flags. */
int dme_solver_gain(dme_solver *sv, double *K, int64_t ldk);

/* Phase timing with HIP events recorded on the solver's stream around each
 * launch group of a phase (enable = 1 turns it on and clears the totals;
 * enable = 2 times DME_PHASE_STEP_KERNEL alone, so that the other phases add
 * no events to the stream; 0 turns it off; other values: DME_EINVAL).
 * Phases: DME_PHASE_STEP_GEMM (e^{tA^T} L products), DME_PHASE_COMPRESS
 * (QR + eigen compression), DME_PHASE_RICCATI (T3), DME_PHASE_S (S L, S^2 L).
 * For each: number of launches, summed device milliseconds, and the
 * algorithmic flops and HBM bytes of the method's operation (not counting
 * split-precision emulation). */
#define DME_PHASE_STEP_GEMM 0
#define DME_PHASE_COMPRESS 1
#define DME_PHASE_RICCATI 2
#define DME_PHASE_S 3
/* the main kernel of each step product alone (skinny FP64 or split-BF16),
 * with the algorithmic work of that launch                                 */
#define DME_PHASE_STEP_KERNEL 4
int dme_solver_profile(dme_solver *sv, int enable);
int dme_solver_profile_get(dme_solver *sv, int phase, int64_t *count, double *ms, double *flops,
                           double *bytes);
void dme_solver_free(dme_solver *sv);

/* ------------------------------------------------------------- results */
/* n, rank r and steps taken of a result, and err_est: the estimated relative
 * Frobenius distance ||P - P64||_F / ||P64||_F between this P = L D L^T and the
 * same scheme computed in FP64 throughout (the precision of the paper's
 * method).  err_est = 2 N_p max(delta, sqrt(n) u) with N_p the products
 * e^{tA^T} L the solve applied, u = 2^-53, and delta = 0 for DME_FP64 results;
 * for DME_MIXED results delta is the relative Frobenius error of one
 * split-BF16 product, measured when the result is taken by forming e^{tA^T} L
 * of the final factor both ways (two products on the device).  It assumes
 * that the per-product errors add without amplification (the flows are
 * contractive): a first-order upper estimate, not a rigorous bound.  Any
 * output pointer may be NULL.                                               */
int dme_result_info(const dme_result *res, int64_t *n, int64_t *r, int64_t *steps, double *err_est);
/* L: n x r host buffer, D: r x r host buffer, both caller-allocated. */
int dme_result_copy(const dme_result *res, double *L, double *D);
void dme_result_free(dme_result *res);

/* ------------------------------------------ step-level calls (device)  */
/* Each is one row of the method's hot path, on device pointers, enqueued on
 * the context's stream.  Used by the solvers above and by parity tests.     */

/* E = e^{t X} for an n x n X (Higham 2005 Alg. 2.3: Pade degree m and
 * scaling s from ||tX||_1, [m/m] Pade numerator/denominator, LU solve, s
 * squarings).  Writes m and s to *m_out, *s_out (host) when non-NULL.
 * X and E device, n x n, must not alias.  Synchronises the stream.          */
int dme_expm(dme_ctx *ctx, int64_t n, const double *X, double t, double *E, int *m_out, int *s_out);

/* C = alpha op(A) op(B) + beta C with FP64 MFMA; trans = 'N' or 'T'. */
int dme_gemm_f64(dme_ctx *ctx, char transa, char transb, int64_t M, int64_t N, int64_t K,
                 double alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                 double beta, double *C, int64_t ldc);

/* Y = E X in the mixed-precision mode (the split-precision form of the step
 * product e^{tA^T} L of Sec. 2.1, eq. for T1): E is rounded to FP32 and X to
 * FP32, each is split into three BF16 pieces, the six leading piece products
 * run on BF16 MFMA with FP32 accumulation per K chunk, and the chunks are summed
 * in FP64.  Relative error per entry is about 2^-24 times the sum of |E||X|.
 * E: n x n device (FP64, ld n), X: n x r device (ld ldx), Y: n x r device
 * (ld ldy).  The FP32 copy of E is built on every call (the solver keeps its
 * copy resident instead).  E and Y must not alias.                         */
int dme_gemm_mixed(dme_ctx *ctx, int64_t n, int64_t r, const double *E, const double *X,
                   int64_t ldx, double *Y, int64_t ldy);

/* Y = e^{t A^T} X by the Leja-interpolation action (the paper's expleja,
 * Sec. 3 and Sec. 4): Gershgorin interval of A, Newton interpolation of
 * e^{t z} at Leja points in S substeps of degree m (chosen so that each
 * substep errs by at most 1e-14 relative for a symmetric A), products with A^T
 * only.  A is either dense on the device (n x n, ld n; A_rowptr NULL) or in
 * CSR form on the host (A_rowptr n + 1, A_colind / A_val nnz; A_dev NULL).
 * A must be symmetric (DME_EINVAL otherwise).  X, Y: n x ncols device (ld n),
 * may alias.  *S_out, *m_out (host, optional) get the substeps and degree.
 * Synchronises the stream.                                                  */
int dme_expmv_leja(dme_ctx *ctx, int64_t n, const double *A_dev, const int64_t *A_rowptr,
                   const int64_t *A_colind, const double *A_val, double t, int64_t ncols,
                   const double *X, double *Y, int *S_out, int *m_out);

/* Column compression (Sec. 3 after Alg. 2): Householder QR W = Q R,
 * M = R Dhat R^T, M = V Lam V^T, keep |lam_i| > tol max|lam| (sorted by |lam|
 * descending), L = Q V_I, D = diag(lam_I).
 * W: n x k device (destroyed), Dhat: k x k device, L: n x max_rank device
 * (ld n), D: max_rank x max_rank device (ld max_rank).  *r_out (host) gets the
 * kept rank; DME_ERANK if it exceeds max_rank.  Synchronises the stream.    */
int dme_compress(dme_ctx *ctx, int64_t n, int64_t k, double *W, const double *Dhat, double tol,
                 int64_t max_rank, double *L, double *D, int64_t *r_out);

/* Riccati subflow T3(t) of Sec. 2.2 on the small factor: with W_B = L^T B,
 * D <- (I + t D W_B R^-1 W_B^T)^-1 D, evaluated as the symmetric m x m
 * Woodbury form D - t D W_B (R + t W_B^T D W_B)^-1 W_B^T D.
 * L: n x r, B: n x m, R: m x m, D: r x r (in place), all device.           */
int dme_riccati(dme_ctx *ctx, int64_t n, int64_t r, int64_t m, const double *L, const double *B,
                const double *R, double t, double *D);

/* Allocation-free form of dme_riccati for callers that cannot allocate device
 * memory during a call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same computation, arguments and
 * result, with its temporaries (W_B = L^T B, the split-K partial sums of that
 * product, the m-column staging of the update) in a static 8 MiB device
 * scratch per device instead of the context's arena.  Returns DME_EINVAL when
 * they do not fit (about 8 (2 + nsplit) r m bytes, nsplit <= 256 the split of
 * L^T B over n).  Every call on a device shares that device's scratch, so
 * calls that overlap on one device race.  Synchronises the stream.          */
int dme_riccati_noalloc(dme_ctx *ctx, int64_t n, int64_t r, int64_t m, const double *L,
                        const double *B, const double *R, double t, double *D);

/* Symmetric eigen-decomposition of a k x k matrix M (device), eigenvalues
 * ordered by |lambda| descending; eigenvectors only for the kept ones
 * (|lambda| > tol max|lambda|, at most max_keep).  lam: k, V: k x max_keep. */
int dme_syev(dme_ctx *ctx, int64_t k, const double *M, double tol, int64_t max_keep, double *lam,
             double *V, int64_t *keep_out);

/* ------------------------------------------------------------- serving */
/* A request server on a context: solves submitted as they arrive run with
 * continuous batching.  A scheduler thread admits waiting requests in
 * arrival order whenever a slot is free and the device-memory ledger
 * (cached operators + per-solve state) stays within the budget, advances all
 * admitted solves one time step per tick (solves that share an operator
 * e^{tA^T} get one product over their concatenated factors; compressions and
 * Riccati updates of different solves overlap on their own streams), and
 * retires finished solves.  A solve's result is the same alone and in any mix.
 * Mixed-precision requests are re-run from the start in FP64 when a numerical
 * guard trips (non-finite values, rank cap).                                */
typedef struct dme_server dme_server;

typedef struct {
  int64_t completed, failed, fallbacks; /* requests                            */
  int64_t steps;                        /* time steps advanced, all requests    */
  int64_t cold_builds;                  /* operator sets built on demand        */
  int64_t in_flight;                    /* submitted, not finished              */
  int64_t peak_bytes;                   /* high-water mark of the ledger        */
  double p50_s, p99_s;                  /* arrival-to-completion latency        */
  double queue_p50_s, queue_p99_s;      /* arrival-to-admission                 */
  double req_per_s, steps_per_s;        /* over first arrival .. last completion */
  double cold_build_s;                  /* time in on-demand operator builds    */
} dme_server_stats;

/* Register an operator A (host, n x n, the A of the Sec. 1 equation) on the
 * context: it is copied to the device once and named by *op_id in later
 * submissions.  The registration lives as long as the context.             */
int dme_register_operator(dme_ctx *ctx, const double *A, int64_t n, uint64_t *op_id);
/* Start a server on ctx with a device-memory budget (bytes) for cached
 * operators and solve state, and at most max_slots solves admitted at once. */
int dme_server_start(dme_ctx *ctx, size_t hbm_budget_bytes, int max_slots, dme_server **srv);
/* Build and cache the operator set of op_id for step fraction t (e^{tA^T},
 * its FP32 copy in DME_MIXED, and the quad_nodes Gauss-Legendre node
 * exponentials on [0, t]).  Call before submitting requests.              */
int dme_server_warm(dme_server *srv, uint64_t op_id, double t, int precision, int quad_nodes);
/* Submit a solve (prob.A is ignored: the operator is op_id; all host arrays
 * are copied before return).  is_dre as in dme_solver_create.             */
int dme_submit(dme_server *srv, uint64_t op_id, const dme_problem *prob, const dme_opts *opts,
               int is_dre, uint64_t *ticket);
/* DME_OK and *out (owned by the caller, free with dme_result_free) when the
 * request finished, DME_EAGAIN while it is in flight, the request's error
 * code if it failed.  A ticket can be collected once.                      */
int dme_poll(dme_server *srv, uint64_t ticket, dme_result **out);
int dme_server_stats_get(dme_server *srv, dme_server_stats *out);
/* Finish every submitted request, stop the scheduler, free the server and
 * results that were never collected.                                        */
int dme_server_stop(dme_server *srv);
/* Serving details of a result: precision used (dme_precision), whether it
 * fell back to FP64, latency and queueing time in seconds.                 */
int dme_result_serving(const dme_result *res, int *precision, int *fell_back, double *latency_s,
                       double *queue_s);

#ifdef __cplusplus
}
#endif
#endif /* DME_H */
