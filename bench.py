"""Benchmark: DRE Strang steps/s at n = 16384 on one MI355X, FP64 (the
paper's arithmetic, the headline) and mixed precision, plus served latency
(p50/p99) of a continuous-batching request mix.

Workload (the heat-equation Riccati setting of the paper's Sec. 5.1 at the size
of the headline metric): A = 5-point Dirichlet Laplacian on a 128 x 128 grid
(n = 16384) scaled by 1/dx^2; B = the four quadrant indicators (n x 4);
R = I_4; C = 8 x n with i.i.d. N(0,1)/sqrt(n) entries (numpy default_rng(0));
P0 = 0; h = 1e-3; two-term Strang splitting T12(h/2) T3(h) T12(h/2) with a
7-node Gauss-Legendre quadrature factor; compression tolerance 1e-10.

A "step" is one Strang time step of the whole hot path (two e^{(h/2)A^T} L
products, two compressions, one Riccati update) with every operand resident
in HBM.  Setup (operator and quadrature factor) runs once before the timed
region and is reported separately.  --warmup W steps run untimed, then exactly
--steps K are timed between two device synchronisations.

Printed: one JSON line.  `value` is the FP64 steps/s (`mixed_steps_per_s`
beside it, with the mixed result's distance to the FP64 one and its stated
estimate), `roofline` is the FP64 step product's main kernel timed with HIP
events on the library's stream inside the timed region (`roofline_mixed` the
split-BF16 kernel), `cpu_baseline` the CPU oracle on a bounded sample of the
same workload, `serving` the request-mix statistics.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
GIB = 1 << 30

KERNEL_SOURCES = {
    "gemm_mixed_kernel": "paper_1805_08990_amd/csrc/gemm_mixed.hip",
    "gemm_f64_skinny_kernel": "paper_1805_08990_amd/csrc/gemm_f64.hip",
    "leja_csr_term_kernel": "paper_1805_08990_amd/csrc/leja.hip",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nx", type=int, default=128, help="grid side (n = nx^2)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "leja", "both", "all"], default="all",
                    help="fp64 / mixed: dense e^{tA^T} products; leja: FP64 Leja-interpolation "
                         "action on the CSR Laplacian (the paper's expleja); both = fp64 + mixed; "
                         "all = the three")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget for the CPU oracle sample (0 disables it)")
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests in the served mix (0 disables the serving leg)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one device copy of known size (counter calibration)")
    ap.add_argument("--product-only", type=int, default=0, metavar="R",
                    help="run only the step product E X (n x n times n x R, random E and X, 3 "
                         "launches) for hardware counters, and exit")
    ap.add_argument("--product-precision", choices=["fp64", "mixed", "leja"], default="mixed",
                    help="which step product --product-only runs (leja: the Leja action "
                         "e^{(h/2)A^T} X on the CSR Laplacian, its Newton terms at rank R)")
    ap.add_argument("--serve-sweep", type=int, default=0, metavar="COUNT",
                    help="instead of the steps/s line: serve COUNT requests at 0.5, 0.7 and 0.9 x "
                         "the measured capacity and the same stream one request at a time (FIFO)")
    ap.add_argument("--sweep-parts", default="0.5,0.7,0.9,fifo",
                    help="which parts of the serving sweep run (comma list of 0.5, 0.7, 0.9, fifo)")
    ap.add_argument("--serve-capacity", type=float, default=None,
                    help="capacity (requests/s) the sweep's rates are fractions of, instead of a burst")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", flush=True)


def workload(nx):
    import workloads as wl
    return wl.config_dre_quadrant(nx=nx, seed=0, p=8, m=4, T=0.1, h=1e-3)


def lowrank_rel_diff(L1, D1, L2, D2):
    """||L1 D1 L1^T - L2 D2 L2^T||_F / ||L2 D2 L2^T||_F without forming n x n
    matrices: with [L1, L2] = Q R, both are Q (R_i D_i R_i^T) Q^T."""
    import numpy as np
    L1, L2 = np.asarray(L1, dtype=np.float64), np.asarray(L2, dtype=np.float64)
    D1, D2 = np.asarray(D1, dtype=np.float64), np.asarray(D2, dtype=np.float64)
    _, R = np.linalg.qr(np.hstack([L1, L2]))
    r1 = L1.shape[1]
    M1 = R[:, :r1] @ D1 @ R[:, :r1].T
    M2 = R[:, r1:] @ D2 @ R[:, r1:].T
    return float(np.linalg.norm(M1 - M2) / np.linalg.norm(M2))


def run_gpu(ctx, prob, precision, steps, warmup):
    import torch
    from paper_1805_08990_amd import _binding as b

    A = prob.A
    if precision == "leja":
        import numpy as np
        import scipy.sparse as sp
        Ms = sp.csr_matrix(prob.A)
        A = (Ms.indptr.astype(np.int64), Ms.indices.astype(np.int64), Ms.data.astype(np.float64))
        opts = b.SolveOptions(T=prob.T, h=prob.h, tol=prob.tol, scheme="strang", split="F12",
                              precision="fp64", quad_nodes=prob.quad_nodes, action="leja")
        log(f"leja: setup (CSR A, nnz {len(A[2])}, Leja plan for e^(h/2 A^T), quadrature factor)")
    else:
        opts = b.SolveOptions(T=prob.T, h=prob.h, tol=prob.tol, scheme="strang", split="F12",
                              precision=precision, quad_nodes=prob.quad_nodes)
        log(f"{precision}: setup (operator e^(h/2 A^T), quadrature factor)")
    t0 = time.perf_counter()
    sv = ctx.solver("dre", opts, A, prob.C, B=prob.B, R=prob.R)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    setup = sv.setup_info()
    log(f"{precision}: setup {setup_s:.2f} s (expm {setup['expm_ms']:.0f} ms, quadrature "
        f"{setup['quad_ms']:.0f} ms, rank L_I {setup['rank_quad']})")
    if warmup:
        sv.step(warmup)
    torch.cuda.synchronize()
    # timed steps: HIP events around the step product kernel only
    sv.profile(True, kernel_only=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st, tot, rank = sv.state()
    prof = {"step_kernel": sv.profile_get("step_kernel")}
    log(f"{precision}: {steps} steps in {elapsed:.3f} s ({steps / elapsed:.1f} steps/s), rank {rank}")
    # phase breakdown from a few more steps with events around every phase
    # (outside the timed region: the events cost the stream a little time)
    phase_steps = min(steps, 5)
    sv.profile(True)
    sv.step(phase_steps)
    torch.cuda.synchronize()
    for ph in ("step_gemm", "compress", "riccati"):
        prof[ph] = sv.profile_get(ph)
    prof["phase_steps"] = phase_steps
    sv.profile(False)
    # LQR feedback gain K = R^-1 B^T L D L^T at the last step (device work and
    # the m x n copy to the host)
    sv.gain()
    t1 = time.perf_counter()
    for _ in range(3):
        sv.gain()
    gain_ms = (time.perf_counter() - t1) / 3 * 1e3
    L, D, _, err_est = sv.result(err_est=True)
    sv.close()
    return {"elapsed_s": elapsed, "setup_s": setup_s, "setup": setup, "rank": rank, "prof": prof,
            "L": L, "D": D, "gain_ms": gain_ms, "err_est": err_est}


def kernel_source_hash(kernel):
    path = os.path.join(ROOT, KERNEL_SOURCES[kernel])
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, alg_bytes_per_launch):
    """HBM bytes per launch of `kernel`: the committed counter summary's
    measured-over-algorithmic ratio (FETCH_SIZE + WRITE_SIZE of whole-product
    launches, copy-calibrated) times this run's algorithmic bytes per launch
    (the split-BF16 steps launch the product in two row ranges); None unless
    the summary was taken on the current source of the kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256_16") != kernel_source_hash(kernel):
        return None
    return int(round(rec["traffic_over_algorithmic"] * alg_bytes_per_launch))


def roofline_from(prof, precision):
    g = prof.get("step_kernel")
    if not g or g["count"] == 0 or g["ms"] <= 0:
        return None
    avg_s = g["ms"] / g["count"] * 1e-3
    if precision == "fp64":
        kernel = "gemm_f64_skinny_kernel"
        achieved = g["flops"] / g["count"] / avg_s / 1e12
        out = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
               "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4)}
    elif precision == "leja":
        # one Newton term of the Leja action: the CSR operator, the basis block
        # read and written, the accumulator read and written by every second
        # term (HBM-bound form, averaged over the terms)
        kernel = "leja_csr_term_kernel"
        achieved = g["bytes"] / g["count"] / avg_s / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": round(achieved / PEAK_HBM_GBS, 4)}
    else:
        # the FP32 operator is streamed once per launch: HBM-bound form on the
        # algorithmic bytes; the six BF16 piece products it executes (12 n^2 r
        # flops) are reported beside it against the BF16 MFMA peak
        kernel = "gemm_mixed_kernel"
        achieved = g["bytes"] / g["count"] / avg_s / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": round(achieved / PEAK_HBM_GBS, 4)}
        executed = 6.0 * g["flops"] / g["count"] / avg_s / 1e12
        out["executed_bf16_tflops"] = round(executed, 1)
        out["executed_bf16_frac"] = round(executed / PEAK_BF16_TFLOPS, 4)
    out["traffic"] = measured_traffic(kernel, g["bytes"] / g["count"])
    out.update({"kernel": kernel, "avg_launch_ms": round(avg_s * 1e3, 4), "launches": g["count"],
                "algorithmic_per_launch": {"flops": g["flops"] / g["count"],
                                           "bytes": g["bytes"] / g["count"]}})
    return out


def host_description():
    """CPU model, logical CPUs and the BLAS numpy uses (for the baseline)."""
    import platform
    from threadpoolctl import threadpool_info
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = [f"{i.get('internal_api')} {i.get('version')} ({i.get('threading_layer')}, "
            f"{i.get('architecture')})" for i in threadpool_info() if i.get("user_api") == "blas"]
    return {"cpu_model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)), "blas": blas[0] if blas else "unknown"}


def cpu_baseline(prob, budget_s):
    """The oracle as it stands, on the host cores, over a bounded sample: its
    operator setup through the Kronecker-sum route (e^{tA} = e^{tA1} (x) e^{tA1}),
    then the first Strang steps from P0 = 0.  Three samples with every BLAS
    thread (the median is `value`) and one with a single thread."""
    import numpy as np
    import oracle
    import workloads as wl
    from threadpoolctl import threadpool_info, threadpool_limits

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    A1 = wl.laplacian_1d(prob.nx)
    t = 0.5 * prob.h
    t0 = time.perf_counter()
    E = oracle.laplacian_expm_kron(A1, t)
    LI, DI = oracle.quadrature_factor_kron(A1, prob.C, t, prob.quad_nodes, prob.tol)
    setup_s = time.perf_counter() - t0
    per_sample = budget_s / 4.0

    def sample(max_steps):
        L = np.zeros((prob.n, 0))
        D = np.zeros((0, 0))
        done = 0
        t0 = time.perf_counter()
        while True:
            L, D = oracle.t12(L, D, E, LI, DI, prob.tol)
            D = oracle.t3(L, D, prob.B, prob.R, prob.h)
            L, D = oracle.t12(L, D, E, LI, DI, prob.tol)
            done += 1
            el = time.perf_counter() - t0
            if el >= per_sample or done >= max_steps:
                return done, el, L.shape[1]

    runs = [sample(prob.nsteps) for _ in range(3)]
    rates = sorted(d / el for d, el, _ in runs)
    with threadpool_limits(limits=1):
        d1, el1, _ = sample(prob.nsteps)
    done, el, rank = runs[0]
    out = {"value": round(rates[1], 4), "unit": "steps/s", "cores": threads, "kind": "oracle",
           "sample": f"first {done} Strang steps from P0 = 0 (rank {rank} at the end) of the "
                     f"n = {prob.n} workload, numpy FP64, median of 3 samples of ~{per_sample:.0f} s, "
                     f"setup {setup_s:.1f} s excluded",
           "samples_steps_per_s": [round(r, 4) for r in rates],
           "one_thread_steps_per_s": round(d1 / el1, 4), "one_thread_steps": d1}
    out.update(host_description())
    return out


def _serving_setup(ctx, max_slots):
    import workloads as wl
    h = 1e-3
    srv = ctx.server(160 * GIB, max_slots=max_slots)
    ops = {}
    t0 = time.perf_counter()
    for nx in wl.SERVE_GRID_SIDES:
        ops[nx] = ctx.register_operator(wl.laplacian_2d(nx))
        for t in (0.5 * h, h):  # DRE Strang half step, DLE full step
            srv.warm(ops[nx], t, "mixed", 7)
        log(f"serving: operator nx={nx} warm ({time.perf_counter() - t0:.1f} s)")
    return srv, ops, time.perf_counter() - t0


def _serve_stream(srv, ops, stream, label=None):
    """Submit the stream at its arrival times, wait for every result (with a
    progress line every 64 results when `label` is given)."""
    import numpy as np
    import workloads as wl
    from paper_1805_08990_amd import _binding as b

    def submit(req):
        p = wl.request_problem(req)
        opts = b.SolveOptions(T=p.T, h=req.h, tol=p.tol, scheme="strang", split="F12",
                              precision="mixed")
        return srv.submit(ops[req.nx], p.kind, opts, p.C, p.n, B=p.B, R=p.R)

    t0 = time.perf_counter()
    tickets, res = {}, {}
    reported = [0]

    def collect():
        for i, tk in list(tickets.items()):
            if i not in res:
                got = srv.poll(tk)
                if got is not None:
                    res[i] = got
        if label and len(res) >= reported[0] + 64:
            reported[0] = len(res) // 64 * 64
            log(f"{label}: {len(res)} of {len(stream)} done at {time.perf_counter() - t0:.0f} s")

    for r in stream:
        while True:  # collect finished requests while waiting for the next arrival
            wait = r.arrival_s - (time.perf_counter() - t0)
            collect()
            if wait <= 0:
                break
            time.sleep(min(wait, 0.002))
        tickets[r.index] = submit(r)
    while len(res) < len(tickets):
        collect()
        time.sleep(0.001)
    span = time.perf_counter() - t0
    lat = np.array([res[r.index][3]["latency_s"] for r in stream])
    queue = np.array([res[r.index][3]["queue_s"] for r in stream])
    est = np.array([res[r.index][3]["err_est"] for r in stream])
    steps = sum(r.nsteps for r in stream)
    return {"requests": len(stream), "p50_s": round(float(np.percentile(lat, 50)), 4),
            "p99_s": round(float(np.percentile(lat, 99)), 4),
            "mean_latency_s": round(float(lat.mean()), 4),
            "queue_p50_s": round(float(np.percentile(queue, 50)), 4),
            "req_per_s": round(len(stream) / span, 3), "steps_per_s": round(steps / span, 1),
            "fallbacks": sum(1 for v in res.values() if v[3]["fell_back"]),
            "err_est_max": float(est.max()) if len(est) else 0.0, "span_s": round(span, 1)}


def _capacity(srv, ops, count, seed):
    import workloads as wl
    burst = wl.request_stream(count, rate_per_s=1e9, base_seed=5000, stream_seed=seed)
    t0 = time.perf_counter()
    _serve_stream(srv, ops, burst)
    return len(burst) / (time.perf_counter() - t0)


def serve_mix(ctx, count, seed=7):
    """Served request mix: grid sides in {32, 48, 64, 96, 128}, DLE or DRE,
    m in 1..4, p in 1..8, N in 50..200 steps of h = 1e-3, mixed precision.
    Capacity is measured first with a burst of count/2 requests, then `count`
    requests arrive as a Poisson stream at 0.7 x capacity."""
    import workloads as wl
    srv, ops, warm_s = _serving_setup(ctx, 16)
    cap = _capacity(srv, ops, max(1, count // 2), seed)
    log(f"serving: capacity {cap:.2f} requests/s from a burst of {max(1, count // 2)}")
    rate = 0.7 * cap
    out = _serve_stream(srv, ops, wl.request_stream(count, rate_per_s=rate, base_seed=1000,
                                                    stream_seed=seed))
    st = srv.stats()
    srv.stop()
    log(f"serving: {count} requests at {rate:.2f}/s, p50 {out['p50_s']:.3f} s, p99 {out['p99_s']:.3f} s")
    out.update({"arrival_rate_per_s": round(rate, 3), "capacity_req_per_s": round(cap, 3),
                "failed": st["failed"], "cold_builds": st["cold_builds"],
                "warm_operators_s": round(warm_s, 1), "max_slots": 16, "hbm_budget_gib": 160,
                "peak_ledger_gib": round(st["peak_bytes"] / GIB, 2)})
    return out


def serve_sweep(ctx, count, parts=("0.5", "0.7", "0.9", "fifo"), capacity=None, seed=7):
    """The served mix at its full size: capacity from a burst of 64 (or as
    given), then `count` Poisson arrivals at 0.5, 0.7 and 0.9 x capacity with
    continuous batching (16 slots), and the 0.7 stream served one request at
    a time in arrival order (one slot: FIFO, no batching) as the baseline.
    `parts` picks which of these run (each takes minutes at count = 512)."""
    import workloads as wl
    srv, ops, warm_s = _serving_setup(ctx, 16)
    if capacity is None:
        cap = _capacity(srv, ops, 64, seed)
        log(f"serving sweep: capacity {cap:.2f} requests/s (burst of 64)")
    else:
        cap = float(capacity)
        log(f"serving sweep: capacity {cap:.2f} requests/s (given)")
    out = {"requests": count, "capacity_req_per_s": round(cap, 3), "capacity_given": capacity is not None,
           "warm_operators_s": round(warm_s, 1), "batched": {}, "max_slots": 16, "hbm_budget_gib": 160}
    for frac in ("0.5", "0.7", "0.9"):
        if frac not in parts:
            continue
        rate = float(frac) * cap
        stream = wl.request_stream(count, rate_per_s=rate, base_seed=1000, stream_seed=seed)
        res = _serve_stream(srv, ops, stream, label=f"serving sweep {frac} x capacity")
        res["arrival_rate_per_s"] = round(rate, 3)
        out["batched"][frac] = res
        log(f"serving sweep: {frac} x capacity: p50 {res['p50_s']:.3f} s p99 {res['p99_s']:.3f} s "
            f"{res['req_per_s']:.2f} req/s")
    st = srv.stats()
    out["failed"] = st["failed"]
    out["peak_ledger_gib"] = round(st["peak_bytes"] / GIB, 2)
    srv.stop()
    if "fifo" in parts:
        fifo, fops, _ = _serving_setup(ctx, 1)
        stream = wl.request_stream(count, rate_per_s=0.7 * cap, base_seed=1000, stream_seed=seed)
        res = _serve_stream(fifo, fops, stream, label="serving sweep FIFO")
        res["arrival_rate_per_s"] = round(0.7 * cap, 3)
        out["failed"] += fifo.stats()["failed"]
        fifo.stop()
        out["fifo_0.7"] = res
        log(f"serving sweep: FIFO at 0.7 x capacity: p50 {res['p50_s']:.3f} s p99 {res['p99_s']:.3f} s")
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the path is built "
              "for one GPU; sharding E by rows across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1805_08990_amd import _binding as b

    ctx = b.Context(0)
    if args.calibrate_copy:
        # one plain device copy of 1 GiB, for the HBM counter calibration
        x = torch.ones(GIB // 8, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.product_only > 0:
        # the step product alone, at the workload's n, with no operator set-up
        # (its LU issues ~10^5 small launches, which counter collection does not bear)
        n, r = args.nx * args.nx, args.product_only
        g = torch.Generator(device="cuda").manual_seed(0)
        info = {"n": n, "r": r, "launches": 3, "precision": args.product_precision}
        if args.product_precision == "leja":
            # three actions of the workload's half step; every Newton term is
            # one leja_csr_term_kernel launch over the n x r block
            import numpy as np
            import scipy.sparse as sp
            import workloads as wl
            X = torch.randn((n, r), dtype=torch.float64, device="cuda", generator=g)
            Ms = sp.csr_matrix(wl.laplacian_2d(args.nx))
            A = (Ms.indptr.astype(np.int64), Ms.indices.astype(np.int64), Ms.data.astype(np.float64))
            for _ in range(3):
                _, S, m = ctx.expmv_leja(A, 0.5e-3, X)  # the workload's half step, h = 1e-3
                torch.cuda.synchronize()
            # per term the operator and the basis block read and written; the
            # accumulator read and written by every second term
            per_term = 12 * int(Ms.nnz) + 8 * n + 16 * n * r + 16 * n * r * ((m + 1) // 2) / m
            info.update({"substeps": S, "degree": m, "term_launches": 3 * S * m, "nnz": int(Ms.nnz),
                         "algorithmic_bytes_per_term": round(per_term)})
        else:
            E = torch.randn((n, n), dtype=torch.float64, device="cuda", generator=g) / math.sqrt(n)
            X = torch.randn((n, r), dtype=torch.float64, device="cuda", generator=g)
            for _ in range(3):
                if args.product_precision == "mixed":
                    ctx.gemm_mixed(E, X)
                else:
                    ctx.gemm(E, X)
                torch.cuda.synchronize()
        print(json.dumps({"product_only": info}), flush=True)
        return
    if args.serve_sweep > 0:
        parts = tuple(x.strip() for x in args.sweep_parts.split(","))
        print(json.dumps({"serving_sweep": serve_sweep(ctx, args.serve_sweep, parts, args.serve_capacity)}),
              flush=True)
        ctx.close()
        return
    prob = workload(args.nx)
    precisions = {"both": ["fp64", "mixed"], "all": ["fp64", "mixed", "leja"]}.get(
        args.precision, [args.precision])
    results = {p: run_gpu(ctx, prob, p, args.steps, args.warmup) for p in precisions}
    main_prec = "fp64" if "fp64" in results else precisions[0]
    res = results[main_prec]
    value = args.steps / res["elapsed_s"]
    line = {
        "metric": "DRE Strang steps/s at n=16384, FP64 vs mixed; p50/p99 served latency",
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["elapsed_s"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x3-split products, f64 elsewhere" if main_prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"dre_strang_f12f3_quadrant_n{prob.n}", "n": prob.n, "m": 4, "p": 8,
                   "h": prob.h, "tol": prob.tol, "quad_nodes": prob.quad_nodes,
                   "precision": main_prec, "rank_end": res["rank"],
                   "setup_s": round(res["setup_s"], 3)},
        "roofline": roofline_from(res["prof"], main_prec),
    }
    for prec, r in results.items():
        line[f"{prec}_steps_per_s"] = round(args.steps / r["elapsed_s"], 4)
        line[f"{prec}_gain_ms"] = round(r["gain_ms"], 3)
        pr = r["prof"]
        line[f"{prec}_phase_ms_per_step"] = {
            k: round(v["ms"] / (args.steps if k == "step_kernel" else pr["phase_steps"]), 4)
            for k, v in pr.items() if k != "phase_steps"}
        if prec != main_prec:
            line[f"roofline_{prec}"] = roofline_from(r["prof"], prec)
    for prec, r in results.items():
        line[f"{prec}_err_est"] = r["err_est"]
        line[f"{prec}_setup"] = {"total_s": round(r["setup_s"], 3),
                                 "expm_ms": round(r["setup"]["expm_ms"], 1),
                                 "quad_ms": round(r["setup"]["quad_ms"], 1),
                                 "rank_quad": r["setup"]["rank_quad"]}
    if "fp64" in results and "mixed" in results:
        rf, rm = results["fp64"], results["mixed"]
        line["mixed_vs_fp64_rel_err"] = lowrank_rel_diff(rm["L"], rm["D"], rf["L"], rf["D"])
    if "fp64" in results and "leja" in results:
        rf, rl = results["fp64"], results["leja"]
        line["leja_vs_fp64_rel_err"] = lowrank_rel_diff(rl["L"], rl["D"], rf["L"], rf["D"])
    if args.serve_requests > 0:
        try:
            line["serving"] = serve_mix(ctx, args.serve_requests)
        except Exception as e:  # the steps/s line is still reported
            line["serving"] = {"error": str(e)}
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
