"""Benchmark: DRE Strang steps/s at n = 16384 on one MI355X, FP64 and mixed.

Workload (the paper's heat-equation Riccati setting, Sec. 5.1, at the size
named by the headline metric): A = 5-point Dirichlet Laplacian on a 128 x 128
grid (n = 16384) scaled by 1/dx^2; B = the four quadrant indicators (n x 4);
R = I_4; C = 8 x n with i.i.d. N(0,1)/sqrt(n) entries (numpy default_rng(0));
P0 = 0; h = 1e-3 (T = 0.1, N = 100); two-term Strang splitting
T12(h/2) T3(h) T12(h/2) with a 7-node Gauss-Legendre quadrature factor;
compression tolerance 1e-10.

A "step" is one Strang time step of the whole hot path (two e^{(h/2)A^T} L
products, two compressions, one Riccati update) with all operands resident in
HBM.  Setup (operator and quadrature factor) is done once before the timed
region and reported separately.  --warmup W steps run untimed, then exactly
--steps K are timed between two device synchronisations.

Printed: one JSON line with the throughput of the (default) precision, the
roofline position of the dominant kernel (the step product e^{tA^T} L,
FP64 MFMA-bound) from HIP events recorded by the library on its own stream,
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 matrix
PEAK_BF16_TFLOPS = 2500.0    # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=90)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--nx", type=int, default=128, help="grid side (n = nx^2)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "both"], default="fp64")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="budget for the CPU oracle sample (0 disables it)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-launch event timing of the step product")
    return ap.parse_args()


def workload(nx):
    import workloads as wl
    return wl.config_dre_quadrant(nx=nx, seed=0, p=8, m=4, T=0.1, h=1e-3)


def run_gpu(prob, precision, steps, warmup, profile=True):
    import torch
    from paper_1805_08990_amd import _binding as b

    ctx = b.Context(0)
    opts = b.SolveOptions(T=prob.T, h=prob.h, tol=prob.tol, scheme="strang", split="F12",
                          precision=precision, quad_nodes=prob.quad_nodes)
    t0 = time.perf_counter()
    sv = ctx.solver("dre", opts, prob.A, prob.C, B=prob.B, R=prob.R)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    setup = sv.setup_info()
    print(f"[bench] {precision}: setup {setup_s:.2f} s (expm {setup['expm_ms']:.0f} ms, "
          f"quadrature {setup['quad_ms']:.0f} ms, rank L_I {setup['rank_quad']})", flush=True)
    if warmup:
        sv.step(warmup)
    torch.cuda.synchronize()
    if profile:
        sv.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sv.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st, tot, rank = sv.state()
    prof = {ph: sv.profile_get(ph) for ph in ("step_gemm", "compress", "riccati")} if profile else {}
    print(f"[bench] {precision}: {steps} steps in {elapsed:.3f} s, rank {rank}", flush=True)
    sv.close()
    ctx.close()
    return {"elapsed_s": elapsed, "setup_s": setup_s, "setup": setup, "rank": rank, "prof": prof}


def roofline_from(prof, precision):
    g = prof.get("step_gemm")
    if not g or g["count"] == 0 or g["ms"] <= 0:
        return None
    avg_ms = g["ms"] / g["count"]
    if precision == "fp64":
        achieved = g["flops"] / g["count"] / (avg_ms * 1e-3) / 1e12
        return {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4), "traffic": None,
                "kernel": "gemm_f64 (e^{tA^T} L)", "avg_launch_ms": round(avg_ms, 4),
                "launches": g["count"]}
    achieved = g["bytes"] / g["count"] / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
            "kernel": "gemm split-bf16 (e^{tA^T} L)", "avg_launch_ms": round(avg_ms, 4),
            "launches": g["count"]}


def cpu_baseline(prob, budget_s):
    """The oracle as it stands, on the host cores, over a bounded sample: its
    operator setup through the Kronecker-sum route (e^{tA} = e^{tA1} (x) e^{tA1}),
    then as many Strang steps from P0 = 0 as fit in the budget."""
    import numpy as np
    import oracle
    import workloads as wl
    from threadpoolctl import threadpool_info

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    A1 = wl.laplacian_1d(prob.nx)
    t = 0.5 * prob.h
    t0 = time.perf_counter()
    E = oracle.laplacian_expm_kron(A1, t)
    LI, DI = oracle.quadrature_factor_kron(A1, prob.C, t, prob.quad_nodes, prob.tol)
    setup_s = time.perf_counter() - t0
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
        if el >= budget_s or done >= prob.nsteps:
            break
    return {"value": round(done / el, 4), "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} Strang steps from P0 = 0 (rank {L.shape[1]} at the end) of the "
                      f"n = {prob.n} workload, numpy FP64, setup {setup_s:.1f} s excluded",
            "elapsed_s": round(el, 2)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the path would shard E row-wise across GPUs, see the design notes)", file=sys.stderr)
        sys.exit(2)
    prob = workload(args.nx)
    precisions = ["fp64", "mixed"] if args.precision == "both" else [args.precision]
    results = {}
    for prec in precisions:
        results[prec] = run_gpu(prob, prec, args.steps, args.warmup, profile=not args.no_profile)
    main_prec = precisions[-1]
    res = results[main_prec]
    value = args.steps / res["elapsed_s"]
    line = {
        "metric": "DRE Strang steps/s at n=16384 (two-term splitting, quadrature linear part)",
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * res["elapsed_s"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "bf16-split x3 + f32 acc + f64",
        "data": "synthetic",
        "config": {"workload": f"dre_strang_f12f3_quadrant_n{prob.n}", "n": prob.n, "m": 4, "p": 8,
                   "h": prob.h, "T": prob.T, "tol": prob.tol, "quad_nodes": prob.quad_nodes,
                   "precision": main_prec, "rank_end": res["rank"],
                   "setup_s": round(res["setup_s"], 3)},
        "roofline": roofline_from(res["prof"], main_prec),
    }
    for prec, r in results.items():
        line[f"{prec}_steps_per_s"] = round(args.steps / r["elapsed_s"], 4)
        line[f"{prec}_phases_ms"] = {k: round(v["ms"], 3) for k, v in r["prof"].items()}
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(prob, args.cpu_seconds)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
