"""Whole solves at the workload sizes (64 x 64 and 128 x 128 grids) against
the oracle, which evaluates the same exponentials through the Kronecker-sum
structure of the Laplacian (e^{tA} = e^{tA1} (x) e^{tA1}; pinned against the
dense exponential in the oracle tests), and the observed orders of the Lie and
Strang schemes at n = 4096 (Sec. 5, order plots)."""
import math

import numpy as np
import pytest

import oracle
import workloads as wl
from paper_1805_08990_amd import _binding as b
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu


def gpu_solve(ctx, p, precision="fp64"):
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split,
                          quad_nodes=p.quad_nodes, precision=precision)
    return ctx.solve(p.kind, opts, p.A, p.C, B=p.B, R=p.R, S=p.S, L0=p.L0, D0=p.D0)


def oracle_kron(p):
    A1 = wl.laplacian_1d(p.nx)
    return oracle.solve(p.A, p.C, p.T, p.h, kind=p.kind, B=p.B, R=p.R, S=p.S, split=p.split,
                        scheme=p.scheme, tol=p.tol, quad_nodes=p.quad_nodes,
                        expm_fn=lambda t: oracle.laplacian_expm_kron(A1, t),
                        quad_fn=lambda t: oracle.quadrature_factor_kron(A1, p.C, t, p.quad_nodes,
                                                                        p.tol))


@pytest.mark.parametrize("scheme", ["lie", "strang"])
def test_dre_halfplane_n4096_matches_oracle(ctx, scheme):
    """64 x 64 Laplacian, B = 1[x < 1/2], R = 1, C = ones, h = 1e-2 (10 steps)."""
    p = wl.config_dre_halfplane(nx=64, h=1e-2, scheme=scheme)
    announce("dre n4096", scheme)
    L, D, steps = gpu_solve(ctx, p)
    Lo, Do, info = oracle_kron(p)
    assert steps == info["steps"] == 10
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank gpu {L.shape[1]} oracle {Lo.shape[1]} rel err {err:.3e}", flush=True)
    assert err < 1e-10


@pytest.mark.parametrize("scheme,order", [("lie", 1), ("strang", 2)])
def test_dre_halfplane_n4096_observed_order(ctx, scheme, order):
    """Errors at h = 1e-4, 5e-5, 2.5e-5 (T = 1e-3) against a Strang solve at
    h = 3.125e-6 fall by 2^order per halving (order 1 for Lie, 2 for Strang).
    The 64 x 64 Laplacian has ||A|| h >> 1 at the h of the parity test above
    (1e-2), where both schemes are still pre-asymptotic (relative errors of
    order one, the oracle gives the same values), so the order is measured at
    steps where ||A|| h is of order one."""
    announce("order n4096", scheme)
    ref = wl.config_dre_halfplane(nx=64, h=3.125e-6, scheme="strang", T=1e-3)
    Lr, Dr, _ = gpu_solve(ctx, ref)
    errs = []
    for h in (1e-4, 5e-5, 2.5e-5):
        p = wl.config_dre_halfplane(nx=64, h=h, scheme=scheme, T=1e-3)
        L, D, _ = gpu_solve(ctx, p)
        errs.append(oracle.lowrank_rel_err(L, D, Lr, Dr))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print(f"  errors {['%.3e' % e for e in errs]} observed orders {['%.2f' % r for r in rates]}",
          flush=True)
    for r in rates:
        assert abs(r - order) < 0.15


def test_gdre_n4096_matches_oracle(ctx):
    """Generalized DRE on the 64 x 64 grid, S = 0.1 tridiag(1, 0, 1), h = 1e-3
    (20 steps of the five-stage Strang composition)."""
    p = wl.config_gdre(nx=64, h=1e-3, T=0.02)
    announce("gdre n4096")
    L, D, steps = gpu_solve(ctx, p)
    Lo, Do, info = oracle_kron(p)
    assert steps == info["steps"] == 20
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank gpu {L.shape[1]} oracle {Lo.shape[1]} rel err {err:.3e}", flush=True)
    assert err < 1e-10


def test_dre_quadrant_n16384_fp64_and_mixed(ctx):
    """The 128 x 128 workload of the benchmark (B = quadrant indicators, R = I4,
    C = 8 x n N(0,1)/sqrt(n), seed 0), first 5 steps of h = 1e-3: FP64 within
    1e-10 and the split-BF16 products within 1e-6 of the oracle."""
    p = wl.config_dre_quadrant(nx=128, T=5e-3, h=1e-3)
    announce("dre n16384 fp64/mixed")
    Lo, Do, info = oracle_kron(p)
    L, D, steps = gpu_solve(ctx, p, "fp64")
    assert steps == info["steps"] == 5
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    Lm, Dm, _ = gpu_solve(ctx, p, "mixed")
    errm = oracle.lowrank_rel_err(Lm, Dm, Lo, Do)
    print(f"  rank gpu {L.shape[1]} oracle {Lo.shape[1]} fp64 {err:.3e} mixed {errm:.3e}", flush=True)
    assert err < 1e-10
    assert errm < 1e-6
