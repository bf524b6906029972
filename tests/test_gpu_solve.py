"""Whole solves through the C ABI (dle_solve / dre_solve / stepwise solver)
against the oracle, on seeded synthetic inputs; relative Frobenius error of
P = L D L^T at 1e-10 (FP64)."""
import numpy as np
import pytest

import oracle
import workloads as wl
from paper_1805_08990_amd import _binding as b
from tests.gpu_common import announce

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10


def run_gpu(ctx, prob, **kw):
    opts = b.SolveOptions(T=prob.T, h=prob.h, tol=prob.tol, scheme=prob.scheme, split=prob.split,
                          quad_nodes=prob.quad_nodes, **kw)
    return ctx.solve(prob.kind, opts, prob.A, prob.C, B=prob.B, R=prob.R, S=prob.S,
                     L0=prob.L0, D0=prob.D0)


def run_oracle(prob, **kw):
    return oracle.solve(prob.A, prob.C, prob.T, prob.h, kind=prob.kind, B=prob.B, R=prob.R,
                        S=prob.S, L0=prob.L0, D0=prob.D0, split=prob.split, scheme=prob.scheme,
                        tol=prob.tol, quad_nodes=prob.quad_nodes, **kw)


def check(ctx, prob, tol=TOL_FP64, **okw):
    announce(prob.name, prob.kind, prob.split, prob.scheme, "n", prob.n, "h", prob.h)
    L, D, steps = run_gpu(ctx, prob)
    Lo, Do, info = run_oracle(prob, **okw)
    assert steps == info["steps"]
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank gpu {L.shape[1]} oracle {Lo.shape[1]} rel err {err:.3e}", flush=True)
    assert err < tol
    return L, D, Lo, Do


def test_config_dle_strang_f1f2_n256(ctx):
    """16 x 16 Laplacian, C = ones, P0 = 0, T = 0.1, h = 1e-3, tol 1e-12 (Alg. 1)."""
    check(ctx, wl.config_dle_small(16))


@pytest.mark.parametrize("scheme", ["strang", "lie"])
@pytest.mark.parametrize("split", ["F12", "F1F2"])
def test_dle_small(ctx, scheme, split):
    p = wl.config_dle_small(8)
    p.scheme, p.split, p.h, p.tol = scheme, split, 1e-2, 1e-12
    check(ctx, p)


@pytest.mark.parametrize("scheme", ["strang", "lie"])
@pytest.mark.parametrize("split", ["F12", "F1F2", "F1F3F2"])
def test_dre_small(ctx, scheme, split):
    p = wl.config_dre_halfplane(nx=8, h=1e-2, scheme=scheme)
    p.split = split
    check(ctx, p)


def test_gdre_small(ctx):
    p = wl.config_gdre(nx=8, h=1e-2)
    check(ctx, p)


def test_dre_quadrant_random_C(ctx):
    p = wl.config_dre_quadrant(nx=12, seed=0, p=8, m=4, h=1e-2)
    check(ctx, p)


@pytest.mark.parametrize("n", [60, 61, 1001])
def test_dre_nonsymmetric_A_with_P0(ctx, n):
    """Odd n and row counts off the kernels' 32- and 64-row tiles (ragged tails,
    unaligned column starts in the tall-skinny projections)."""
    A = wl.random_nonsymmetric(n, seed=3, scale=5.0)
    C = wl.random_C(3, n, seed=4)
    L0, D0 = wl.random_lowrank_P0(n, 5, seed=6)
    p = wl.Problem(name="nonsym", A=A, C=C, B=wl.random_C(2, n, seed=7).T.copy(order="F"),
                   R=np.diag([1.0, 2.0]), L0=L0, D0=D0, T=0.05, h=5e-3, tol=1e-12)
    check(ctx, p)


@pytest.mark.parametrize("m", [1, 3, 5, 8])
def test_dre_input_widths(ctx, m):
    """m = 1 .. 8 input columns: every width of the compile-time factor of the
    Riccati-updated D (the compression's D-hat), against the oracle."""
    n = 144
    A = wl.laplacian_2d(12)
    C = wl.random_C(3, n, seed=11)
    B = wl.random_C(m, n, seed=12).T.copy(order="F")
    R = np.diag(1.0 + 0.25 * np.arange(m))
    p = wl.Problem(name=f"dre m={m}", A=A, C=C, B=B, R=R, T=0.03, h=3e-3, tol=1e-12)
    check(ctx, p)


@pytest.mark.parametrize("n", [200, 1030])
def test_dre_nonsymmetric_mixed(ctx, n):
    """DME_MIXED with a nonsymmetric A: the quadrature node products
    e^{s_k A^T} C^T go through the split-BF16 product as well as the step
    products; within 1e-6 of the oracle, and the stated estimate bounds the
    measured distance."""
    A = wl.random_nonsymmetric(n, seed=3, scale=5.0)
    C = wl.random_C(3, n, seed=4)
    p = wl.Problem(name="nonsym mixed", A=A, C=C, B=wl.random_C(2, n, seed=7).T.copy(order="F"),
                   R=np.diag([1.0, 2.0]), T=0.05, h=5e-3, tol=1e-12)
    announce(p.name, "n", n)
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split,
                          quad_nodes=p.quad_nodes, precision="mixed")
    L, D, steps, est = ctx.solve(p.kind, opts, p.A, p.C, B=p.B, R=p.R, err_est=True)
    Lo, Do, info = run_oracle(p)
    assert steps == info["steps"]
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank gpu {L.shape[1]} oracle {Lo.shape[1]} rel err {err:.3e} err_est {est:.3e}", flush=True)
    assert err < 1e-6
    assert err <= est < 1e-3


def test_stepwise_equals_whole_solve(ctx):
    p = wl.config_dre_halfplane(nx=8, h=1e-2)
    announce("stepwise")
    L, D, _ = run_gpu(ctx, p)
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split)
    sv = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    sv.step(3)
    sv.step(7)
    st, tot, r = sv.state()
    assert (st, tot) == (10, 10)
    L2, D2, _ = sv.result()
    assert np.array_equal(L, L2) and np.array_equal(D, D2)
    sv.close()


def test_mixed_stepwise_ahead_products(ctx):
    """The split-BF16 mode forms each step product ahead of need (its first
    rows beside the compression's eigensolver, the rest at the next T12):
    stepping in pieces repeats the whole solve's arithmetic exactly, and an
    error estimate between the pieces (which uses W as scratch and so drops
    the product formed ahead) changes only the association, within the
    split-BF16 error of the oracle."""
    p = wl.config_dre_quadrant(nx=32, T=1e-2, h=1e-3)
    announce("mixed stepwise ahead", "n", p.A.shape[0])
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split, quad_nodes=p.quad_nodes,
                          precision="mixed")
    L, D, _ = ctx.solve(p.kind, opts, p.A, p.C, B=p.B, R=p.R)
    sv = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    sv.step(4)
    sv.step(6)
    L2, D2, _ = sv.result()
    sv.close()
    assert np.array_equal(L, L2) and np.array_equal(D, D2)
    sv = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    sv.step(4)
    _, _, _, est = sv.result(err_est=True)
    sv.step(6)
    L3, D3, _ = sv.result()
    sv.close()
    Lo, Do, _ = run_oracle(p)
    e_whole = oracle.lowrank_rel_err(L, D, Lo, Do)
    e_split = oracle.lowrank_rel_err(L3, D3, Lo, Do)
    print(f"  rank {L.shape[1]} err whole {e_whole:.2e} split {e_split:.2e} est {est:.2e}", flush=True)
    assert e_whole < 1e-6 and e_split < 1e-6
    assert oracle.lowrank_rel_err(L3, D3, L, D) < 1e-6


def test_profiling_levels(ctx):
    """Level 1 times every phase, level 2 the step product kernel alone; the
    timing does not change the result; other levels are rejected.  n = 1024,
    so that the step product takes the skinny kernel that level 2 times."""
    p = wl.config_dre_halfplane(nx=32, h=1e-2)
    announce("profiling levels")
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split)
    ref = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    ref.step(4)
    L0, D0, _ = ref.result()
    ref.close()
    sv = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    sv.profile(True, kernel_only=True)
    sv.step(2)
    assert sv.profile_get("step_kernel")["count"] > 0
    assert sv.profile_get("compress")["count"] == 0 and sv.profile_get("step_gemm")["count"] == 0
    sv.profile(True)
    sv.step(2)
    assert sv.profile_get("compress")["count"] > 0 and sv.profile_get("step_gemm")["count"] > 0
    with pytest.raises(b.DmeError) as e:
        b._check(b._lib_solver_profile(sv._h, 3), "dme_solver_profile")
    assert e.value.code == b.DME_EINVAL
    sv.profile(False)
    L1, D1, _ = sv.result()
    sv.close()
    assert np.array_equal(L0, L1) and np.array_equal(D0, D1)


def test_errors_are_reported(ctx):
    p = wl.config_dre_halfplane(nx=4, h=1e-2)
    announce("errors")
    with pytest.raises(b.DmeError) as e:
        ctx.solve("dre", b.SolveOptions(T=0.1, h=0.03), p.A, p.C, B=p.B, R=p.R)
    assert e.value.code == b.DME_EINVAL
    with pytest.raises(b.DmeError) as e:
        ctx.solve("dre", b.SolveOptions(T=0.1, h=0.01), p.A, p.C, B=p.B, R=-np.eye(1))
    assert e.value.code == b.DME_EINVAL
    with pytest.raises(b.DmeError) as e:
        ctx.solve("dle", b.SolveOptions(T=0.1, h=0.01, max_rank=1), p.A, wl.random_C(3, 16, 1))
    assert e.value.code == b.DME_ERANK


@pytest.mark.parametrize("nx", [12, 32])
def test_feedback_gain(ctx, nx):
    """K = R^-1 B^T L D L^T on the device against the oracle's gain, both from
    the GPU factors (element by element) and from the oracle's own solve; a
    DLE solver has no gain."""
    p = wl.config_dre_quadrant(nx=nx, seed=0, p=8, m=4, h=1e-2)
    announce("feedback gain", "n", p.n)
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split,
                          quad_nodes=p.quad_nodes)
    sv = ctx.solver("dre", opts, p.A, p.C, B=p.B, R=p.R)
    sv.step(5)
    K = sv.gain()
    L, D, _ = sv.result()
    sv.close()
    Kf = oracle.feedback_gain(L, D, p.B, p.R)
    scale = np.abs(Kf).max()
    assert K.shape == Kf.shape
    assert np.abs(K - Kf).max() <= 1e-12 * scale
    Lo, Do, _ = oracle.solve(p.A, p.C, 5 * p.h, p.h, kind="dre", B=p.B, R=p.R, split=p.split,
                             scheme=p.scheme, tol=p.tol, quad_nodes=p.quad_nodes)
    Ko = oracle.feedback_gain(Lo, Do, p.B, p.R)
    err = np.abs(K - Ko).max() / np.abs(Ko).max()
    print(f"  gain vs oracle solve {err:.3e}", flush=True)
    assert err < 1e-10
    dle = ctx.solver("dle", b.SolveOptions(T=p.T, h=p.h), p.A, p.C)
    with pytest.raises(b.DmeError) as e:
        b._check(b._lib_solver_gain(dle._h, K.ctypes.data_as(b._p), 4), "dme_solver_gain")
    assert e.value.code == b.DME_EINVAL
    dle.close()


@pytest.mark.parametrize("scheme", ["strang", "lie"])
@pytest.mark.parametrize("split", ["F12", "F1F2", "F1F3F2"])
def test_gdle_small(ctx, split, scheme):
    """Generalized DLE (S P S^T term, no Riccati term) on the 8 x 8 grid: the
    schemes F12F4, F1F2F4 and F1F4F2 of Sec. 3 (T4 of Alg. 4 in place of T3),
    T = 0.1 with h = 1e-2."""
    p = wl.config_gdle(nx=8, h=1e-2, T=0.1, split=split, scheme=scheme)
    check(ctx, p)


@pytest.mark.parametrize("split,nx", [("F12", 10), ("F1F2", 10), ("F12", 12)])
def test_dle_indefinite_P0(ctx, split, nx):
    """P0 = L0 D0 L0^T with an indefinite D0: the compressions see an
    indefinite Dhat, which the Gram-matrix route declines, so the Householder
    route compresses; the P of both schemes matches the oracle.  At n = 144
    the F12 steps also form their next product ahead beside the compression,
    which a Householder compression then discards."""
    n = nx * nx
    A = wl.laplacian_2d(nx)
    C = wl.random_C(2, n, seed=8)
    L0, _ = wl.random_lowrank_P0(n, 4, seed=9)
    D0 = np.diag([1.0, -0.5, 0.25, -2.0])
    p = wl.Problem(name="dle_indefinite", A=A, C=C, L0=L0, D0=D0, T=0.02, h=2e-3, tol=1e-12,
                   kind="dle", split=split, scheme="strang")
    check(ctx, p)


def test_gram_compression_orthonormality(ctx):
    """The compression through the Gram matrix leaves L orthonormal to well
    below the square root of the unit roundoff times 1/tol (the columns of the
    smallest kept eigenvalues are the least orthonormal); P itself matches the
    oracle at 1e-10 (the check above)."""
    p = wl.config_dre_quadrant(nx=16, T=2e-2, h=1e-3)
    L, D, Lo, Do = check(ctx, p)
    off = np.abs(L.T @ L - np.eye(L.shape[1])).max()
    print(f"  max |L^T L - I| = {off:.2e}", flush=True)
    assert off < 1e-5
