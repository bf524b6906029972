"""The Leja-interpolation action (the paper's expleja, Sec. 3 and Sec. 4) on
the device: step-level e^{tA^T} X against the oracle's action and the exact
one, and whole solves with DME_ACTION_LEJA (dense and CSR A) and with the
mass-matrix form (Sec. 5.1, Ex. 4) against the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import workloads as wl
from paper_1805_08990_amd import _binding as b
from tests.gpu_common import announce, to_np
from tests.laplace_closed_form import eig2d

pytestmark = pytest.mark.gpu


def csr(A):
    M = sp.csr_matrix(np.asarray(A))
    return (M.indptr.astype(np.int64), M.indices.astype(np.int64), M.data.astype(np.float64))


@pytest.mark.parametrize("nx,t,c", [(8, 5e-4, 3), (24, 1e-3, 17), (64, 5e-4, 40), (31, 1e-2, 5)])
@pytest.mark.parametrize("form", ["dense", "csr"])
def test_expmv_leja_matches_exact_action(ctx, nx, t, c, form):
    """e^{tA} X for the Dirichlet Laplacian against its closed-form eigenpairs
    (nx = 31, t = 1e-2 takes several substeps; ragged column counts)."""
    announce("expmv_leja", form, nx, t, c)
    A = wl.laplacian_2d(nx)
    X = np.random.default_rng(nx + c).standard_normal((nx * nx, c))
    Y, S, m = ctx.expmv_leja(A if form == "dense" else csr(A), t, X)
    lam, U = eig2d(nx)
    ref = U @ (np.exp(t * lam)[:, None] * (U.T @ X))
    err = np.linalg.norm(to_np(Y) - ref) / np.linalg.norm(X)
    print(f"  S {S} m {m} err {err:.2e}", flush=True)
    assert err < 1e-12
    if nx <= 24:
        ref_o = oracle.leja_expmv(A, t, X)
        assert np.linalg.norm(to_np(Y) - ref_o) <= 1e-12 * np.linalg.norm(X)


@pytest.mark.parametrize("t,c", [(5e-4, 7), (1e-2, 3)])
def test_expmv_leja_csr_wide_rows(ctx, t, c):
    """A symmetric CSR operator whose rows hold 3 to 9 entries (the 24 x 24
    Laplacian with symmetric couplings i <-> i + {37, 53, 71, 97} on every
    fifth row): rows of more than 8 entries rule out the fixed-width form, so
    the rows of up to 8 entries and the wider ones take the two CSR-walking
    paths of the term kernel.  Against the exact action from the
    eigendecomposition of A and against the oracle's action."""
    announce("expmv_leja wide rows", t, c)
    nx = 24
    n = nx * nx
    A = wl.laplacian_2d(nx).copy()
    for i in range(0, n, 5):
        for d in (37, 53, 71, 97):
            if i + d < n:
                A[i, i + d] = A[i + d, i] = 40.0
    widths = np.count_nonzero(A, axis=1)
    assert widths.max() > 8 and widths.min() <= 8
    X = np.random.default_rng(11 + c).standard_normal((n, c))
    Y, S, m = ctx.expmv_leja(csr(A), t, X)
    lam, U = np.linalg.eigh(A)
    ref = U @ (np.exp(t * lam)[:, None] * (U.T @ X))
    err = np.linalg.norm(to_np(Y) - ref) / np.linalg.norm(ref)
    print(f"  S {S} m {m} err {err:.2e}", flush=True)
    assert err < 1e-12
    ref_o = oracle.leja_expmv(A, t, X)
    assert np.linalg.norm(to_np(Y) - ref_o) <= 1e-12 * np.linalg.norm(ref)


def test_expmv_leja_rejects_nonsymmetric(ctx):
    A = wl.random_nonsymmetric(30, seed=4)
    X = np.ones((30, 2))
    for form in (A, csr(A)):
        with pytest.raises(b.DmeError) as e:
            ctx.expmv_leja(form, 1e-3, X)
        assert e.value.code == b.DME_EINVAL


def _solve(ctx, p, A=None, **kw):
    opts = b.SolveOptions(T=p.T, h=p.h, tol=p.tol, scheme=p.scheme, split=p.split,
                          quad_nodes=p.quad_nodes, **kw)
    return ctx.solve(p.kind, opts, p.A if A is None else A, p.C, B=p.B, R=p.R, S=p.S, L0=p.L0,
                     D0=p.D0, M=p.M)


def _oracle(p):
    return oracle.solve(p.A, p.C, p.T, p.h, kind=p.kind, B=p.B, R=p.R, S=p.S, L0=p.L0, D0=p.D0,
                        split=p.split, scheme=p.scheme, tol=p.tol, quad_nodes=p.quad_nodes, M=p.M)


@pytest.mark.parametrize("split", ["F12", "F1F2", "F1F3F2"])
@pytest.mark.parametrize("form", ["dense", "csr"])
def test_leja_solves_match_oracle(ctx, split, form):
    """DRE Strang with the operator action instead of the dense exponential,
    every split, 16 x 16 grid, h = 1e-2: the same P as the oracle's Pade
    route within 1e-10."""
    p = wl.config_dre_halfplane(nx=16, h=1e-2)
    p.split = split
    announce("leja solve", split, form)
    L, D, steps = _solve(ctx, p, A=(p.A if form == "dense" else csr(p.A)), action="leja")
    Lo, Do, info = _oracle(p)
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank {L.shape[1]} / {Lo.shape[1]} err {err:.2e}", flush=True)
    assert steps == info["steps"] and err < 1e-10


def test_leja_generalized_dre_csr_n4096(ctx):
    """Generalized DRE (T12 T3 T4 T3 T12) on the 64 x 64 grid with A in CSR
    form and the Leja action, 20 steps, against the oracle."""
    p = wl.config_gdre(nx=64, h=1e-3, T=0.02)
    announce("leja gdre n4096 csr")
    L, D, steps = _solve(ctx, p, A=csr(p.A), action="leja")
    A1 = wl.laplacian_1d(p.nx)
    Lo, Do, info = oracle.solve(p.A, p.C, p.T, p.h, kind=p.kind, B=p.B, R=p.R, S=p.S, split=p.split,
                                scheme=p.scheme, tol=p.tol,
                                expm_fn=lambda t: oracle.KronExpm(A1, t),
                                quad_fn=lambda t: oracle.quadrature_factor_kron(A1, p.C, t, 7, p.tol))
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank {L.shape[1]} / {Lo.shape[1]} err {err:.2e}", flush=True)
    assert steps == info["steps"] == 20 and err < 1e-10


def test_leja_rejects_bad_combinations(ctx):
    p = wl.config_dre_halfplane(nx=6, h=1e-2)
    with pytest.raises(b.DmeError) as e:
        _solve(ctx, p, action="leja", precision="mixed")
    assert e.value.code == b.DME_EINVAL
    q = wl.config_dre_halfplane(nx=6, h=1e-2)
    q.A = wl.random_nonsymmetric(36, seed=1, scale=10.0)
    with pytest.raises(b.DmeError) as e:
        _solve(ctx, q, action="leja")
    assert e.value.code == b.DME_EINVAL
    with pytest.raises(b.DmeError) as e:   # a CSR A needs the Leja action
        _solve(ctx, p, A=csr(p.A))
    assert e.value.code == b.DME_EINVAL


@pytest.mark.parametrize("nx,scheme,h", [(8, "strang", 1e-3), (8, "lie", 1e-3), (32, "strang", 2e-4)])
def test_mass_matrix_dre_matches_oracle(ctx, nx, scheme, h):
    """DRE in mass-matrix form (graded bilinear finite elements, M^T dP/dt M =
    A^T P M + M^T P A + Q - M^T P B R^-1 B^T P M) against the oracle."""
    p = wl.config_dre_mass(nx=nx, h=h, T=20 * h, scheme=scheme)
    announce("mass dre", nx, scheme)
    L, D, steps = _solve(ctx, p)
    Lo, Do, info = _oracle(p)
    err = oracle.lowrank_rel_err(L, D, Lo, Do)
    print(f"  rank {L.shape[1]} / {Lo.shape[1]} err {err:.2e}", flush=True)
    assert steps == info["steps"] == 20 and err < 1e-10


def test_mass_matrix_identity_equals_plain(ctx):
    p = wl.config_dre_halfplane(nx=8, h=1e-2)
    L1, D1, _ = _solve(ctx, p)
    p.M = np.eye(p.n)
    L2, D2, _ = _solve(ctx, p)
    assert oracle.lowrank_rel_err(L2, D2, L1, D1) < 1e-12
