"""Parity of each hot-path kernel (through the C ABI) with numpy / the oracle."""
import numpy as np
import pytest

import oracle
import workloads as wl
from tests.gpu_common import announce, rel_fro, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,N,K,ta,tb", [
    (64, 64, 64, "N", "N"), (200, 150, 130, "N", "N"), (129, 65, 300, "T", "N"),
    (33, 257, 17, "N", "T"), (70, 90, 1000, "T", "T"), (1, 1, 1, "N", "N"),
    (32, 40, 5000, "T", "N"), (1000, 7, 1000, "N", "N"), (256, 256, 0, "N", "N"),
    # the small-product path at its limits (M, N <= 256, K <= 2048), ragged
    (256, 256, 2048, "T", "T"), (250, 17, 2047, "N", "T"), (178, 178, 178, "T", "N"),
    # few tiles and a long K (L^T B of the Riccati step): K split over the grid
    (122, 4, 16384, "T", "N"), (33, 40, 5000, "T", "N"), (16, 16, 2049, "N", "N"), (64, 64, 70001, "T", "T"),
    # tall-square times narrow: the skinny split-K path (ragged rows, K and N)
    (2048, 150, 2048, "N", "N"), (1500, 7, 1100, "N", "N"), (4097, 256, 3000, "N", "N"),
    (1024, 33, 1024, "N", "N"),
])
def test_gemm_f64(ctx, M, N, K, ta, tb):
    announce("gemm", M, N, K, ta, tb)
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((K, M) if ta == "T" else (M, K))
    B = rng.standard_normal((N, K) if tb == "T" else (K, N))
    C = rng.standard_normal((M, N))
    opA = A.T if ta == "T" else A
    opB = B.T if tb == "T" else B
    got = to_np(ctx.gemm(A, B, alpha=0.75, beta=-0.5, C=C, transa=ta, transb=tb))
    ref = 0.75 * opA @ opB - 0.5 * C
    assert rel_fro(got, ref) < 1e-13
    # entrywise: the dot-product error bound, K units of roundoff on |A||B| (+ |C|)
    scale = 0.75 * np.abs(opA) @ np.abs(opB) + 0.5 * np.abs(C)
    assert np.all(np.abs(got - ref) <= (K + 2) * 2.3e-16 * scale)


@pytest.mark.parametrize("n,k,beta", [(2048, 178, 0.0), (16384, 192, 0.0), (5000, 33, -0.5), (3001, 1, 0.0),
                                       (70000, 120, 0.0), (16384, 176, 0.5)])
def test_gemm_gram(ctx, n, k, beta):
    """A^T A of a tall A (the compression's W^T W): the symmetric Gram path,
    ragged row blocks and tiles; the result is exactly symmetric."""
    announce("gemm gram", n, k, beta)
    rng = np.random.default_rng(n + k)
    W = rng.standard_normal((n, k))
    C = rng.standard_normal((k, k))
    C = C + C.T
    got = to_np(ctx.gemm(W, W, alpha=0.75, beta=beta, C=C, transa="T"))
    ref = 0.75 * W.T @ W + beta * C
    assert rel_fro(got, ref) < 1e-13
    assert np.array_equal(got, got.T)


def test_gemm_beta_zero_ignores_nan(ctx):
    announce("gemm beta0 nan")
    rng = np.random.default_rng(1)
    A, B = rng.standard_normal((50, 40)), rng.standard_normal((40, 30))
    C = np.full((50, 30), np.nan)
    got = to_np(ctx.gemm(A, B, beta=0.0, C=C))
    assert np.all(np.isfinite(got)) and rel_fro(got, A @ B) < 1e-14


@pytest.mark.parametrize("nx,t", [(16, 5e-4), (16, 1e-6), (16, 2e-5), (16, 1e-3), (16, 2e-2), (10, 1e-1)])
def test_expm_laplacian(ctx, nx, t):
    announce("expm laplacian", nx, t)
    A = wl.laplacian_2d(nx)
    E, m, s = ctx.expm(A.T, t)
    ref = oracle.expm(t * A.T)
    mo, so = oracle.expm_params(oracle.norm1(t * A.T))
    assert (m, s) == (mo, so)
    assert rel_fro(to_np(E), ref) < 1e-12


@pytest.mark.parametrize("n,t", [(100, 1.0), (130, 0.05), (1, 2.0), (257, 0.3)])
def test_expm_nonsymmetric(ctx, n, t):
    announce("expm nonsym", n, t)
    X = wl.random_nonsymmetric(n, seed=n)
    E, m, s = ctx.expm(X, t)
    assert rel_fro(to_np(E), oracle.expm(t * X)) < 1e-12


def _sym_with_spectrum(k, lam, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (Q * lam) @ Q.T


@pytest.mark.parametrize("case", ["random", "graded", "clusters", "psd_lowrank", "k2", "k1", "k150",
                                  "k180", "k300", "k600"])
def test_syev(ctx, case):
    announce("syev", case)
    rng = np.random.default_rng(5)
    if case == "random":
        k = 60
        X = rng.standard_normal((k, k)); M = 0.5 * (X + X.T)
    elif case == "graded":
        k = 120
        M = _sym_with_spectrum(k, 10.0 ** -rng.uniform(0, 12, k), 2)
    elif case == "clusters":
        k = 50
        lam = np.repeat([3.0, 2.0, 1.0, 0.5, -1.0], 10)
        M = _sym_with_spectrum(k, lam, 3)
    elif case == "psd_lowrank":
        k = 80
        F = rng.standard_normal((k, 20)); M = F @ F.T
    elif case == "k2":
        k = 2
        M = np.array([[2.0, 1.0], [1.0, 3.0]])
    elif case == "k1":
        k = 1
        M = np.array([[-4.0]])
    elif case == "k150":  # register-resident reduction sizes
        k = 150
        M = _sym_with_spectrum(k, np.exp(-0.15 * np.arange(k)) * np.where(np.arange(k) % 7 == 3, -1, 1), 6)
    elif case == "k180":
        k = 180
        F = rng.standard_normal((k, 120)); M = F @ np.diag(10.0 ** -np.linspace(0, 9, 120)) @ F.T
    elif case == "k300":  # LDS-staged reduction
        k = 300
        M = _sym_with_spectrum(k, np.exp(-0.1 * np.arange(k)), 4)
    else:  # global-memory reduction
        k = 600
        X = rng.standard_normal((k, k)); M = 0.5 * (X + X.T)
    tol = 1e-12
    lam, V, kk = ctx.syev(M, tol=tol)
    lam, V = to_np(lam), to_np(V)
    ref = np.linalg.eigvalsh(M)
    ref = ref[np.argsort(-np.abs(ref), kind="stable")]
    keep = np.abs(ref) > tol * np.abs(ref).max()
    assert kk == int(keep.sum())
    nrm = np.abs(ref).max()
    bound = 1e-13 * nrm * max(1, np.sqrt(k))
    # equal |lambda| may come in either order: compare the sets, then the order
    assert np.max(np.abs(np.sort(lam[:kk]) - np.sort(ref[:kk]))) < bound
    assert np.max(np.abs(np.sort(lam) - np.sort(ref))) < bound
    assert np.all(np.abs(lam[1:kk]) <= np.abs(lam[:kk - 1]) + bound)
    # kept part reproduces M up to the dropped eigenvalues
    Mk = (V * lam[:kk]) @ V.T
    drop = np.sqrt(np.sum(ref[kk:] ** 2))
    assert np.linalg.norm(Mk - M) <= 1e-12 * np.linalg.norm(M) + 1.01 * drop
    orth = np.max(np.abs(V.T @ V - np.eye(kk))) if kk else 0.0
    print(f"  max |V^T V - I| {orth:.2e}", flush=True)
    assert orth < 1e-12 * max(1, np.sqrt(k))


@pytest.mark.parametrize("k", [3, 33, 64, 65, 96, 128, 129, 160, 161, 191, 192, 193])
def test_syev_tile_sizes(ctx, k):
    """Sizes at the edges of the register-tiled reductions (k <= 64, 128, 160, 192)."""
    announce("syev size", k)
    rng = np.random.default_rng(100 + k)
    X = rng.standard_normal((k, k))
    M = 0.5 * (X + X.T)
    lam, V, kk = ctx.syev(M, tol=1e-14)
    lam, V = to_np(lam), to_np(V)
    ref = np.linalg.eigvalsh(M)
    assert kk == k
    bound = 1e-13 * np.abs(ref).max() * np.sqrt(k)
    assert np.max(np.abs(np.sort(lam) - np.sort(ref))) < bound
    assert np.linalg.norm((V * lam) @ V.T - M) <= 1e-12 * np.linalg.norm(M) * np.sqrt(k)
    orth = np.max(np.abs(V.T @ V - np.eye(k)))
    print(f"  max |V^T V - I| {orth:.2e}", flush=True)
    assert orth < 1e-12 * np.sqrt(k)


def _compress_case(name):
    rng = np.random.default_rng(11)
    if name == "random":
        n, k = 300, 40
        W = rng.standard_normal((n, k)); F = rng.standard_normal((k, k)); Dh = F @ F.T / k
    elif name == "rankdef":
        n, k = 500, 60
        W = rng.standard_normal((n, 20)) @ rng.standard_normal((20, k)); Dh = np.diag(rng.uniform(0.5, 2, k))
    elif name == "wide":
        n, k = 20, 33
        W = rng.standard_normal((n, k)); Dh = np.diag(rng.uniform(0.1, 1, k))
    elif name == "zero":
        n, k = 64, 5
        W = rng.standard_normal((n, k)); Dh = np.zeros((k, k))
    elif name == "identity":
        n, k = 200, 30
        W, _ = np.linalg.qr(rng.standard_normal((n, k))); Dh = np.eye(k)
    elif name == "graded":
        n, k = 1000, 100
        W = rng.standard_normal((n, k)) * (10.0 ** -np.linspace(0, 9, k)); Dh = np.eye(k)
    elif name == "tall_multi_panel":
        n, k = 4097, 97
        W = rng.standard_normal((n, k)) / np.sqrt(n); Dh = np.diag(np.exp(-0.2 * np.arange(k)))
    elif name == "tree_ragged":  # tree QR: last block 476 rows, last panel 6 columns
        n, k = 1500, 70
        W = rng.standard_normal((n, k)) * (10.0 ** -np.linspace(0, 6, k)); Dh = np.eye(k)
    elif name == "tree_two_levels":  # product-like columns, rank-deficient
        n, k = 2048, 200
        W = rng.standard_normal((n, 150)) @ rng.standard_normal((150, k)) / np.sqrt(n)
        F = rng.standard_normal((k, k)); Dh = F @ F.T / k
    elif name == "tree_full_size":  # n of the headline workload: three tree levels
        n, k = 16384, 180
        W = rng.standard_normal((n, k)) / np.sqrt(n) * np.exp(-0.05 * np.arange(k)); Dh = np.eye(k)
    else:
        raise KeyError(name)
    return W, Dh


@pytest.mark.parametrize("name", ["random", "rankdef", "wide", "zero", "identity", "graded",
                                  "tall_multi_panel", "tree_ragged", "tree_two_levels",
                                  "tree_full_size"])
def test_compress_matches_oracle(ctx, name):
    announce("compress", name)
    W, Dh = _compress_case(name)
    tol = 1e-10
    L, D = ctx.compress(W, Dh, tol)
    L, D = to_np(L), to_np(D)
    Lo, Do = oracle.compress(W, Dh, tol)
    assert L.shape[1] == Lo.shape[1]
    if Lo.shape[1] == 0:
        return
    assert oracle.lowrank_rel_err(L, D, Lo, Do) < 1e-11
    # L^T L = I up to the Gram route's error: entry (i, j) is off by about
    # eps ||G|| / sqrt(lam_i lam_j) (G = W^T W-type Gram matrix, lam = diag D),
    # so the scaled deviation is a roundoff-level quantity for every column
    lam = np.abs(np.diag(D))
    dev = np.abs(L.T @ L - np.eye(L.shape[1])) * np.sqrt(np.outer(lam, lam))
    print(f"  scaled max |L^T L - I| {dev.max() / lam.max():.2e}, unscaled "
          f"{np.abs(L.T @ L - np.eye(L.shape[1])).max():.2e}", flush=True)
    assert dev.max() <= 1e-13 * lam.max() * L.shape[1]
    assert np.max(np.abs(L.T @ L - np.eye(L.shape[1]))) < 1e-11


@pytest.mark.parametrize("n,r,m", [(200, 12, 1), (300, 40, 4), (50, 3, 2), (4096, 60, 4)])
def test_riccati_matches_oracle(ctx, n, r, m):
    announce("riccati", n, r, m)
    rng = np.random.default_rng(n + r)
    L = rng.standard_normal((n, r)) / np.sqrt(n)
    F = rng.standard_normal((r, r)); D = F @ F.T
    B = rng.standard_normal((n, m))
    G = rng.standard_normal((m, m)); R = G @ G.T + m * np.eye(m)
    t = 1e-2
    got = to_np(ctx.riccati(L, B, R, t, D))
    ref = oracle.t3(L, D, B, R, t)
    assert rel_fro(got, ref) < 1e-12


@pytest.mark.parametrize("n,r", [(1, 1), (31, 7), (257, 16), (1000, 150), (2304, 33), (1296, 300)])
def test_gemm_mixed(ctx, n, r):
    """Split-BF16 product: error bounded by the FP32 representation of E and X
    plus FP32 chunk accumulation, elementwise against |E||X|."""
    announce("gemm_mixed", n, r)
    rng = np.random.default_rng(n + r)
    E = rng.standard_normal((n, n)) / np.sqrt(n)
    X = rng.standard_normal((n, r))
    got = to_np(ctx.gemm_mixed(E, X))
    ref = E @ X
    scale = np.abs(E) @ np.abs(X)
    # FP32 representation of E and X plus the dropped piece products: a few
    # units of 2^-24 of |E||X| per entry (FP64 accumulation across K steps)
    assert np.all(np.abs(got - ref) <= 4e-7 * scale + 1e-300)
    assert rel_fro(got, ref) < 1e-6


def test_gemm_mixed_heat_operator(ctx):
    """On the heat semigroup of the 2-D Laplacian (the operator the mixed mode
    applies) the relative error of E L stays near FP32 resolution: the FP32
    representation of E and X (2^-24 per entry) plus FP32 accumulation over
    128-term spans."""
    announce("gemm_mixed heat")
    A = wl.laplacian_2d(24)
    E = oracle.expm(5e-4 * A.T)
    rng = np.random.default_rng(3)
    X, _ = np.linalg.qr(rng.standard_normal((A.shape[0], 40)))
    got = to_np(ctx.gemm_mixed(E, X))
    assert rel_fro(got, E @ X) < 2e-7
