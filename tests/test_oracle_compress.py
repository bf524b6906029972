"""Pins for column compression and the low-rank error metric."""
import numpy as np
import pytest

import oracle as o


def _rand_lowrank(n, k, seed, decay=0.5):
    rng = np.random.default_rng(seed)
    L = rng.standard_normal((n, k))
    D = np.diag(decay ** np.arange(k))
    return L, D


def test_full_rank_exact():
    L, D = _rand_lowrank(50, 8, 1)
    Lc, Dc = o.compress(L, D, tol=1e-14)
    assert Lc.shape[1] == 8
    assert np.linalg.norm(Lc @ Dc @ Lc.T - L @ D @ L.T) < 1e-12 * np.linalg.norm(L @ D @ L.T)
    assert np.abs(Lc.T @ Lc - np.eye(8)).max() < 1e-13
    lam = np.diag(Dc)
    assert np.all(np.diff(np.abs(lam)) <= 0)  # sorted by |lam| descending
    assert np.abs(Dc - np.diag(lam)).max() == 0.0


def test_truncation_drops_small_eigenvalues():
    # P = U diag(l) U^T with known eigenvalues; tol removes exactly those below.
    rng = np.random.default_rng(2)
    U, _ = np.linalg.qr(rng.standard_normal((40, 10)))
    lam = np.array([1.0, 0.5, 1e-3, 1e-6, 1e-9, 2e-11, 1e-12, 1e-14, 0.0, 0.0])
    L = U @ np.diag(np.sqrt(lam))
    # duplicate columns make L rank-deficient like a concatenation does
    Lc, Dc = o.compress(np.hstack([L, L[:, :3]]), np.eye(13), tol=1e-10)
    assert Lc.shape[1] == 5
    np.testing.assert_allclose(np.sort(np.diag(Dc))[::-1], [2.0, 1.0, 2e-3, 1e-6, 1e-9], rtol=1e-6)
    P = L @ L.T + L[:, :3] @ L[:, :3].T
    err = np.linalg.norm(Lc @ Dc @ Lc.T - P)
    assert err == pytest.approx(np.sqrt(2e-11 ** 2 + 1e-12 ** 2 + 1e-14 ** 2), rel=1e-3)


def test_indefinite_and_zero():
    rng = np.random.default_rng(3)
    L = rng.standard_normal((20, 4))
    D = np.diag([1.0, -2.0, 0.5, 0.0])
    Lc, Dc = o.compress(L, D, 1e-12)
    assert Lc.shape[1] == 3
    assert np.linalg.norm(Lc @ Dc @ Lc.T - L @ D @ L.T) < 1e-12 * np.linalg.norm(L @ D @ L.T)
    assert abs(Dc[0, 0]) == np.abs(np.diag(Dc)).max()
    Lz, Dz = o.compress(np.zeros((7, 3)), np.eye(3), 1e-10)
    assert Lz.shape == (7, 0) and Dz.shape == (0, 0)
    Le, De = o.compress(np.zeros((7, 0)), np.zeros((0, 0)), 1e-10)
    assert Le.shape == (7, 0)


def test_nondiagonal_D():
    rng = np.random.default_rng(4)
    L = rng.standard_normal((30, 6))
    G = rng.standard_normal((6, 6))
    D = G @ G.T
    Lc, Dc = o.compress(L, D, 1e-14)
    assert np.linalg.norm(Lc @ Dc @ Lc.T - L @ D @ L.T) < 1e-12 * np.linalg.norm(L @ D @ L.T)


def test_lowrank_error_metric_matches_dense():
    rng = np.random.default_rng(5)
    L1, D1 = _rand_lowrank(60, 5, 6)
    L2 = L1 + 1e-3 * rng.standard_normal(L1.shape)
    D2 = D1.copy()
    D2[0, 0] *= 1.01
    P1 = L1 @ D1 @ L1.T
    P2 = L2 @ D2 @ L2.T
    ref = np.linalg.norm(P1 - P2) / np.linalg.norm(P2)
    assert o.lowrank_rel_err(L1, D1, L2, D2) == pytest.approx(ref, rel=1e-9)
    assert o.lowrank_fro(L1, D1) == pytest.approx(np.linalg.norm(P1), rel=1e-12)
    assert o.lowrank_rel_err(L1, D1, L1, D1) < 1e-14
