"""Pins for the subflow solvers T1, T2, T3 (Alg. 3) and T4 (Alg. 4)."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as o
import workloads as w


def _psd_factor(n, r, seed):
    return w.random_lowrank_P0(n, r, seed)


def test_t3_equals_dense_formula():
    # T3(t) P = (I + t P B R^-1 B^T)^-1 P  (Sec. 2.2, eq. nonlinear)
    n, r, m = 30, 5, 2
    L, D = _psd_factor(n, r, 1)
    rng = np.random.default_rng(2)
    B = rng.standard_normal((n, m))
    G0 = rng.standard_normal((m, m))
    R = G0 @ G0.T + m * np.eye(m)
    t = 0.3
    Dn = o.t3(L, D, B, R, t)
    P = L @ D @ L.T
    ref = np.linalg.solve(np.eye(n) + t * P @ B @ np.linalg.solve(R, B.T), P)
    assert np.linalg.norm(L @ Dn @ L.T - ref) < 1e-13 * np.linalg.norm(ref)
    assert np.abs(Dn - Dn.T).max() == 0.0


def test_t3_semigroup_and_ode():
    n, r = 20, 4
    L, D = _psd_factor(n, r, 3)
    B = w.random_C(2, n, 4).T.copy()
    R = np.diag([0.5, 2.0])
    a, b = 0.2, 0.5
    D_ab = o.t3(L, o.t3(L, D, B, R, a), B, R, b)
    D_sum = o.t3(L, D, B, R, a + b)
    assert np.abs(D_ab - D_sum).max() < 1e-13 * np.abs(D_sum).max()
    # derivative: d/dt T3(t)P at t=0 equals -P B R^-1 B^T P
    P = L @ D @ L.T
    eps = 1e-6
    dP = (L @ o.t3(L, D, B, R, eps) @ L.T - L @ o.t3(L, D, B, R, -eps) @ L.T) / (2 * eps)
    ref = -P @ B @ np.linalg.solve(R, B.T) @ P
    assert np.linalg.norm(dP - ref) < 1e-6 * np.linalg.norm(ref)


def test_t3_woodbury_form():
    # the m x m form D - tDW(R + tW^T D W)^-1 W^T D, W = L^T B, is the same map
    n, r, m = 25, 6, 3
    L, D = _psd_factor(n, r, 5)
    B = np.random.default_rng(6).standard_normal((n, m))
    R = np.diag([1.0, 0.3, 3.0])
    t = 0.7
    W = L.T @ B
    wood = D - t * D @ W @ np.linalg.solve(R + t * W.T @ D @ W, W.T @ D)
    assert np.abs(o.t3(L, D, B, R, t) - wood).max() < 1e-13 * np.abs(wood).max()


def test_t3_empty():
    D = o.t3(np.zeros((5, 0)), np.zeros((0, 0)), np.ones((5, 1)), np.eye(1), 0.1)
    assert D.shape == (0, 0)


def test_t4_midpoint_formula():
    # T4(t)P = P + t S P S^T + t^2/2 S^2 P (S^2)^T (Sec. 2.3), before truncation
    n, r = 24, 3
    L, D = _psd_factor(n, r, 7)
    S = w.tridiag_S(n, 0.1) + 0.05 * np.random.default_rng(8).standard_normal((n, n))
    t = 0.4
    Ln, Dn = o.t4(L, D, S, t, tol=1e-15)
    P = L @ D @ L.T
    S2 = S @ S
    ref = P + t * S @ P @ S.T + 0.5 * t * t * S2 @ P @ S2.T
    assert np.linalg.norm(Ln @ Dn @ Ln.T - ref) < 1e-13 * np.linalg.norm(ref)
    # second-order accurate for the linear flow dP/dt = S P S^T
    n2 = 6
    S = np.random.default_rng(9).standard_normal((n2, n2)) * 0.5
    P0 = np.eye(n2)
    Kop = np.kron(S, S)  # vec(S P S^T) = (S (x) S) vec(P) (column-major vec)
    errs = []
    for t in (0.1, 0.05):
        ex = (sl.expm(t * Kop) @ P0.reshape(-1, order="F")).reshape(n2, n2, order="F")
        Ln, Dn = o.t4(np.eye(n2), np.eye(n2), S, t, tol=1e-15)
        errs.append(np.linalg.norm(Ln @ Dn @ Ln.T - ex))
    assert math.log2(errs[0] / errs[1]) == pytest.approx(3.0, abs=0.3)  # local error O(t^3)


def test_t2_and_t1():
    n = 16
    L, D = _psd_factor(n, 2, 10)
    C = w.random_C(3, n, 11)
    t = 0.25
    Ln, Dn = o.t2(L, D, C, t, tol=1e-15)
    ref = L @ D @ L.T + t * C.T @ C
    assert np.linalg.norm(Ln @ Dn @ Ln.T - ref) < 1e-13 * np.linalg.norm(ref)
    A = w.random_nonsymmetric(n, 12)
    E = o.expm(0.1 * A.T)
    P = L @ D @ L.T
    L1 = o.t1(L, E)
    ref = sl.expm(0.1 * A.T) @ P @ sl.expm(0.1 * A)
    assert np.linalg.norm(L1 @ D @ L1.T - ref) < 1e-13 * np.linalg.norm(ref)


def test_feedback_gain_basis_invariance_and_R():
    """K = R^-1 B^T L D L^T depends on P = L D L^T only, and scales as R^-1."""
    rng = np.random.default_rng(11)
    n, r, m = 30, 5, 3
    L = rng.standard_normal((n, r))
    D = np.diag(rng.uniform(0.5, 2.0, r))
    B = rng.standard_normal((n, m))
    R = np.diag([1.0, 2.0, 4.0])
    K = o.feedback_gain(L, D, B, R)
    assert K.shape == (m, n)
    G = np.linalg.qr(rng.standard_normal((r, r)))[0] @ np.diag(np.linspace(1.0, 2.0, r))  # cond 2
    Gi = np.linalg.inv(G)
    K2 = o.feedback_gain(L @ G, Gi @ D @ Gi.T, B, R)
    assert np.allclose(K, K2, rtol=1e-12, atol=1e-12)
    K3 = o.feedback_gain(L, D, B, 0.5 * R)
    assert np.allclose(K3, 2.0 * K, rtol=1e-13, atol=1e-13)
    assert np.array_equal(o.feedback_gain(L[:, :0], D[:0, :0], B, R), np.zeros((m, n)))


def test_feedback_gain_scalar_closed_form():
    """n = 1: p' = 2 a p + c^2 - (b^2 / r) p^2, p(0) = 0, has
    p(t) = c^2 sinh(mu t) / (mu cosh(mu t) - a sinh(mu t)), mu = sqrt(a^2 + b^2 c^2 / r),
    and K(t) = b p(t) / r; the Strang solution's gain is second-order close."""
    a, b, c, r, T = -1.0, 0.7, 1.3, 2.0, 0.5
    mu = math.sqrt(a * a + b * b * c * c / r)
    p_exact = c * c * math.sinh(mu * T) / (mu * math.cosh(mu * T) - a * math.sinh(mu * T))
    errs = []
    for h in (0.05, 0.025):
        L, D, _ = o.solve(np.array([[a]]), np.array([[c]]), T, h, kind="dre", B=np.array([[b]]),
                          R=np.array([[r]]), split="F12", scheme="strang", tol=1e-14)
        K = o.feedback_gain(L, D, np.array([[b]]), np.array([[r]]))
        errs.append(abs(K[0, 0] - b * p_exact / r))
    assert errs[1] < 1e-3 * abs(b * p_exact / r)
    assert 3.0 < errs[0] / errs[1] < 5.0  # second order
