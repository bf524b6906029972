"""Brute-force pins: the schemes against a high-accuracy Runge-Kutta solution
of the vectorised matrix ODE at n <= 25 (the paper's verification method,
Sec. 5.2, with a DOP853 integrator in place of ode15s), observed orders, and
invariants of the solution."""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle as o
import workloads as w


def _rk_reference(A, Q, T, G=None, S=None, P0=None):
    n = A.shape[0]
    P0 = np.zeros((n, n)) if P0 is None else P0

    def f(_, y):
        P = y.reshape(n, n)
        dP = A.T @ P + P @ A + Q
        if G is not None:
            dP -= P @ G @ P
        if S is not None:
            dP += S @ P @ S.T
        return dP.reshape(-1)

    sol = solve_ivp(f, (0.0, T), P0.reshape(-1), method="DOP853", rtol=1e-13, atol=1e-15)
    assert sol.success
    return sol.y[:, -1].reshape(n, n)


def _orders(errs):
    return [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


HS = (1e-2, 5e-3, 2.5e-3, 1.25e-3)


@pytest.fixture(scope="module")
def dre25():
    nx = 5
    A = w.laplacian_2d(nx)
    B = w.half_plane_B(nx)
    C = w.ones_C(nx * nx)
    R = np.eye(1)
    T = 0.1
    ref = _rk_reference(A, C.T @ C, T, G=B @ B.T)
    return A, B, C, R, T, ref


@pytest.mark.parametrize("split,scheme,order", [("F12", "lie", 1), ("F12", "strang", 2),
                                                ("F1F2", "strang", 2), ("F1F3F2", "strang", 2),
                                                ("F1F2", "lie", 1)])
def test_dre_observed_order(dre25, split, scheme, order):
    A, B, C, R, T, ref = dre25
    errs = []
    for h in HS:
        L, D, _ = o.solve(A, C, T, h, kind="dre", B=B, R=R, split=split, scheme=scheme,
                          tol=1e-14)
        errs.append(np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref))
    rates = _orders(errs)
    assert abs(rates[-1] - order) < 0.15, (errs, rates)
    assert errs[-1] < errs[0]


def test_generalized_dre_order_two():
    nx = 4
    n = nx * nx
    A = w.laplacian_2d(nx)
    B = w.half_plane_B(nx)
    C = w.ones_C(n)
    S = w.tridiag_S(n, 0.1) * 30.0    # make the S P S^T term visible at this size
    T = 0.1
    ref = _rk_reference(A, C.T @ C, T, G=B @ B.T, S=S)
    errs = []
    for h in HS:
        L, D, _ = o.solve(A, C, T, h, kind="dre", B=B, R=np.eye(1), S=S, split="F12",
                          scheme="strang", tol=1e-14)
        errs.append(np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref))
    rates = _orders(errs)
    assert abs(rates[-1] - 2.0) < 0.15, (errs, rates)


def test_generalized_dle_orders():
    nx = 4
    n = nx * nx
    A = w.laplacian_2d(nx)
    C = w.ones_C(n)
    S = w.tridiag_S(n, 0.1) * 30.0
    T = 0.1
    ref = _rk_reference(A, C.T @ C, T, S=S)
    for split, order in (("F12", 2), ("F1F2", 2), ("F1F3F2", 2)):
        errs = []
        for h in HS:
            L, D, _ = o.solve(A, C, T, h, kind="dle", S=S, split=split, scheme="strang",
                              tol=1e-14)
            errs.append(np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref))
        assert abs(_orders(errs)[-1] - order) < 0.15, (split, errs)


def test_nonsymmetric_dle_quadrature_exact():
    # Alg. 2 with a nonsymmetric A: only quadrature error remains, and it is tiny.
    # Using e^{tA} instead of e^{tA^T} would be off by O(1).
    n = 12
    A = w.random_nonsymmetric(n, seed=21, scale=3.0)
    C = w.random_C(2, n, seed=22)
    L0, D0 = w.random_lowrank_P0(n, 2, seed=23)
    T = 0.2
    ref = _rk_reference(A, C.T @ C, T, P0=L0 @ D0 @ L0.T)
    L, D, _ = o.solve(A, C, T, 0.05, kind="dle", split="F12", L0=L0, D0=D0, tol=1e-15)
    assert np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref) < 1e-11


def test_nonsymmetric_dre_strang_order():
    n = 10
    A = w.random_nonsymmetric(n, seed=31, scale=2.0)
    C = w.random_C(2, n, seed=32)
    B = w.random_C(2, n, seed=33).T.copy()
    R = np.diag([0.5, 2.0])
    T = 0.2
    ref = _rk_reference(A, C.T @ C, T, G=B @ np.linalg.solve(R, B.T))
    errs = []
    for h in (0.02, 0.01, 0.005):
        L, D, _ = o.solve(A, C, T, h, kind="dre", B=B, R=R, split="F12", scheme="strang",
                          tol=1e-15)
        errs.append(np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref))
    assert abs(_orders(errs)[-1] - 2.0) < 0.15, errs


def test_invariants_dre():
    p = w.config_dre_halfplane(12, h=2e-3, T=0.04)
    L, D, info = o.solve(p.A, p.C, p.T, p.h, kind="dre", B=p.B, R=p.R, tol=1e-10,
                         record_ranks=True)
    assert np.abs(D - D.T).max() == 0.0
    assert np.abs(L.T @ L - np.eye(L.shape[1])).max() < 1e-13  # last op compresses
    lam = np.linalg.eigvalsh(L @ D @ L.T)
    assert lam.min() >= -1e-10 * lam.max()
    assert max(info["ranks"]) <= p.n


def test_dle_monotone_from_zero():
    # P0 = 0 => P(t) is nondecreasing in the Loewner order for the DLE.
    p = w.config_dle_small(8)
    prev = None
    for T in (0.02, 0.04, 0.06):
        L, D, _ = o.solve(p.A, p.C, T, 2e-3, kind="dle", split="F12", tol=1e-14)
        P = L @ D @ L.T
        if prev is not None:
            assert np.linalg.eigvalsh(P - prev).min() > -1e-12 * np.abs(P).max()
        prev = P
