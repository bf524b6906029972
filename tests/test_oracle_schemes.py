"""Pins for the splitting schemes: discrete closed forms in the Laplacian
eigenbasis (DLE) and exact scalar recursions in commuting DRE cases."""
import math

import numpy as np
import pytest

import oracle as o
import workloads as w
from tests.laplace_closed_form import eig2d


def _dle_closed_form(nx, C, h, N, kind):
    lam, V = eig2d(nx)
    mu = lam[:, None] + lam[None, :]
    Qt = V.T @ (C.T @ C) @ V
    geo = (1.0 - np.exp(mu * h * N)) / (1.0 - np.exp(mu * h))
    if kind == "lie":        # T2(h) T1(h)
        F = h * geo
    elif kind == "strang":   # T1(h/2) T2(h) T1(h/2)  (Alg. 1)
        F = h * np.exp(mu * h / 2) * geo
    elif kind == "quad":     # Alg. 2 with K-point GL on [0, h]
        s, wt = o.gauss_legendre(7, h)
        F = sum(wk * np.exp(mu * sk) for sk, wk in zip(s, wt)) * geo
    return V @ (Qt * F) @ V.T


@pytest.mark.parametrize("split,scheme,kind", [("F1F2", "strang", "strang"),
                                                ("F1F2", "lie", "lie"),
                                                ("F12", "strang", "quad")])
def test_dle_discrete_closed_form_config_small(split, scheme, kind):
    # 16x16 Laplacian, C = ones, P0 = 0, T = 0.1, h = 1e-3, tol 1e-12.
    p = w.config_dle_small()
    L, D, info = o.solve(p.A, p.C, p.T, p.h, kind="dle", split=split, scheme=scheme,
                         tol=p.tol)
    ref = _dle_closed_form(16, p.C, p.h, 100, kind)
    err = np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref)
    assert err < 1e-10
    assert info["steps"] == 100


def test_dle_splitting_error_size():
    # Strang F1F2 differs from the exact solution (eq. full) by its splitting
    # error; the quadrature method is exact to quadrature accuracy.
    nx, h, T = 16, 1e-3, 0.1
    p = w.config_dle_small(nx)
    lam, V = eig2d(nx)
    mu = lam[:, None] + lam[None, :]
    Qt = V.T @ (p.C.T @ p.C) @ V
    exact = V @ (Qt * (np.expm1(mu * T) / mu)) @ V.T
    for split, lo, hi in (("F1F2", 1e-4, 1e-3), ("F12", 0.0, 1e-12)):
        L, D, _ = o.solve(p.A, p.C, T, h, kind="dle", split=split, scheme="strang", tol=1e-12)
        err = np.linalg.norm(L @ D @ L.T - exact) / np.linalg.norm(exact)
        assert lo <= err < hi, (split, err)


def _commuting_setup(nx, modes_B, modes_C, q, g):
    n = nx * nx
    B = np.stack([w.sine_mode(nx, a, b) for a, b in modes_B], axis=1) * np.sqrt(g)[None, :]
    C = np.stack([w.sine_mode(nx, a, b) for a, b in modes_C], axis=0) * np.sqrt(q)[:, None]
    return B, C


def _scalar_recursion(lam, q, g, h, N, seq, quad_nodes=7):
    """Per-mode recursion of the scheme when Q and B R^-1 B^T are diagonal in
    the eigenbasis: T1: p <- e^{2 lam t} p; T2: p <- p + t q;
    T12: p <- e^{2 lam t} p + q sum_k w_k e^{2 lam s_k}; T3: p <- p/(1 + t g p)."""
    p = 0.0
    for _ in range(N):
        for name, frac in seq:
            t = frac * h
            if name == "T1":
                p = math.exp(2 * lam * t) * p
            elif name == "T2":
                p = p + t * q
            elif name == "T12":
                s, wt = o.gauss_legendre(quad_nodes, t)
                p = math.exp(2 * lam * t) * p + q * float(np.sum(wt * np.exp(2 * lam * s)))
            elif name == "T3":
                p = p / (1.0 + t * g * p)
    return p


@pytest.mark.parametrize("split,scheme", [("F12", "strang"), ("F12", "lie"),
                                          ("F1F2", "strang"), ("F1F2", "lie"),
                                          ("F1F3F2", "strang"), ("F1F3F2", "lie")])
def test_dre_commuting_modes(split, scheme):
    nx, h, T = 12, 2e-3, 0.06
    modes = [(1, 1), (1, 3), (2, 1)]
    q = np.array([40.0, 25.0, 10.0])
    g = np.array([3.0, 0.0, 8.0])          # mode (1,3) has no control
    B, C = _commuting_setup(nx, modes, modes, q, g)
    R = np.eye(B.shape[1])
    A = w.laplacian_2d(nx)
    L, D, info = o.solve(A, C, T, h, kind="dre", B=B, R=R, split=split, scheme=scheme,
                         tol=1e-14)
    lam, _ = eig2d(nx)
    ref = np.zeros((nx * nx, nx * nx))
    for (a, b), qi, gi in zip(modes, q, g):
        v = w.sine_mode(nx, a, b)
        lm = lam[(a - 1) + nx * (b - 1)]
        pm = _scalar_recursion(lm, qi, gi, h, info["steps"], info["sequence"])
        ref += pm * np.outer(v, v)
    err = np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref)
    assert err < 1e-12, err


def test_dre_commuting_continuous_limit():
    # the scalar Riccati ODE p' = 2 lam p + q - g p^2, p(0)=0, has the solution
    # p(t) = q sinh(bt) / (b cosh(bt) - lam sinh(bt)), b = sqrt(lam^2 + g q);
    # the Strang F12F3 scheme converges to it with order 2.
    nx = 8
    modes = [(1, 1)]
    q, g = np.array([30.0]), np.array([5.0])
    B, C = _commuting_setup(nx, modes, modes, q, g)
    A = w.laplacian_2d(nx)
    lam, _ = eig2d(nx)
    lm = lam[0]
    T = 0.08
    beta = math.sqrt(lm * lm + g[0] * q[0])
    pex = q[0] * math.sinh(beta * T) / (beta * math.cosh(beta * T) - lm * math.sinh(beta * T))
    v = w.sine_mode(nx, 1, 1)
    errs = []
    for h in (4e-3, 2e-3, 1e-3):
        L, D, _ = o.solve(A, C, T, h, kind="dre", B=B, R=np.eye(1), split="F12",
                          scheme="strang", tol=1e-14)
        errs.append(abs(v @ L @ D @ L.T @ v - pex) / pex)
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(r - 2.0) < 0.1 for r in rates), rates


def test_generalized_commuting_S():
    # S = 0.1 (I (x) tridiag(1,0,1)) commutes with A: eigenvalue sigma = 0.2 cos(a pi/(nx+1)),
    # so T4(t): p <- p (1 + t sigma^2 + t^2 sigma^4 / 2).
    nx, h, T = 10, 2e-3, 0.04
    modes = [(1, 1), (2, 3)]
    q = np.array([20.0, 12.0])
    g = np.array([2.0, 4.0])
    B, C = _commuting_setup(nx, modes, modes, q, g)
    S = 0.1 * np.kron(np.eye(nx), w.tridiag_1d(nx, diag=0.0, off=1.0))
    A = w.laplacian_2d(nx)
    L, D, info = o.solve(A, C, T, h, kind="dre", B=B, R=np.eye(2), S=S, split="F12",
                         scheme="strang", tol=1e-14)
    lam, _ = eig2d(nx)
    ref = 0.0
    for (a, b), qi, gi in zip(modes, q, g):
        lm = lam[(a - 1) + nx * (b - 1)]
        sig2 = (0.2 * math.cos(a * math.pi / (nx + 1))) ** 2
        p = 0.0
        for _ in range(info["steps"]):
            for name, frac in info["sequence"]:
                t = frac * h
                if name == "T12":
                    s, wt = o.gauss_legendre(7, t)
                    p = math.exp(2 * lm * t) * p + qi * float(np.sum(wt * np.exp(2 * lm * s)))
                elif name == "T3":
                    p = p / (1.0 + t * gi * p)
                elif name == "T4":
                    p = p * (1.0 + t * sig2 + 0.5 * t * t * sig2 * sig2)
        v = w.sine_mode(nx, a, b)
        ref = ref + p * np.outer(v, v)
    err = np.linalg.norm(L @ D @ L.T - ref) / np.linalg.norm(ref)
    assert err < 1e-12, err


def test_step_sequences():
    seq = o.step_sequence
    assert seq("dle", False, "F12", "strang") == [("T12", 1.0)]
    assert seq("dle", False, "F1F2", "strang") == [("T1", 0.5), ("T2", 1.0), ("T1", 0.5)]
    assert seq("dre", False, "F12", "strang") == [("T12", 0.5), ("T3", 1.0), ("T12", 0.5)]
    assert seq("dre", False, "F12", "lie") == [("T12", 1.0), ("T3", 1.0)]
    assert seq("dre", True, "F12", "strang") == [("T12", 0.5), ("T3", 0.5), ("T4", 1.0),
                                                 ("T3", 0.5), ("T12", 0.5)]
    assert seq("dre", False, "F1F3F2", "strang") == [("T1", 0.5), ("T3", 0.5), ("T2", 1.0),
                                                     ("T3", 0.5), ("T1", 0.5)]
    with pytest.raises(o.OracleError):
        seq("dre", True, "F1F2", "strang")
    with pytest.raises(o.OracleError):
        o.num_steps(0.1, 0.03)
    assert o.num_steps(0.1, 1e-3) == 100
