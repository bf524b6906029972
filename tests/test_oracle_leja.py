"""Pins for the Leja-interpolation action e^{tA} V of the oracle (the paper's
expleja, Sec. 3 and Sec. 4): Gershgorin interval, Leja points, divided
differences of the exponential, and the action against the exact one."""
import math

import numpy as np
import pytest

import oracle as o
from oracle import dme_oracle as od
import workloads as w
from tests.laplace_closed_form import eig2d


def _sym(n, seed, shift=0.0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, n))
    return 0.5 * (X + X.T) + shift * np.eye(n)


def test_gershgorin_contains_spectrum_and_laplacian_closed_form():
    for seed in range(4):
        A = _sym(30, seed, shift=-3.0)
        a, b = o.gershgorin_interval(A)
        lam = np.linalg.eigvalsh(A)
        assert a <= lam.min() and lam.max() <= b
    nx = 9
    dx = 1.0 / (nx + 1)
    a, b = o.gershgorin_interval(w.laplacian_2d(nx))
    assert abs(a + 8.0 / dx ** 2) < 1e-9 and abs(b) < 1e-9


def test_leja_points_maximise_the_node_polynomial():
    m, grid = 40, 20001
    xi = o.leja_points(m, grid)
    assert xi[0] == 2.0 and xi[1] == -2.0
    assert len(np.unique(xi)) == m + 1 and np.all(np.abs(xi) <= 2.0)
    x = np.linspace(-2.0, 2.0, grid)
    for j in range(1, m + 1):
        wj = np.prod(np.abs(x[:, None] - xi[None, :j]), axis=1)
        wxi = np.prod(np.abs(xi[j] - xi[:j]))
        assert wxi >= wj.max() * (1 - 1e-12)


@pytest.mark.parametrize("rho", [0.5, 4.0, 8.0])
def test_divided_differences_of_exp(rho):
    xi = o.leja_points(30)
    d = o.exp_divided_differences(rho, xi)
    # two points: the difference quotient
    assert abs(d[1] - (math.exp(rho * xi[1]) - math.exp(rho * xi[0])) / (xi[1] - xi[0])) \
        <= 1e-15 * math.exp(2 * rho)
    # mean value theorem: f[x_0..x_j] = f^(j)(eta) / j! with eta in [-2, 2]
    for j in range(len(d)):
        lo = rho ** j * math.exp(-2 * rho) / math.factorial(j)
        hi = rho ** j * math.exp(2 * rho) / math.factorial(j)
        assert lo * (1 - 1e-12) <= d[j] <= hi * (1 + 1e-12), j
    # the Newton form interpolates at the nodes
    p = o.newton_eval(d, xi, xi)
    assert np.max(np.abs(p - np.exp(rho * xi))) <= 1e-13 * math.exp(2 * rho)


@pytest.mark.parametrize("t", [1e-5, 5e-4, 1e-2])
def test_leja_action_equals_laplacian_eigenbasis(t):
    """e^{tA} V = U e^{t Lam} U^T V for the 2-D Laplacian (closed-form
    eigenpairs); t = 1e-2 needs several substeps (t g / rho_max ~ 20)."""
    nx = 12
    A = w.laplacian_2d(nx)
    lam, U = eig2d(nx)
    V = np.random.default_rng(3).standard_normal((nx * nx, 4))
    ref = U @ (np.exp(t * lam)[:, None] * (U.T @ V))
    got = o.leja_expmv(A, t, V)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(V)


@pytest.mark.parametrize("t,seed", [(0.3, 1), (2.5, 2), (0.01, 3)])
def test_leja_action_equals_dense_exponential(t, seed):
    A = _sym(40, seed, shift=-1.0)
    V = np.random.default_rng(seed + 10).standard_normal((40, 3))
    ref = o.expm(t * A) @ V
    got = o.leja_expmv(A, t, V)
    a, b = o.gershgorin_interval(A)
    assert np.linalg.norm(got - ref) <= 1e-12 * math.exp(t * b) * np.linalg.norm(V)


def test_leja_params_substeps_and_degree():
    S, m, rho, xi, d = o.leja_params(20.0)
    assert S == 3 and abs(rho - 20.0 / 3) < 1e-15 and 10 < m <= 100
    z = np.linspace(-2, 2, 1001)
    assert np.max(np.abs(o.newton_eval(d, xi, z) - np.exp(rho * z))) <= 1e-14 * math.exp(2 * rho)


def test_quadrature_factor_leja_equals_expm_route():
    nx, t, K, p = 10, 5e-4, 7, 3
    A = w.laplacian_2d(nx)
    C = w.random_C(p, nx * nx, seed=6)
    Lg, Dg = o.quadrature_factor(A, C, t, K, tol=1e-15)
    Ll, Dl = o.quadrature_factor_leja(A, C, t, K, tol=1e-15)
    Pg, Pl = Lg @ Dg @ Lg.T, Ll @ Dl @ Ll.T
    assert np.linalg.norm(Pl - Pg) / np.linalg.norm(Pg) < 1e-12


def test_solve_with_leja_operator_equals_pade_route():
    """A whole DRE solve with the action-based T12 (LejaExpm) equals the one
    with the dense Pade exponential."""
    p = w.config_dre_halfplane(nx=8, h=1e-2)
    Lp, Dp, _ = o.solve(p.A, p.C, p.T, p.h, kind="dre", B=p.B, R=p.R, tol=p.tol)
    Ll, Dl, _ = o.solve(p.A, p.C, p.T, p.h, kind="dre", B=p.B, R=p.R, tol=p.tol,
                        expm_fn=lambda t: o.LejaExpm(p.A, t),
                        quad_fn=lambda t: o.quadrature_factor_leja(p.A, p.C, t, 7, p.tol))
    assert o.lowrank_rel_err(Ll, Dl, Lp, Dp) < 1e-11


_orig_leja = od.leja_expmv


def _leja_wrong_shift(A, t, V, tol=1e-14):   # e^{-tc} instead of e^{tc} per substep
    a, b = od.gershgorin_interval(np.asarray(A))
    c = 0.5 * (a + b)
    return math.exp(-2.0 * t * c) * _orig_leja(A, t, V, tol)


def _leja_wrong_node(A, t, V, tol=1e-14):    # Newton basis built with xi_{j+1}
    A = np.asarray(A, dtype=np.float64)
    a, b = od.gershgorin_interval(A)
    c, g = 0.5 * (a + b), 0.25 * (b - a)
    S, m, rho, xi, d = od.leja_params(t * g, tol)
    xi2 = od.leja_points(m + 1)
    As = (A - c * np.eye(A.shape[0])) / g
    V = np.array(V, dtype=np.float64)
    for _ in range(S):
        W, P = V, d[0] * V
        for j in range(m):
            W = As @ W - xi2[j + 1] * W
            P = P + d[j + 1] * W
        V = math.exp(t * c / S) * P
    return V


@pytest.mark.parametrize("bad", [_leja_wrong_shift, _leja_wrong_node])
def test_planted_leja_mistake_is_caught(monkeypatch, bad):
    monkeypatch.setattr(od, "leja_expmv", bad)
    monkeypatch.setattr(o, "leja_expmv", bad)
    with pytest.raises(AssertionError):
        test_leja_action_equals_laplacian_eigenbasis(5e-4)
