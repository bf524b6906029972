"""Pins for the oracle's matrix exponential (Higham 2005, Alg. 2.3)."""
import math

import numpy as np
import pytest
import scipy.linalg as sl

import oracle as o
from oracle import dme_oracle as od
import workloads as w
from tests.laplace_closed_form import eig2d


@pytest.mark.parametrize("m", [3, 5, 7, 9, 13])
def test_pade_order(m):
    # Defining property of the [m/m] Pade approximant p(x)/p(-x) of e^x: the
    # Taylor coefficients of p(-x) e^x - p(x) vanish up to x^(2m) and the
    # x^(2m+1) one does not.
    c = o.pade_coefficients(m)
    assert c[0] == 1.0
    q = [cj * (-1) ** j for j, cj in enumerate(c)]
    ex = [1.0 / math.factorial(j) for j in range(2 * m + 2)]
    for k in range(2 * m + 2):
        coef = sum(q[j] * ex[k - j] for j in range(min(k, m) + 1))
        coef -= c[k] if k <= m else 0.0
        scale = sum(abs(q[j] * ex[k - j]) for j in range(min(k, m) + 1)) + (abs(c[k]) if k <= m else 0)
        if k <= 2 * m:
            assert abs(coef) <= 4e-16 * scale, (m, k, coef)
        else:
            assert abs(coef) > 1e3 * 4e-16 * scale  # clearly above rounding level


def test_pade_13_known_ratio():
    # c_1 = 1/2 for every m (the [m/m] Pade numerator is 1 + x/2 + ...).
    for m in (3, 5, 7, 9, 13):
        assert o.pade_coefficients(m)[1] == pytest.approx(0.5, abs=0)


@pytest.mark.parametrize("m", [3, 5, 7, 9, 13])
def test_theta_accuracy_boundary(m):
    # theta_m is where the degree-m approximant stops being accurate to working
    # precision: unscaled r_m(X) at ||X||_1 = theta_m matches the library
    # exponential, while at 4 theta_m it is clearly worse.
    # A nonnegative matrix with constant column sums has rho(X) = ||X||_1, the
    # worst case for a norm-based rule.
    M = np.ones((30, 30)) / 30.0
    errs = []
    for f in (1.0, 4.0):
        X = f * o.THETA[m] * M
        U, V = od._pade_uv(X, m)
        F = np.linalg.solve(V - U, V + U)
        ref = sl.expm(X)
        errs.append(np.linalg.norm(F - ref) / np.linalg.norm(ref))
    assert errs[0] < 3e-14
    assert errs[1] > 5 * errs[0]


def test_params_selection():
    assert o.expm_params(0.0) == (3, 0)
    assert o.expm_params(1.0)[0] == 9
    assert o.expm_params(5.0) == (13, 0)
    assert o.expm_params(5.4) == (13, 1)
    # ||tA||_1 = 8 t / dx^2 for the Laplacian: 16x16 grid, t = h/2 = 5e-4
    A = w.laplacian_2d(16)
    assert o.norm1(5e-4 * A) == pytest.approx(8 * 5e-4 * 17 ** 2)
    assert o.expm_params(o.norm1(5e-4 * A)) == (9, 0)
    # 64x64 grid: 16.9 -> s = 2; 128x128 grid: 66.6 -> s = 4
    assert o.expm_params(8 * 5e-4 * 65 ** 2) == (13, 2)
    assert o.expm_params(8 * 5e-4 * 129 ** 2) == (13, 4)


@pytest.mark.parametrize("scale", [0.005, 0.1, 0.5, 1.5, 4.0, 40.0])
def test_expm_vs_scipy_nonsymmetric(scale):
    A = w.random_nonsymmetric(40, seed=11, scale=scale)
    E = o.expm(A)
    ref = sl.expm(A)
    assert np.linalg.norm(E - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("nx,t", [(8, 5e-4), (12, 1e-3), (16, 1e-2)])
def test_expm_laplacian_eigenpairs(nx, t):
    A = w.laplacian_2d(nx)
    lam, V = eig2d(nx)
    E = o.expm(t * A)
    # E v = e^{t lam} v for every analytic eigenvector
    res = E @ V - V * np.exp(t * lam)[None, :]
    assert np.abs(res).max() < 1e-13
    ref = (V * np.exp(t * lam)) @ V.T
    assert np.abs(E - ref).max() < 1e-13


def test_expm_semigroup():
    A = w.laplacian_2d(10)
    E1 = o.expm(1e-3 * A)
    Eh = o.expm(5e-4 * A)
    assert np.abs(Eh @ Eh - E1).max() < 1e-14


def test_expm_scalar_and_empty():
    for x in (-60.0, -3.0, 0.0, 0.7, 9.0):
        e = o.expm(np.array([[x]]))[0, 0]
        # squaring s times amplifies the relative error by about 2^s
        _, s = o.expm_params(abs(x))
        assert e == pytest.approx(math.exp(x), rel=(2 ** s) * 2e-14, abs=1e-300)
    assert o.expm(np.zeros((0, 0))).shape == (0, 0)


def test_expm_transpose_convention():
    # e^{A^T} = (e^A)^T: the solver uses e^{tA^T}; make sure it is not e^{tA}.
    A = w.random_nonsymmetric(20, seed=5, scale=2.0)
    assert np.abs(o.expm(A.T) - o.expm(A).T).max() < 1e-13
    assert np.abs(o.expm(A.T) - o.expm(A)).max() > 1e-3


def test_kron_path_equals_generic():
    nx = 9
    A = w.laplacian_2d(nx)
    A1 = w.laplacian_1d(nx)
    for t in (5e-4, 3e-3):
        Ek = o.laplacian_expm_kron(A1, t)
        Eg = o.expm(t * A)
        assert np.abs(Ek - Eg).max() < 1e-14
        V = np.random.default_rng(1).standard_normal((nx * nx, 3))
        E1 = o.expm(t * A1.T)
        assert np.abs(o.kron_apply_expm(E1, V) - Eg @ V).max() < 1e-13


def test_kron_operator_matches_dense_kron():
    """KronExpm @ V equals laplacian_expm_kron(A1, t) @ V (the operator form
    used by the large-n oracle runs)."""
    nx, t = 9, 7e-4
    A1 = w.laplacian_1d(nx)
    V = np.random.default_rng(1).standard_normal((nx * nx, 5))
    got = o.KronExpm(A1, t) @ V
    ref = o.laplacian_expm_kron(A1, t) @ V
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()
