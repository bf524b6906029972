"""Pins for Gauss-Legendre nodes and the quadrature factor of Alg. 2."""
import numpy as np
import pytest

import oracle as o
import workloads as w
from tests.laplace_closed_form import eig2d


@pytest.mark.parametrize("K", [1, 3, 7, 14])
def test_gl_exact_monomials(K):
    t = 0.37
    s, wt = o.gauss_legendre(K, t)
    assert np.all((s > 0) & (s < t))
    for d in range(2 * K):
        exact = t ** (d + 1) / (d + 1)
        assert abs(np.sum(wt * s ** d) - exact) <= 1e-14 * max(1.0, exact)
    # not exact for degree 2K (detectable in double precision for small K)
    if K <= 3:
        d = 2 * K
        exact = t ** (d + 1) / (d + 1)
        assert abs(np.sum(wt * s ** d) - exact) > 1e-6 * exact


def test_quadrature_factor_eigenbasis():
    # In the eigenbasis: L_I D_I L_I^T = V (Qt o sum_k w_k e^{mu s_k}) V^T,
    # mu_ij = lam_i + lam_j, Qt = V^T Q V.
    nx, t, K = 8, 5e-4, 7
    A = w.laplacian_2d(nx)
    lam, V = eig2d(nx)
    C = w.random_C(3, nx * nx, seed=4)
    LI, DI = o.quadrature_factor(A, C, t, K, tol=1e-15)
    s, wt = o.gauss_legendre(K, t)
    mu = lam[:, None] + lam[None, :]
    Qt = V.T @ (C.T @ C) @ V
    F = sum(wk * np.exp(mu * sk) for sk, wk in zip(s, wt))
    ref = V @ (Qt * F) @ V.T
    got = LI @ DI @ LI.T
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    # and the rule integrates the exact integral (Qt o (e^{mu t}-1)/mu) closely
    exact = V @ (Qt * (np.expm1(mu * t) / mu)) @ V.T
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 1e-10


@pytest.mark.parametrize("nx,t,p,K", [(9, 5e-4, 1, 7), (12, 1e-3, 3, 7), (16, 5e-4, 8, 7),
                                      (10, 2.5e-3, 2, 14), (13, 1e-4, 5, 3)])
def test_quadrature_factor_kron_equals_generic(nx, t, p, K):
    """The Kronecker-sum route (e^{sA} = e^{sA1} (x) e^{sA1} applied column by
    column) gives the same factor L_I D_I L_I^T as the generic quadrature factor
    of Alg. 2, and both match the eigenbasis closed form Qt o sum_k w_k e^{mu s_k}."""
    A = w.laplacian_2d(nx)
    A1 = w.laplacian_1d(nx)
    C = w.random_C(p, nx * nx, seed=nx + p)
    Lg, Dg = o.quadrature_factor(A, C, t, K, tol=1e-15)
    Lk, Dk = o.quadrature_factor_kron(A1, C, t, K, tol=1e-15)
    Pg = Lg @ Dg @ Lg.T
    Pk = Lk @ Dk @ Lk.T
    assert np.linalg.norm(Pk - Pg) / np.linalg.norm(Pg) < 1e-13
    lam, V = eig2d(nx)
    s, wt = o.gauss_legendre(K, t)
    mu = lam[:, None] + lam[None, :]
    Qt = V.T @ (C.T @ C) @ V
    ref = V @ (Qt * sum(wk * np.exp(mu * sk) for sk, wk in zip(s, wt))) @ V.T
    assert np.linalg.norm(Pk - ref) / np.linalg.norm(ref) < 1e-12
    # at the workloads' compression tolerance the two routes keep the same rank
    Lg2, Dg2 = o.quadrature_factor(A, C, t, K, tol=1e-10)
    Lk2, Dk2 = o.quadrature_factor_kron(A1, C, t, K, tol=1e-10)
    assert Lg2.shape[1] == Lk2.shape[1]
    assert o.lowrank_rel_err(Lk2, Dk2, Lg2, Dg2) < 1e-12


def test_quadrature_factor_kron_detects_block_order():
    """A factor whose weights are attached to the wrong nodes (weights shifted by
    one node; the Gauss-Legendre weights are symmetric, so a reversal would not
    show) differs from the Kronecker route by far more than the bar above."""
    nx, t, p, K = 10, 1e-3, 2, 7
    A = w.laplacian_2d(nx)
    A1 = w.laplacian_1d(nx)
    C = w.random_C(p, nx * nx, seed=3)
    Lk, Dk = o.quadrature_factor_kron(A1, C, t, K, tol=1e-15)
    s, wt = o.gauss_legendre(K, t)
    AT = np.ascontiguousarray(A.T)
    cols = [o.expm(sk * AT) @ C.T for sk in s]
    blocks = [wk * np.eye(p) for wk in np.roll(wt, 1)]
    L = np.hstack(cols)
    D = np.zeros((K * p, K * p))
    for q, b in enumerate(blocks):
        D[q * p:(q + 1) * p, q * p:(q + 1) * p] = b
    err = np.linalg.norm(L @ D @ L.T - Lk @ Dk @ Lk.T) / np.linalg.norm(Lk @ Dk @ Lk.T)
    assert err > 1e-6
