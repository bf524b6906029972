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
