"""Closed forms for the Dirichlet finite-difference Laplacian used as pins.

These are textbook facts, independent of the oracle and of the HIP path:
the 1-D matrix tridiag(1,-2,1)/dx^2 (dx = 1/(nx+1)) has eigenvalues
-(4/dx^2) sin^2(j pi / (2(nx+1))) with orthonormal eigenvectors
sqrt(2/(nx+1)) sin(j i pi/(nx+1)); the 2-D Laplacian is the Kronecker sum.
"""
import math

import numpy as np


def eig1d(nx):
    dx = 1.0 / (nx + 1)
    j = np.arange(1, nx + 1)
    lam = -(4.0 / dx ** 2) * np.sin(j * math.pi / (2 * (nx + 1))) ** 2
    i = np.arange(1, nx + 1)
    V = math.sqrt(2.0 / (nx + 1)) * np.sin(np.outer(i, j) * math.pi / (nx + 1))
    return lam, V


def eig2d(nx):
    """Eigenvalues (length n) and orthonormal eigenvectors (n x n) of the 2-D
    Laplacian with index i + nx*j (x fastest); mode (a, b) sits at column a + nx*b."""
    lam1, V1 = eig1d(nx)
    lam = (lam1[:, None] + lam1[None, :]).T.reshape(-1)  # index a + nx*b
    V = np.kron(V1, V1)
    return lam, V
