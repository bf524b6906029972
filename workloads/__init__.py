"""Seeded synthetic inputs for the differential Lyapunov / Riccati workloads.

This module only *generates* problem data (A, B, C, R, S, P0, time grid,
request streams).  It holds none of the solution method's arithmetic and is
imported both by the CPU oracle's tests and by the GPU tests / benchmark, so
that both sides see byte-identical inputs.

Conventions (all matrices float64, returned Fortran-ordered = column-major):
  * 2-D grid with ``nx`` interior points per direction, spacing
    ``dx = 1/(nx+1)``, lexicographic index ``i + nx*j`` with the x index ``i``
    fastest.  This is the central second-order finite-difference Laplacian on
    the unit square with homogeneous Dirichlet conditions used by the paper's
    heat-equation examples (Sec. 5.1, Examples 1 and 2).
  * ``C`` is p x n (output matrix, Q = C^T C), ``B`` is n x m, ``R`` is m x m.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np


# ----------------------------------------------------------------------------
# operators
# ----------------------------------------------------------------------------
def tridiag_1d(nx: int, diag: float = -2.0, off: float = 1.0) -> np.ndarray:
    """nx x nx tridiagonal matrix with constant diagonal / off-diagonals."""
    T = np.zeros((nx, nx))
    idx = np.arange(nx)
    T[idx, idx] = diag
    T[idx[:-1], idx[:-1] + 1] = off
    T[idx[:-1] + 1, idx[:-1]] = off
    return T


def laplacian_2d(nx: int) -> np.ndarray:
    """Dense 5-point Dirichlet Laplacian on an nx x nx interior grid, scaled by 1/dx^2.

    A = (T (x) I + I (x) T) / dx^2 with T = tridiag(1, -2, 1), index i + nx*j.
    """
    dx = 1.0 / (nx + 1)
    T = tridiag_1d(nx)
    I = np.eye(nx)
    # x is the fastest index: kron(I_y, T_x) acts on x, kron(T_y, I_x) on y.
    A = (np.kron(I, T) + np.kron(T, I)) / (dx * dx)
    return np.asfortranarray(A)


def laplacian_1d(nx: int) -> np.ndarray:
    """The 1-D factor T/dx^2 of the 2-D Laplacian (A = I(x)A1 + A1(x)I)."""
    dx = 1.0 / (nx + 1)
    return np.asfortranarray(tridiag_1d(nx) / (dx * dx))


def fe_heat_2d(nx: int, grading: float = 1.3):
    """Bilinear finite elements for the heat equation on the unit square with
    Dirichlet boundary on a tensor mesh graded towards x = 0 and y = 0 (1-D
    nodes x_i = (i / (nx + 1))^grading, nx interior nodes per side, x
    fastest): returns (A, M) with the mass matrix M = M1 (x) M1 and the
    stiffness A = -(K1 (x) M1 + M1 (x) K1), M1 and K1 the 1-D linear-element
    mass and stiffness matrices on the interior nodes.  On a graded mesh M1 and
    K1 do not commute, so A M^-1 differs from M^-1 A.  A synthetic stand-in for
    the mass / stiffness pair of the steel-cooling example (whose
    finite-element data is not available)."""
    x = (np.arange(nx + 2) / (nx + 1.0)) ** grading
    he = np.diff(x)                      # element lengths, nx + 1 of them
    M1 = np.zeros((nx, nx))
    K1 = np.zeros((nx, nx))
    for i in range(nx):                  # interior node i + 1 between elements i and i + 1
        M1[i, i] = (he[i] + he[i + 1]) / 3.0
        K1[i, i] = 1.0 / he[i] + 1.0 / he[i + 1]
        if i + 1 < nx:
            M1[i, i + 1] = M1[i + 1, i] = he[i + 1] / 6.0
            K1[i, i + 1] = K1[i + 1, i] = -1.0 / he[i + 1]
    M = np.asfortranarray(np.kron(M1, M1))
    A = np.asfortranarray(-(np.kron(K1, M1) + np.kron(M1, K1)))
    return A, M


def grid_coords(nx: int):
    """x and y coordinates (length n) of the interior grid points, x fastest."""
    dx = 1.0 / (nx + 1)
    g = (np.arange(nx) + 1) * dx
    x = np.tile(g, nx)
    y = np.repeat(g, nx)
    return x, y


def half_plane_B(nx: int) -> np.ndarray:
    """n x 1 indicator of the grid cells with x < 1/2."""
    x, _ = grid_coords(nx)
    return np.asfortranarray((x < 0.5).astype(np.float64)[:, None])


def quadrant_B(nx: int, m: int = 4) -> np.ndarray:
    """First m of the four quadrant indicators, ordered
    (x<1/2,y<1/2), (x>=1/2,y<1/2), (x<1/2,y>=1/2), (x>=1/2,y>=1/2)."""
    if not 1 <= m <= 4:
        raise ValueError("m must be in 1..4")
    x, y = grid_coords(nx)
    cols = [(x < 0.5) & (y < 0.5), (x >= 0.5) & (y < 0.5),
            (x < 0.5) & (y >= 0.5), (x >= 0.5) & (y >= 0.5)]
    return np.asfortranarray(np.stack(cols[:m], axis=1).astype(np.float64))


def ones_C(n: int) -> np.ndarray:
    """1 x n row of ones (Q = C^T C)."""
    return np.asfortranarray(np.ones((1, n)))


def random_C(p: int, n: int, seed: int) -> np.ndarray:
    """p x n with i.i.d. N(0,1)/sqrt(n) entries from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((p, n)) / math.sqrt(n))


def tridiag_S(n: int, scale: float = 0.1) -> np.ndarray:
    """S = scale * tridiag(1, 0, 1) (n x n, lexicographic order)."""
    return np.asfortranarray(scale * tridiag_1d(n, diag=0.0, off=1.0))


def random_nonsymmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """A dense nonsymmetric test operator: a shifted random matrix (stable)."""
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n)) / math.sqrt(n)
    return np.asfortranarray(scale * (M - 1.5 * np.eye(n)))


def sine_mode(nx: int, j: int, k: int) -> np.ndarray:
    """Orthonormal discrete sine product s_j(x) s_k(y) on the grid (length n).

    These are the eigenvectors of the Dirichlet finite-difference Laplacian;
    they are returned here only as *input* vectors (columns of B, rows of C)
    for commuting special cases.
    """
    i = np.arange(1, nx + 1)
    sj = math.sqrt(2.0 / (nx + 1)) * np.sin(j * i * math.pi / (nx + 1))
    sk = math.sqrt(2.0 / (nx + 1)) * np.sin(k * i * math.pi / (nx + 1))
    return np.kron(sk, sj)  # x (j) fastest


def random_lowrank_P0(n: int, r: int, seed: int):
    """Random PSD initial value P0 = L0 D0 L0^T (L0 n x r, D0 r x r diagonal > 0)."""
    rng = np.random.default_rng(seed)
    L0 = rng.standard_normal((n, r)) / math.sqrt(n)
    D0 = np.diag(rng.uniform(0.5, 1.5, size=r))
    return np.asfortranarray(L0), np.asfortranarray(D0)


# ----------------------------------------------------------------------------
# named configurations
# ----------------------------------------------------------------------------
@dataclass
class Problem:
    """One differential matrix equation instance (all arrays column-major)."""
    name: str
    A: np.ndarray
    C: np.ndarray
    B: Optional[np.ndarray] = None
    R: Optional[np.ndarray] = None
    S: Optional[np.ndarray] = None
    L0: Optional[np.ndarray] = None
    D0: Optional[np.ndarray] = None
    M: Optional[np.ndarray] = None      # mass matrix (None: identity)
    T: float = 0.1
    h: float = 1e-3
    tol: float = 1e-10
    kind: str = "dre"          # "dle" (G = 0) or "dre" (G = -P B R^-1 B^T P)
    split: str = "F12"         # "F12", "F1F2", "F1F3F2"
    scheme: str = "strang"     # "strang" or "lie"
    quad_nodes: int = 7
    nx: Optional[int] = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.A.shape[0]

    @property
    def nsteps(self) -> int:
        return int(round(self.T / self.h))


def config_dle_small(nx: int = 16) -> Problem:
    """DLE, plain Strang splitting (F1F2, Alg. 1): 16x16 Laplacian, C = ones, P0 = 0."""
    n = nx * nx
    return Problem(name=f"dle_strang_f1f2_n{n}", A=laplacian_2d(nx), C=ones_C(n),
                   T=0.1, h=1e-3, tol=1e-12, kind="dle", split="F1F2",
                   scheme="strang", nx=nx)


def config_dre_halfplane(nx: int = 64, h: float = 1e-3, scheme: str = "strang",
                         T: float = 0.1) -> Problem:
    """DRE with B = 1[x<1/2], R = 1, C = ones, P0 = 0; F12F3 splitting."""
    n = nx * nx
    return Problem(name=f"dre_{scheme}_f12f3_n{n}_h{h:g}", A=laplacian_2d(nx),
                   C=ones_C(n), B=half_plane_B(nx), R=np.eye(1, order="F"),
                   T=T, h=h, tol=1e-10, kind="dre", split="F12", scheme=scheme,
                   nx=nx)


def config_gdre(nx: int = 64, h: float = 1e-3, T: float = 0.1) -> Problem:
    """Generalized DRE: the half-plane DRE plus S = 0.1 tridiag(1,0,1) (F12F3F4)."""
    p = config_dre_halfplane(nx, h=h, T=T)
    p.S = tridiag_S(p.n, 0.1)
    p.name = f"gdre_strang_f12f3f4_n{p.n}"
    p.meta["seed"] = 0
    return p


def config_gdle(nx: int = 64, h: float = 1e-3, T: float = 0.1, split: str = "F12",
                scheme: str = "strang") -> Problem:
    """Generalized DLE: C = ones, P0 = 0, S = 0.1 tridiag(1,0,1), no B; split
    F12 (T12 and T4), F1F2 (T1 T2 T4) or F1F3F2 (T1 T4 T2)."""
    n = nx * nx
    return Problem(name=f"gdle_{scheme}_{split.lower()}_n{n}_h{h:g}", A=laplacian_2d(nx),
                   C=ones_C(n), S=tridiag_S(n, 0.1), T=T, h=h, tol=1e-10, kind="dle",
                   split=split, scheme=scheme, nx=nx, meta={"seed": 0})


def config_dre_mass(nx: int = 8, h: float = 1e-3, T: float = 0.05, scheme: str = "strang",
                    split: str = "F12", p: int = 3, m: int = 2, seed: int = 0) -> Problem:
    """DRE in mass-matrix form (M^T dP/dt M = A^T P M + M^T P A + C^T C - ...)
    with the bilinear finite-element pair of ``fe_heat_2d``, B = the first m
    quadrant indicators, R = I, C = p x n N(0,1)/sqrt(n)."""
    n = nx * nx
    A, M = fe_heat_2d(nx)
    return Problem(name=f"dre_mass_{scheme}_n{n}", A=A, C=random_C(p, n, seed), B=quadrant_B(nx, m),
                   R=np.eye(m, order="F"), M=M, T=T, h=h, tol=1e-10, kind="dre", split=split,
                   scheme=scheme, nx=nx, meta={"seed": seed})


def config_dre_quadrant(nx: int = 128, seed: int = 0, p: int = 8, m: int = 4,
                        T: float = 0.1, h: float = 1e-3) -> Problem:
    """DRE with B = 4 quadrant indicators, R = I_4, C = 8 x n N(0,1)/sqrt(n) (seed 0)."""
    n = nx * nx
    return Problem(name=f"dre_strang_f12f3_quadrant_n{n}", A=laplacian_2d(nx),
                   C=random_C(p, n, seed), B=quadrant_B(nx, m),
                   R=np.eye(m, order="F"), T=T, h=h, tol=1e-10, kind="dre",
                   split="F12", scheme="strang", nx=nx, meta={"seed": seed})


# ----------------------------------------------------------------------------
# served request stream
# ----------------------------------------------------------------------------
SERVE_GRID_SIDES = (32, 48, 64, 96, 128)


@dataclass
class Request:
    index: int
    arrival_s: float
    nx: int
    kind: str
    m: int
    p: int
    nsteps: int
    h: float
    seed: int

    @property
    def n(self) -> int:
        return self.nx * self.nx

    @property
    def T(self) -> float:
        return self.nsteps * self.h


def request_stream(count: int, rate_per_s: float, base_seed: int = 1000,
                   stream_seed: int = 7, sides=SERVE_GRID_SIDES,
                   nsteps_range=(50, 200), h: float = 1e-3):
    """Poisson arrivals at ``rate_per_s``; per-request shape drawn with seed base_seed+i."""
    arr_rng = np.random.default_rng(stream_seed)
    gaps = arr_rng.exponential(1.0 / rate_per_s, size=count) if count else np.zeros(0)
    t = np.cumsum(gaps) - (gaps[0] if count else 0.0)
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        nx = int(rng.choice(sides))
        kind = "dre" if rng.integers(0, 2) else "dle"
        m = int(rng.integers(1, 5))
        p = int(rng.integers(1, 9))
        nsteps = int(rng.integers(nsteps_range[0], nsteps_range[1] + 1))
        out.append(Request(i, float(t[i]), nx, kind, m, p, nsteps, h, base_seed + i))
    return out


def request_problem(req: Request) -> Problem:
    """Materialise the matrices of one served request."""
    n = req.n
    C = random_C(req.p, n, req.seed)
    if req.kind == "dre":
        B = quadrant_B(req.nx, req.m)
        R = np.eye(req.m, order="F")
    else:
        B = None
        R = None
    return Problem(name=f"req{req.index}", A=laplacian_2d(req.nx), C=C, B=B, R=R,
                   T=req.T, h=req.h, tol=1e-10, kind=req.kind, split="F12",
                   scheme="strang", nx=req.nx, meta={"seed": req.seed})
