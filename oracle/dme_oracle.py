"""FP64 CPU oracle for low-rank splitting schemes for differential matrix equations.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
module: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP implementation.

What it computes (Mena, Pfurtscheller, Stillfjord, "GPU acceleration of
splitting schemes applied to differential matrix equations", 2018):

    dP/dt = A^T P + P A + Q + G(P),   P(0) = P0,   Q = C^T C,
    G = 0                       (DLE, Sec. 2.1)
    G = -P B R^-1 B^T P         (DRE, Sec. 2.2)
    plus S P S^T when S is given (generalized DLE/DRE, Sec. 2.3-2.4),

with P kept as P = L D L^T (Sec. 2, low-rank paragraph) and advanced by Lie or
Strang compositions of the subflows (Sec. 2 and the scheme list of Sec. 3):

    T1(t) P = e^{tA^T} P e^{tA}          -> L <- e^{tA^T} L            (Sec. 2.1)
    T2(t) P = P + t Q                     -> [L, L_Q], blkdiag(D, t D_Q) (Sec. 2.1)
    T12(t)P = e^{tA^T} P e^{tA} + int_0^t e^{sA^T} Q e^{sA} ds
              (integral by a quadrature rule, Alg. 2)                   (Sec. 2.1, Sec. 3)
    T3(t) P = (I + t P B R^-1 B^T)^-1 P   -> D <- (I + t D L^T B R^-1 B^T L)^-1 D
                                                                        (Sec. 2.2, Alg. 3)
    T4(t) P ~ P + t S (P + t/2 S P S^T) S^T
           -> [L, sqrt(t) S L, t/sqrt(2) S^2 L], blkdiag(D, D, D)      (Sec. 2.3, Alg. 4)

and column compression after every concatenation (Alg. 1, 2, 4; Sec. 3).

The matrix exponential is formed by scaling and squaring with a diagonal Pade
approximant, choosing the degree and the scaling from the 1-norm as in
N. J. Higham, "The scaling and squaring method for the matrix exponential
revisited", SIAM J. Matrix Anal. Appl. 26(4), 2005, Algorithm 2.3.  The paper
itself uses a Leja-interpolation action instead (Sec. 3); the dense operator is
the approach this project takes, and both sides of the parity comparison use
the same (m, s) rule.

Readings of points the paper leaves open:
  * Operators act right to left; lists below are in application order.
  * Alg. 3 as printed drops B^T; the formula of Sec. 2.2 is used.
  * Alg. 4 uses the pre-update L in S^2 L.
  * Compression: Householder QR W = QR, M = R D R^T, symmetric eigen-
    decomposition M = V Lam V^T, keep |lam_i| > tol * max|lam|, sorted by
    |lam| descending, L <- Q V_I, D <- diag(lam_I).
  * Quadrature: Gauss-Legendre with K nodes on [0, t] for the T12(t) applied.
  * N = round(T/h) steps, rejected unless |N h - T| <= 1e-12 T.

Every function below is pinned by a CPU test in tests/test_oracle_*.py against
closed forms, library routines, brute-force integration or invariants; see the
docstring of each function for its pin.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

__all__ = [
    "THETA", "pade_coefficients", "norm1", "expm_params", "expm", "num_steps", "gauss_legendre",
    "compress", "quadrature_factor", "t1", "t2", "t12", "t3", "t4", "feedback_gain",
    "step_sequence", "solve", "lowrank_fro", "lowrank_rel_err",
    "laplacian_expm_kron", "kron_apply_expm", "quadrature_factor_kron", "KronExpm",
    "gershgorin_interval", "leja_points", "exp_divided_differences", "newton_eval", "leja_params",
    "leja_expmv", "LejaExpm", "quadrature_factor_leja", "mass_matrix_form",
    "OracleError",
]


class OracleError(ValueError):
    pass


# ----------------------------------------------------------------------------
# Matrix exponential: Higham (2005), Algorithm 2.3
# ----------------------------------------------------------------------------
# theta_m: largest 1-norm for which the [m/m] Pade approximant has backward
# error <= 2^-53 (Higham 2005, Table 2.3, double precision column).
THETA = {
    3: 1.495585217958292e-2,
    5: 2.539398330063230e-1,
    7: 9.504178996162932e-1,
    9: 2.097847961257068e0,
    13: 5.371920351148152e0,
}


def pade_coefficients(m: int) -> list:
    """Coefficients c_0..c_m of the numerator p_m(x) = sum c_j x^j of the [m/m]
    Pade approximant of e^x (denominator q_m(x) = p_m(-x)):

        c_j = (2m - j)! m! / ((2m)! j! (m - j)!)

    Pin: tests check r_m(x) - e^x = O(x^(2m+1)) as x -> 0.
    """
    f = math.factorial
    return [float(Fraction(f(2 * m - j) * f(m), f(2 * m) * f(j) * f(m - j)))
            for j in range(m + 1)]


def norm1(A: np.ndarray) -> float:
    """Matrix 1-norm (max column absolute sum)."""
    return float(np.max(np.sum(np.abs(A), axis=0))) if A.size else 0.0


def expm_params(nrm1: float):
    """Pade degree m and scaling s of Higham (2005) Alg. 2.3 for ||X||_1 = nrm1."""
    for m in (3, 5, 7, 9):
        if nrm1 <= THETA[m]:
            return m, 0
    s = max(0, int(math.ceil(math.log2(nrm1 / THETA[13])))) if nrm1 > 0 else 0
    return 13, s


def _pade_uv(X: np.ndarray, m: int):
    """U (odd part) and V (even part) of p_m(X) = V + U, so q_m(X) = V - U."""
    c = pade_coefficients(m)
    n = X.shape[0]
    I = np.eye(n)
    X2 = X @ X
    if m == 13:
        X4 = X2 @ X2
        X6 = X4 @ X2
        U = X @ (X6 @ (c[13] * X6 + c[11] * X4 + c[9] * X2)
                 + c[7] * X6 + c[5] * X4 + c[3] * X2 + c[1] * I)
        V = (X6 @ (c[12] * X6 + c[10] * X4 + c[8] * X2)
             + c[6] * X6 + c[4] * X4 + c[2] * X2 + c[0] * I)
        return U, V
    # m in {3, 5, 7, 9}: plain even powers X^2, X^4, ...
    pows = [I, X2]
    for _ in range(2, m // 2 + 1):
        pows.append(pows[-1] @ X2)
    odd = sum(c[2 * k + 1] * pows[k] for k in range(m // 2 + 1))
    even = sum(c[2 * k] * pows[k] for k in range(m // 2 + 1))
    return X @ odd, even


def expm(X: np.ndarray) -> np.ndarray:
    """e^X by scaling and squaring with the [m/m] Pade approximant (Higham 2005,
    Alg. 2.3): pick (m, s) from ||X||_1, form U and V, solve (V - U) F = V + U
    with LU and partial pivoting, then square s times.

    Pins: scipy.linalg.expm; the analytic Laplacian eigenpairs; the semigroup
    identity e^{X/2} e^{X/2} = e^X; scalar exponentials.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if n == 0:
        return np.zeros((0, 0))
    m, s = expm_params(norm1(X))
    Xs = X / (2.0 ** s)
    U, V = _pade_uv(Xs, m)
    F = np.linalg.solve(V - U, V + U)
    for _ in range(s):
        F = F @ F
    return F


# ----------------------------------------------------------------------------
# Action e^{tA} V by Newton interpolation at Leja points (the paper's
# "expleja", Sec. 3 and Sec. 4: a one-time spectral estimate by Gershgorin
# discs, one-time interpolation parameters, then Newton interpolation built
# from products with A), for A with a real spectrum (symmetric A).
#
# With [a, b] an interval holding the spectrum, c = (a + b) / 2 and
# g = (b - a) / 4, the matrix As = (A - c I) / g has its spectrum in [-2, 2]
# and e^{tA} = e^{tc} e^{t g As}.  The time t is cut into S substeps of
# t / S; in each, e^{rho z} (rho = t g / S) is interpolated at Leja points
# xi_0 .. xi_m of [-2, 2] in Newton form
#     p(z) = sum_j d_j w_j(z),  w_0 = 1,  w_{j+1} = (z - xi_j) w_j,
# with d_j the divided differences of e^{rho z}, and applied to the block:
#     W <- V, P <- d_0 V;  for j: W <- (As - xi_j I) W, P <- P + d_{j+1} W;
#     V <- e^{t c / S} P.
# For a symmetric A the error of one substep is at most
# max_{z in [-2, 2]} |e^{rho z} - p(z)| times ||V||, so (S, m) are chosen
# from that scalar error.
# ----------------------------------------------------------------------------
def gershgorin_interval(A: np.ndarray):
    """[a, b] = [min_i (a_ii - R_i), max_i (a_ii + R_i)], R_i the off-diagonal
    absolute row sum: the union of the Gershgorin discs meets the real line
    inside it, so for a symmetric A it contains every eigenvalue.

    Pin: contains the eigenvalues of symmetric matrices; equals the closed
    form [-8/dx^2, 0] for the Dirichlet Laplacian.
    """
    A = np.asarray(A, dtype=np.float64)
    d = np.diag(A)
    rad = np.sum(np.abs(A), axis=1) - np.abs(d)
    return float(np.min(d - rad)), float(np.max(d + rad))


def leja_points(m: int, grid: int = 20001) -> np.ndarray:
    """m + 1 (discrete) Leja points of [-2, 2]: xi_0 = 2, then each xi_j is a
    point of a uniform grid of [-2, 2] where prod_{i<j} |x - xi_i| is largest.

    Pin: every xi_j maximises |w_j| over the grid (w_j = prod_{i<j}(x - xi_i))
    and the points are distinct.
    """
    x = np.linspace(-2.0, 2.0, grid)
    pts = [2.0]
    logw = np.log(np.abs(x - 2.0) + 1e-300)
    for _ in range(m):
        i = int(np.argmax(logw))
        pts.append(float(x[i]))
        logw = logw + np.log(np.abs(x - x[i]) + 1e-300)
    return np.array(pts)


def exp_divided_differences(rho: float, xi: np.ndarray, digits: int = 80) -> np.ndarray:
    """d_j = f[xi_0, ..., xi_j] of f(z) = e^{rho z}, by the recursive definition
    f[x_i..x_k] = (f[x_{i+1}..x_k] - f[x_i..x_{k-1}]) / (x_k - x_i), evaluated in
    decimal arithmetic with `digits` significant digits.

    Pins: two-point closed form; the mean-value bounds
    rho^j e^{-2 rho} / j! <= d_j <= rho^j e^{2 rho} / j!; the Newton form
    reproduces e^{rho xi_j} at the nodes.
    """
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = digits
        X = [Decimal(repr(float(v))) for v in xi]
        R = Decimal(repr(float(rho)))
        col = [(R * x).exp() for x in X]
        d = [col[0]]
        for k in range(1, len(X)):
            col = [(col[i + 1] - col[i]) / (X[i + k] - X[i]) for i in range(len(col) - 1)]
            d.append(col[0])
        return np.array([float(v) for v in d])


def newton_eval(d: np.ndarray, xi: np.ndarray, z: np.ndarray) -> np.ndarray:
    """p(z) = sum_j d_j prod_{i<j} (z - xi_i) at the points z."""
    z = np.asarray(z, dtype=np.float64)
    p = np.zeros_like(z)
    w = np.ones_like(z)
    for j in range(len(d)):
        p = p + d[j] * w
        w = w * (z - xi[j])
    return p


def leja_params(rho_total: float, tol: float = 1e-14, rho_max: float = 8.0, m_max: int = 100):
    """Substeps S and degree m for e^{rho_total z} on [-2, 2]: S substeps of
    rho = rho_total / S <= rho_max, and the smallest m <= m_max whose Newton
    interpolant at the Leja points has max |e^{rho z} - p(z)| <= tol e^{2 rho}
    on a fine grid of [-2, 2] (e^{2 rho} = max of e^{rho z} there).
    Returns (S, m, rho, xi, d)."""
    S = max(1, int(math.ceil(rho_total / rho_max)))
    rho = rho_total / S
    xi = leja_points(m_max)
    d = exp_divided_differences(rho, xi)
    z = np.linspace(-2.0, 2.0, 4001)
    f = np.exp(rho * z)
    scale = math.exp(2.0 * rho)
    for m in range(1, m_max + 1):
        if np.max(np.abs(newton_eval(d[:m + 1], xi, z) - f)) <= tol * scale:
            return S, m, rho, xi[:m + 1], d[:m + 1]
    raise OracleError("Leja interpolation: no degree <= m_max meets the tolerance")


def leja_expmv(A: np.ndarray, t: float, V: np.ndarray, tol: float = 1e-14) -> np.ndarray:
    """e^{tA} V for a symmetric A by Newton interpolation at Leja points (see
    the section comment): Gershgorin interval, shift and scale to [-2, 2], S
    substeps of degree m.

    Pins: the exact action V e^{t Lam} V^T of the Laplacian's eigenpairs;
    ``expm(t A) @ V`` on random symmetric matrices, including t g >> rho_max
    (several substeps).
    """
    A = np.asarray(A, dtype=np.float64)
    V = np.array(V, dtype=np.float64)
    a, b = gershgorin_interval(A)
    c = 0.5 * (a + b)
    g = 0.25 * (b - a)
    if g == 0.0:
        return math.exp(t * c) * V
    S, m, rho, xi, d = leja_params(t * g, tol)
    n = A.shape[0]
    As = (A - c * np.eye(n)) / g
    for _ in range(S):
        W = V
        P = d[0] * V
        for j in range(m):
            W = As @ W - xi[j] * W
            P = P + d[j + 1] * W
        V = math.exp(t * c / S) * P
    return V


class LejaExpm:
    """e^{tA^T} as an operator whose ``@`` is ``leja_expmv`` (for
    ``solve(expm_fn=...)``: the paper's action-based step)."""

    def __init__(self, A: np.ndarray, t: float, tol: float = 1e-14):
        self.AT = np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)
        self.t = t
        self.tol = tol

    def __matmul__(self, V: np.ndarray) -> np.ndarray:
        return leja_expmv(self.AT, self.t, V, self.tol)


def quadrature_factor_leja(A, C, t, K, tol, leja_tol: float = 1e-14):
    """``quadrature_factor`` with the node actions e^{s_k A^T} C^T by
    ``leja_expmv`` (Alg. 2 with expleja, as in the paper's Sec. 3)."""
    s, w = gauss_legendre(K, t)
    p = C.shape[0]
    AT = np.ascontiguousarray(np.asarray(A, dtype=np.float64).T)
    cols = [leja_expmv(AT, sk, np.ascontiguousarray(C.T), leja_tol) for sk in s]
    blocks = [wk * np.eye(p) for wk in w]
    return compress(np.hstack(cols), _blkdiag(*blocks), tol)


# ----------------------------------------------------------------------------
# Quadrature (Alg. 2, "Approximate integral")
# ----------------------------------------------------------------------------
def gauss_legendre(K: int, t: float):
    """K-point Gauss-Legendre nodes s_k and weights w_k on [0, t].

    Pin: exact integration of monomials of degree <= 2K-1 on [0, t].
    """
    x, w = np.polynomial.legendre.leggauss(K)
    return 0.5 * t * (x + 1.0), 0.5 * t * w


# ----------------------------------------------------------------------------
# Column compression (Sec. 3, after Alg. 2)
# ----------------------------------------------------------------------------
def compress(L: np.ndarray, D: np.ndarray, tol: float):
    """Column compression of P = L D L^T.

    Householder QR L = Q R (numpy/LAPACK geqrf), M = R D R^T, M = V Lam V^T,
    keep |lam_i| > tol * max_j |lam_j| (sorted by |lam| descending), return
    (Q V_I, diag(lam_I)).

    Pins: the kept part reproduces L D L^T up to the dropped eigenvalues;
    L^T L = I; the full-rank case is exact.
    """
    n, k = L.shape
    if k == 0:
        return np.zeros((n, 0)), np.zeros((0, 0))
    Q, R = np.linalg.qr(L, mode="reduced")
    M = R @ D @ R.T
    M = 0.5 * (M + M.T)
    lam, V = np.linalg.eigh(M)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam = lam[order]
    V = V[:, order]
    amax = abs(lam[0]) if lam.size else 0.0
    if amax == 0.0:
        return np.zeros((n, 0)), np.zeros((0, 0))
    keep = np.abs(lam) > tol * amax
    lam = lam[keep]
    V = V[:, keep]
    return Q @ V, np.diag(lam)


# ----------------------------------------------------------------------------
# Subflows
# ----------------------------------------------------------------------------
def t1(L: np.ndarray, E: np.ndarray) -> np.ndarray:
    """T1(t): L <- e^{tA^T} L, with E = e^{tA^T} (Sec. 2.1, eq. F_sol_LDL)."""
    return E @ L


def t2(L, D, C, t, tol):
    """T2(t): P + t Q with Q = C^T C = L_Q D_Q L_Q^T, L_Q = C^T, D_Q = I (Sec. 2.1);
    concatenate and compress (Alg. 1)."""
    p = C.shape[0]
    Lc = np.hstack([L, C.T])
    Dc = _blkdiag(D, t * np.eye(p))
    return compress(Lc, Dc, tol)


def quadrature_factor(A, C, t, K, tol):
    """(L_I, D_I) of Alg. 2: L_I = [e^{s_1 A^T} L_Q, ..., e^{s_K A^T} L_Q],
    D_I = blkdiag(w_1 D_Q, ..., w_K D_Q), compressed, with L_Q = C^T, D_Q = I.

    Pin: in the eigenbasis of a symmetric A the result equals
    Qt o sum_k w_k e^{mu s_k} (mu_ij = lam_i + lam_j).
    """
    s, w = gauss_legendre(K, t)
    p = C.shape[0]
    cols, blocks = [], []
    AT = np.ascontiguousarray(A.T)
    for sk, wk in zip(s, w):
        cols.append(expm(sk * AT) @ C.T)
        blocks.append(wk * np.eye(p))
    return compress(np.hstack(cols), _blkdiag(*blocks), tol)


def t12(L, D, E, LI, DI, tol):
    """T12(t) of Alg. 2: L <- [e^{tA^T} L, L_I], D <- blkdiag(D, D_I), compress."""
    return compress(np.hstack([E @ L, LI]), _blkdiag(D, DI), tol)


def t3(L, D, B, R, t):
    """T3(t) of Sec. 2.2 / Alg. 3 (with the B^T of the Sec. 2.2 formula):
    D <- (I + t D L^T B R^-1 B^T L)^-1 D, symmetrised.

    Pins: equals the dense (I + t P B R^-1 B^T)^-1 P; T3(a) T3(b) = T3(a + b);
    scalar recursion p <- p / (1 + t g p) in the commuting case.
    """
    r = L.shape[1]
    if r == 0:
        return D
    W = L.T @ B
    G = W @ np.linalg.solve(R, W.T)
    X = np.linalg.solve(np.eye(r) + t * D @ G, D)
    return 0.5 * (X + X.T)


def feedback_gain(L, D, B, R):
    """Feedback gain K = R^-1 B^T P (m x n) of the LQR problem behind the DRE
    (Sec. 1, the LQR setting; the optimal input is u = -K x with P the DRE
    solution at the remaining horizon), from the factors P = L D L^T.

    Pins: invariant under L -> L G, D -> G^-1 D G^-T (the same P); linear in
    R^-1; the scalar DRE's closed-form solution gives K = b p(t) / r.
    """
    m, n = B.shape[1], B.shape[0]
    if L.shape[1] == 0:
        return np.zeros((m, n))
    return np.linalg.solve(R, ((B.T @ L) @ D) @ L.T)


def t4(L, D, S, t, tol):
    """T4(t) of Sec. 2.3 / Alg. 4 (midpoint rule):
    L <- [L, sqrt(t) S L, t/sqrt(2) S^2 L], D <- blkdiag(D, D, D), compress.

    Pin: reproduces P + t S P S^T + t^2/2 S^2 P S^2^T exactly before truncation.
    """
    SL = S @ L
    S2L = S @ SL
    Lc = np.hstack([L, math.sqrt(t) * SL, (t / math.sqrt(2.0)) * S2L])
    return compress(Lc, _blkdiag(D, D, D), tol)


def _blkdiag(*blocks):
    n = sum(b.shape[0] for b in blocks)
    out = np.zeros((n, n))
    o = 0
    for b in blocks:
        k = b.shape[0]
        out[o:o + k, o:o + k] = b
        o += k
    return out


# ----------------------------------------------------------------------------
# Mass-matrix form (Sec. 5.1, Example 4)
# ----------------------------------------------------------------------------
def mass_matrix_form(A, C, M):
    """Standard-form data of M^T dP/dt M = A^T P M + M^T P A + C^T C + G
    (G = -M^T P B R^-1 B^T P M for the DRE): multiplying by M^-T on the left
    and M^-1 on the right gives dP/dt = At^T P + P At + Ct^T Ct - P B R^-1 B^T P
    with At = A M^-1 and Ct = C M^-1 (B, R unchanged).  Returns (At, Ct).

    Pins: At^T P + P At + Ct^T Ct equals M^-T (A^T P M + M^T P A + Q) M^-1 for
    any P; a brute-force integration of the equation with M reproduces the
    split solution at its order; M = I changes nothing.
    """
    A = np.asarray(A, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    At = np.linalg.solve(M.T, A.T).T   # A M^-1
    Ct = np.linalg.solve(M.T, C.T).T   # C M^-1
    return At, Ct


# ----------------------------------------------------------------------------
# Schemes (Sec. 2, Sec. 3)
# ----------------------------------------------------------------------------
def step_sequence(kind: str, has_S: bool, split: str, scheme: str):
    """Subflows of one step, in application order, as (name, fraction of h).

    kind: "dle" (G = 0) or "dre"; has_S: generalized equation; split: "F12"
    (linear part solved with the quadrature formula), "F1F2" (Q split off;
    three-term for DRE), "F1F3F2" (reversed three-term); scheme: "lie"/"strang".
    """
    strang = scheme == "strang"
    if scheme not in ("lie", "strang"):
        raise OracleError(f"unknown scheme {scheme}")
    G = "T3" if kind == "dre" else None
    if kind not in ("dle", "dre"):
        raise OracleError(f"unknown kind {kind}")
    if split == "F12":
        inner = [x for x in (G, "T4" if has_S else None) if x]
        if not inner:
            return [("T12", 1.0)]                                   # Alg. 2
        if not strang:
            return [("T12", 1.0)] + [(x, 1.0) for x in inner]
        if len(inner) == 1:
            return [("T12", 0.5), (inner[0], 1.0), ("T12", 0.5)]    # Sec. 3
        # generalized DRE: T12(h/2) T3(h/2) T4(h) T3(h/2) T12(h/2)
        return [("T12", 0.5), ("T3", 0.5), ("T4", 1.0), ("T3", 0.5), ("T12", 0.5)]
    if split == "F1F2":
        third = [x for x in (G, "T4" if has_S else None) if x]
        if len(third) > 1:
            raise OracleError("four-term splitting is not part of the method")
        if not third:
            if not strang:
                return [("T1", 1.0), ("T2", 1.0)]
            return [("T1", 0.5), ("T2", 1.0), ("T1", 0.5)]          # Alg. 1
        x = third[0]
        if not strang:
            return [("T1", 1.0), ("T2", 1.0), (x, 1.0)]
        return [("T1", 0.5), ("T2", 0.5), (x, 1.0), ("T2", 0.5), ("T1", 0.5)]
    if split == "F1F3F2":
        third = [x for x in (G, "T4" if has_S else None) if x]
        if len(third) != 1:
            raise OracleError("F1F3F2 needs exactly one of B (DRE) or S")
        x = third[0]
        if not strang:
            return [("T1", 1.0), (x, 1.0), ("T2", 1.0)]
        return [("T1", 0.5), (x, 0.5), ("T2", 1.0), (x, 0.5), ("T1", 0.5)]
    raise OracleError(f"unknown split {split}")


def num_steps(T: float, h: float) -> int:
    if not (h > 0 and T > 0):
        raise OracleError("T and h must be positive")
    N = int(round(T / h))
    if N < 1 or abs(N * h - T) > 1e-12 * T:
        raise OracleError("T/h is not an integer")
    return N


def solve(A, C, T, h, *, kind="dle", B=None, R=None, S=None, L0=None, D0=None,
          split="F12", scheme="strang", tol=1e-10, quad_nodes=7,
          expm_fn=None, quad_fn=None, record_ranks=False, M=None):
    """Run the splitting scheme from P0 = L0 D0 L0^T to time T with step h.

    expm_fn(t) -> e^{tA^T} and quad_fn(t) -> (L_I, D_I) may be supplied (used
    for the Kronecker-structured Laplacian at large n); by default they are
    the generic ``expm`` and ``quadrature_factor`` above.  With a mass matrix
    M the equation M^T dP/dt M = ... is first put in standard form
    (``mass_matrix_form``).

    Returns (L, D, info) with P(T) ~ L D L^T.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    C = np.asarray(C, dtype=np.float64)
    if M is not None:
        A, C = mass_matrix_form(A, C, M)
    N = num_steps(T, h)
    seq = step_sequence(kind, S is not None, split, scheme)
    if kind == "dre":
        if B is None or R is None:
            raise OracleError("DRE needs B and R")
        B = np.asarray(B, dtype=np.float64)
        R = np.asarray(R, dtype=np.float64)
        np.linalg.cholesky(R)  # R must be SPD
    if L0 is None or (hasattr(L0, "shape") and L0.shape[1] == 0):
        L = np.zeros((n, 0))
        D = np.zeros((0, 0))
    else:
        L = np.asarray(L0, dtype=np.float64).copy()
        D = np.asarray(D0, dtype=np.float64).copy()
    AT = np.ascontiguousarray(A.T)
    if expm_fn is None:
        expm_fn = lambda t: expm(t * AT)  # noqa: E731
    if quad_fn is None:
        quad_fn = lambda t: quadrature_factor(A, C, t, quad_nodes, tol)  # noqa: E731
    E_cache, Q_cache = {}, {}
    for name, frac in seq:
        t = frac * h
        if name in ("T1", "T12") and t not in E_cache:
            E_cache[t] = expm_fn(t)
        if name == "T12" and t not in Q_cache:
            Q_cache[t] = quad_fn(t)
    ranks = []
    for _ in range(N):
        for name, frac in seq:
            t = frac * h
            if name == "T1":
                L = t1(L, E_cache[t])
            elif name == "T2":
                L, D = t2(L, D, C, t, tol)
            elif name == "T12":
                LI, DI = Q_cache[t]
                L, D = t12(L, D, E_cache[t], LI, DI, tol)
            elif name == "T3":
                D = t3(L, D, B, R, t)
            elif name == "T4":
                L, D = t4(L, D, np.asarray(S, dtype=np.float64), t, tol)
        if record_ranks:
            ranks.append(L.shape[1])
    return L, D, {"steps": N, "sequence": seq, "ranks": ranks}


# ----------------------------------------------------------------------------
# Low-rank error metric
# ----------------------------------------------------------------------------
def lowrank_fro(L, D) -> float:
    """||L D L^T||_F without forming the n x n product."""
    if L.shape[1] == 0:
        return 0.0
    _, Rz = np.linalg.qr(L, mode="reduced")
    return float(np.linalg.norm(Rz @ D @ Rz.T, "fro"))


def lowrank_rel_err(L1, D1, L2, D2) -> float:
    """||L1 D1 L1^T - L2 D2 L2^T||_F / ||L2 D2 L2^T||_F via one thin QR of [L1, L2]."""
    diff = lowrank_fro(np.hstack([L1, L2]), _blkdiag(D1, -D2))
    ref = lowrank_fro(L2, D2)
    if ref == 0.0:
        return diff
    return diff / ref


# ----------------------------------------------------------------------------
# Kronecker-sum Laplacian (large-n evaluation of the same exponentials)
# ----------------------------------------------------------------------------
def laplacian_expm_kron(A1: np.ndarray, t: float) -> np.ndarray:
    """e^{tA} for A = I (x) A1 + A1 (x) I (x index fastest), using
    e^{t(A1 (+) A1)} = e^{tA1} (x) e^{tA1}; the 1-D factor comes from ``expm``.

    Pin: equals ``expm(t A)`` at small n.
    """
    E1 = expm(t * np.ascontiguousarray(A1.T))
    return np.kron(E1, E1)


def kron_apply_expm(E1: np.ndarray, V: np.ndarray) -> np.ndarray:
    """(E1 (x) E1) V without forming the Kronecker product (columns of V are
    vec(X) with X nx x nx, x fastest): vec(E1 X E1^T)."""
    nx = E1.shape[0]
    out = np.empty_like(V)
    for j in range(V.shape[1]):
        X = V[:, j].reshape(nx, nx, order="F")
        out[:, j] = (E1 @ X @ E1.T).reshape(-1, order="F")
    return out


class KronExpm:
    """e^{tA^T} for A = I (x) A1 + A1 (x) I as an operator: ``E @ V`` applies
    e^{tA1^T} (x) e^{tA1^T} through ``kron_apply_expm`` instead of forming the
    n x n matrix (for ``solve(expm_fn=...)`` at large n; same values as
    ``laplacian_expm_kron(A1, t) @ V``)."""

    def __init__(self, A1: np.ndarray, t: float):
        self.E1 = expm(t * np.ascontiguousarray(A1.T))

    def __matmul__(self, V: np.ndarray) -> np.ndarray:
        return kron_apply_expm(self.E1, np.asarray(V, dtype=np.float64))


def quadrature_factor_kron(A1, C, t, K, tol):
    """``quadrature_factor`` for the Kronecker-sum Laplacian."""
    s, w = gauss_legendre(K, t)
    p = C.shape[0]
    cols, blocks = [], []
    for sk, wk in zip(s, w):
        E1 = expm(sk * np.ascontiguousarray(A1.T))
        cols.append(kron_apply_expm(E1, np.ascontiguousarray(C.T)))
        blocks.append(wk * np.eye(p))
    return compress(np.hstack(cols), _blkdiag(*blocks), tol)
