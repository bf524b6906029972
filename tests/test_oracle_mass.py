"""Pins for the mass-matrix form of the oracle (Sec. 5.1, Example 4):
M^T dP/dt M = A^T P M + M^T P A + Q - M^T P B R^-1 B^T P M."""
import numpy as np
import pytest

import oracle as o
from oracle import dme_oracle as od
import workloads as w


def _generalized_rhs(A, M, C, B, R, P):
    """dP/dt of the equation with M, straight from its definition: solve
    M^T X M = A^T P M + M^T P A + C^T C - M^T P B R^-1 B^T P M for X."""
    F = A.T @ P @ M + M.T @ P @ A + C.T @ C - M.T @ P @ B @ np.linalg.solve(R, B.T) @ P @ M
    return np.linalg.solve(M.T, np.linalg.solve(M.T, F.T).T)  # M^-T F M^-1


def test_standard_form_has_the_same_right_hand_side():
    nx = 4
    A, M = w.fe_heat_2d(nx)
    n = nx * nx
    rng = np.random.default_rng(2)
    C = rng.standard_normal((3, n))
    B = w.quadrant_B(nx, 2)
    R = np.eye(2) * 1.5
    X = rng.standard_normal((n, n))
    P = X @ X.T
    At, Ct = o.mass_matrix_form(A, C, M)
    std = At.T @ P + P @ At + Ct.T @ Ct - P @ B @ np.linalg.solve(R, B.T) @ P
    ref = _generalized_rhs(A, M, C, B, R, P)
    assert np.linalg.norm(std - ref) <= 1e-12 * np.linalg.norm(ref)


def test_identity_mass_matrix_changes_nothing():
    p = w.config_dre_halfplane(nx=6, h=1e-2)
    L1, D1, _ = o.solve(p.A, p.C, p.T, p.h, kind="dre", B=p.B, R=p.R, tol=p.tol)
    L2, D2, _ = o.solve(p.A, p.C, p.T, p.h, kind="dre", B=p.B, R=p.R, tol=p.tol, M=np.eye(p.n))
    assert o.lowrank_rel_err(L2, D2, L1, D1) < 1e-13


def _rk4_reference(A, M, C, B, R, T, dt):
    n = A.shape[0]
    P = np.zeros((n, n))
    for _ in range(int(round(T / dt))):
        k1 = _generalized_rhs(A, M, C, B, R, P)
        k2 = _generalized_rhs(A, M, C, B, R, P + 0.5 * dt * k1)
        k3 = _generalized_rhs(A, M, C, B, R, P + 0.5 * dt * k2)
        k4 = _generalized_rhs(A, M, C, B, R, P + dt * k3)
        P = P + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return P


def test_split_solution_converges_to_the_equation_with_M():
    """Strang F12F3 on the mass-matrix DRE against a brute-force RK4 solution
    of M^T dP/dt M = ... (built from the definition, not from the transformed
    data): second-order decrease of the error as h halves."""
    p = w.config_dre_mass(nx=3, T=0.02, h=4e-3)
    Pref = _rk4_reference(p.A, p.M, p.C, p.B, p.R, p.T, 2.5e-5)
    errs = []
    for h in (4e-3, 2e-3, 1e-3):
        L, D, _ = o.solve(p.A, p.C, p.T, h, kind="dre", B=p.B, R=p.R, M=p.M, tol=1e-14)
        errs.append(np.linalg.norm(L @ D @ L.T - Pref) / np.linalg.norm(Pref))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 1e-4
    assert all(abs(r - 2.0) < 0.25 for r in rates), (errs, rates)


def _wrong_mass_form(A, C, M):  # M^-1 A (the order of the paper's phrase) in place of A M^-1
    return np.linalg.solve(M, A), np.linalg.solve(M.T, C.T).T


def test_planted_mass_mistake_is_caught(monkeypatch):
    monkeypatch.setattr(od, "mass_matrix_form", _wrong_mass_form)
    monkeypatch.setattr(o, "mass_matrix_form", _wrong_mass_form)
    with pytest.raises(AssertionError):
        test_standard_form_has_the_same_right_hand_side()
    with pytest.raises(AssertionError):
        test_split_solution_converges_to_the_equation_with_M()
