"""Plant plausible mistakes in the oracle (on the CPU, via monkeypatch) and
check that the pins catch each one."""
import math

import numpy as np
import pytest

import oracle as o
from oracle import dme_oracle as od
import workloads as w
from tests import test_oracle_order as t_order
from tests import test_oracle_schemes as t_schemes
from tests import test_oracle_subflows as t_sub
from tests import test_oracle_quadrature as t_quad


_orig_expm = od.expm


def _wrong_expm(X):             # e^{tA} used where e^{tA^T} is meant
    return _orig_expm(np.ascontiguousarray(X.T))


def _wrong_t3(L, D, B, R, t):   # R instead of R^-1
    r = L.shape[1]
    if r == 0:
        return D
    W = L.T @ B
    X = np.linalg.solve(np.eye(r) + t * D @ W @ R @ W.T, D)
    return 0.5 * (X + X.T)


def _wrong_t4(L, D, S, t, tol):  # t/2 instead of t/sqrt(2)
    SL = S @ L
    Lc = np.hstack([L, math.sqrt(t) * SL, 0.5 * t * (S @ SL)])
    return od.compress(Lc, od._blkdiag(D, D, D), tol)


def _wrong_gl(K, t):             # weights not mapped to [0, t]
    x, wt = np.polynomial.legendre.leggauss(K)
    return 0.5 * t * (x + 1.0), wt


def _wrong_seq(kind, has_S, split, scheme):  # Strang with full-step T12 halves
    seq = _orig_seq(kind, has_S, split, scheme)
    return [(n, 1.0 if n == "T12" else f) for n, f in seq]


_orig_seq = od.step_sequence


def _run_nonsym_dle():
    t_order.test_nonsymmetric_dle_quadrature_exact()


def _run_t3_dense():
    t_sub.test_t3_equals_dense_formula()


def _run_t4():
    t_sub.test_t4_midpoint_formula()


def _run_quad():
    t_quad.test_quadrature_factor_eigenbasis()


def _run_commuting():
    t_schemes.test_dre_commuting_continuous_limit()


@pytest.mark.parametrize("target,replacement,check", [
    ("expm", _wrong_expm, _run_nonsym_dle),
    ("t3", _wrong_t3, _run_t3_dense),
    ("t4", _wrong_t4, _run_t4),
    ("gauss_legendre", _wrong_gl, _run_quad),
    ("step_sequence", _wrong_seq, _run_commuting),
])
def test_planted_mistake_is_caught(monkeypatch, target, replacement, check):
    monkeypatch.setattr(od, target, replacement)
    monkeypatch.setattr(o, target, replacement, raising=False)
    with pytest.raises(AssertionError):
        check()
