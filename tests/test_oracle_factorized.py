"""Pins of the oracle's factorised solve (Corollary 6 applied to a right-hand
side): x_s = prod_{n<s} (I + P^(2^n)) phi B with P = I - phi A.

Each check fixes the result by something other than the function itself:
exact rational arithmetic of the corollary (pinned in test_oracle_exact
against the truncated Neumann series), the equality with s Newton nests
applied to B (nn_ref with d = 1), spectral and diagonal closed forms,
numpy.linalg.solve at convergence, and the monotone residual of Hermitian
inputs.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact as ex
from paper_2212_02406_amd import workloads as W


def _rel(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY])
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_matches_exact_corollary6(x0, s):
    A = [[4, 1, 0], [1, 3, 1], [0, 1, 2]]
    B = [[1, 2], [0, -1], [3, 1]]
    Af, Bf = ex.to_frac(A), ex.to_frac(B)
    phi = ex.x0_transpose(Af) if x0 == oracle.X0_TRANSPOSE else ex.x0_scaled_identity(Af)
    P = ex.sub(ex.eye(3), ex.matmul(phi, Af))
    want = ex.matmul(ex.factorised_series(P, phi, s), Bf)
    want = np.array([[float(v) for v in r] for r in want])
    x, info = oracle.nn_factorized_solve_ref(np.array(A, float), np.array(B, float), x0=x0,
                                             fixed_factors=s)
    assert info["status"] == oracle.OK and info["factors"] == s
    assert _rel(x, want) < 1e-13


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY])
def test_equals_newton_nests_applied_to_b(x0):
    """s factors give the series of order 2^s - 1, which is also what s
    Newton nests (d = 1) produce (Corollary 2)."""
    A = W.dense_spd(40, 1.0, 30.0, 71)
    B = W.rng(72).standard_normal((40, 5))
    for s in (1, 3, 6):
        x, _ = oracle.nn_factorized_solve_ref(A, B, x0=x0, fixed_factors=s)
        X, _ = oracle.nn_ref(A, d=1, x0=x0, fixed_iter=s)
        assert _rel(x, X @ B) < 1e-11, s


def test_diagonal_closed_forms():
    a = np.array([0.5, 1.0, 2.5, 4.0, 7.0])
    A = np.diag(a)
    B = np.arange(1.0, 11.0).reshape(5, 2)
    for s in (1, 2, 5):
        m = 2 ** s
        x, _ = oracle.nn_factorized_solve_ref(A, B, x0=oracle.X0_TRANSPOSE, fixed_factors=s)
        c = (1.0 - (1.0 - a ** 2 / a.max() ** 2) ** m) / a
        assert _rel(x, c[:, None] * B) < 1e-14
        x, _ = oracle.nn_factorized_solve_ref(A, B, x0=oracle.X0_SCALED_IDENTITY, fixed_factors=s)
        c = (1.0 - (1.0 - a / a.sum()) ** m) / a
        assert _rel(x, c[:, None] * B) < 1e-14


def test_spectral_closed_form_identity_start():
    n = 30
    A, lam, Q = W.dense_spd(n, 1.0, 20.0, 73, return_factors=True)
    B = W.rng(74).standard_normal((n, 3))
    tr = lam.sum()
    for s in (2, 4, 7):
        x, _ = oracle.nn_factorized_solve_ref(A, B, x0=oracle.X0_SCALED_IDENTITY, fixed_factors=s)
        f = (1.0 - (1.0 - lam / tr) ** (2 ** s)) / lam
        ref = (Q * f) @ (Q.T @ B)
        assert _rel(x, ref) < 1e-12, s


@pytest.mark.parametrize("cplx", [False, True])
def test_converged_solution_matches_numpy(cplx):
    n = 48
    A = W.dense_spd(n, 1.0, 50.0, 75, complex_=cplx)
    g = W.rng(76)
    B = g.standard_normal((n, 4)) + (1j * g.standard_normal((n, 4)) if cplx else 0.0)
    x, info = oracle.nn_factorized_solve_ref(A, B, tol=1e-12)
    assert info["status"] == oracle.OK and info["rel_residual"] < 1e-12
    ref = np.linalg.solve(A, B)
    # x - A^-1 B = -A^-1 r: relative error <= kappa * rel_residual
    assert _rel(x, ref) <= 50.0 * 1e-12 * 1.01
    # the series order reached is 2^factors - 1; for the transpose start the
    # slowest mode decays like (1 - lam_min^2 / den)^(2^s)
    assert info["factors"] >= 1


def test_residual_never_increases_for_hermitian_input():
    A = W.dense_spd(64, 1.0, 100.0, 77)
    B = W.rng(78).standard_normal((64, 2))
    for x0 in (oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY):
        _, info = oracle.nn_factorized_solve_ref(A, B, x0=x0, fixed_factors=20)
        tr = info["trace"]
        assert all(b <= a * (1 + 1e-12) + 1e-15 for a, b in zip(tr, tr[1:]))


def test_statuses():
    n = 16
    B = np.ones((n, 1))
    _, info = oracle.nn_factorized_solve_ref(-np.eye(n), B, x0=oracle.X0_SCALED_IDENTITY)
    assert info["status"] == oracle.ERR_DIVERGED and info["factors"] == 0
    A = W.dense_spd(n, 1.0, 10.0, 79)
    An = A.copy()
    An[2, 3] = np.nan
    _, info = oracle.nn_factorized_solve_ref(An, B)
    assert info["status"] == oracle.ERR_NONFINITE
    _, info = oracle.nn_factorized_solve_ref(A, B, tol=1e-14, max_factors=2)
    assert info["status"] == oracle.NOT_CONVERGED and info["factors"] == 2
    x, info = oracle.nn_factorized_solve_ref(A, B, tol=0.0)
    assert info["status"] == oracle.STAGNATED
    assert info["rel_residual"] < 1e-13
    assert info["trace"][info["factors"]] == info["rel_residual"]
