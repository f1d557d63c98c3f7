"""Pins of the oracle's Chebyshev-Neumann series solve (CNS):
x_T = sum_{k<=T} (I - phi A)^k phi B with phi = X_m, the NN iterate.

* exact rationals: with phi from m nests at depth d, I - phi A = P^((d+1)^m)
  (P = I - phi_0 A), so the CNS is the plain Neumann series of order
  (d+1)^m (T+1) - 1 in P applied to B (the reading of the order formula the
  paper prints garbled) — checked against exact.neumann_series;
* the series equals T steps of refinement x <- x + phi (B - A x) from phi B
  (Horner form, the form the device evaluates);
* T = 0 is phi B; convergence to numpy.linalg.solve; statuses.
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


@pytest.mark.parametrize("d,m,T", [(2, 1, 0), (2, 1, 2), (2, 2, 1), (1, 2, 3), (3, 1, 1)])
def test_exact_order_formula(d, m, T):
    A = [[5, 1, 0], [1, 4, 1], [0, 1, 3]]
    B = [[1, 0], [2, 1], [0, 3]]
    Af, Bf = ex.to_frac(A), ex.to_frac(B)
    phi0 = ex.x0_transpose(Af)
    P = ex.sub(ex.eye(3), ex.matmul(phi0, Af))
    order = (d + 1) ** m * (T + 1) - 1
    want = ex.matmul(ex.neumann_series(P, phi0, order), Bf)
    want = np.array([[float(v) for v in r] for r in want])
    x, info = oracle.nn_cns_solve_ref(np.array(A, float), np.array(B, float), d=d,
                                      nests=m, fixed_terms=T)
    assert info["status"] == oracle.OK and info["terms"] == T and info["nests"] == m
    assert _rel(x, want) < 1e-12


def test_series_equals_refinement_steps():
    A = W.dense_spd(60, 1.0, 200.0, 81)
    B = W.rng(82).standard_normal((60, 4))
    X2, _ = oracle.nn_ref(A, d=2, fixed_iter=3)
    for T in (0, 1, 5):
        x, _ = oracle.nn_cns_solve_ref(A, B, nests=3, fixed_terms=T)
        y = X2 @ B
        for _ in range(T):
            y = y + X2 @ (B - A @ y)
        assert _rel(x, y) < 1e-12, T


def test_zero_terms_is_phi_b():
    A = W.dense_spd(30, 1.0, 20.0, 83)
    B = W.rng(84).standard_normal((30, 2))
    X, _ = oracle.nn_ref(A, d=2, fixed_iter=2)
    x, info = oracle.nn_cns_solve_ref(A, B, nests=2, fixed_terms=0)
    assert np.array_equal(x, X @ B)
    assert info["trace"] == [info["rel_residual"]]


@pytest.mark.parametrize("cplx", [False, True])
def test_converges_to_numpy_solve(cplx):
    n = 50
    A = W.dense_spd(n, 1.0, 300.0, 85, complex_=cplx)
    g = W.rng(86)
    B = g.standard_normal((n, 3)) + (1j * g.standard_normal((n, 3)) if cplx else 0.0)
    # the series as printed forms Q = I - phi A once, so it floors near
    # kappa-scaled rounding of Q (~2e-13 here): ask for 1e-12
    x, info = oracle.nn_cns_solve_ref(A, B, nests=0, precond_tol=1e-2, tol=1e-12)
    assert info["status"] == oracle.OK and info["rel_residual"] < 1e-12
    assert info["precond_rms"] < 1e-2 and info["terms"] >= 1
    assert _rel(x, np.linalg.solve(A, B)) <= 300.0 * 1e-12 * 1.01


def test_statuses():
    n = 20
    B = np.ones((n, 1))
    _, info = oracle.nn_cns_solve_ref(-np.eye(n), B, x0=oracle.X0_SCALED_IDENTITY, nests=2)
    assert info["status"] == oracle.ERR_DIVERGED
    A = W.dense_spd(n, 1.0, 30.0, 87)
    _, info = oracle.nn_cns_solve_ref(A, B, nests=1, tol=1e-15, max_terms=2)
    assert info["status"] == oracle.NOT_CONVERGED and info["terms"] == 2
    _, info = oracle.nn_cns_solve_ref(A, B, nests=12, tol=0.0)
    assert info["status"] == oracle.STAGNATED and info["rel_residual"] < 1e-13
