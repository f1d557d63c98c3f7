"""Pins of the exact-rational oracle against the paper's closed forms.

Every assertion here is an equality of rational matrices: the NN iteration
(Sec. II-D, Theorem) against its closed forms —
  T1  Corollary 2 / Appendix 4: k nests = Neumann series with (L+1)^k terms
  T2  Appendix 2 (norm step, written as an equality): R_k = R_0^((L+1)^k)
  T3  Corollary 1 / Appendix 3: the explicit product form
  T4  Corollary 4: L = 1 is Newton's step (Sec. II-B), L = 2 Chebyshev's
      (Sec. II-C)
  T5  Corollary 6 / Appendix 7: the binary factorisation of the series
and the reading that the right form X * sum (I - A X)^n equals the printed
left form sum (I - phi W)^n phi.  Matrix products in this file are written
out here (``_mm``), not borrowed from the oracle, so a slip in the oracle's
own helpers shows.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import exact as ex

# Small integer matrices: SPD, non-symmetric, 2x2 and 4x4.
MATS = {
    "spd3": [[4, 1, 0], [1, 3, 1], [0, 1, 2]],
    "nonsym3": [[5, 2, -1], [1, 4, 0], [2, -1, 6]],
    "spd2": [[3, 1], [1, 2]],
    "nonsym4": [[2, 1, 0, 0], [0, 3, 1, 0], [1, 0, 4, 1], [0, 1, 0, 5]],
}
SPD = {"spd3", "spd2"}


def _F(A):
    return [[Fraction(v) for v in r] for r in A]


def _mm(A, B):
    n, m, p = len(A), len(B), len(B[0])
    return [[sum((A[i][t] * B[t][j] for t in range(m)), Fraction(0)) for j in range(p)]
            for i in range(n)]


def _I(n):
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


def _sub(A, B):
    return [[a - b for a, b in zip(x, y)] for x, y in zip(A, B)]


def _add(A, B):
    return [[a + b for a, b in zip(x, y)] for x, y in zip(A, B)]


def _pow(P, e):
    out = _I(len(P))
    for _ in range(e):
        out = _mm(out, P)
    return out


def _x0(A, kind):
    n = len(A)
    if kind == "transpose":
        n1 = max(sum(abs(A[i][j]) for i in range(n)) for j in range(n))
        ni = max(sum(abs(v) for v in row) for row in A)
        s = Fraction(1, 1) / (n1 * ni)
        return [[s * A[j][i] for j in range(n)] for i in range(n)]
    tr = sum(A[i][i] for i in range(n))
    return [[Fraction(int(i == j)) / tr for j in range(n)] for i in range(n)]


def _cases():
    for name in MATS:
        kinds = ["transpose", "identity"] if name in SPD else ["transpose"]
        for kind in kinds:
            for d in (1, 2, 3):
                for k in (1, 2):
                    yield name, kind, d, k


def test_helpers_match_numpy():
    """The oracle's rational matmul/transpose/norms agree with NumPy on integers."""
    for A in MATS.values():
        An = np.array(A, dtype=np.int64)
        F = ex.to_frac(A)
        assert ex.matmul(F, F) == _F((An @ An).tolist())
        assert ex.transpose(F) == _F(An.T.tolist())
        assert ex.norm_1(F) == np.abs(An).sum(axis=0).max()
        assert ex.norm_inf(F) == np.abs(An).sum(axis=1).max()
        assert ex.x0_transpose(F) == _x0(F, "transpose")


@pytest.mark.parametrize("name,kind,d,k", list(_cases()))
def test_T1_T2_nests_equal_neumann_series(name, kind, d, k):
    A = _F(MATS[name])
    n = len(A)
    X0 = _x0(A, kind)
    X = ex.nn_iterate(A, X0, d, k)
    R0 = _sub(_I(n), _mm(A, X0))
    terms = (d + 1) ** k
    # T1 (right form): X_k = X_0 sum_{m < (d+1)^k} R_0^m
    S = _I(n)
    Rm = _I(n)
    for _ in range(terms - 1):
        Rm = _mm(Rm, R0)
        S = _add(S, Rm)
    assert X == _mm(X0, S)
    # T1 (left form, as printed): sum_{m < (d+1)^k} P_0^m phi_0, P_0 = I - phi_0 W
    P0 = _sub(_I(n), _mm(X0, A))
    Sl = _I(n)
    Pm = _I(n)
    for _ in range(terms - 1):
        Pm = _mm(Pm, P0)
        Sl = _add(Sl, Pm)
    assert X == _mm(Sl, X0)
    # T2: R_k = R_0^((d+1)^k)
    assert _sub(_I(n), _mm(A, X)) == _pow(R0, terms)
    # the oracle's own series helper agrees
    assert ex.neumann_series(P0, X0, terms - 1) == X


@pytest.mark.parametrize("name,kind,d,k", list(_cases()))
def test_left_form_equals_right_form(name, kind, d, k):
    A = _F(MATS[name])
    X0 = _x0(A, kind)
    assert ex.nn_iterate(A, X0, d, k, left=True) == ex.nn_iterate(A, X0, d, k, left=False)


@pytest.mark.parametrize("name", sorted(SPD))
@pytest.mark.parametrize("d", [1, 2, 3])
def test_theta_folding(name, d):
    """The paper iterates phi on W~ = Theta W from phi^(0) = I and returns
    phi Theta (Theorem of Sec. II-D, Algorithm 1).  We iterate X directly
    from X_0 = Theta I.  After k nests phi_k Theta == X_k exactly."""
    A = _F(MATS[name])
    n = len(A)
    theta = Fraction(1) / sum(A[i][i] for i in range(n))
    Wt = [[theta * v for v in row] for row in A]
    phi = _I(n)
    X = _x0(A, "identity")
    for _ in range(3):
        phi = ex.nn_step_left(Wt, phi, d)
        X = ex.nn_step_right(A, X, d)
        assert [[theta * v for v in row] for row in phi] == X


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("L", [1, 2, 3])
@pytest.mark.parametrize("i", [0, 1, 2])
def test_T3_product_form(name, L, i):
    """Corollary 1: phi^(i+1) = prod_j sum_n P0^(n (L+1)^j) phi0 — checked
    against i+1 nests of the printed (left) recursion."""
    W = _F(MATS[name])
    phi0 = _x0(W, "transpose")
    assert ex.product_form(W, phi0, L, i) == ex.nn_iterate(W, phi0, L, i + 1, left=True)


@pytest.mark.parametrize("name", sorted(MATS))
def test_T4_newton_chebyshev(name):
    A = _F(MATS[name])
    X = _x0(A, "transpose")
    for _ in range(2):
        assert ex.nn_step_right(A, X, 1) == ex.newton_step(A, X)
        assert ex.nn_step_right(A, X, 2) == ex.chebyshev_step(A, X)
        # written out here once more: Newton X(2I - AX), Chebyshev X(3I - AX(3I - AX))
        n = len(A)
        AX = _mm(A, X)
        two = [[2 * v for v in r] for r in _I(n)]
        three = [[3 * v for v in r] for r in _I(n)]
        assert ex.nn_step_right(A, X, 1) == _mm(X, _sub(two, AX))
        assert ex.nn_step_right(A, X, 2) == _mm(X, _sub(three, _mm(AX, _sub(three, AX))))
        X = ex.nn_step_right(A, X, 2)


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("s", [1, 2, 3, 4])
def test_T5_factorisation(name, s):
    """Corollary 6: sum_{n=0}^{2^s - 1} P^n phi = prod_{n<s} (I + P^(2^n)) phi."""
    A = _F(MATS[name])
    phi = _x0(A, "transpose")
    n = len(A)
    P = _sub(_I(n), _mm(phi, A))
    series = _I(n)
    Pm = _I(n)
    for _ in range(2 ** s - 1):
        Pm = _mm(Pm, P)
        series = _add(series, Pm)
    assert ex.factorised_series(P, phi, s) == _mm(series, phi)


def _gauss_jordan_inverse(A):
    """Textbook Gauss-Jordan elimination with pivoting, exact rationals."""
    n = len(A)
    M = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(A)]
    for c in range(n):
        p = max(range(c, n), key=lambda r: abs(M[r][c]))
        assert M[p][c] != 0, "singular"
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [row[n:] for row in M]


@pytest.mark.parametrize("name", sorted(MATS))
@pytest.mark.parametrize("d", [1, 2, 3])
def test_limit_is_gauss_jordan_inverse(name, d):
    """X_k = A^-1 (I - R_0^((d+1)^k)) exactly, with A^-1 from Gauss-Jordan:
    the NN iterate approaches the textbook inverse with exactly the error
    the truncated series leaves."""
    A = _F(MATS[name])
    n = len(A)
    Ainv = _gauss_jordan_inverse(A)
    assert _mm(A, Ainv) == _I(n)
    X0 = _x0(A, "transpose")
    R0 = _sub(_I(n), _mm(A, X0))
    for k in (1, 2):
        X = ex.nn_iterate(A, X0, d, k)
        assert X == _mm(Ainv, _sub(_I(n), _pow(R0, (d + 1) ** k)))
