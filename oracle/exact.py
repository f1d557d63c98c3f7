"""Exact rational arithmetic for the NN iteration — TEST INFRASTRUCTURE ONLY.

Paper: Engsig, Yang, Mehouachi, arXiv 2212.02406.

Matrices are lists of lists of ``fractions.Fraction``; sizes are tiny (N <= 5).
Everything here is exact, so identities the paper states as equalities can be
checked as equalities:

* ``nn_step_right``   one nest in the right form X * sum_{n<=d} (I - A X)^n
* ``nn_step_left``    one nest as printed in the Theorem of Sec. II-D,
                      sum_{n<=L} (I - phi W~)^n phi
* ``neumann_series``  the truncated Neumann series of Sec. II-A,
                      sum_{n=0..m} P^n phi (Corollary 2 says k nests equal it
                      with m = (L+1)^k - 1)
* ``product_form``    Corollary 1: prod_{j=0..i} sum_{n=0..L} P0^(n (L+1)^j) phi0
* ``factorised_series`` Corollary 6: prod_{n<s} (I + P^(2^n)) phi
* ``newton_step``, ``chebyshev_step``  the Newton (Sec. II-B) and Chebyshev
                      (Sec. II-C) matrix iterations as printed (tildes read
                      as W~ Z, the garbled placement in Sec. II-B corrected)

These are deliberately written independently of ``nn_ref``.
"""

from __future__ import annotations

from fractions import Fraction

Mat = list  # list[list[Fraction]]


def to_frac(A) -> Mat:
    return [[Fraction(v) for v in row] for row in A]


def eye(n: int) -> Mat:
    return [[Fraction(int(i == j)) for j in range(n)] for i in range(n)]


def zeros(n: int) -> Mat:
    return [[Fraction(0) for _ in range(n)] for _ in range(n)]


def add(A: Mat, B: Mat) -> Mat:
    return [[a + b for a, b in zip(ra, rb)] for ra, rb in zip(A, B)]


def sub(A: Mat, B: Mat) -> Mat:
    return [[a - b for a, b in zip(ra, rb)] for ra, rb in zip(A, B)]


def scale(c, A: Mat) -> Mat:
    return [[c * a for a in row] for row in A]


def transpose(A: Mat) -> Mat:
    return [list(col) for col in zip(*A)]


def matmul(A: Mat, B: Mat) -> Mat:
    Bt = transpose(B)
    return [[sum((a * b for a, b in zip(row, col)), Fraction(0)) for col in Bt] for row in A]


def matpow(P: Mat, e: int) -> Mat:
    """P^e by repeated multiplication (e >= 0)."""
    out = eye(len(P))
    for _ in range(e):
        out = matmul(out, P)
    return out


def norm_1(A: Mat) -> Fraction:
    n = len(A)
    return max(sum(abs(A[i][j]) for i in range(n)) for j in range(n))


def norm_inf(A: Mat) -> Fraction:
    return max(sum(abs(v) for v in row) for row in A)


def trace(A: Mat) -> Fraction:
    return sum((A[i][i] for i in range(len(A))), Fraction(0))


def x0_transpose(A: Mat) -> Mat:
    """X_0 = A^T / (||A||_1 ||A||_inf) for a real A (exact)."""
    return scale(Fraction(1) / (norm_1(A) * norm_inf(A)), transpose(A))


def x0_scaled_identity(A: Mat) -> Mat:
    """X_0 = I / Tr(A) (Sec. II-A trace normalisation with phi^(0) = I)."""
    return scale(Fraction(1) / trace(A), eye(len(A)))


def nn_step_right(A: Mat, X: Mat, d: int) -> Mat:
    """X * sum_{n=0..d} (I - A X)^n, powers accumulated term by term."""
    n = len(A)
    R = sub(eye(n), matmul(A, X))
    S, Rn = eye(n), eye(n)
    for _ in range(d):
        Rn = matmul(Rn, R)
        S = add(S, Rn)
    return matmul(X, S)


def nn_step_left(W: Mat, phi: Mat, L: int) -> Mat:
    """sum_{n=0..L} (I - phi W)^n phi, the Theorem of Sec. II-D as printed."""
    n = len(W)
    P = sub(eye(n), matmul(phi, W))
    S, Pn = eye(n), eye(n)
    for _ in range(L):
        Pn = matmul(Pn, P)
        S = add(S, Pn)
    return matmul(S, phi)


def nn_iterate(A: Mat, X0: Mat, d: int, k: int, left: bool = False) -> Mat:
    X = X0
    for _ in range(k):
        X = nn_step_left(A, X, d) if left else nn_step_right(A, X, d)
    return X


def neumann_series(P: Mat, phi: Mat, m: int) -> Mat:
    """sum_{n=0..m} P^n phi (Sec. II-A, truncated Neumann series)."""
    n = len(P)
    S, Pn = eye(n), eye(n)
    for _ in range(m):
        Pn = matmul(Pn, P)
        S = add(S, Pn)
    return matmul(S, phi)


def product_form(W: Mat, phi0: Mat, L: int, i: int) -> Mat:
    """Corollary 1: phi^(i+1) = prod_{j=0..i} sum_{n=0..L} P0^(n (L+1)^j) phi0.

    P0 = I - phi0 W.  The factors are polynomials in P0 and commute; they are
    multiplied in the order j = 0..i, and phi0 is applied once on the right
    (the placement that Appendix 3's derivation produces).
    """
    n = len(W)
    P0 = sub(eye(n), matmul(phi0, W))
    prod = eye(n)
    for j in range(i + 1):
        base = matpow(P0, (L + 1) ** j)
        S, Bn = eye(n), eye(n)
        for _ in range(L):
            Bn = matmul(Bn, base)
            S = add(S, Bn)
        prod = matmul(prod, S)
    return matmul(prod, phi0)


def factorised_series(P: Mat, phi: Mat, s: int) -> Mat:
    """Corollary 6: prod_{n=0..s-1} (I + P^(2^n)) phi."""
    n = len(P)
    prod = eye(n)
    Pp = P
    for _ in range(s):
        prod = matmul(prod, add(eye(n), Pp))
        Pp = matmul(Pp, Pp)
    return matmul(prod, phi)


def newton_step(W: Mat, Z: Mat) -> Mat:
    """Sec. II-B: Z (2I - W Z)."""
    n = len(W)
    return matmul(Z, sub(scale(2, eye(n)), matmul(W, Z)))


def chebyshev_step(W: Mat, Z: Mat) -> Mat:
    """Sec. II-C: Z [3I - W Z (3I - W Z)]."""
    n = len(W)
    WZ = matmul(W, Z)
    inner = sub(scale(3, eye(n)), WZ)
    return matmul(Z, sub(scale(3, eye(n)), matmul(WZ, inner)))
