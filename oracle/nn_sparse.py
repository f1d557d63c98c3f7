"""Oracle of the sparse form: the NN / factorised Neumann series applied to
a right-hand side of a sparse system without storing any power of P.

TEST INFRASTRUCTURE ONLY: used by ``tests/`` (and nothing in the product
path).  Paper: Engsig, Yang, Mehouachi, arXiv 2212.02406.

What is computed (Algorithm 2; Corollary 6 and the sparse-system passage
after it; the NN explicit form of Sec. II-D): with a preconditioner phi that
keeps sparsity (a scalar Theta, or the diagonal diag(W)^-1) and
P = I - phi W, the solution of W x = B is approximated by the Neumann series

    x_T = sum_{m=0}^{T} P^m phi B,

which Algorithm 2 evaluates for T = 2^s - 1 as prod_{n<s} (I + P^(2^n)) phi B,
forming P^(2^n) Z by 2^n applications of P (never storing P^k); and which i
nests of depth L give for T = (L+1)^i - 1 (Corollary 2).  P is applied as
P y = y - phi (W y): one sparse product per application.

Readings (listed in the design notes):
* Algorithm 2 starts from B and applies phi at the end; for a scalar phi
  that is the same as starting from phi B.  For the diagonal
  preconditioner (which does not commute with W) the series is taken in the
  form of Corollary 6, prod (I + P^(2^n)) phi B with P = I - phi W.
* Control: the rules of the dense factorised solve, on the phi-weighted
  relative residual ||phi_w^(1/2) (B - W x)||_F / ||phi_w^(1/2) B||_F with
  phi_w the weights |phi_r| (all equal for a scalar phi, so then it is the
  plain relative residual).  For Hermitian PD W the iteration is a
  contraction in that norm (r_{t+1} = (I - W phi) r_t and
  phi^(1/2) (I - W phi) phi^(-1/2) is Hermitian), so the residual never
  rises and the stagnation rule only fires at the rounding floor.  The
  plain relative residual of the returned x is reported too.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .nn_fp64 import (OK, NOT_CONVERGED, STAGNATED, ERR_DIVERGED, ERR_NONFINITE,
                      X0_SCALED_IDENTITY, X0_POWER_IDENTITY, X0_JACOBI, power_vector, theta2)


def csr_matrix(indptr, indices, data, n: int):
    """The CSR arrays as a scipy sparse matrix (its product is the sparse
    matrix-times-dense primitive the oracle's steps use)."""
    return sp.csr_matrix((np.asarray(data), np.asarray(indices), np.asarray(indptr)), shape=(n, n))


def sparse_preconditioner(W, x0: int, power_k: int = 8):
    """phi for the sparse series, as a length-n vector of row factors
    (phi = diag(f)) plus a scale check value ``den``:

    * SCALED_IDENTITY: f_r = 1 / Re Tr(W)  (Theta_1, Sec. II-A);
    * POWER_IDENTITY: f_r = Theta_2(power_k) of W (Sec. II-A, read with
      plain norms; v the SplitMix64 vector);
    * JACOBI: f_r = 1 / w_rr  (the diagonal preconditioner).

    den: the denominator of the scalar starts (1 / Theta), min_r |w_rr| for
    JACOBI; not finite -> NONFINITE, <= 0 -> DIVERGED, as for the dense
    starts."""
    n = W.shape[0]
    diag = W.diagonal()
    if x0 == X0_SCALED_IDENTITY:
        den = float(np.real(np.sum(diag)))
        f = np.full(n, 1.0 / den if den > 0 and math.isfinite(den) else math.nan)
    elif x0 == X0_POWER_IDENTITY:
        th = theta2(lambda w: W @ w, power_vector(n), power_k)
        den = 1.0 / th if math.isfinite(th) and th > 0 else (math.nan if math.isnan(th) else 0.0)
        f = np.full(n, th)
    elif x0 == X0_JACOBI:
        den = float(np.min(np.abs(diag))) if np.all(np.isfinite(diag)) else math.nan
        with np.errstate(divide="ignore", invalid="ignore"):
            f = 1.0 / diag
    else:
        raise ValueError(f"start {x0} has no sparse form")
    return den, f


def nn_sparse_solve_ref(indptr, indices, data, B, x0: int = X0_SCALED_IDENTITY,
                        power_k: int = 8, tol: float = 1e-10, max_terms: int = 1000,
                        fixed_terms: int | None = None):
    """Solve W x = B for sparse W (CSR arrays) with the Neumann series in
    P = I - phi W applied to phi B.  Returns (x, info) with info = {"terms",
    "rel_residual" (plain ||B - W x||_F / ||B||_F of x), "control" (the
    phi-weighted residual the rules use), "status", "trace" (control values
    after 0, 1, ... terms), "den"}.

    fixed_terms = 2^s - 1: the factorised form of Corollary 6 that Algorithm 2
    evaluates, prod_{n<s} (I + P^(2^n)) phi B with each P^(2^n) y formed by
    2^n applications of P.  Other fixed_terms: the series term by term,
    t_{m+1} = P t_m, x = sum t_m.
    Tolerance mode (fixed_terms None): term by term, with the control value
    after each term and the rules of the dense factorised solve, at most
    max_terms terms.
    """
    B = np.asarray(B)
    n = len(indptr) - 1
    cplx = np.iscomplexobj(data) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    W = csr_matrix(indptr, indices, np.asarray(data).astype(dt), n)
    B = B.astype(dt)
    den, f = sparse_preconditioner(W, x0, power_k)
    info = {"terms": 0, "rel_residual": math.nan, "control": math.nan, "status": OK,
            "trace": [], "den": den}
    if not math.isfinite(den):
        info["status"] = ERR_NONFINITE
        return np.full_like(B, math.nan), info
    if den <= 0.0:
        info["status"] = ERR_DIVERGED
        return np.full_like(B, math.nan), info
    f = f.astype(dt)
    wgt = np.abs(f)[:, None]

    def apply_p(y):
        return y - f[:, None] * (W @ y)

    bnorm = float(np.linalg.norm(B))
    bw = float(np.sqrt(np.sum(wgt * np.abs(B) ** 2)))

    def measures(x):
        r = B - W @ x
        plain = float(np.linalg.norm(r)) / bnorm if bnorm > 0 else 0.0
        ctl = float(np.sqrt(np.sum(wgt * np.abs(r) ** 2))) / bw if bw > 0 else 0.0
        return plain, ctl

    phiB = f[:, None] * B
    if fixed_terms is not None:
        T = int(fixed_terms)
        s = (T + 1).bit_length() - 1
        if T >= 1 and (1 << s) == T + 1:
            # Corollary 6's product form, the one Algorithm 2 evaluates:
            # x = prod_{e<s} (I + P^(2^e)) phi B, each factor applied to the
            # running product, its power P^(2^e) y formed as 2^e applications
            # of P (no power of P is stored).
            def apply_power(y, m):
                for _ in range(m):
                    y = apply_p(y)
                return y

            x = phiB.copy()
            for e in range(s):
                x = x + apply_power(x, 1 << e)
        else:
            # the truncated series itself, sum_{m<=T} P^m phi B, term by term
            t = phiB.copy()
            x = t.copy()
            for _ in range(T):
                t = apply_p(t)
                x = x + t
        plain, ctl = measures(x)
        info.update(terms=T, rel_residual=plain, control=ctl, trace=[ctl],
                    status=OK if math.isfinite(ctl) else ERR_NONFINITE)
        return x, info

    t = phiB.copy()
    x = t.copy()
    x_prev, c_prev, p_prev = None, math.nan, math.nan
    T = 0
    while True:
        plain, ctl = measures(x)
        info["trace"].append(ctl)
        done = None
        if not math.isfinite(ctl):
            done = (ERR_NONFINITE, x, T, plain, ctl)
        elif ctl < tol:
            done = (OK, x, T, plain, ctl)
        elif T > 0 and ctl >= 1.0 and ctl > c_prev:
            done = (ERR_DIVERGED, x, T, plain, ctl)
        elif T > 0 and c_prev < 0.1 and ctl >= c_prev:
            done = (STAGNATED, x_prev, T - 1, p_prev, c_prev)
        elif T == max_terms:
            done = (NOT_CONVERGED, x, T, plain, ctl)
        if done is not None:
            st, xr, Tr, pr, cr = done
            info.update(status=st, terms=Tr, rel_residual=pr, control=cr)
            return xr, info
        t = apply_p(t)
        x_prev, c_prev, p_prev = x, ctl, plain
        x = x + t
        T += 1
