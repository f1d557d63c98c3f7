"""FP64 / complex128 NumPy oracle of the Nested Neumann (NN) iteration.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and
``bench.py``'s CPU baseline; never by the product path.

Paper: Engsig, Yang, Mehouachi, arXiv 2212.02406.

What is computed (Sec. II-D, Theorem; Algorithm 1 of Sec. III):
    starting from an initial iterate X_0 with ||I - A X_0||_2 < 1, each nest
    (step) replaces X by X * sum_{n=0..d} (I - A X)^n, where d is the
    inception depth L.  d = 1 is Newton's iteration (Sec. II-B), d = 2 is the
    Chebyshev iteration (Sec. II-C; Corollary 4).

Readings taken where the paper is silent or garbled (each is listed in the
design notes of the repository):

* Right form.  The paper writes the polynomial on the left,
  sum_n (I - phi W~)^n phi.  We iterate X = Theta * phi directly with the
  residual on the right, X * sum_n (I - A X)^n.  The two are equal in exact
  arithmetic because X (A X)^n = (X A)^n X; ``tests/test_oracle_exact.py``
  checks that equality in rational arithmetic.
* Algorithm 1 sets its scale to the trace of W itself and subtracts the
  product from a scalar one; both are read as in Sec. II-A and the Theorem:
  the scale is the trace normalisation 1/Tr(W), the residual is I - Z W.
* Initial iterates.  ``X0_SCALED_IDENTITY`` is the paper's own choice
  phi^(0) = I with Theta = 1/Tr(W) (Sec. II-A, Sec. II-D), i.e.
  X_0 = I / Re Tr(A), for Hermitian positive definite A.
  ``X0_TRANSPOSE`` is X_0 = A^H / (||A||_1 ||A||_inf), the Pan-Schreiber
  start that Sec. II-C and Corollary 5 refer to; it is the normal-equation
  route of Corollary 3 (A X_0 is Hermitian PSD) and works for any
  nonsingular A.  ``X0_GIVEN`` takes a caller-supplied X_0 (restart).
* Other normalisations (Sec. II-A and the linear-system form of Sec. II-D):
  ``X0_TRANSPOSE_FROB`` X_0 = A^H / ||A||_F^2 (Theta = 1/Tr(A^H A));
  ``X0_POWER_IDENTITY`` / ``X0_POWER_TRANSPOSE`` scale I or A^H by the
  power-iteration estimate Theta_2(k), printed with squared norms (which
  would tend to 1/lambda^2) and read here with plain norms (1/lambda_max);
  its random vector comes from SplitMix64 so that the device draws the same
  one; ``X0_JACOBI`` X_0 = diag(A)^-1, the diagonal preconditioner.
* Accuracy measure.  rms = ||I - A X||_F / sqrt(N), the root-mean Frobenius
  error of Sec. II divided by sqrt(N), not N.  The paper iterates a fixed number of nests; a
  tolerance stop on this rms, tested before each update, is our addition.
* Status rules (the paper has none): see ``nn_ref``.
"""

from __future__ import annotations

import math

import numpy as np

# Status codes (same values as the C ABI; defined here independently).
OK = 0
NOT_CONVERGED = 1
STAGNATED = 2
ERR_ARG = -1
ERR_DIVERGED = -2
ERR_NONFINITE = -3

# Initial-iterate choices.
X0_TRANSPOSE = 0
X0_SCALED_IDENTITY = 1
X0_GIVEN = 2
X0_TRANSPOSE_FROB = 3
X0_POWER_IDENTITY = 4
X0_POWER_TRANSPOSE = 5
X0_JACOBI = 6

# Odd constant of SplitMix64 (Steele, Lea and Flood, "Fast splittable
# pseudorandom number generators", OOPSLA 2014): the state advances by it.
_SM64_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(state: int) -> int:
    """The SplitMix64 output function applied to a 64-bit state (the state
    after its increment): two xor-shift-multiply rounds and a final
    xor-shift, all modulo 2^64."""
    z = state & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def power_vector(n: int) -> np.ndarray:
    """The random vector v of the Theta_2 estimate (Sec. II-A), drawn from a
    counter-based generator so that any implementation reproduces it: entry i
    is the (i+1)-th SplitMix64 output from seed 0, its top 53 bits scaled to
    u in [0, 1), and v_i = 2 u - 1."""
    out = np.empty(n)
    for i in range(n):
        z = splitmix64(((i + 1) * _SM64_GAMMA) & _M64)
        out[i] = 2.0 * ((z >> 11) * 2.0 ** -53) - 1.0
    return out


def theta2(apply_w, v: np.ndarray, k: int) -> float:
    """Theta_2(k) = k ||W^k v||_2 / ((k + 1) ||W^(k+1) v||_2)  (Sec. II-A,
    the normalisation equation; the norms are read unsquared, so that
    Theta_2 estimates 1 / lambda_max of W, the scale the normalisation
    needs).  W is given as a function w -> W w.  The powers are formed one
    product at a time; between products the vector is rescaled by a power of
    two (exact in binary floating point, and the ratio is unchanged) so that
    W^k v cannot overflow."""
    w = np.asarray(v, dtype=np.complex128 if np.iscomplexobj(v) else np.float64)
    for _ in range(k):
        w = apply_w(w)
        m = float(np.max(np.abs(w)))
        if m > 0.0 and math.isfinite(m):
            w = w * 2.0 ** (-math.frexp(m)[1])
    num = float(np.linalg.norm(w))
    den = float(np.linalg.norm(apply_w(w)))
    if not (math.isfinite(num) and math.isfinite(den)):
        return math.nan
    return k * num / ((k + 1) * den) if den > 0.0 else math.inf


def norm_1(A: np.ndarray) -> float:
    """Maximum over columns of the sum of moduli (induced 1-norm)."""
    return float(np.max(np.sum(np.abs(A), axis=0)))


def norm_inf(A: np.ndarray) -> float:
    """Maximum over rows of the sum of moduli (induced inf-norm)."""
    return float(np.max(np.sum(np.abs(A), axis=1)))


def initial_guess(A: np.ndarray, x0: int, X_init: np.ndarray | None = None,
                  power_k: int = 8):
    """Return (den, X_0), where X_0 = X_init for GIVEN, else (1/den) * M.

    * TRANSPOSE: den = ||A||_1 ||A||_inf, M = A^H.  Since
      ||A||_2^2 <= ||A||_1 ||A||_inf, A X_0 = A A^H / den has its eigenvalues
      in (0, 1] for nonsingular A, so ||I - A X_0||_2 < 1 (the normalisation
      condition of Sec. II-A).
    * SCALED_IDENTITY: den = Re Tr(A), M = I (Sec. II-A, trace
      normalisation Theta_1, with phi^(0) = I of Sec. II-D).
    * GIVEN: den = nan, X_0 = X_init.
    * TRANSPOSE_FROB: den = ||A||_F^2 = Tr(A^H A), M = A^H: the Theta of the
      normal-equation solve (Sec. II-D, linear systems), 1/Tr(A^H A).
    * POWER_IDENTITY: den = 1 / Theta_2(power_k) of W = A, M = I.
    * POWER_TRANSPOSE: den = 1 / Theta_2(power_k) of W = A A^H, M = A^H
      (A X_0 = Theta_2 A A^H, the matrix whose top eigenvalue is estimated).
    * JACOBI: X_0 = D^-1, D = diag(A) (the diagonal preconditioner of the
      CNS discussion, Sec. II-D); den = min_i |a_ii| only flags a zero or
      non-finite diagonal.  ||I - A D^-1||_2 < 1 is the caller's condition
      (diagonally dominant A); for diagonal A, X_0 = A^-1 exactly.
    """
    n = A.shape[0]
    if x0 == X0_TRANSPOSE_FROB:
        den = float(np.sum(np.abs(A) ** 2))
        s = 1.0 / den if den > 0.0 and math.isfinite(den) else math.nan
        return den, s * A.conj().T
    if x0 in (X0_POWER_IDENTITY, X0_POWER_TRANSPOSE):
        if power_k < 1:
            raise ValueError("power_k must be >= 1")
        v = power_vector(n)
        if x0 == X0_POWER_IDENTITY:
            th = theta2(lambda w: A @ w, v, power_k)
            M = np.eye(n, dtype=A.dtype)
        else:
            AH = A.conj().T
            th = theta2(lambda w: A @ (AH @ w), v, power_k)
            M = AH
        den = 1.0 / th if th > 0.0 else math.nan
        if not math.isfinite(th):
            den = math.nan if math.isnan(th) else 0.0
        s = 1.0 / den if math.isfinite(den) and den > 0.0 else math.nan
        return den, s * M
    if x0 == X0_JACOBI:
        dg = np.diag(A)
        den = float(np.min(np.abs(dg))) if np.all(np.isfinite(dg)) else math.nan
        if not (math.isfinite(den) and den > 0.0):
            return den, np.full(A.shape, math.nan, dtype=A.dtype)
        return den, np.diag(1.0 / dg).astype(A.dtype)
    if x0 == X0_TRANSPOSE:
        den = norm_1(A) * norm_inf(A)
        s = 1.0 / den if den > 0.0 and math.isfinite(den) else math.nan
        return den, s * A.conj().T
    if x0 == X0_SCALED_IDENTITY:
        den = float(np.real(np.trace(A)))
        s = 1.0 / den if den > 0.0 and math.isfinite(den) else math.nan
        return den, s * np.eye(n, dtype=A.dtype)
    if x0 == X0_GIVEN:
        if X_init is None or np.shape(X_init) != A.shape:
            raise ValueError("X0_GIVEN needs X_init of the same shape as A")
        return math.nan, np.array(X_init, dtype=A.dtype, copy=True)
    raise ValueError(f"unknown x0 choice {x0}")


def residual(A: np.ndarray, X: np.ndarray) -> np.ndarray:
    """R = I - A X (Algorithm 1's P, in the right form)."""
    n = A.shape[0]
    return np.eye(n, dtype=A.dtype) - A @ X


def rms_of(R: np.ndarray) -> float:
    """||R||_F / sqrt(N), with |.| the complex modulus."""
    n = R.shape[0]
    return float(math.sqrt(float(np.sum(np.abs(R) ** 2)) / n))


def nn_step(X: np.ndarray, R: np.ndarray, d: int) -> np.ndarray:
    """One nest, given the residual R = I - A X of the current iterate.

    The Theorem of Sec. II-D in the right form: the next iterate is the
    current one times the truncated Neumann polynomial of degree d in its own
    residual, X_{k+1} = X_k * sum_{n=0..d} R^n.  The polynomial is summed
    term by term as defined, every power R^n taken from
    ``numpy.linalg.matrix_power`` (R^0 = I); no Horner form, no reuse of one
    power for the next.
    """
    S = sum(np.linalg.matrix_power(R, m) for m in range(d + 1))
    return X @ S


def nn_ref(A, d: int = 2, x0: int = X0_TRANSPOSE, tol: float = 1e-12,
           max_iter: int = 100, fixed_iter: int | None = None,
           X_init=None, trace_max: int = 1 << 20, power_k: int = 8):
    """Run the NN iteration on A; return (X, info).

    info = {"iters", "rms", "status", "trace", "den"}.  ``iters`` is the
    number of nests applied to X_0 to obtain the returned X, and ``rms`` is
    that X's rms; ``trace`` lists rms_0, rms_1, ... as computed.

    Control, for k = 0, 1, 2, ... with R_k = I - A X_k and rms_k its rms:

    * fixed_iter mode (fixed_iter is not None): exactly fixed_iter nests; the
      returned X is X_fixed_iter, status OK unless its rms is not finite.
    * tolerance mode, tested in this order:
        - rms_k not finite                         -> ERR_NONFINITE
        - rms_k < tol                              -> OK (X_k returned)
        - k > 0, rms_k >= 1 and rms_k > rms_{k-1}  -> ERR_DIVERGED
          (a valid start keeps rms <= ||R||_2 < 1 for ever: Appendix 2)
        - k > 0, sqrt(N) rms_{k-1} < 0.1 and rms_k >= rms_{k-1}
                                                   -> STAGNATED, X_{k-1}
          (then ||R_{k-1}||_2 < 0.1 and an exact nest would have taken it
          below 0.1^(d+1); no decrease means the rounding floor)
        - k == max_iter                            -> NOT_CONVERGED, X_k
    * Before the loop (not for X0_GIVEN): the scale denominator den of
      ``initial_guess`` not finite -> ERR_NONFINITE; den <= 0 -> ERR_DIVERGED
      (the normalisation of Sec. II-A cannot hold: A = 0, or a trace that
      is not positive, so A is not positive definite).
    """
    A = np.asarray(A)
    if A.ndim != 2 or A.shape[0] != A.shape[1] or A.shape[0] < 1:
        raise ValueError("A must be a non-empty square matrix")
    if d < 1:
        raise ValueError("inception depth d must be >= 1")
    if A.dtype not in (np.float64, np.complex128):
        A = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64)
    n = A.shape[0]
    den, X = initial_guess(A, x0, X_init, power_k)
    info = {"iters": 0, "rms": math.nan, "status": OK, "trace": [], "den": den}
    if x0 != X0_GIVEN:
        if not math.isfinite(den):
            info["status"] = ERR_NONFINITE
            return X, info
        if den <= 0.0:
            info["status"] = ERR_DIVERGED
            return X, info

    X_prev, rms_prev = None, math.nan
    k = 0
    while True:
        R = residual(A, X)
        rms = rms_of(R)
        if len(info["trace"]) < trace_max:
            info["trace"].append(rms)
        if fixed_iter is not None:
            if k == fixed_iter:
                info.update(iters=k, rms=rms,
                            status=OK if math.isfinite(rms) else ERR_NONFINITE)
                return X, info
        else:
            if not math.isfinite(rms):
                info.update(iters=k, rms=rms, status=ERR_NONFINITE)
                return X, info
            if rms < tol:
                info.update(iters=k, rms=rms, status=OK)
                return X, info
            if k > 0 and rms >= 1.0 and rms > rms_prev:
                info.update(iters=k, rms=rms, status=ERR_DIVERGED)
                return X, info
            if k > 0 and math.sqrt(n) * rms_prev < 0.1 and rms >= rms_prev:
                info.update(iters=k - 1, rms=rms_prev, status=STAGNATED)
                return X_prev, info
            if k == max_iter:
                info.update(iters=k, rms=rms, status=NOT_CONVERGED)
                return X, info
        X_prev, rms_prev = X, rms
        X = nn_step(X, R, d)
        k += 1


def nn_solve_ref(A, B, d: int = 2, x0: int = X0_TRANSPOSE, tol: float = 1e-12,
                 max_iter: int = 100, fixed_iter: int | None = None, power_k: int = 8):
    """Solve A x = B (Corollary 3): x = X B with X the NN inverse of A.

    With X0_TRANSPOSE this is the normal-equation route of Corollary 3
    (A X_0 is Hermitian PSD for any nonsingular A).  Returns (x, info);
    info also gets "rel_residual" = ||B - A x||_F / ||B||_F.
    """
    X, info = nn_ref(A, d=d, x0=x0, tol=tol, max_iter=max_iter, fixed_iter=fixed_iter,
                     power_k=power_k)
    x = X @ np.asarray(B, dtype=X.dtype)
    bnorm = float(np.linalg.norm(B))
    info["rel_residual"] = float(np.linalg.norm(B - A @ x)) / bnorm if bnorm > 0 else 0.0
    return x, info


def nn_factorized_solve_ref(A, B, x0: int = X0_TRANSPOSE, tol: float = 1e-10,
                            max_factors: int = 60, fixed_factors: int | None = None,
                            power_k: int = 8):
    """Solve A x = B with the factorised Neumann series applied to B, without
    forming the inverse (Corollary 6 and the linear-solve form after it):

        x = prod_{n=0}^{s-1} (I + P^(2^n)) phi B,   P = I - phi A,

    which equals the truncated series sum_{n=0}^{2^s-1} P^n phi B.  phi is
    the start of ``initial_guess`` (transpose or scaled identity).  Steps, in
    the paper's order: phi and P; y_0 = phi B; factor n maps y_n to
    y_{n+1} = (I + P^(2^n)) y_n, the power P^(2^n) being the square of
    P^(2^(n-1)).

    Control, for s = 0, 1, ... with rel_s = ||B - A y_s||_F / ||B||_F of
    the iterate after s factors:
      * fixed mode (fixed_factors given): exactly fixed_factors factors,
        status OK unless rel is not finite;
      * tolerance mode, in this order:
          rel_s not finite                               -> ERR_NONFINITE
          rel_s < tol                                    -> OK, y_s
          s > 0, rel_s >= 1 and rel_s > rel_{s-1}        -> ERR_DIVERGED
          s > 0, rel_{s-1} < 0.1 and rel_s >= rel_{s-1}  -> STAGNATED, y_{s-1}
          s == max_factors                               -> NOT_CONVERGED, y_s
      * before the loop: den not finite -> ERR_NONFINITE, den <= 0 ->
        ERR_DIVERGED (as in nn_ref).
    (For Hermitian A both starts make A P^m A^-1 Hermitian with eigenvalues
    in [0, 1), so rel_s never increases in exact arithmetic: an increase in
    the asymptotic regime is the rounding floor.)

    Returns (x, info) with info = {"factors", "rel_residual", "status",
    "trace", "den"}; the power P^(2^n) is formed only when factor n is
    applied.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    if A.ndim != 2 or A.shape[0] != A.shape[1] or A.shape[0] < 1:
        raise ValueError("A must be a non-empty square matrix")
    if B.ndim != 2 or B.shape[0] != A.shape[0]:
        raise ValueError("B must have A's row count")
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    A = A.astype(dt)
    B = B.astype(dt)
    n = A.shape[0]
    den, phi = initial_guess(A, x0, power_k=power_k)
    info = {"factors": 0, "rel_residual": math.nan, "status": OK, "trace": [], "den": den}
    if not math.isfinite(den):
        info["status"] = ERR_NONFINITE
        return phi @ B, info
    if den <= 0.0:
        info["status"] = ERR_DIVERGED
        return phi @ B, info
    P = np.eye(n, dtype=dt) - phi @ A
    y = phi @ B
    bnorm = float(np.linalg.norm(B))
    Pk = None          # P^(2^(s-1)) once factor s-1 has been applied
    y_prev, rel_prev = None, math.nan
    s = 0
    while True:
        rel = float(np.linalg.norm(B - A @ y)) / bnorm if bnorm > 0 else 0.0
        info["trace"].append(rel)
        if fixed_factors is not None:
            if s == fixed_factors:
                info.update(factors=s, rel_residual=rel,
                            status=OK if math.isfinite(rel) else ERR_NONFINITE)
                return y, info
        else:
            if not math.isfinite(rel):
                info.update(factors=s, rel_residual=rel, status=ERR_NONFINITE)
                return y, info
            if rel < tol:
                info.update(factors=s, rel_residual=rel, status=OK)
                return y, info
            if s > 0 and rel >= 1.0 and rel > rel_prev:
                info.update(factors=s, rel_residual=rel, status=ERR_DIVERGED)
                return y, info
            if s > 0 and rel_prev < 0.1 and rel >= rel_prev:
                info.update(factors=s - 1, rel_residual=rel_prev, status=STAGNATED)
                return y_prev, info
            if s == max_factors:
                info.update(factors=s, rel_residual=rel, status=NOT_CONVERGED)
                return y, info
        # factor s: (I + P^(2^s)) applied to y
        Pk = P if Pk is None else Pk @ Pk
        y_prev, rel_prev = y, rel
        y = y + Pk @ y
        s += 1


def nn_cns_solve_ref(A, B, d: int = 2, x0: int = X0_TRANSPOSE, nests: int = 1,
                     precond_tol: float = 1e-2, max_nests: int = 100, tol: float = 1e-12,
                     max_terms: int = 100, fixed_terms: int | None = None,
                     power_k: int = 8):
    """Chebyshev-Neumann series solve, CNS (Sec. II-D, the CNS equation after
    Corollary 2; d = 1 is the Newton-Neumann series): the NN iterate phi = X_m
    is the preconditioner of a Neumann series applied to B,

        x = sum_{k=0}^{T} (I - phi A)^k phi B,

    the series of order (d+1)^m (T + 1) - 1 in the start's P = I - X_0 A (the
    order printed in the paper is garbled; this is the reading that follows
    from I - phi A = P^((d+1)^m)).  phi comes from nn_ref: ``nests`` > 0 fixed nests,
    ``nests`` == 0 tolerance mode down to rms < precond_tol.  The series is
    summed term by term as printed: t_0 = phi B, t_{k+1} = (I - phi A) t_k,
    x_T = t_0 + ... + t_T.

    Control on rel_T = ||B - A x_T||_F / ||B||_F, for T = 0, 1, ...: fixed
    mode (fixed_terms given) stops at T == fixed_terms; tolerance mode uses the
    rules of nn_factorized_solve_ref with max_terms.  A failed preconditioner
    (status < 0) is returned as is.

    Returns (x, info) with info = {"nests", "precond_rms", "terms",
    "rel_residual", "status", "trace"}.
    """
    A = np.asarray(A)
    B = np.asarray(B)
    cplx = np.iscomplexobj(A) or np.iscomplexobj(B)
    dt = np.complex128 if cplx else np.float64
    A = A.astype(dt)
    B = B.astype(dt)
    if nests > 0:
        phi, pinfo = nn_ref(A, d=d, x0=x0, fixed_iter=nests, power_k=power_k)
    else:
        phi, pinfo = nn_ref(A, d=d, x0=x0, tol=precond_tol, max_iter=max_nests,
                            power_k=power_k)
    info = {"nests": pinfo["iters"], "precond_rms": pinfo["rms"], "terms": 0,
            "rel_residual": math.nan, "status": OK, "trace": []}
    if pinfo["status"] < 0:
        info["status"] = pinfo["status"]
        return phi @ B, info
    n = A.shape[0]
    Q = np.eye(n, dtype=dt) - phi @ A
    t = phi @ B
    x = t.copy()
    bnorm = float(np.linalg.norm(B))
    x_prev, rel_prev = None, math.nan
    T = 0
    while True:
        rel = float(np.linalg.norm(B - A @ x)) / bnorm if bnorm > 0 else 0.0
        info["trace"].append(rel)
        if fixed_terms is not None:
            if T == fixed_terms:
                info.update(terms=T, rel_residual=rel,
                            status=OK if math.isfinite(rel) else ERR_NONFINITE)
                return x, info
        else:
            if not math.isfinite(rel):
                info.update(terms=T, rel_residual=rel, status=ERR_NONFINITE)
                return x, info
            if rel < tol:
                info.update(terms=T, rel_residual=rel, status=OK)
                return x, info
            if T > 0 and rel >= 1.0 and rel > rel_prev:
                info.update(terms=T, rel_residual=rel, status=ERR_DIVERGED)
                return x, info
            if T > 0 and rel_prev < 0.1 and rel >= rel_prev:
                info.update(terms=T - 1, rel_residual=rel_prev, status=STAGNATED)
                return x_prev, info
            if T == max_terms:
                info.update(terms=T, rel_residual=rel, status=NOT_CONVERGED)
                return x, info
        t = Q @ t
        x_prev, rel_prev = x, rel
        x = x + t
        T += 1
