"""Pins of the FP64 / complex128 oracle ``oracle.nn_ref``.

What fixes each value (none of it is the oracle re-run):
* exact rational results of ``oracle.exact`` (themselves pinned to the
  paper's closed forms) — FP64 must agree to rounding;
* the identity and diagonal special cases, closed form
  x_i = (1 - (1 - mu_i)^((d+1)^k)) / a_i (Corollary 2 on a diagonal);
* the spectral trajectory of A = Q diag(lam) Q^T: with R_k = R_0^((d+1)^k)
  (Appendix 2), rms_k^2 = mean_j (1 - mu_j)^(2 (d+1)^k) where
  mu_j = lam_j^2 / (||A||_1 ||A||_inf) (transpose start) or lam_j / Tr A
  (identity start); norms from numpy.linalg.norm, an independent routine;
* the known inverse Q diag(1/lam) Q^T and numpy.linalg.solve;
* the order of convergence d+1 (Appendix 5) and monotone decrease
  (Appendix 2);
* status rules on inputs that force each outcome.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import exact as ex
from oracle import nn_fp64 as R
from paper_2212_02406_amd import workloads as W

INT_MATS = {
    "spd3": [[4, 1, 0], [1, 3, 1], [0, 1, 2]],
    "nonsym3": [[5, 2, -1], [1, 4, 0], [2, -1, 6]],
    "nonsym4": [[2, 1, 0, 0], [0, 3, 1, 0], [1, 0, 4, 1], [0, 1, 0, 5]],
}


def _relF(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


@pytest.mark.parametrize("name", sorted(INT_MATS))
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_fp64_matches_exact(name, d, k):
    A = INT_MATS[name]
    F = ex.to_frac(A)
    Xe = ex.nn_iterate(F, ex.x0_transpose(F), d, k)
    Xe = np.array([[float(v) for v in r] for r in Xe])
    X, info = oracle.nn_ref(np.array(A, float), d=d, x0=oracle.X0_TRANSPOSE, fixed_iter=k)
    assert info["iters"] == k and info["status"] == oracle.OK
    assert _relF(X, Xe) < 1e-13


@pytest.mark.parametrize("d", [1, 2, 3])
def test_fp64_identity_start_matches_exact(d):
    A = INT_MATS["spd3"]
    F = ex.to_frac(A)
    Xe = ex.nn_iterate(F, ex.x0_scaled_identity(F), d, 2)
    Xe = np.array([[float(v) for v in r] for r in Xe])
    X, _ = oracle.nn_ref(np.array(A, float), d=d, x0=oracle.X0_SCALED_IDENTITY, fixed_iter=2)
    assert _relF(X, Xe) < 1e-13


def test_x0_norms_match_numpy():
    g = np.random.default_rng(11)
    for A in (g.standard_normal((7, 7)), g.standard_normal((5, 5)) + 1j * g.standard_normal((5, 5))):
        assert math.isclose(R.norm_1(A), np.linalg.norm(A, 1), rel_tol=1e-14)
        assert math.isclose(R.norm_inf(A), np.linalg.norm(A, np.inf), rel_tol=1e-14)
        den, X0 = R.initial_guess(A, R.X0_TRANSPOSE)
        np.testing.assert_allclose(X0, A.conj().T / (np.linalg.norm(A, 1) * np.linalg.norm(A, np.inf)),
                                   rtol=1e-14)


@pytest.mark.parametrize("alpha", [1.0, 2.0, 0.25, 8.0])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_identity_input_one_nest_exact(alpha, d):
    """A = alpha I with alpha a power of two: X_0 = I/alpha exactly, R_0 = 0,
    and one nest returns X_0 bitwise."""
    n = 6
    A = alpha * np.eye(n)
    X, info = oracle.nn_ref(A, d=d, fixed_iter=1)
    assert np.array_equal(X, np.eye(n) / alpha)
    assert info["trace"][0] == 0.0
    X, info = oracle.nn_ref(A, d=d, tol=1e-12)
    assert info["iters"] == 0 and info["status"] == oracle.OK


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY])
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_diagonal_closed_form(x0, d, k):
    g = np.random.default_rng(100 + d)
    a = g.uniform(0.5, 20.0, 9)
    if x0 == oracle.X0_TRANSPOSE:
        a[::2] *= -1.0  # the transpose start also handles indefinite diagonals
        mu = a * a / (np.max(np.abs(a)) ** 2)
    else:
        mu = a / np.sum(a)
    A = np.diag(a)
    X, _ = oracle.nn_ref(A, d=d, x0=x0, fixed_iter=k)
    expect = (1.0 - (1.0 - mu) ** ((d + 1) ** k)) / a
    assert np.count_nonzero(X - np.diag(np.diag(X))) == 0
    np.testing.assert_allclose(np.diag(X), expect, rtol=1e-12)


@pytest.mark.parametrize("d", [1, 2])
def test_complex_diagonal_closed_form(d):
    """Complex diagonal: X_0 = s conj(A) — a dropped conjugate fails here."""
    g = np.random.default_rng(7)
    a = g.uniform(0.5, 4.0, 6) * np.exp(1j * g.uniform(0, 2 * np.pi, 6))
    A = np.diag(a)
    mu = np.abs(a) ** 2 / np.max(np.abs(a)) ** 2
    for k in (1, 2, 4):
        X, _ = oracle.nn_ref(A, d=d, fixed_iter=k)
        np.testing.assert_allclose(np.diag(X), (1 - (1 - mu) ** ((d + 1) ** k)) / a, rtol=1e-12)


def test_complex_matches_real_embedding():
    """Complex iteration == the real 2N x 2N embedding [[Re, -Im], [Im, Re]]
    iterated from the embedded start (catches conjugate/transposition slips
    in the complex path)."""
    g = np.random.default_rng(5)
    n = 6
    A = W.dense_spd(n, 1.0, 10.0, 9, complex_=True)
    A = A + 0.3 * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))  # non-Hermitian

    def emb(M):
        return np.block([[M.real, -M.imag], [M.imag, M.real]])

    _, X0 = R.initial_guess(A, R.X0_TRANSPOSE)
    for d in (1, 2, 3):
        Xc, _ = oracle.nn_ref(A, d=d, x0=oracle.X0_GIVEN, X_init=X0, fixed_iter=3)
        Xr, _ = oracle.nn_ref(emb(A), d=d, x0=oracle.X0_GIVEN, X_init=emb(X0), fixed_iter=3)
        np.testing.assert_allclose(emb(Xc), Xr, rtol=0, atol=1e-13 * np.abs(Xr).max())


def _spectral_rms(mu, d, k):
    e = 2 * (d + 1) ** k
    return math.sqrt(float(np.mean(np.exp(e * np.log1p(-mu)))))


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_spectral_trajectory(x0, d):
    n = 128
    A, lam, Q = W.dense_spd(n, 1.0, 100.0, 1, return_factors=True)
    if x0 == oracle.X0_TRANSPOSE:
        mu = lam ** 2 / (np.linalg.norm(A, 1) * np.linalg.norm(A, np.inf))
    else:
        mu = lam / np.sum(lam)
    _, info = oracle.nn_ref(A, d=d, x0=x0, tol=1e-13, max_iter=80)
    assert info["status"] in (oracle.OK, oracle.STAGNATED)
    tr = info["trace"]
    for k, r in enumerate(tr):
        pred = _spectral_rms(mu, d, k)
        if pred > 1e-10:
            assert abs(r - pred) <= 1e-9 * max(pred, 1e-3) + 1e-13, (k, r, pred)
    # steps to tolerance: the closed-form prediction and the oracle agree to +-1
    kpred = next(k for k in range(200) if _spectral_rms(mu, d, k) < 1e-13)
    if info["status"] == oracle.OK:
        assert abs(info["iters"] - kpred) <= 1


@pytest.mark.parametrize("d", [1, 2, 3])
def test_order_of_convergence(d):
    """Appendix 5: order d+1. Estimate log(e_{k+1}/e_k)/log(e_k/e_{k-1})."""
    A = W.dense_spd(96, 1.0, 50.0, 4)
    _, info = oracle.nn_ref(A, d=d, tol=1e-14, max_iter=80)
    e = info["trace"]
    qs = []
    for k in range(1, len(e) - 1):
        if 1e-1 > e[k] > 1e-9 and e[k + 1] > 1e-12:
            qs.append(math.log(e[k + 1] / e[k]) / math.log(e[k] / e[k - 1]))
    assert qs, e
    assert abs(qs[-1] - (d + 1)) < 0.2, qs


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE, oracle.X0_SCALED_IDENTITY])
def test_monotone_until_floor(x0):
    A = W.dense_spd(64, 1.0, 1e3, 6, log_spectrum=True)
    _, info = oracle.nn_ref(A, d=2, x0=x0, tol=0.0, max_iter=60)
    tr = info["trace"]
    for a, b in zip(tr, tr[1:]):
        if a > 1e-12:
            assert b <= a * (1 + 1e-12), tr
    assert info["status"] == oracle.STAGNATED


def test_converged_inverse_error_bound():
    """||X - A^-1||_F <= ||A^-1||_2 ||R||_F with A^-1 = Q diag(1/lam) Q^T known
    by construction; also agrees with numpy.linalg.inv."""
    A, lam, Q = W.dense_spd(200, 1.0, 100.0, 1, return_factors=True)
    Ainv = (Q / lam[None, :]) @ Q.T
    X, info = oracle.nn_ref(A, d=2, tol=1e-12)
    assert info["status"] == oracle.OK and info["rms"] < 1e-12
    Rf = math.sqrt(200) * info["rms"]
    assert np.linalg.norm(X - Ainv) <= (1 / lam.min()) * Rf * 1.01 + 1e-14
    assert _relF(X, np.linalg.inv(A)) < 1e-11


def test_solve_matches_numpy():
    g = np.random.default_rng(3)
    n = 40
    A = g.standard_normal((n, n)) + n ** 0.5 * np.eye(n)  # non-symmetric, nonsingular
    B = g.standard_normal((n, 3))
    x, info = oracle.nn_solve_ref(A, B, d=2, tol=1e-13, max_iter=200)
    assert info["status"] in (oracle.OK, oracle.STAGNATED)
    np.testing.assert_allclose(x, np.linalg.solve(A, B), rtol=1e-9, atol=1e-10)
    assert info["rel_residual"] < 1e-10


def test_depth_ordering_closed_form():
    """Sec. II-D / Appendix 6: depth 2 reaches a tolerance with the fewest
    products; depths 1 and 3 tie asymptotically (4 = 2^2).  Products to
    tolerance = k (d+1) + 1 (the last residual)."""
    A, lam, _ = W.dense_spd(256, 1.0, 100.0, 1, return_factors=True)
    mu = lam ** 2 / (np.linalg.norm(A, 1) * np.linalg.norm(A, np.inf))
    cost = {}
    for d in (1, 2, 3):
        k = next(k for k in range(200) if _spectral_rms(mu, d, k) < 1e-12)
        cost[d] = k * (d + 1) + 1
        _, info = oracle.nn_ref(A, d=d, tol=1e-12)
        assert abs(info["iters"] - k) <= 1
    assert cost[2] <= min(cost[1], cost[3])
    # "2^3 < 3^2": six products buy 8 series terms at depth 1, 9 at depth 2
    assert 2 ** (6 // 2) < 3 ** (6 // 3)


def test_status_nonfinite():
    A = W.dense_spd(8, 1.0, 10.0, 2)
    A[3, 4] = np.nan
    _, info = oracle.nn_ref(A)
    assert info["status"] == oracle.ERR_NONFINITE
    A[3, 4] = np.inf
    _, info = oracle.nn_ref(A, x0=oracle.X0_SCALED_IDENTITY)
    assert info["status"] == oracle.ERR_NONFINITE


def test_status_indefinite_identity_start_diverges():
    lam = np.array([5.0, 4.0, 3.0, 2.0, 1.0, -3.0])
    Q = W.haar_unitary(6, W.rng(1))
    A = (Q * lam) @ Q.T
    _, info = oracle.nn_ref(A, x0=oracle.X0_SCALED_IDENTITY, max_iter=200)
    assert info["status"] == oracle.ERR_DIVERGED


def test_status_nonpositive_trace():
    A = -W.dense_spd(5, 1.0, 2.0, 2)
    _, info = oracle.nn_ref(A, x0=oracle.X0_SCALED_IDENTITY)
    assert info["status"] == oracle.ERR_DIVERGED and info["trace"] == []


def test_status_overscaled_start_diverges():
    """X_0 = 3 A^T / ||A||_2^2: the top eigenvalue of A X_0 is 3, so
    |1 - 3| > 1 breaks the normalisation condition and the iteration grows."""
    A = W.dense_spd(16, 1.0, 10.0, 3)
    X0 = 3.0 * A.T / np.linalg.norm(A, 2) ** 2
    _, info = oracle.nn_ref(A, x0=oracle.X0_GIVEN, X_init=X0, max_iter=100)
    assert info["status"] == oracle.ERR_DIVERGED


def test_status_not_converged_and_singular():
    A = W.dense_spd(32, 1.0, 1e3, 3, log_spectrum=True)
    _, info = oracle.nn_ref(A, tol=1e-12, max_iter=3)
    assert info["status"] == oracle.NOT_CONVERGED and info["iters"] == 3
    # rank deficient: the transpose start converges to the pseudo-inverse, so
    # rms settles at sqrt(nullity / N) and the tolerance is never met.  (Much
    # later, rounding noise in the null directions is amplified and the run
    # ends as ERR_DIVERGED; both outcomes report failure.)
    lam = np.r_[np.linspace(1, 10, 30), 0.0, 0.0]
    Q = W.haar_unitary(32, W.rng(2))
    S = (Q * lam) @ Q.T
    _, info = oracle.nn_ref(S, tol=1e-12, max_iter=40)
    assert info["status"] == oracle.NOT_CONVERGED
    assert abs(info["rms"] - math.sqrt(2 / 32)) < 1e-6
    _, info = oracle.nn_ref(S, tol=1e-12, max_iter=400)
    assert info["status"] in (oracle.NOT_CONVERGED, oracle.STAGNATED, oracle.ERR_DIVERGED)


def test_stagnation_returns_previous_iterate():
    A = W.dense_spd(64, 1.0, 100.0, 8)
    X, info = oracle.nn_ref(A, d=2, tol=0.0, max_iter=100)
    assert info["status"] == oracle.STAGNATED
    assert info["rms"] == min(info["trace"][:-1]) or info["rms"] <= info["trace"][-1]
    assert len(info["trace"]) == info["iters"] + 2
    assert info["rms"] == info["trace"][info["iters"]]


def test_paper_cond_1e6_thirty_seven_nests():
    """Corollary 3's remark: cond(A) = 1e6, phi^(0) = I, Theta = 1/Tr(A^* A),
    L = 2 — 37 nests are more than enough.  In exact arithmetic the residual
    eigenvalue of the worst direction after 37 nests is
    (1 - sigma_min^2 / Tr(A^* A))^(3^37); for N <= 1e4 and sigma in
    [1e-6, 1], sigma_min^2/Tr >= 1e-12 / N.  Corollary 5's bound gives 17."""
    for N in (10, 100, 1000, 10000):
        mu = 1e-12 / N
        log_res = 3 ** 37 * math.log1p(-mu)
        assert log_res < math.log(1e-16)
    kappa = 1e6
    i_bound = math.log(2 * kappa ** (2 / math.log2(math.e))) / math.log(3) - 1
    assert 16.5 < i_bound < 37


def test_paper_cond_1e6_oracle_run():
    """The same remark on the oracle: normal equations of a cond-1e6 A, trace
    start, depth 2 — the residual of W X reaches its rounding floor well
    within 37 nests."""
    n = 24
    g = W.rng(10)
    U = W.haar_unitary(n, g)
    V = W.haar_unitary(n, g)
    sig = W.spectrum_loguniform(n, 1e-6, 1.0, g)
    A = (U * sig) @ V.T
    Wm = A.T @ A
    _, info = oracle.nn_ref(Wm, d=2, x0=oracle.X0_SCALED_IDENTITY, tol=0.0, max_iter=37)
    # in exact arithmetic the error would be below 1e-16 by nest 37 (n = 24):
    assert info["status"] in (oracle.STAGNATED, oracle.NOT_CONVERGED)
    assert min(info["trace"]) < 1e-3  # rounding floor of cond(W) = 1e12 in FP64
