"""Pins of the oracle's other normalisations (start iterates): the Frobenius
transpose start, the power-iteration scale Theta_2(k) (Sec. II-A) applied to
I or A^H, and the diagonal (Jacobi) preconditioner.

What fixes them, other than the functions themselves:
* SplitMix64 against its published output sequences (seed 0 and seed
  1234567), which pins the random vector both sides draw;
* Theta_2 closed forms: W = c I gives k / ((k + 1) c); the Rayleigh bound
  Theta_2 lambda_max >= k / (k + 1) for any Hermitian PSD W; the limit
  k / (k + 1) for a gapped spectrum; the paper's remark that Theta_1 and
  Theta_2 meet when one eigenvalue dominates;
* the normalisation condition ||I - A X_0||_2 < 1 by numpy's spectral norm;
* exact rational nests from the Frobenius start; Jacobi exact for diagonal A;
* convergence to numpy.linalg.inv; statuses of degenerate inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact as ex
from paper_2212_02406_amd import workloads as W


def test_splitmix64_published_sequences():
    g, m = 0x9E3779B97F4A7C15, (1 << 64) - 1
    seed0 = [oracle.splitmix64(((i + 1) * g) & m) for i in range(4)]
    assert seed0 == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F,
                     0xF88BB8A8724C81EC]
    s = [oracle.splitmix64((1234567 + (i + 1) * g) & m) for i in range(5)]
    assert s == [6457827717110365317, 3203168211198807973, 9817491932198370423,
                 4593380528125082431, 16408922859458223821]


def test_power_vector_entries():
    v = oracle.power_vector(4096)
    assert v[0] == 2.0 * ((0xE220A8397B1DCDAF >> 11) * 2.0 ** -53) - 1.0
    assert v[2] == 2.0 * ((0x06C45D188009454F >> 11) * 2.0 ** -53) - 1.0
    assert np.all(v >= -1.0) and np.all(v < 1.0)
    assert abs(v.mean()) < 0.05 and abs(np.mean(v ** 2) - 1.0 / 3.0) < 0.02


@pytest.mark.parametrize("k", [1, 2, 8, 33])
def test_theta2_scaled_identity_closed_form(k):
    c = 7.25
    v = oracle.power_vector(20)
    th = oracle.theta2(lambda w: c * w, v, k)
    assert abs(th - k / ((k + 1) * c)) <= 1e-15 * th


def test_theta2_rayleigh_bound_and_limit():
    n = 60
    A, lam, _ = W.dense_spd(n, 1.0, 50.0, 91, return_factors=True)
    v = oracle.power_vector(n)
    for k in (1, 2, 4, 16):
        th = oracle.theta2(lambda w: A @ w, v, k)
        # ||W^(k+1) v|| <= lambda_max ||W^k v||  =>  Theta_2 lambda_max >= k/(k+1)
        assert th * lam.max() >= k / (k + 1) * (1 - 1e-14)
    # a spectral gap: lambda = 10 and 1 (x n-1); W^k v aligns with the top
    # eigenvector, so Theta_2 lambda_max -> k / (k + 1)
    B = np.diag(np.r_[10.0, np.ones(n - 1)])
    k = 40
    th = oracle.theta2(lambda w: B @ w, v, k)
    assert abs(th * 10.0 - k / (k + 1)) < 1e-12


def test_theta2_meets_theta1_when_one_eigenvalue_dominates():
    """Sec. II-A: Theta_1 -> Theta_2 when one eigenvector dominates
    (then Tr W ~ lambda_max); with the k/(k+1) margin the ratio is (k+1)/k."""
    n, k = 16, 8
    A = np.diag(np.r_[1e8, np.ones(n - 1)])
    den1, _ = oracle.initial_guess(A, oracle.X0_SCALED_IDENTITY)
    den2, _ = oracle.initial_guess(A, oracle.X0_POWER_IDENTITY, power_k=k)
    theta1, theta2 = 1.0 / den1, 1.0 / den2
    assert abs(theta2 / theta1 - k / (k + 1)) < 1e-6
    # a flat spectrum: Theta_2 is about N times Theta_1 (the benefit)
    A = np.diag(np.linspace(1.0, 2.0, n))
    d1, _ = oracle.initial_guess(A, oracle.X0_SCALED_IDENTITY)
    d2, _ = oracle.initial_guess(A, oracle.X0_POWER_IDENTITY, power_k=k)
    assert d1 / d2 > 0.6 * n


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE_FROB, oracle.X0_POWER_TRANSPOSE])
@pytest.mark.parametrize("cplx", [False, True])
def test_transpose_family_normalisation_any_nonsingular(x0, cplx):
    n = 40
    g = W.rng(92)
    A = g.standard_normal((n, n)) + (1j * g.standard_normal((n, n)) if cplx else 0.0)
    A = A + 3.0 * np.eye(n)
    den, X0 = oracle.initial_guess(A, x0, power_k=8)
    assert den > 0
    # A X_0 = A A^H / den is Hermitian PSD with spectrum in (0, 2): ||I - A X_0||_2 < 1
    assert np.linalg.norm(np.eye(n) - A @ X0, 2) < 1.0
    if x0 == oracle.X0_TRANSPOSE_FROB:
        assert abs(den - np.trace(A.conj().T @ A).real) <= 1e-12 * den
    else:
        smax2 = np.linalg.norm(A, 2) ** 2
        assert smax2 / den >= 8 / 9 * (1 - 1e-12)


def test_power_identity_normalisation_spd():
    n = 50
    A = W.dense_spd(n, 1.0, 1e3, 93, log_spectrum=True)
    den, X0 = oracle.initial_guess(A, oracle.X0_POWER_IDENTITY, power_k=8)
    assert np.linalg.norm(np.eye(n) - A @ X0, 2) < 1.0
    assert np.allclose(X0, np.eye(n) / den, rtol=0, atol=0)


def test_frobenius_start_exact_nests():
    A = [[4, 1, 0], [1, 3, 1], [0, 1, 2]]
    Af = ex.to_frac(A)
    den = sum(v * v for row in Af for v in row)
    X0 = ex.scale(Fraction(1) / den, ex.transpose(Af))
    for k in (1, 2, 3):
        want = ex.nn_iterate(Af, X0, 2, k)
        want = np.array([[float(v) for v in r] for r in want])
        X, info = oracle.nn_ref(np.array(A, float), d=2, x0=oracle.X0_TRANSPOSE_FROB, fixed_iter=k)
        assert np.linalg.norm(X - want) / np.linalg.norm(want) < 1e-13


def test_jacobi_exact_for_diagonal_and_dominant():
    a = np.array([0.5, 2.0, -3.0, 7.0])
    X, info = oracle.nn_ref(np.diag(a), x0=oracle.X0_JACOBI, tol=1e-12)
    assert info["status"] == oracle.OK and info["iters"] == 0 and info["rms"] == 0.0
    assert np.array_equal(X, np.diag(1.0 / a))
    # strictly diagonally dominant (rows and columns): ||I - A D^-1|| < 1
    n = 30
    g = W.rng(94)
    off = g.uniform(-1, 1, (n, n))
    np.fill_diagonal(off, 0.0)
    A = off + np.diag(np.abs(off).sum(1) + np.abs(off).sum(0) + 1.0)
    _, X0 = oracle.initial_guess(A, oracle.X0_JACOBI)
    assert np.linalg.norm(np.eye(n) - A @ X0, 2) < 1.0
    X, info = oracle.nn_ref(A, x0=oracle.X0_JACOBI, tol=1e-13)
    assert info["status"] == oracle.OK
    assert np.linalg.norm(X - np.linalg.inv(A)) / np.linalg.norm(np.linalg.inv(A)) < 1e-12


@pytest.mark.parametrize("x0", [oracle.X0_TRANSPOSE_FROB, oracle.X0_POWER_IDENTITY,
                                oracle.X0_POWER_TRANSPOSE, oracle.X0_JACOBI])
def test_new_starts_converge_to_inverse(x0):
    n = 48
    A = W.dense_spd(n, 1.0, 100.0, 95)
    X, info = oracle.nn_ref(A, d=2, x0=x0, tol=1e-13, power_k=4)
    assert info["status"] == oracle.OK, info
    inv = np.linalg.inv(A)
    assert np.linalg.norm(X - inv) / np.linalg.norm(inv) < 100 * 1e-13 * np.sqrt(n)


def test_power_identity_saves_nests_on_flat_spectrum():
    n = 64
    A = W.dense_spd(n, 1.0, 2.0, 96)
    _, i1 = oracle.nn_ref(A, d=2, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12)
    _, i2 = oracle.nn_ref(A, d=2, x0=oracle.X0_POWER_IDENTITY, tol=1e-12, power_k=8)
    assert i1["status"] == i2["status"] == oracle.OK
    assert i2["iters"] < i1["iters"]


def test_degenerate_statuses():
    n = 8
    A = W.dense_spd(n, 1.0, 10.0, 97)
    Z = A.copy()
    Z[3, 3] = 0.0
    _, info = oracle.nn_ref(Z, x0=oracle.X0_JACOBI)
    assert info["status"] == oracle.ERR_DIVERGED
    Nn = A.copy()
    Nn[2, 5] = np.nan
    for x0 in (oracle.X0_TRANSPOSE_FROB, oracle.X0_POWER_IDENTITY, oracle.X0_POWER_TRANSPOSE):
        _, info = oracle.nn_ref(Nn, x0=x0)
        assert info["status"] == oracle.ERR_NONFINITE, x0
    Nn = A.copy()
    Nn[4, 4] = np.inf
    _, info = oracle.nn_ref(Nn, x0=oracle.X0_JACOBI)
    assert info["status"] == oracle.ERR_NONFINITE
    for x0 in (oracle.X0_TRANSPOSE_FROB, oracle.X0_POWER_IDENTITY, oracle.X0_POWER_TRANSPOSE):
        _, info = oracle.nn_ref(np.zeros((n, n)), x0=x0)
        assert info["status"] == oracle.ERR_DIVERGED, x0
