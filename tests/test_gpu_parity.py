"""Parity of the HIP NN path (through the C ABI) with the oracle.

Tolerances:
* FP64 / complex128: relative Frobenius difference <= 1e-10 between the HIP
  result and the oracle's, at a forced identical number of nests and in
  tolerance mode (where the two may stop one nest apart; each converged
  result is within sqrt(N) rms of A^-1).
* FP32 / complex64: the inputs are the same FP32-rounded bits, promoted to
  FP64 for the oracle.  The HIP result carries FP32 rounding from every
  product; its distance to the FP64 iterate is bounded by
  c * u32 * kappa(A) with u32 = 2^-24 (forward error of an inverse computed
  in FP32).  We use c = 64: rel <= 64 * 2^-24 * kappa.
Each case prints its name before its GPU step so a failure names it.
"""
import json
import math
import os
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2212_02406_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2212_02406_amd import nn  # noqa: E402  (fails loudly if libnn.so is missing)

DEV = torch.device("cuda:0")
U32 = 2.0 ** -24


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _relF(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


def _relmax(X, Y):
    """Largest entrywise difference relative to the largest entry of Y: a
    wrong tile or block of X shows here at its own size, where the Frobenius
    norm of the whole matrix would dilute it."""
    return float(np.abs(X - Y).max() / np.abs(Y).max())


def _to_dev(A, ld=None):
    """Upload A; with ld > n the matrix is a view with leading dimension ld."""
    n = A.shape[0]
    if ld is None or ld == n:
        return torch.from_numpy(np.ascontiguousarray(A)).to(DEV)
    big = np.zeros((n, ld), dtype=A.dtype)
    big[:, :n] = A
    return torch.from_numpy(big).to(DEV)[:, :n]


def _gpu_invert(A, ld=None, **kw):
    At = _to_dev(A, ld)
    X, info = nn.invert(At, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), info


GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "exact_small.json")))


@pytest.mark.parametrize("case", GOLD["cases"], ids=lambda c: f"{c['name']}-{c['x0']}-d{c['d']}-k{c['k']}")
def test_exact_golden_fp64(case):
    _say(f"golden {case['name']} x0={case['x0']} d={case['d']} k={case['k']}")
    A = np.array(case["A"], dtype=np.float64)
    Xe = np.array([[float(Fraction(v)) for v in r] for r in case["X"]])
    X, info = _gpu_invert(A, depth=case["d"], x0=case["x0"], fixed_iter=case["k"])
    assert info["status"] == nn.NN_OK and info["iters"] == case["k"]
    assert info["gemms"] == case["k"] * (case["d"] + 1) + 1
    assert _relF(X, Xe) < 1e-13


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("x0", ["transpose", "identity"])
def test_config1_n256_fp64(d, x0):
    """N = 256 SPD, lambda ~ U[1,100], tol 1e-12 (rms)."""
    _say(f"n256 fp64 d={d} x0={x0}")
    A = W.dense_spd(256, 1.0, 100.0, 1)
    x0c = oracle.X0_TRANSPOSE if x0 == "transpose" else oracle.X0_SCALED_IDENTITY
    Xo, io = oracle.nn_ref(A, d=d, x0=x0c, tol=1e-12)
    X, info = _gpu_invert(A, depth=d, x0=x0, tol=1e-12)
    assert info["status"] == nn.NN_OK, info
    assert abs(info["iters"] - io["iters"]) <= 1
    assert info["rms"] < 1e-12
    assert _relF(X, Xo) < 1e-10
    # forced identical k: strict parity, and the traces agree nest by nest
    X, info = _gpu_invert(A, depth=d, x0=x0, fixed_iter=io["iters"])
    assert _relF(X, Xo) < 1e-10
    assert _relmax(X, Xo) < 1e-10
    tr = info["trace"]
    for a, b in zip(tr, io["trace"]):
        assert abs(a - b) <= 1e-9 * b + 1e-14


@pytest.mark.parametrize("n,ld", [(1, 1), (2, 2), (3, 5), (17, 17), (33, 40), (100, 100),
                                  (129, 131), (257, 257), (300, 301), (520, 520)])
def test_ragged_sizes_fp64(n, ld):
    """Sizes that leave ragged tails in every tile configuration, and odd
    leading dimensions (unaligned load path)."""
    _say(f"ragged fp64 n={n} ld={ld}")
    A = W.dense_spd(n, 1.0, 50.0, 100 + n)
    Xo, io = oracle.nn_ref(A, d=2, fixed_iter=6)
    X, info = _gpu_invert(A, ld=ld, depth=2, fixed_iter=6)
    assert info["status"] == nn.NN_OK
    assert _relF(X, Xo) < 1e-10
    assert _relmax(X, Xo) < 1e-10
    assert abs(info["rms"] - io["rms"]) <= 1e-9 * io["rms"] + 1e-15


@pytest.mark.parametrize("tile", ["T128", "T128W8", "T128K8", "T128W8K8", "T256K8", "T256",
                                  "T64", "T32", "T16"])
@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.complex128, np.complex64])
@pytest.mark.parametrize("n", [197, 256, 320])
def test_every_tile_config(tile, dtype, n, monkeypatch):
    """Each GEMM tile configuration, forced for every product, on a size with
    ragged tails in both dimensions (n = 197: the bounds-checked kernels) and
    on one every tile divides (n = 256: the kernels without bounds checks),
    and on one whose k extent is not a multiple of the small-product kernel's
    64-deep chunks (n = 320, complex k = 640 is), each with an odd leading
    dimension too."""
    _say(f"tile {tile} {np.dtype(dtype).name} n={n}")
    monkeypatch.setenv("NN_GEMM_TILE", tile)
    cplx = np.dtype(dtype).kind == "c"
    A = W.dense_spd(n, 1.0, 40.0, 31, complex_=cplx, dtype=dtype)
    ref = A.astype(np.complex128 if cplx else np.float64)
    Xo, io = oracle.nn_ref(ref, d=3, fixed_iter=5)
    for ld in (n, n + 1):
        X, info = _gpu_invert(A, ld=ld, depth=3, fixed_iter=5)
        assert info["status"] == nn.NN_OK
        single = np.dtype(dtype) in (np.dtype(np.float32), np.dtype(np.complex64))
        tol = 64 * U32 * np.linalg.cond(ref) if single else 1e-10
        assert _relF(X.astype(ref.dtype), Xo) < tol
        assert _relmax(X.astype(ref.dtype), Xo) < tol


@pytest.mark.parametrize("n", [5, 64, 130, 300])
def test_nonsymmetric_fp64(n):
    _say(f"nonsym fp64 n={n}")
    g = np.random.default_rng(n)
    A = g.standard_normal((n, n)) + 2.0 * math.sqrt(n) * np.eye(n)
    Xo, io = oracle.nn_ref(A, d=2, fixed_iter=8)
    X, info = _gpu_invert(A, depth=2, fixed_iter=8)
    assert _relF(X, Xo) < 1e-10
    assert _relmax(X, Xo) < 1e-10


@pytest.mark.parametrize("n,ld", [(16, 16), (100, 101), (256, 256), (390, 390)])
@pytest.mark.parametrize("d", [1, 2])
def test_fp32(n, ld, d):
    _say(f"fp32 n={n} ld={ld} d={d}")
    A32 = W.dense_spd(n, 1.0, 100.0, 7 + n, dtype=np.float32)
    A64 = A32.astype(np.float64)
    kappa = np.linalg.cond(A64)
    Xo, io = oracle.nn_ref(A64, d=d, fixed_iter=12 if d == 2 else 18)
    X, info = _gpu_invert(A32, ld=ld, depth=d, fixed_iter=12 if d == 2 else 18)
    assert info["status"] == nn.NN_OK
    assert _relF(X.astype(np.float64), Xo) < 64 * U32 * kappa
    assert _relmax(X.astype(np.float64), Xo) < 64 * U32 * kappa


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
@pytest.mark.parametrize("n", [3, 40, 150])
def test_complex(dtype, n):
    _say(f"complex {np.dtype(dtype).name} n={n}")
    A = W.dense_spd(n, 1.0, 30.0, 50 + n, complex_=True, dtype=dtype)
    g = np.random.default_rng(n)
    A = (A + 0.2 * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))).astype(dtype)
    A128 = A.astype(np.complex128)
    Xo, io = oracle.nn_ref(A128, d=2, fixed_iter=10)
    X, info = _gpu_invert(A, depth=2, fixed_iter=10)
    tol = 1e-10 if dtype == np.complex128 else 64 * U32 * np.linalg.cond(A128)
    assert _relF(X.astype(np.complex128), Xo) < tol
    assert _relmax(X.astype(np.complex128), Xo) < tol


@pytest.mark.parametrize("dtype", [np.complex128, np.complex64])
def test_complex_hpd_identity_start(dtype):
    _say(f"complex hpd identity {np.dtype(dtype).name}")
    A = W.dense_spd(70, 1.0, 20.0, 77, complex_=True, dtype=dtype)
    A128 = A.astype(np.complex128)
    Xo, io = oracle.nn_ref(A128, d=3, x0=oracle.X0_SCALED_IDENTITY, fixed_iter=6)
    X, info = _gpu_invert(A, depth=3, x0="identity", fixed_iter=6)
    tol = 1e-10 if dtype == np.complex128 else 64 * U32 * np.linalg.cond(A128)
    assert _relF(X.astype(np.complex128), Xo) < tol
    assert _relmax(X.astype(np.complex128), Xo) < tol


def test_restart_from_given_iterate():
    """Three nests, then a restart from that iterate for three more, equal
    six nests in one call (the iterate is the whole state)."""
    _say("restart")
    A = W.dense_spd(200, 1.0, 100.0, 3)
    At = _to_dev(A)
    X3, _ = nn.invert(At, depth=2, fixed_iter=3)
    X6, _ = nn.invert(At, depth=2, fixed_iter=3, x0="given", X=X3.clone())
    Xd, _ = nn.invert(At, depth=2, fixed_iter=6)
    torch.cuda.synchronize()
    assert torch.equal(X6, Xd)


def test_bitwise_reproducible():
    _say("reproducible")
    A = W.dense_spd(333, 1.0, 100.0, 4)
    At = _to_dev(A)
    X1, i1 = nn.invert(At, depth=2, tol=1e-12)
    X2, i2 = nn.invert(At, depth=2, tol=1e-12)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2) and i1["trace"] == i2["trace"]


def test_status_outcomes():
    _say("status nonfinite")
    A = W.dense_spd(64, 1.0, 10.0, 2)
    B = A.copy()
    B[3, 4] = np.nan
    _, info = _gpu_invert(B)
    assert info["status"] == nn.NN_ERR_NONFINITE
    _, info = _gpu_invert(B, x0="identity")
    assert info["status"] == nn.NN_ERR_NONFINITE
    _say("status nonpositive trace")
    _, info = _gpu_invert(-A, x0="identity")
    assert info["status"] == nn.NN_ERR_DIVERGED and info["iters"] == 0
    _say("status indefinite")
    lam = np.r_[np.linspace(1.0, 5.0, 60), [-3.0, -2.0, -1.0, -0.5]]
    Q = W.haar_unitary(64, W.rng(1))
    S = (Q * lam) @ Q.T
    Xo, io = oracle.nn_ref(S, x0=oracle.X0_SCALED_IDENTITY, max_iter=200)
    _, info = _gpu_invert(S, x0="identity", max_iter=200)
    assert info["status"] == io["status"] == nn.NN_ERR_DIVERGED
    assert info["iters"] == io["iters"]
    _say("status max_iter")
    C = W.dense_spd(64, 1.0, 1e3, 3, log_spectrum=True)
    _, info = _gpu_invert(C, tol=1e-12, max_iter=3)
    assert info["status"] == nn.NN_NOT_CONVERGED and info["iters"] == 3
    _say("status stagnation")
    Xo, io = oracle.nn_ref(C, d=2, tol=0.0, max_iter=100)
    X, info = _gpu_invert(C, depth=2, tol=0.0, max_iter=100)
    assert info["status"] == io["status"] == nn.NN_STAGNATED
    assert abs(info["iters"] - io["iters"]) <= 1
    assert info["rms"] == min(info["trace"])
    assert _relF(X, Xo) < 1e-10
    _say("status overscaled start")
    X0 = np.ascontiguousarray(3.0 * C.T / np.linalg.norm(C, 2) ** 2)
    Ct = _to_dev(C)
    Xs = torch.from_numpy(X0).to(DEV)
    _, info = nn.invert(Ct, x0="given", X=Xs, max_iter=100)
    assert info["status"] == nn.NN_ERR_DIVERGED


def test_argument_errors_leave_x_untouched():
    _say("arg errors")
    import ctypes
    A = _to_dev(W.dense_spd(32, 1.0, 10.0, 5))
    X = torch.full((32, 32), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(nn.NNError):
        nn.invert(A, depth=0, X=X)
    with pytest.raises(nn.NNError):
        nn.invert(A, tol=float("nan"), X=X)
    ctx = nn.default_context(0)
    p = nn.make_params()
    need = nn.nn_workspace_size(32, nn.NN_F64, ctypes.byref(p))
    hold, wsp, wsb = nn.workspace(need, DEV)
    info = nn.nn_info()
    args = [ctx.ptr, ctypes.c_void_p(A.data_ptr()), 32, ctypes.c_void_p(X.data_ptr()), 32, 32,
            nn.NN_F64, ctypes.byref(p), ctypes.c_void_p(wsp), wsb, ctypes.byref(info)]
    bad_lda = list(args)
    bad_lda[2] = 31
    assert nn.nn_invert(*bad_lda) == nn.NN_ERR_ARG
    alias = list(args)
    alias[3] = ctypes.c_void_p(A.data_ptr())
    assert nn.nn_invert(*alias) == nn.NN_ERR_ARG
    small = list(args)
    small[9] = wsb - 8
    assert nn.nn_invert(*small) == nn.NN_ERR_WORKSPACE
    mis = list(args)
    mis[8] = ctypes.c_void_p(wsp + 8)
    assert nn.nn_invert(*mis) == nn.NN_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((X == 7.0).all())


@pytest.mark.parametrize("dtype", [np.float64, np.complex128])
def test_solve(dtype):
    _say(f"solve {np.dtype(dtype).name}")
    n, k = 120, 5
    g = np.random.default_rng(9)
    A = g.standard_normal((n, n)) + 2 * math.sqrt(n) * np.eye(n)
    B = g.standard_normal((n, k))
    if dtype == np.complex128:
        A = A + 1j * g.standard_normal((n, n))
        B = B + 1j * g.standard_normal((n, k))
    xo, io = oracle.nn_solve_ref(A, B, d=2, tol=1e-13, max_iter=200)
    xs, info = nn.solve(_to_dev(A), _to_dev(B), depth=2, tol=1e-13, max_iter=200)
    torch.cuda.synchronize()
    x = xs.cpu().numpy()
    assert info["status"] in (nn.NN_OK, nn.NN_STAGNATED)
    assert _relF(x, xo) < 1e-10
    assert info["rel_residual"] < 1e-10
    assert abs(info["rel_residual"] - io["rel_residual"]) < 1e-10
