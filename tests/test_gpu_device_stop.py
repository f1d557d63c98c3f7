"""The device-side stopping rules (NN_FLAG_DEVICE_STOP) against the host
rules, through the C ABI.

The flag moves the tolerance-mode rules into a kernel after each residual and
lets the host read their outcome only every few nests; products enqueued past
the stop return at once.  The rules and the arithmetic are the host loop's,
so every case must give the same X bit for bit, and the same status, nests,
rms, trace and product count.  The host loop itself is checked against the
oracle in the parity tests; one case here also goes to the oracle directly.
Each case prints its name before its GPU step.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2212_02406_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
from paper_2212_02406_amd import nn  # noqa: E402

DEV = torch.device("cuda:0")


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _both(A, X0=None, **kw):
    """(X, info) with host rules and with device rules, same arguments."""
    At = torch.from_numpy(np.ascontiguousarray(A)).to(DEV)
    out = []
    for flags in (0, nn.NN_FLAG_DEVICE_STOP):
        X = None if X0 is None else torch.from_numpy(np.ascontiguousarray(X0)).to(DEV)
        Xr, info = nn.invert(At, X=X, flags=flags, **kw)
        torch.cuda.synchronize()
        out.append((Xr.cpu().numpy(), info))
    return out


def _same(host, dev, check_x=True):
    (Xh, ih), (Xd, idv) = host, dev
    for key in ("status", "iters", "gemms"):
        assert ih[key] == idv[key], (key, ih[key], idv[key])
    assert np.array_equal(np.array(ih["trace"]), np.array(idv["trace"]), equal_nan=True)
    assert (np.isnan(ih["rms"]) and np.isnan(idv["rms"])) or ih["rms"] == idv["rms"]
    assert ih["prec_gemms"] == idv["prec_gemms"]
    if check_x:
        assert np.array_equal(Xh, Xd, equal_nan=True)


@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("x0", ["transpose", "identity"])
def test_n256_fp64_same_bits(d, x0):
    """The small single-matrix workload: N = 256 SPD, lambda ~ U[1, 100]."""
    _say(f"device stop n256 d={d} x0={x0}")
    A = W.dense_spd(256, 1.0, 100.0, 1)
    h, dv = _both(A, depth=d, x0=x0, tol=1e-12, max_iter=100)
    assert h[1]["status"] == nn.NN_OK
    _same(h, dv)
    x0c = oracle.X0_TRANSPOSE if x0 == "transpose" else oracle.X0_SCALED_IDENTITY
    Xo, io = oracle.nn_ref(A, d=d, x0=x0c, tol=1e-12)
    assert abs(dv[1]["iters"] - io["iters"]) <= 1
    assert np.linalg.norm(dv[0] - Xo) / np.linalg.norm(Xo) < 1e-10


@pytest.mark.parametrize("dtype", [np.float64, np.float32, np.complex128, np.complex64])
@pytest.mark.parametrize("n", [1, 37, 200, 513])
def test_dtypes_and_ragged_sizes(dtype, n):
    """Every dtype, sizes with ragged tiles; single precision to its floor
    (STAGNATED) and double to a tolerance."""
    _say(f"device stop {np.dtype(dtype).name} n={n}")
    cplx = np.dtype(dtype).kind == "c"
    A = W.dense_spd(n, 1.0, 60.0, 40 + n, complex_=cplx, dtype=dtype)
    single = np.dtype(dtype) in (np.dtype(np.float32), np.dtype(np.complex64))
    h, dv = _both(A, depth=2, tol=1e-5 if single else 1e-12, max_iter=60)
    _same(h, dv)
    h, dv = _both(A, depth=3, x0="identity", tol=0.0, max_iter=60)
    assert h[1]["status"] == nn.NN_STAGNATED
    _same(h, dv)


def test_status_outcomes_same():
    _say("device stop status nonfinite")
    A = W.dense_spd(64, 1.0, 10.0, 2)
    B = A.copy()
    B[3, 4] = np.nan
    for x0 in ("transpose", "identity"):
        h, dv = _both(B, x0=x0)
        assert h[1]["status"] == nn.NN_ERR_NONFINITE
        _same(h, dv, check_x=False)
    _say("device stop nonpositive trace")
    h, dv = _both(-A, x0="identity")
    assert h[1]["status"] == nn.NN_ERR_DIVERGED and h[1]["iters"] == 0
    _same(h, dv, check_x=False)
    _say("device stop zero matrix")
    h, dv = _both(np.zeros((40, 40)), x0="transpose")
    assert h[1]["status"] == nn.NN_ERR_DIVERGED
    _same(h, dv, check_x=False)
    _say("device stop indefinite")
    lam = np.r_[np.linspace(1.0, 5.0, 60), [-3.0, -2.0, -1.0, -0.5]]
    Q = W.haar_unitary(64, W.rng(1))
    S = (Q * lam) @ Q.T
    h, dv = _both(S, x0="identity", max_iter=200)
    assert h[1]["status"] == nn.NN_ERR_DIVERGED
    _same(h, dv, check_x=False)
    _say("device stop max_iter")
    C = W.dense_spd(64, 1.0, 1e3, 3, log_spectrum=True)
    for m in (1, 2, 3, 17):
        h, dv = _both(C, tol=1e-12, max_iter=m)
        assert h[1]["status"] == nn.NN_NOT_CONVERGED and h[1]["iters"] == m
        _same(h, dv)
    _say("device stop stagnation")
    h, dv = _both(C, depth=2, tol=0.0, max_iter=100)
    assert h[1]["status"] == nn.NN_STAGNATED
    _same(h, dv)
    _say("device stop overscaled start")
    X0 = 3.0 * C.T / np.linalg.norm(C, 2) ** 2
    h, dv = _both(C, X0=X0, x0="given", max_iter=100)
    assert h[1]["status"] == nn.NN_ERR_DIVERGED
    _same(h, dv, check_x=False)
    _say("device stop given start, converged")
    X0 = C.T / np.linalg.norm(C, 2) ** 2
    h, dv = _both(C, X0=X0, x0="given", tol=1e-12, max_iter=100)
    assert h[1]["status"] == nn.NN_OK
    _same(h, dv)


def test_timing_and_solve():
    """GEMM event timing counts only the products that did work; nn_solve
    takes the flag through its inverse."""
    _say("device stop timing")
    A = W.dense_spd(300, 1.0, 100.0, 5)
    At = torch.from_numpy(A).to(DEV)
    X, info = nn.invert(At, tol=1e-12, flags=nn.NN_FLAG_DEVICE_STOP | nn.NN_FLAG_TIME_GEMMS)
    torch.cuda.synchronize()
    assert info["status"] == nn.NN_OK and info["gemm_ms"] > 0
    assert info["gemms"] == info["iters"] * 3 + 1
    _say("device stop solve")
    B = torch.from_numpy(W.rng(3).standard_normal((300, 7))).to(DEV)
    import ctypes
    outs = []
    for flags in (0, nn.NN_FLAG_DEVICE_STOP):
        p = nn.make_params(depth=2, tol=1e-12, flags=flags)
        need = nn.nn_solve_workspace_size(300, 7, nn.NN_F64, ctypes.byref(p))
        hold, wsp, wsb = nn.workspace(need, DEV)
        Xs = torch.empty((300, 7), dtype=torch.float64, device=DEV)
        info = nn.nn_info()
        rel = ctypes.c_double()
        st = nn.nn_solve(nn.default_context(0).ptr, ctypes.c_void_p(At.data_ptr()), 300,
                         ctypes.c_void_p(B.data_ptr()), 7, ctypes.c_void_p(Xs.data_ptr()), 7,
                         300, 7, nn.NN_F64, ctypes.byref(p), ctypes.c_void_p(wsp), wsb,
                         ctypes.byref(info), ctypes.byref(rel))
        torch.cuda.synchronize()
        assert st == nn.NN_OK
        outs.append((Xs.cpu().numpy(), info.iters, rel.value))
        del hold
    assert np.array_equal(outs[0][0], outs[1][0]) and outs[0][1:] == outs[1][1:]
