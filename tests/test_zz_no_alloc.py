"""nn_invert_noalloc (static device scratch, no allocation) against
nn_invert with a caller workspace, through the C ABI.

Both run the same kernels on the same inputs, so X, status, nests, rms and
trace must be identical bit for bit.  Each case makes two calls in a row, the
second on a smaller matrix, so the second runs on scratch the first left
behind.  Sizes beyond the scratch are refused before any launch.
"""
import ctypes
import sys

import numpy as np
import pytest

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


def _pair(A, **kw):
    """(X, info) from nn_invert (workspace) and from nn_invert_noalloc."""
    At = torch.from_numpy(np.ascontiguousarray(A)).to(DEV)
    Xw, iw = nn.invert(At, **kw)
    torch.cuda.synchronize()
    Xs = torch.full_like(At, float("nan"))
    st, is_ = nn.invert_noalloc(At, Xs, **kw)
    torch.cuda.synchronize()
    assert st == iw["status"], (st, iw["status"])
    return Xw.cpu().numpy(), iw, Xs.cpu().numpy(), is_


def _same(Xw, iw, Xs, is_):
    for key in ("status", "iters", "gemms", "prec_gemms", "phase_iters"):
        assert iw[key] == is_[key], (key, iw[key], is_[key])
    assert np.array_equal(np.array(iw["trace"]), np.array(is_["trace"]), equal_nan=True)
    assert iw["rms"] == is_["rms"] or (np.isnan(iw["rms"]) and np.isnan(is_["rms"]))
    assert np.array_equal(Xw, Xs)


@pytest.mark.parametrize("dtype,sizes,kw", [
    (np.float64, (1176, 256), dict(depth=2, tol=1e-12)),
    (np.float64, (600, 37), dict(depth=3, x0="identity", tol=1e-12,
                                 flags=nn.NN_FLAG_DEVICE_STOP)),
    (np.float32, (1000, 129), dict(depth=2, tol=1e-5)),
    (np.complex64, (700, 65), dict(depth=1, fixed_iter=9)),
    (np.complex128, (830, 100), dict(depth=2, tol=1e-12)),
    (np.float64, (698, 300), dict(depth=2, x0="identity", prec="mixed", tol=1e-11)),
])
def test_noalloc_matches_workspace_path(dtype, sizes, kw):
    for n in sizes:
        _say(f"noalloc {np.dtype(dtype).name} n={n} {kw}")
        cplx = np.dtype(dtype).kind == "c"
        A = W.dense_spd(n, 1.0, 100.0, 60 + n, complex_=cplx, dtype=dtype)
        Xw, iw, Xs, is_ = _pair(A, **kw)
        assert iw["status"] in (nn.NN_OK, nn.NN_STAGNATED), iw
        _same(Xw, iw, Xs, is_)


def test_noalloc_refuses_what_does_not_fit():
    _say("noalloc too large")
    n = 1177  # FP64 depth 2: one past the scratch
    A = torch.eye(n, dtype=torch.float64, device=DEV)
    X = torch.full_like(A, 7.0)
    st, _ = nn.invert_noalloc(A, X, depth=2)
    torch.cuda.synchronize()
    assert st == nn.NN_ERR_WORKSPACE
    assert bool((X == 7.0).all())
    _say("noalloc timing flag refused")
    B = torch.eye(64, dtype=torch.float64, device=DEV) * 2.0
    Y = torch.full_like(B, 7.0)
    st, _ = nn.invert_noalloc(B, Y, flags=nn.NN_FLAG_TIME_GEMMS)
    torch.cuda.synchronize()
    assert st == nn.NN_ERR_ARG and bool((Y == 7.0).all())
    _say("noalloc after a refusal")
    A = W.dense_spd(64, 1.0, 10.0, 3)
    _same(*_pair(A, depth=2, tol=1e-12))
