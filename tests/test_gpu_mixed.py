"""Mixed-precision schedule (BF16 -> FP32 -> FP64) against the FP64 oracle.

The schedule's trajectory is not pinned nest by nest (its BF16 and FP32
phases carry their own rounding); what is pinned:
* the final iterate: relative Frobenius difference to the oracle's converged
  FP64 iterate (identity start, same tolerance) <= 1e-10, and its FP64 rms
  < tol;
* the BF16 phase products: its first nests' rms follows the oracle's FP64
  trajectory within the BF16 perturbation (relative 2e-2), which a wrong
  operand layout or a missing term in the BF16 GEMM would break;
* the phase accounting: nests in phases B + F + D = iters.
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


@pytest.mark.parametrize("n,cond,d", [(512, 1e4, 2), (1000, 1e4, 2), (1001, 1e3, 2), (256, 100.0, 2),
                                      (384, 1e4, 3), (320, 1e3, 1)])
def test_mixed_matches_fp64_oracle(n, cond, d):
    _say(f"mixed n={n} cond={cond:g} d={d}")
    A = W.dense_spd(n, 1.0, cond, 40 + n, log_spectrum=True)
    Xo, io = oracle.nn_ref(A, d=d, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12, max_iter=200)
    assert io["status"] == oracle.OK
    X, info = nn.invert(torch.from_numpy(A).to(DEV), depth=d, x0="identity", tol=1e-12,
                        max_iter=200, prec="mixed")
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    assert info["status"] == nn.NN_OK, info
    assert info["rms"] < 1e-12
    rel = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    assert rel < 1e-10, rel
    pb, pf, pd = info["phase_iters"]
    assert pb + pf + pd == info["iters"]
    assert pd >= 1
    if n % 8 == 0:
        assert pb >= 2, info["phase_iters"]
        for k in range(min(pb, 6)):
            a, b = info["trace"][k], io["trace"][k]
            assert abs(a - b) <= 2e-2 * b, (k, a, b)
    else:
        assert pb == 0


def test_mixed_unsupported_combinations():
    _say("mixed unsupported")
    A = torch.from_numpy(W.dense_spd(64, 1.0, 10.0, 3)).to(DEV)
    for kw in (dict(x0="transpose"), dict(x0="identity", fixed_iter=3)):
        _, info = nn.invert(A, prec="mixed", check=False, **kw)
        assert info["status"] == nn.NN_ERR_UNSUPPORTED
    with pytest.raises(nn.NNError):  # no workspace size exists for a non-FP64 mixed call
        nn.invert(A.to(torch.float32), prec="mixed", x0="identity", check=False)


def test_mixed_status_nonpositive_trace():
    _say("mixed nonpositive trace")
    A = torch.from_numpy(-W.dense_spd(64, 1.0, 10.0, 3)).to(DEV)
    _, info = nn.invert(A, prec="mixed", x0="identity", check=False)
    assert info["status"] == nn.NN_ERR_DIVERGED


@pytest.mark.parametrize("n,tol", [(512, 1e-3), (1000, 1e-2)])
def test_mixed_loose_tolerance_ends_in_fp32(n, tol):
    """A tolerance far above the FP32 floor (a preconditioner's) is met by the
    FP32 iterate: no FP64 nest, the FP64 check of the returned X below tol."""
    _say(f"mixed loose n={n} tol={tol:g}")
    A = W.dense_spd(n, 1.0, 1e3, 60 + n, log_spectrum=True)
    X, info = nn.invert(torch.from_numpy(A).to(DEV), depth=2, x0="identity", tol=tol,
                        max_iter=200, prec="mixed")
    torch.cuda.synchronize()
    assert info["status"] == nn.NN_OK, info
    pb, pf, pd = info["phase_iters"]
    assert pd == 0 and pb + pf == info["iters"], info["phase_iters"]
    Xh = X.cpu().numpy()
    rms = np.linalg.norm(np.eye(n) - A @ Xh) / np.sqrt(n)
    assert rms < tol and abs(rms - info["rms"]) <= 1e-9 * rms + 1e-13
    # the iterate is the oracle's NN trajectory to within the single-precision
    # perturbation: the oracle's rms after the same number of nests is close
    _, io = oracle.nn_ref(A, d=2, x0=oracle.X0_SCALED_IDENTITY, fixed_iter=info["iters"])
    assert rms <= 4.0 * io["rms"] + 1e-6


@pytest.mark.parametrize("n,cond", [(512, 1e4), (1000, 1e3)])
def test_mixed_power_identity_start(n, cond):
    """The mixed schedule from Theta_2(8) I: against the oracle's converged
    FP64 iterate from the same start (1e-10), in fewer nests than I / Tr A."""
    _say(f"mixed power_identity n={n} cond={cond:g}")
    A = W.dense_spd(n, 1.0, cond, 70 + n, log_spectrum=True)
    At = torch.from_numpy(A).to(DEV)
    Xo, io = oracle.nn_ref(A, d=2, x0=oracle.X0_POWER_IDENTITY, tol=1e-12, max_iter=200, power_k=8)
    X, info = nn.invert(At, depth=2, x0="power_identity", tol=1e-12, max_iter=200, prec="mixed",
                        power_k=8)
    _, i1 = nn.invert(At, depth=2, x0="identity", tol=1e-12, max_iter=200, prec="mixed")
    torch.cuda.synchronize()
    assert io["status"] == oracle.OK and info["status"] == nn.NN_OK, info
    assert info["rms"] < 1e-12
    assert np.linalg.norm(X.cpu().numpy() - Xo) / np.linalg.norm(Xo) < 1e-10
    assert info["iters"] <= i1["iters"]


@pytest.mark.parametrize("n", [512, 768, 1000])
def test_bf16_tilings_agree(n, monkeypatch):
    """The 256 x 256 and 128 x 128 BF16 tilings, each staged through registers
    or loaded straight into LDS (the latter for exact tilings: n = 512, 768),
    accumulate every output element over the same k in the same order, so the
    schedule takes the same steps: equal phase counts, BF16-phase rms equal up
    to the partials' summation order, and the same final iterate.  n = 1000
    exercises the bounds-checked form (not a multiple of either tile)."""
    _say(f"bf16 tilings n={n}")
    A = torch.from_numpy(W.dense_spd(n, 1.0, 1e4, 60 + n, log_spectrum=True)).to(DEV)
    res = {}
    for tile, dma in (("128", "0"), ("128", "1"), ("256", "0"), ("256", "1")):
        monkeypatch.setenv("NN_BF16_TILE", tile)
        monkeypatch.setenv("NN_BF16_DMA", dma)
        X, info = nn.invert(A, depth=2, x0="identity", tol=1e-12, max_iter=200, prec="mixed")
        torch.cuda.synchronize()
        assert info["status"] == nn.NN_OK, (tile, dma, info)
        res[tile + dma] = (X.cpu().numpy(), info)
    X1, i1 = res["1280"]
    pb = i1["phase_iters"][0]
    if n % 8 == 0:
        assert pb >= 2
    for key in ("1281", "2560", "2561"):
        X2, i2 = res[key]
        assert i1["phase_iters"] == i2["phase_iters"], key
        for k in range(pb + 1):
            a, b = i1["trace"][k], i2["trace"][k]
            assert abs(a - b) <= 1e-12 * b, (key, k, a, b)
        assert np.linalg.norm(X1 - X2) <= 1e-13 * np.linalg.norm(X1), key


@pytest.mark.parametrize("n", [1024, 1536])
def test_single_fp64_nest_from_the_fp32_floor(n):
    """From the FP32 floor the FP64 residual falls at full order, so one FP64
    nest, of the smallest depth predicted to finish, takes it below tol: one
    FP64 nest, rms < tol, and the iterate agrees with LAPACK's inverse within
    the residual bound."""
    _say(f"mixed one FP64 nest n={n}")
    A = W.dense_spd(n, 1.0, 1e4, 80 + n, log_spectrum=True)
    X, info = nn.invert(torch.from_numpy(A).to(DEV), depth=2, x0="identity", tol=1e-11,
                        max_iter=200, prec="mixed")
    torch.cuda.synchronize()
    assert info["status"] == nn.NN_OK and info["rms"] < 1e-11, info
    pb, pf, pd = info["phase_iters"]
    assert pd == 1, info["phase_iters"]
    Xi = np.linalg.inv(A)
    rel = np.linalg.norm(X.cpu().numpy() - Xi) / np.linalg.norm(Xi)
    # X - A^-1 = -A^-1 R: relative error <= sqrt(n) rms, plus LAPACK's own cond * u
    assert rel < 2.0 * np.sqrt(n) * info["rms"] + 1e-11, rel
