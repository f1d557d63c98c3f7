"""Parity at the full workload sizes, in the launch configurations bench.py
times, on sampled outputs with references that hold at any size.

* Dense N = 8192 FP64 (cond 1e3, transpose start, depth 2): A = Q diag(lam)
  Q^T is built from known factors, so at a forced nest count k the exact
  iterate is X_k = Q diag(x_k(lam)) Q^T with x_k(l) = (1 - (1 - l^2/s)^m) / l,
  m = (d+1)^k, s = ||A||_1 ||A||_inf (R_0 = I - A^2/s and R_k = R_0^m, the
  Sec. II-D Theorem / Corollary 2 with the transpose start).  Sampled columns
  of X_k cost O(N^2) each.  Bar 1e-10 relative per column: FP64 products of
  these iterates carry errors of order N u ||A|| ||X|| << 1e-10.
* Tolerance mode: the returned X satisfies X - A^-1 = -A^-1 R, so a column's
  error relative to ||A^-1 e_j|| >= 1/lam_max is at most kappa ||R||_F =
  kappa sqrt(N) rms.
* Mixed N = 16384 (cond 1e4, tol 1e-11): sampled columns against the exact
  inverse within kappa sqrt(N) rms, and the whole result against plain FP64 at
  relative Frobenius 1e-10.
* Batched: all 4096 MIMO matrices with the autotuned configuration, every
  one against the oracle as in the batched parity tests.
* Serving: requests drawn from the serving pool (N up to 4096); the true rms
  of every result is recomputed in FP64 on the host.
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
U32 = 2.0 ** -24


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dense8192():
    A, lam, Q = W.dense_spd(8192, 1.0, 1e3, 2, log_spectrum=True, device="cuda",
                            return_factors=True)
    return A, lam, Q


def _cols(n, k=8, seed=0):
    return sorted(np.random.default_rng(seed).choice(n, k, replace=False).tolist())


def test_n8192_fp64_forced_k_closed_form(dense8192):
    A, lam, Q = dense8192
    n, d, k = 8192, 2, 6
    _say(f"n8192 fp64 transpose forced k={k}")
    X, info = nn.invert(torch.from_numpy(A).to(DEV), depth=d, x0="transpose", fixed_iter=k)
    torch.cuda.synchronize()
    assert info["status"] == nn.NN_OK and info["iters"] == k
    s = np.abs(A).sum(axis=0).max() * np.abs(A).sum(axis=1).max()
    m = (d + 1) ** k
    xk = (1.0 - (1.0 - lam ** 2 / s) ** m) / lam
    cols = _cols(n)
    Xc = X[:, cols].cpu().numpy()
    for t, j in enumerate(cols):
        ref = Q @ (xk * Q[j, :])
        assert np.linalg.norm(Xc[:, t] - ref) / np.linalg.norm(ref) < 1e-10, j


def test_n8192_fp64_tolerance_mode(dense8192):
    A, lam, Q = dense8192
    n = 8192
    _say("n8192 fp64 transpose tol 1e-12")
    X, info = nn.invert(torch.from_numpy(A).to(DEV), depth=2, x0="transpose", tol=1e-12,
                        max_iter=100)
    torch.cuda.synchronize()
    assert info["status"] == nn.NN_OK and info["rms"] < 1e-12
    kappa = lam.max() / lam.min()
    cols = _cols(n, seed=1)
    Xc = X[:, cols].cpu().numpy()
    for t, j in enumerate(cols):
        ref = Q @ (Q[j, :] / lam)
        assert np.linalg.norm(Xc[:, t] - ref) / np.linalg.norm(ref) <= kappa * np.sqrt(n) * 1e-12


def test_n8192_fp32_to_floor(dense8192):
    """FP32: tol 1e-6 is below the single-precision floor; the run ends
    STAGNATED (or OK) with sampled columns within 64 u32 kappa of A^-1."""
    A, lam, Q = dense8192
    n = 8192
    _say("n8192 fp32 transpose tol 1e-6")
    A32 = torch.from_numpy(A).to(DEV).to(torch.float32)
    X, info = nn.invert(A32, depth=2, x0="transpose", tol=1e-6, max_iter=100)
    torch.cuda.synchronize()
    assert info["status"] in (nn.NN_OK, nn.NN_STAGNATED), info
    kappa = lam.max() / lam.min()
    cols = _cols(n, seed=2)
    Xc = X[:, cols].cpu().numpy().astype(np.float64)
    for t, j in enumerate(cols):
        ref = Q @ (Q[j, :] / lam)
        assert np.linalg.norm(Xc[:, t] - ref) / np.linalg.norm(ref) < 64 * U32 * kappa


def test_n16384_mixed_vs_exact_and_plain():
    n = 16384
    _say("n16384 mixed cond 1e4 tol 1e-11")
    A, lam, Q = W.dense_spd(n, 1.0, 1e4, 4, log_spectrum=True, device="cuda",
                            return_factors=True)
    At = torch.from_numpy(A).to(DEV)
    Xm, im = nn.invert(At, depth=2, x0="identity", tol=1e-11, max_iter=100, prec="mixed")
    torch.cuda.synchronize()
    assert im["status"] == nn.NN_OK and im["rms"] < 1e-11, im
    assert im["phase_iters"][0] > 0 and im["phase_iters"][1] > 0
    Xp, ip = nn.invert(At, depth=2, x0="identity", tol=1e-11, max_iter=100)
    torch.cuda.synchronize()
    assert ip["status"] == nn.NN_OK
    rel = (torch.linalg.norm(Xm - Xp) / torch.linalg.norm(Xp)).item()
    assert rel < 1e-10, rel
    # entrywise as well: a wrong tile would be diluted in the Frobenius norm
    relmax = ((Xm - Xp).abs().max() / Xp.abs().max()).item()
    assert relmax < 1e-10, relmax
    kappa = lam.max() / lam.min()
    cols = _cols(n, k=4, seed=3)
    Xc = Xm[:, cols].cpu().numpy()
    for t, j in enumerate(cols):
        ref = Q @ (Q[j, :] / lam)
        # x - A^-1 e_j = A^-1 (A x - e_j) and |A^-1 e_j| >= 1 / lambda_max, so the
        # relative error of the column is at most kappa |r_j|, r_j = e_j - A x
        # (the column's own residual, computed here in FP64); 1e-11 covers the
        # rounding of the reference column itself
        r = -(A @ Xc[:, t])
        r[j] += 1.0
        err = np.linalg.norm(Xc[:, t] - ref) / np.linalg.norm(ref)
        assert err <= kappa * np.linalg.norm(r) * 1.01 + 1e-11, (j, err, np.linalg.norm(r))


def test_batched_4096_autotuned_all():
    """Every one of the 4096 matrices against the oracle, both starts."""
    _say("batched 4096 mimo autotuned")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=4096, seed=3)
    P = torch.from_numpy(packed).to(DEV)
    O = torch.from_numpy(offsets).to(DEV)
    S = torch.from_numpy(sizes).to(DEV)
    nn.batched_autotune(P, O, S, 64, fixed_iter=4)
    for x0, x0c in (("transpose", oracle.X0_TRANSPOSE), ("identity", oracle.X0_SCALED_IDENTITY)):
        X, info = nn.invert_batched(P, O, S, 64, x0=x0, fixed_iter=4)
        torch.cuda.synchronize()
        Xh = X.cpu().numpy()
        it, st, rms = nn.decode_batched_info(info)
        assert np.all(st == nn.NN_OK) and np.all(it == 4)
        for b in range(4096):
            G = mats[b].astype(np.complex128)
            K = G.shape[0]
            Xo, io = oracle.nn_ref(G, d=2, x0=x0c, fixed_iter=4)
            Xg = Xh[offsets[b]:offsets[b] + K * K].reshape(K, K).astype(np.complex128)
            assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < 1e-5, (x0, b, K)
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)


def test_serving_pool_requests_true_rms():
    _say("serving pool requests up to N=4096")
    pool = W.serving_pool(64, seed=5)
    pick = list(dict.fromkeys(sorted(range(64), key=lambda i: -pool[i]["n"])[:6] + list(range(6))))
    srv = nn.Server(48 << 30, max_active=64)
    src = {}
    for i in pick:
        A = W.build_request(pool[i], device="cuda" if pool[i]["n"] >= 512 else None)
        src[i] = A
        srv.submit(i, torch.from_numpy(A).to(DEV), pool[i]["tol"], 100)
    torch.cuda.synchronize()
    seen = 0
    for _ in range(10000):
        s = srv.tick()
        for r in srv.poll():
            i = r["id"]
            A = src[i]
            assert r["status"] == nn.NN_OK, r
            X = srv.fetch(i, r["n"], r["out_dtype"], out_device="cpu").numpy()
            Ad = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64)
            R = np.eye(A.shape[0]) - Ad @ X.astype(Ad.dtype)
            rt = float(np.sqrt(np.sum(np.abs(R) ** 2) / A.shape[0]))
            tol = pool[i]["tol"]
            if r["wide_iters"] > 0:
                assert rt < tol * (1 + 1e-6) + 1e-13, (r, rt)
            else:
                # residual formed in FP32: its rms differs from the FP64 one by at
                # most the single-precision floor 2 N u32 ||A||_F ||X||_F / sqrt(N)
                floor = 2 * A.shape[0] * U32 * np.linalg.norm(Ad) * np.linalg.norm(X) / np.sqrt(
                    A.shape[0])
                assert rt < tol + floor, (r, rt, floor)
            seen += 1
        if s.active == 0 and s.queued == 0:
            break
    srv.close()
    assert seen == len(pick)
