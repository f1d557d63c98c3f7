"""Parity of nn_invert_batched (persistent, graph-launched) with the oracle.

Tolerance: per matrix, relative Frobenius difference <= 1e-5 between the
complex64 (or FP32) batched result after a fixed number of nests and the
oracle's complex128 (FP64) iterate from the same dtype-rounded input.  Running
the oracle's own step functions on complex64 arrays (a single-precision
emulation) differs from complex128 by at most 4.3e-7 on these inputs (K <= 64,
4 nests, depth 2); 1e-5 leaves a factor ~20 for the different summation order
of the MFMA products.  The per-matrix rms gets that relative bound plus the
proven floor of a residual formed in single precision (see _check).
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
TOL = 1e-5


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def _upload(packed, offsets, sizes):
    return (torch.from_numpy(packed).to(DEV), torch.from_numpy(offsets).to(DEV),
            torch.from_numpy(sizes).to(DEV))


def _run(packed, offsets, sizes, max_n, **kw):
    P, O, S = _upload(packed, offsets, sizes)
    X, info = nn.invert_batched(P, O, S, max_n, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy(), nn.decode_batched_info(info)


def _check(mats, offsets, X, info, d, x0, iters, sample=None):
    it, st, rms = info
    idx = range(len(mats)) if sample is None else sample
    x0c = oracle.X0_TRANSPOSE if x0 == "transpose" else oracle.X0_SCALED_IDENTITY
    worst = 0.0
    for b in idx:
        G = mats[b]
        K = G.shape[0]
        ref_dt = np.complex128 if np.iscomplexobj(G) else np.float64
        Xo, io = oracle.nn_ref(G.astype(ref_dt), d=d, x0=x0c, fixed_iter=iters)
        Xg = X[offsets[b]:offsets[b] + K * K].reshape(K, K).astype(ref_dt)
        e = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
        worst = max(worst, e)
        assert e < TOL, (b, K, e)
        assert st[b] == nn.NN_OK and it[b] == iters
        # the kernel forms I - G X in single precision: |R^ - R| <= gamma_{2K}|G||X|
        # entrywise, so |rms^ - rms| <= 2K u32 ||G||_F ||X||_F / sqrt(K)
        floor = 2 * K * 2.0 ** -24 * np.linalg.norm(G) * np.linalg.norm(Xo) / np.sqrt(K)
        assert abs(rms[b] - io["rms"]) <= TOL * io["rms"] + floor, (b, rms[b], io["rms"], floor)
    return worst


@pytest.mark.parametrize("x0", ["transpose", "identity"])
def test_mimo_batch_parity(x0):
    _say(f"mimo batch 512 x0={x0}")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=512, seed=3)
    X, info = _run(packed, offsets, sizes, 64, depth=2, x0=x0, fixed_iter=4)
    _check(mats, offsets, X, info, 2, x0, 4)


@pytest.mark.parametrize("d", [1, 3])
def test_depths(d):
    _say(f"mimo batch depth {d}")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=96, seed=11)
    X, info = _run(packed, offsets, sizes, 64, depth=d, fixed_iter=3)
    _check(mats, offsets, X, info, d, "transpose", 3)


def test_ragged_sizes_real_and_complex():
    """Every size 1..64 (ragged MFMA tiles), complex64 and FP32."""
    sizes = list(range(1, 65))
    for cplx, dt in ((True, np.complex64), (False, np.float32)):
        _say(f"ragged 1..64 complex={cplx}")
        packed, offsets, sz, mats = W.ragged_batch(sizes, seed=5, lo=1.0, hi=20.0, complex_=cplx,
                                                   dtype=dt)
        X, info = _run(packed, offsets, sz, 64, depth=2, fixed_iter=5)
        _check(mats, offsets, X, info, 2, "transpose", 5)


@pytest.mark.parametrize("wave_max_k,wg", [(0, 1), (8, 2), (16, 1), (32, 1), (32, 4)])
def test_configs_bitwise_identical(wave_max_k, wg):
    """Every kernel configuration gives the same X bits (the per-matrix
    arithmetic does not depend on the work split)."""
    _say(f"config wave_max_k={wave_max_k} wg={wg}")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=160, seed=21)
    P, O, S = _upload(packed, offsets, sizes)
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)
    Xref, _ = nn.invert_batched(P, O, S, 64, fixed_iter=4)
    nn.batched_set_config(nn.NN_C64, 64, wave_max_k, wg)
    X, info = nn.invert_batched(P, O, S, 64, fixed_iter=4)
    torch.cuda.synchronize()
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)
    assert torch.equal(X, Xref)


def test_alone_vs_in_mix_bitwise():
    """A matrix gives the same bits alone and inside a batch."""
    _say("alone vs mix")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=256, seed=4)
    X, _ = _run(packed, offsets, sizes, 64, fixed_iter=4)
    for b in (0, 7, 100, 255):
        p1, o1, s1 = W.pack_batch([mats[b]], np.complex64)
        X1, _ = _run(p1, o1, s1, 64, fixed_iter=4)
        K = mats[b].shape[0]
        assert np.array_equal(X1, X[offsets[b]:offsets[b] + K * K]), b


def test_graph_replay_with_new_inputs():
    """The cached graph is replayed with new contents in the same buffers,
    with eager torch work and synchronisations between replays; every replay
    matches the oracle for the data it saw."""
    _say("graph replay")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=128, seed=8)
    P, O, S = _upload(packed, offsets, sizes)
    X = torch.empty_like(P)
    info = torch.empty(128 * 16, dtype=torch.uint8, device=DEV)
    hold = nn.workspace(nn.nn_batched_workspace_size(128, nn.NN_C64), DEV)
    for rep in range(3):
        packed2, _, _, mats2 = W.mimo_gram_batch(batch=128, seed=8 + rep) if rep else (packed, 0, 0, mats)
        # same sizes as the first draw are required for the same offsets: keep sizes fixed
        if rep:
            mats2 = [W.dense_spd(m.shape[0], 1.0, 10.0 + rep, 1000 * rep + i, complex_=True,
                                 dtype=np.complex64) for i, m in enumerate(mats)]
            packed2, _, _ = W.pack_batch(mats2, np.complex64)
        P.copy_(torch.from_numpy(packed2).to(DEV))
        _ = (P.abs() * 2).sum().item()  # eager work between replays
        nn.invert_batched(P, O, S, 64, fixed_iter=4, X=X, info=info, ws=hold)
        torch.cuda.synchronize()
        _check(mats2, offsets, X.cpu().numpy(), nn.decode_batched_info(info), 2, "transpose", 4,
               sample=range(0, 128, 9))


def test_invalid_sizes_reported_per_matrix():
    _say("invalid sizes")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=32, seed=9)
    bad = sizes.copy()
    bad[3] = 0
    bad[5] = 65
    X, (it, st, rms) = _run(packed, offsets, bad, 64, fixed_iter=4)
    assert st[3] == nn.NN_ERR_ARG and st[5] == nn.NN_ERR_ARG
    good = [b for b in range(32) if b not in (3, 5)]
    _check(mats, offsets, X, (it, st, rms), 2, "transpose", 4, sample=good)


def test_autotune_keeps_results():
    _say("autotune")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=512, seed=12)
    P, O, S = _upload(packed, offsets, sizes)
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)
    Xref, _ = nn.invert_batched(P, O, S, 64, fixed_iter=4)
    best_ms, wk, wg = nn.batched_autotune(P, O, S, 64, fixed_iter=4)
    assert best_ms > 0 and 0 <= wk <= 32 and 1 <= wg <= 8
    X, _ = nn.invert_batched(P, O, S, 64, fixed_iter=4)
    torch.cuda.synchronize()
    assert torch.equal(X, Xref)
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)


def test_argument_errors():
    import ctypes
    _say("batched arg errors")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=8, seed=1)
    P, O, S = _upload(packed, offsets, sizes)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P, O, S, 65, fixed_iter=4)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P, O, S, 64, fixed_iter=-1)
    with pytest.raises(nn.NNError):  # tolerance mode needs 1 <= max_iter <= 4096, tol >= 0
        nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=1e-4, max_iter=0)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=1e-4, max_iter=4097)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=-1.0, max_iter=10)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=float("nan"), max_iter=10)
    with pytest.raises(ValueError):
        nn.invert_batched(P, O, S, 64, x0="given", fixed_iter=2)
    with pytest.raises(nn.NNError):
        nn.invert_batched(P.to(torch.complex128), O, S, 64, fixed_iter=4)


# ---- tolerance mode: every matrix applies nn_invert's stopping rules -------

def _oracle_tol(G, d, x0, tol, max_iter):
    ref_dt = np.complex128 if np.iscomplexobj(G) else np.float64
    return oracle.nn_ref(G.astype(ref_dt), d=d, x0=x0, tol=tol, max_iter=max_iter)


def _fixed_bits(P, O, S, iters, d=2, x0="transpose"):
    X, info = nn.invert_batched(P, O, S, 64, depth=d, x0=x0, fixed_iter=iters)
    torch.cuda.synchronize()
    return X.cpu().numpy(), nn.decode_batched_info(info)


@pytest.mark.parametrize("x0", ["transpose", "identity"])
def test_tolerance_mode_stops_each_matrix(x0):
    """Each matrix stops at its own nest count: the result is bitwise the
    fixed-count result at that count, its rms passed the tolerance, and the
    count agrees with the oracle's complex128 count to within one nest (the
    two may stop one nest apart near the tolerance)."""
    _say(f"tolerance mode mimo 192 x0={x0}")
    tol, mit = 1e-4, 40
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=192, seed=31)
    P, O, S = _upload(packed, offsets, sizes)
    X, info = nn.invert_batched(P, O, S, 64, x0=x0, fixed_iter=0, tol=tol, max_iter=mit)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    it, st, rms = nn.decode_batched_info(info)
    assert np.all(st == nn.NN_OK), st
    assert np.all(rms < tol)
    assert len(set(it.tolist())) >= 3  # the K classes really stop apart
    x0c = oracle.X0_TRANSPOSE if x0 == "transpose" else oracle.X0_SCALED_IDENTITY
    for k in sorted(set(it.tolist())):
        Xf, (itf, stf, rmsf) = _fixed_bits(P, O, S, k, x0=x0)
        for b in np.nonzero(it == k)[0]:
            K = int(sizes[b])
            sl = slice(offsets[b], offsets[b] + K * K)
            assert np.array_equal(X[sl], Xf[sl]), (b, K, k)
            assert rms[b] == rmsf[b], (b, rms[b], rmsf[b])
    for b in range(0, 192, 5):
        Xo, io = _oracle_tol(mats[b], 2, x0c, tol, mit)
        assert io["status"] == oracle.OK
        assert abs(int(it[b]) - io["iters"]) <= 1, (b, it[b], io["iters"])
        if it[b] == io["iters"]:
            K = int(sizes[b])
            Xg = X[offsets[b]:offsets[b] + K * K].reshape(K, K).astype(Xo.dtype)
            assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < TOL, b


def test_tolerance_mode_not_converged_and_stagnated():
    """tol 0 is unreachable: each matrix ends STAGNATED at its single-precision
    floor (returning the iterate before the last nest, bitwise the fixed-count
    result at the reported count) or NOT_CONVERGED at max_iter; a small
    max_iter gives NOT_CONVERGED with exactly max_iter nests."""
    _say("tolerance mode floor / max_iter")
    packed, offsets, sizes, mats = W.ragged_batch([3, 8, 17, 33, 64, 64, 40, 16], seed=41,
                                                 lo=1.0, hi=50.0)
    P, O, S = _upload(packed, offsets, sizes)
    X, info = nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=0.0, max_iter=60)
    torch.cuda.synchronize()
    X = X.cpu().numpy()
    it, st, rms = nn.decode_batched_info(info)
    assert np.all((st == nn.NN_STAGNATED) | (st == nn.NN_NOT_CONVERGED)), st
    assert np.any(st == nn.NN_STAGNATED)
    for b in range(len(mats)):
        K = int(sizes[b])
        Xf, (_, _, rmsf) = _fixed_bits(P, O, S, int(it[b]))
        sl = slice(offsets[b], offsets[b] + K * K)
        assert np.array_equal(X[sl], Xf[sl]), (b, K, it[b], st[b])
        assert rms[b] == rmsf[b]
        # at the floor: within a few single-precision roundings of the exact inverse
        G = mats[b].astype(np.complex128)
        Xg = X[sl].reshape(K, K).astype(np.complex128)
        Xi = np.linalg.inv(G)
        assert np.linalg.norm(Xg - Xi) / np.linalg.norm(Xi) < 1e-4, b
    X2, info2 = nn.invert_batched(P, O, S, 64, fixed_iter=0, tol=1e-30, max_iter=2)
    torch.cuda.synchronize()
    it2, st2, _ = nn.decode_batched_info(info2)
    assert np.all(st2 == nn.NN_NOT_CONVERGED) and np.all(it2 == 2)
    Xf, _ = _fixed_bits(P, O, S, 2)
    assert np.array_equal(X2.cpu().numpy(), Xf)


def test_given_start_continues_the_iteration():
    """x0='given': X holds X_2 from a fixed 2-nest run; two more nests give
    bitwise the fixed 4-nest result, and the tolerance mode from X_2 stops
    where the oracle, started from the same X_2, stops (within one nest)."""
    _say("given start")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=96, seed=33)
    P, O, S = _upload(packed, offsets, sizes)
    X2, _ = nn.invert_batched(P, O, S, 64, fixed_iter=2)
    X4, _ = nn.invert_batched(P, O, S, 64, fixed_iter=4)
    Xg = X2.clone()
    nn.invert_batched(P, O, S, 64, x0="given", fixed_iter=2, X=Xg)
    torch.cuda.synchronize()
    assert torch.equal(Xg, X4)
    Xt = X2.clone()
    _, info = nn.invert_batched(P, O, S, 64, x0="given", fixed_iter=0, tol=1e-4, max_iter=40,
                                X=Xt)
    torch.cuda.synchronize()
    it, st, rms = nn.decode_batched_info(info)
    assert np.all(st == nn.NN_OK) and np.all(rms < 1e-4)
    X2h = X2.cpu().numpy()
    for b in range(0, 96, 7):
        K = int(sizes[b])
        start = X2h[offsets[b]:offsets[b] + K * K].reshape(K, K).astype(np.complex128)
        _, io = oracle.nn_ref(mats[b].astype(np.complex128), d=2, x0=oracle.X0_GIVEN,
                              X_init=start, tol=1e-4, max_iter=40)
        assert io["status"] == oracle.OK
        assert abs(int(it[b]) - io["iters"]) <= 1, (b, it[b], io["iters"])


def test_tolerance_mode_alone_vs_in_mix_bitwise():
    _say("tolerance mode alone vs mix")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=128, seed=34)
    X, info = _run(packed, offsets, sizes, 64, fixed_iter=0, tol=1e-5, max_iter=30)
    it, _, rms = info
    for b in (0, 9, 64, 127):
        p1, o1, s1 = W.pack_batch([mats[b]], np.complex64)
        X1, (it1, _, rms1) = _run(p1, o1, s1, 64, fixed_iter=0, tol=1e-5, max_iter=30)
        K = mats[b].shape[0]
        assert np.array_equal(X1, X[offsets[b]:offsets[b] + K * K]), b
        assert it1[0] == it[b] and rms1[0] == rms[b]


# ---- one workgroup over many items, LDS fitting, persisted autotune --------

@pytest.mark.parametrize("x0", ["transpose", "identity"])
def test_one_workgroup_processes_every_item(x0, monkeypatch):
    """NN_BATCHED_GRID=1: a single persistent workgroup takes all 512 MIMO
    matrices back to back (group items, then wave items after them, on the
    same LDS); every matrix against the oracle, and bitwise equal to the
    default grid."""
    _say(f"one workgroup, 512 mimo, x0={x0}")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=512, seed=3)
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)
    Xref, _ = _run(packed, offsets, sizes, 64, depth=2, x0=x0, fixed_iter=4)
    monkeypatch.setenv("NN_BATCHED_GRID", "1")
    X, info = _run(packed, offsets, sizes, 64, depth=2, x0=x0, fixed_iter=4)
    monkeypatch.delenv("NN_BATCHED_GRID")
    _check(mats, offsets, X, info, 2, x0, 4)
    assert np.array_equal(X, Xref)


@pytest.mark.parametrize("grid", [1, 3])
def test_small_grids_tolerance_mode_bitwise(grid, monkeypatch):
    """The tolerance-mode kernel on one and three workgroups: the same bits as
    the default grid for every matrix (K = 8..64, wave and group items)."""
    _say(f"tolerance mode grid={grid}")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=256, seed=35)
    Xref, iref = _run(packed, offsets, sizes, 64, fixed_iter=0, tol=1e-5, max_iter=30)
    monkeypatch.setenv("NN_BATCHED_GRID", str(grid))
    X, info = _run(packed, offsets, sizes, 64, fixed_iter=0, tol=1e-5, max_iter=30)
    monkeypatch.delenv("NN_BATCHED_GRID")
    assert np.array_equal(X, Xref)
    for a, b in zip(info, iref):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("cplx", [True, False])
def test_depth3_with_wave_max_k_32(cplx):
    """Depth 3 keeps three LDS buffers per matrix; a configured one-wave limit
    of 32 is lowered to what fits (16 for complex64: 32 would need 204 KB of
    LDS), and the results match the oracle and the default configuration."""
    _say(f"depth 3 wave_max_k=32 complex={cplx}")
    dt = nn.NN_C64 if cplx else nn.NN_F32
    if cplx:
        packed, offsets, sizes, mats = W.mimo_gram_batch(batch=128, seed=36)
    else:
        szs = [int(k) for k in np.random.default_rng(36).choice([8, 16, 24, 32, 48, 64], 96)]
        packed, offsets, sizes, mats = W.ragged_batch(szs, seed=36, lo=1.0, hi=20.0,
                                                     complex_=False, dtype=np.float32)
    assert nn.nn_batched_fit_config(dt, 64, 32, 3) == (16 if cplx else 32)
    nn.batched_set_config(dt, 64, 16, 1)
    Xref, _ = _run(packed, offsets, sizes, 64, depth=3, fixed_iter=3)
    nn.batched_set_config(dt, 64, 32, 2)
    X, info = _run(packed, offsets, sizes, 64, depth=3, fixed_iter=3)
    nn.batched_set_config(dt, 64, 16, 1)
    _check(mats, offsets, X, info, 3, "transpose", 3)
    assert np.array_equal(X, Xref)


def test_autotune_depth3_complex():
    """The autotuner skips the candidates whose LDS does not fit at depth 3
    (complex64, one-wave limit 32) instead of failing."""
    _say("autotune depth 3")
    packed, offsets, sizes, mats = W.mimo_gram_batch(batch=256, seed=37)
    P, O, S = _upload(packed, offsets, sizes)
    best_ms, wk, wg = nn.batched_autotune(P, O, S, 64, depth=3, fixed_iter=3)
    assert best_ms > 0 and wk in (0, 8, 16)
    X, info = nn.invert_batched(P, O, S, 64, depth=3, fixed_iter=3)
    torch.cuda.synchronize()
    _check(mats, offsets, X.cpu().numpy(), nn.decode_batched_info(info), 3, "transpose", 3,
           sample=range(0, 256, 5))
    nn.batched_set_config(nn.NN_C64, 64, 16, 1)


_CACHE_CHILD = r"""
import sys, json, torch
sys.path.insert(0, sys.argv[1])
from paper_2212_02406_amd import nn, workloads as W
packed, offsets, sizes, mats = W.mimo_gram_batch(batch=384, seed=38)
P, O, S = (torch.from_numpy(a).to('cuda:0') for a in (packed, offsets, sizes))
best, wk, wg, cached = nn.batched_autotune(P, O, S, 64, fixed_iter=4, with_source=True)
X, _ = nn.invert_batched(P, O, S, 64, fixed_iter=4)
torch.cuda.synchronize()
torch.save(X.cpu(), sys.argv[2])
print(json.dumps({"best": best, "wk": wk, "wg": wg, "cached": cached}), flush=True)
"""


def test_autotune_cache_persists_across_processes(tmp_path):
    """A second process finds the first one's entry in NN_AUTOTUNE_CACHE,
    skips the timing runs, uses the same configuration and gives the same
    bits."""
    import json
    import os
    import subprocess
    _say("autotune cache across processes")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, NN_AUTOTUNE_CACHE=str(tmp_path / "tune.txt"))
    outs = []
    for i in range(2):
        r = subprocess.run([sys.executable, "-c", _CACHE_CHILD, root, str(tmp_path / f"x{i}.pt")],
                           env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    assert not outs[0]["cached"] and outs[1]["cached"]
    assert (outs[0]["wk"], outs[0]["wg"]) == (outs[1]["wk"], outs[1]["wg"])
    assert abs(outs[0]["best"] - outs[1]["best"]) < 1e-3
    lines = open(tmp_path / "tune.txt").read().split()
    assert len(lines) == 6  # one entry, written once
    x0 = torch.load(tmp_path / "x0.pt")
    x1 = torch.load(tmp_path / "x1.pt")
    assert torch.equal(x0, x1)
