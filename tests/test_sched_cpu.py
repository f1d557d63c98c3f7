"""The server's scheduling policy on the CPU, under AddressSanitizer.

paper_2212_02406_amd/csrc/nn_sched.cpp holds what nn_server decides: the pool
allocator, the layout of each request's pool block, admission by footprint
with bounded bypass, and the per-request rules.  tests/sched_harness.cpp
drives that same source with a fake device (each residual answered by the
next value of an rms sequence the test gives, one tick at a time) and host
buffers in place of the pool blocks; it is built here with g++,
-fsanitize=address,undefined, so any write of the carving past a block, any
use after free in the allocator or the request records fails the run.

Rule pins: FP64 requests fed the oracle's own rms trace must end exactly as
the oracle does (status, nests, rms), which ties the server's per-request
rules to the oracle's stopping rules.  Promotion, stagnation, the small
path's records, admission, starvation and footprint are checked on
sequences built for each case.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2212_02406_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F64, F32, C64, C128 = 0, 1, 2, 3
OK, NOT_CONVERGED, STAGNATED = 0, 1, 2
ERR_DIVERGED, ERR_NONFINITE, ERR_HIP = -2, -3, -4
POINT_D2 = 1e-9 ** (1.0 / 3.0)  # promotion point at depth 2


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("sched") / "sched_harness")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "sched_harness.cpp"),
           os.path.join(ROOT, "paper_2212_02406_amd", "csrc", "nn_sched.cpp"), "-o", exe]
    subprocess.run(cmd, check=True)
    return exe


class Req:
    def __init__(self, rid, n, dtype, tol, max_iter=100, arrival=0, den=1.0, narrow=(),
                 wide=(), rec=None):
        self.rid, self.n, self.dtype, self.tol = rid, n, dtype, tol
        self.max_iter, self.arrival, self.den = max_iter, arrival, den
        self.narrow, self.wide, self.rec = list(narrow), list(wide), rec

    def text(self):
        f = lambda v: repr(float(v))  # noqa: E731
        parts = [str(self.rid), str(self.n), str(self.dtype), f(self.tol), str(self.max_iter),
                 str(self.arrival), f(self.den), str(len(self.narrow))]
        parts += [f(v) for v in self.narrow]
        parts += [str(len(self.wide))] + [f(v) for v in self.wide]
        if self.rec is None:
            parts.append("0")
        else:
            parts += ["1", str(self.rec[0]), str(self.rec[1]), f(self.rec[2])]
        return " ".join(parts)


def run(harness, reqs, depth=2, max_active=64, wide_tol=1e-6, pool=1 << 40, batch_max_n=0,
        ticks_max=100000):
    head = f"{depth} {max_active} {wide_tol!r} {pool} {batch_max_n} {ticks_max} {len(reqs)}\n"
    body = "\n".join(r.text() for r in reqs) + "\n"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([harness], input=head + body, capture_output=True, text=True, env=env,
                       timeout=120)
    assert p.returncode == 0, p.stderr[-4000:]
    out = {"req": {}, "violations": []}
    for line in p.stdout.splitlines():
        w = line.split()
        if w[0] == "violation":
            out["violations"].append(line)
        elif w[0] in ("max_used", "max_active", "ticks"):
            out[w[0]] = int(w[1])
        elif w[0] == "end_used":
            out["end_used"], out["end_ranges"] = int(w[1]), int(w[2])
        else:
            rid = int(w[0])
            out["req"][rid] = dict(status=int(w[1]), iters=int(w[2]), wide_iters=int(w[3]),
                                   rms=float(w[4]), result_buf=int(w[5]), admit=int(w[6]),
                                   finish=int(w[7]), bypassed=int(w[8]), promoted=bool(int(w[9])),
                                   small=bool(int(w[10])))
    assert out["violations"] == [], out["violations"]
    assert out["end_used"] == 0 and out["end_ranges"] == 1
    return out


def _oracle_case(A, **kw):
    _, info = oracle.nn_ref(A, **kw)
    return info


@pytest.mark.parametrize("case", ["ok_d2", "ok_d1", "ok_d3", "max_iter", "stagnated",
                                  "diverged", "nonfinite", "bad_den"])
def test_fp64_rules_match_the_oracle(harness, case):
    """An FP64 request fed the oracle's rms trace ends as the oracle does."""
    A = W.dense_spd(48, 1.0, 1e3, 3, log_spectrum=True)
    d, den = 2, 1.0
    if case == "ok_d2":
        info = _oracle_case(A, d=2, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12)
    elif case == "ok_d1":
        d = 1
        info = _oracle_case(A, d=1, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12)
    elif case == "ok_d3":
        d = 3
        info = _oracle_case(A, d=3, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12)
    elif case == "max_iter":
        info = _oracle_case(A, d=2, x0=oracle.X0_SCALED_IDENTITY, tol=1e-12, max_iter=4)
    elif case == "stagnated":
        info = _oracle_case(A, d=2, x0=oracle.X0_SCALED_IDENTITY, tol=0.0)
    elif case == "diverged":
        lam = np.r_[np.linspace(1.0, 5.0, 44), [-3.0, -2.0, -1.0, -0.5]]
        Q = W.haar_unitary(48, W.rng(1))
        A = (Q * lam) @ Q.T
        info = _oracle_case(A, d=2, x0=oracle.X0_SCALED_IDENTITY, max_iter=200)
    elif case == "nonfinite":
        A = A.copy()
        A[2, 3] = np.inf
        info = _oracle_case(A, d=2, x0=oracle.X0_TRANSPOSE)
    else:  # a trace that is not positive
        info = _oracle_case(-A, d=2, x0=oracle.X0_SCALED_IDENTITY)
        den = info["den"]
    tol = {"stagnated": 0.0}.get(case, 1e-12)
    max_iter = {"max_iter": 4, "diverged": 200}.get(case, 100)
    if case == "nonfinite":
        den = info["den"]
    r = Req(1, 48, F64, tol, max_iter=max_iter, den=den, wide=info["trace"] or [0.5])
    got = run(harness, [r], depth=d)["req"][1]
    assert got["status"] == info["status"], (got, info["status"])
    if info["status"] >= 0 or case in ("diverged",):
        assert got["iters"] == info["iters"]
        assert got["wide_iters"] == info["iters"]
    if info["status"] >= 0:
        assert got["rms"] == info["rms"]
        # X_j sits in buffer j mod 2 of the ping-pong
        assert got["result_buf"] == info["iters"] % 2


def test_promotion_at_the_point_when_wide_is_reserved(harness):
    """tol 1e-8 < wide_tol: the narrow phase hands over once the previous rms
    is below the promotion point, continuing from the better iterate."""
    narrow = [0.9, 0.6, 0.2, 8e-3, 5e-4, 2e-7, 2e-7]
    wide = [3e-7, 1e-13]
    got = run(harness, [Req(7, 300, F32, 1e-8, narrow=narrow, wide=wide)])["req"][7]
    # rms_prev first < 1e-3 at the read of X_5 (prev = X_4's 5e-4); X_5 is
    # better than X_4, so the wide phase starts from X_5; one wide nest ends it
    assert got["promoted"] and got["status"] == OK
    assert got["iters"] == 6 and got["wide_iters"] == 1
    assert got["rms"] == 1e-13 and got["result_buf"] == 1


def test_promotion_from_the_previous_iterate(harness):
    narrow = [0.9, 0.2, 5e-4, 7e-4]
    wide = [4e-4, 1e-13]
    got = run(harness, [Req(8, 100, C64, 1e-8, narrow=narrow, wide=wide)])["req"][8]
    # at X_3: prev 5e-4 < point and 5e-4 <= 7e-4: continue from X_2
    assert got["promoted"] and got["status"] == OK
    assert got["iters"] == 3 and got["wide_iters"] == 1


def test_stagnation_promotes_or_retires(harness):
    """tol 1e-4 >= wide_tol: nothing reserved; a narrow floor above tol
    promotes when the wide buffers fit, else ends STAGNATED on the previous
    iterate."""
    narrow = [0.5, 0.1, 1e-3, 3e-4, 3e-4]
    wide = [3e-4, 1e-9]
    got = run(harness, [Req(9, 256, F32, 1e-4, narrow=narrow, wide=wide)])["req"][9]
    assert got["promoted"] and got["status"] == OK and got["wide_iters"] == 1
    assert got["iters"] == 3 + 1  # X_3 promoted (X_4 no better), one wide nest
    # a pool with room for the narrow block only (five 256 x 256 FP32
    # matrices and the control arrays, 1.3 MB; the wide phase needs 2.6 MB)
    got = run(harness, [Req(9, 256, F32, 1e-4, narrow=narrow, wide=wide)], pool=2 << 20)
    g = got["req"][9]
    assert not g["promoted"] and g["status"] == STAGNATED
    assert g["iters"] == 3 and g["rms"] == 3e-4 and g["result_buf"] == 1


def test_small_path_records(harness):
    """Records of the batched narrow phase: OK below tol retires on X_0's
    buffer; OK at the promotion point and STAGNATED promote; a STAGNATED one
    that cannot get wide buffers retires; an error record retires."""
    reqs = [Req(1, 32, F32, 1e-4, rec=(5, OK, 3e-5)),
            Req(2, 40, C64, 1e-8, rec=(6, OK, 9e-4), wide=[9e-4, 1e-12]),
            Req(3, 16, F32, 1e-5, rec=(7, STAGNATED, 2e-5), wide=[2e-5, 1e-9]),
            Req(4, 64, F32, 1e-4, rec=(3, ERR_DIVERGED, 2.0))]
    out = run(harness, reqs, batch_max_n=64)["req"]
    assert out[1]["small"] and out[1]["status"] == OK and out[1]["iters"] == 5
    assert out[1]["result_buf"] == 0 and not out[1]["promoted"]
    assert out[2]["promoted"] and out[2]["status"] == OK and out[2]["iters"] == 7
    assert out[3]["promoted"] and out[3]["status"] == OK and out[3]["wide_iters"] == 1
    assert out[4]["status"] == ERR_DIVERGED and out[4]["iters"] == 3
    # no room for wide buffers: the stagnated record retires as it is
    r = Req(3, 16, F32, 1e-5, rec=(7, STAGNATED, 2e-5), wide=[2e-5, 1e-9])
    g = run(harness, [r], batch_max_n=64, pool=8 * 1024)["req"][3]  # narrow block 6.4 KB, wide 10 KB
    assert g["status"] == STAGNATED and g["iters"] == 7 and not g["promoted"]


def _converging(n_nests, start=0.9, order=3, floor=1e-13):
    v, out = start, []
    for _ in range(n_nests):
        out.append(max(v, floor))
        v = v ** order
    return out


def test_starvation_is_bounded(harness):
    """A request too large for the free pool is passed over at most 8 ticks;
    then nothing behind it is admitted until it fits, and it runs."""
    small = [Req(100 + i, 64, F64, 1e-12, arrival=i, wide=[0.9] * 6 + [1e-13])
             for i in range(60)]
    big = Req(1, 2048, F64, 1e-12, arrival=1, wide=_converging(8))
    # pool: the big request's block is about 4 x 2048^2 x 8 x 5/4 = 168 MB
    pool = 180 * 1024 * 1024
    out = run(harness, [big] + small, pool=pool, max_active=64)
    b = out["req"][1]
    assert b["status"] == OK
    assert b["bypassed"] <= 8
    # every request finished, nothing left in the pool (checked in run)
    assert all(r["status"] == OK for r in out["req"].values())
    assert out["max_used"] <= pool


def test_max_active_and_footprint(harness):
    g = np.random.default_rng(4)
    reqs = [Req(i, int(g.integers(8, 700)), int(g.integers(0, 4)), 1e-12 if i % 2 else 1e-4,
                arrival=int(g.integers(0, 30)), wide=_converging(int(g.integers(6, 12))),
                narrow=_converging(int(g.integers(6, 12)), floor=3e-7)) for i in range(200)]
    out = run(harness, reqs, max_active=7, pool=1 << 30)
    assert out["max_active"] <= 7
    assert out["max_used"] <= 1 << 30
    assert all(r["status"] in (OK, STAGNATED) for r in out["req"].values())


def test_random_stream_under_sanitizers(harness):
    """2000 requests of every dtype and size class, random sequences
    (converging, stagnating, diverging, non-finite), random arrivals, a pool
    that forces queueing and late wide reservations that fail; the run must
    be clean under ASan/UBSan and every invariant of the harness hold."""
    g = np.random.default_rng(11)
    reqs = []
    for i in range(2000):
        n = int(np.rint(np.exp(g.uniform(np.log(4), np.log(700)))))
        kind = g.integers(0, 10)
        if kind < 6:
            wide = _converging(int(g.integers(2, 12)), start=float(g.uniform(0.3, 0.99)))
        elif kind < 8:
            wide = [0.5, 0.1, 1e-3, 1e-3]
        elif kind < 9:
            wide = [0.9, 1.5, 3.0]
        else:
            wide = [0.5, float("nan")]
        narrow = _converging(int(g.integers(2, 10)), floor=float(g.choice([3e-7, 5e-5])))
        rec = None
        if g.uniform() < 0.5:
            rec = (int(g.integers(0, 20)), int(g.choice([OK, STAGNATED, ERR_DIVERGED])),
                   float(g.choice([1e-5, 1e-3, 2.0])))
        reqs.append(Req(i, n, int(g.integers(0, 4)), float(g.choice([1e-4, 1e-8, 1e-12])),
                        max_iter=int(g.integers(1, 40)), arrival=int(g.integers(0, 400)),
                        den=float(g.choice([1.0, 1.0, 1.0, 0.0, -1.0, float("inf")])),
                        narrow=narrow, wide=wide, rec=rec))
    out = run(harness, reqs, depth=int(g.integers(1, 4)), max_active=40, pool=600 << 20,
              batch_max_n=64)
    assert len(out["req"]) == 2000
    assert all(r["status"] != 99 for r in out["req"].values())  # every request retired
