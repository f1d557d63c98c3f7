"""Benchmark of the NN inversion on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu]
                    [--no-extras | --legs small,fp32,factorized,cns,starts,sparse,batched,mixed,serving]

A step is one whole inversion through the C ABI: start-iterate prologue, then
nests of d + 1 GEMMs until rms = ||I - A X||_F / sqrt(N) < tol.  The headline
workload is a dense SPD A of size 8192 in FP64, spectrum log-uniform in
[1, 1e3] (cond 1e3), depth 2, transpose start, tol 1e-12.  Inputs are
synthetic and seeded, resident in HBM before the timed region.

The JSON line carries the whole-job rate (inverses/s), the GEMM roofline
(average GEMM launch duration from HIP events recorded by the library on its
stream during the timed steps, against the FP64 MFMA peak; HBM traffic per
launch from the committed counter summary when it was taken on the current
GEMM source), the oracle timed on the host on a bounded sample, and under
"extra" the other workloads:
  small    dense SPD N=256 FP64 at depths 1, 2, 3 from both starts: us per
           inverse and per nest, GEMMs to 1e-12, the oracle at 1 and all
           host threads;
  fp32     the headline matrix in FP32 (runs to its rounding floor);
  batched  4096 complex64 massive-MIMO Gram matrices, one graph launch;
  mixed    N=16384 cond 1e4: BF16/FP32/FP64 schedule vs plain FP64 at the
           same tolerance;
  serving  a Poisson request stream through the continuous-batching server,
           p50/p99 latency and inverses/s, against plain FP64 one by one;
  factorized  A X = B (64 right-hand sides) on the headline matrix with the
           factorised series of Corollary 6, against nn_solve;
  cns      the same system by the Chebyshev-Neumann series (plain and mixed
           nests for the preconditioner), against nn_solve;
  starts   the other start iterates (Frobenius and power-iteration scales,
           Jacobi on a massive-MIMO Gram matrix) against the default ones;
  sparse   a 2048 x 2048 Laplacian (CSR) by the sparse series, per-term HBM
           roofline.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "inverses/s + TFLOP/s at RMS‖I−AX‖_F≤tol (plain vs mixed/batched); p50/p99"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--depth", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--legs", default="small,fp32,factorized,cns,starts,sparse,batched,mixed,serving",
                    help="comma list of extra workloads to run")
    ap.add_argument("--mixed-n", type=int, default=16384)
    ap.add_argument("--serve-pool", type=int, default=1024)
    ap.add_argument("--serve-requests", type=int, default=256,
                    help="requests of the closed-loop capacity runs")
    ap.add_argument("--serve-window", type=float, default=30.0,
                    help="seconds of each sustained Poisson stream")
    ap.add_argument("--serve-overload", type=float, default=5.0,
                    help="seconds of the 2000 req/s overload window")
    ap.add_argument("--host-input", action="store_true",
                    help="build the headline and mixed-leg matrices with host (NumPy) QR only, no GPU library "
                         "kernels before the NN launches (for counter collection)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run three plain 1 GiB device copies (untimed), the reference "
                         "kernel for scaling HBM counters")
    ap.add_argument("--batched-reps", type=int, default=50,
                    help="timed replays per start in the batched leg")
    ap.add_argument("--profile-report", nargs="+", metavar="DIR",
                    help="no GPU work: summarise the rocprofv3 CSV output under each DIR "
                         "(kernel statistics, counter means per kernel, and the HBM traffic "
                         "per FP64 GEMM launch when FETCH_SIZE / WRITE_SIZE and the copy "
                         "calibration are present), then exit")
    return ap.parse_args()


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "gemm_f64_n8192_traffic.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_2212_02406_amd", "csrc", "nn_gemm.hip")


def traffic_per_launch(n):
    """HBM bytes per FP64 GEMM launch from the committed counter summary, or
    None when it is missing, for another size, or was taken on another
    revision of the GEMM source."""
    import hashlib
    try:
        lines = open(TRAFFIC_SUMMARY).read().splitlines()
        rec = json.loads(next(l[len("json: "):] for l in lines if l.startswith("json: ")))
        sha = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
    except (OSError, StopIteration, ValueError):
        return None
    if rec.get("gemm_source_sha256") != sha or rec.get("n") != n:
        return None
    return rec["hbm_bytes_per_launch"]


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def profile_report(dirs, n=8192):
    """Print a summary of rocprofv3 output (--kernel-trace --stats and --pmc
    runs with --output-format csv) found under dirs."""
    import glob
    import hashlib
    stats, counters = [], {}
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
            stats += _csv_rows(path)
        for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"),
                                     recursive=True)):
            per = {}  # (kernel, dispatch, counter) -> summed value
            for r in _csv_rows(path):
                key = (r["Kernel_Name"], r.get("Dispatch_Id", r.get("Correlation_Id", "")),
                       r["Counter_Name"])
                per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
            for (k, _, c), v in per.items():
                counters.setdefault(k, {}).setdefault(c, []).append(v)
    if stats:
        print("kernel statistics (rocprofv3 --stats): calls, average / min / max duration")
        for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"])):
            print(f"  {int(r['Calls']):7d}  avg {float(r['AverageNs']) / 1e3:11.2f} us  "
                  f"min {float(r['MinNs']) / 1e3:11.2f}  max {float(r['MaxNs']) / 1e3:11.2f}  "
                  f"{float(r['Percentage']):5.1f}%  {r['Name'][:150]}")
    # the same launches by grid size (one kernel runs at several sizes in a run)
    by_grid = {}
    for d in dirs:
        for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
            for r in _csv_rows(path):
                g = r.get("Grid_Size") or r.get("Grid_Size_X")
                w = r.get("Workgroup_Size") or r.get("Workgroup_Size_X")
                dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e6  # ms
                by_grid.setdefault((r["Kernel_Name"], g, w), []).append(dur)
    if by_grid:
        tot = sum(sum(v) for v in by_grid.values())
        print("launches by grid size (ms): kernel | grid (threads) | workgroup | calls | total | "
              "avg | min | max")
        for (k, g, w), v in sorted(by_grid.items(), key=lambda kv: -sum(kv[1]))[:20]:
            if sum(v) < 0.001 * tot:
                break
            print(f"  {k[:110]} | {g} | {w} | {len(v)} | {sum(v):.3f} | {sum(v) / len(v):.4f} | "
                  f"{min(v):.4f} | {max(v):.4f}")
    for k, cs in counters.items():
        print(f"counters per dispatch: {k[:150]}")
        for c, vals in sorted(cs.items()):
            print(f"  {c:32s} dispatches {len(vals):4d}  mean {sum(vals) / len(vals):16.1f}  "
                  f"min {min(vals):16.1f}")
    # HBM traffic of the FP64 GEMM, each counter scaled by its reading for a
    # plain 1 GiB device copy (1 GiB read and 1 GiB written)
    copy = [k for k in counters if "copyBuffer" in k]
    gemm = [k for k in counters if k.startswith("void nn::(anonymous namespace)::gemm_kernel<double")]
    if copy and gemm:
        cc, gc = counters[copy[0]], counters[gemm[0]]
        if all(c in cc and c in gc for c in ("FETCH_SIZE", "WRITE_SIZE")):
            kib = 1024.0 * 1024.0
            big = lambda v: [x for x in v if x > 0.25 * kib]  # noqa: E731  (the 1 GiB copies)
            f_copy = sum(big(cc["FETCH_SIZE"])) / max(len(big(cc["FETCH_SIZE"])), 1)
            w_copy = sum(big(cc["WRITE_SIZE"])) / max(len(big(cc["WRITE_SIZE"])), 1)
            sf, sw = kib / f_copy, kib / w_copy
            f = sum(gc["FETCH_SIZE"]) / len(gc["FETCH_SIZE"])
            w = sum(gc["WRITE_SIZE"]) / len(gc["WRITE_SIZE"])
            hbm = (f * sf + w * sw) * 1024.0
            alg = 3 * 8 * n * n
            sha = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
            rec = {"kernel": gemm[0][len("void nn::(anonymous namespace)::"):].split("(")[0],
                   "n": n, "launches": len(gc["FETCH_SIZE"]), "fetch_kib_per_launch_raw": f,
                   "write_kib_per_launch_raw": w, "copy_scale_fetch": sf, "copy_scale_write": sw,
                   "hbm_bytes_per_launch": hbm, "algorithmic_bytes_per_launch": alg,
                   "traffic_over_algorithmic": hbm / alg, "gemm_source_sha256": sha}
            print(f"FP64 GEMM HBM traffic per launch: {hbm / 1e9:.3f} GB (FETCH_SIZE x {sf:.4f} + "
                  f"WRITE_SIZE x {sw:.4f}), algorithmic {alg / 1e9:.3f} GB, ratio {hbm / alg:.2f}")
            print("json: " + json.dumps(rec))


def time_inversions(nn, torch, A, steps, warmup, **kw):
    """Warm up, then time `steps` inversions with GEMM event timing on."""
    n = A.shape[0]
    X = torch.empty_like(A)
    prm = nn.make_params(**{k: v for k, v in kw.items()})
    import ctypes
    need = nn.nn_workspace_size(n, nn.dtype_code(A), ctypes.byref(prm))
    ws = nn.workspace(need, A.device)
    info = None
    for i in range(warmup):
        X, info = nn.invert(A, X=X, ws=ws, **kw)
        log(f"warmup {i + 1}/{warmup}: status={info['status']} iters={info['iters']} "
            f"rms={info['rms']:.3e} device_ms={info['device_ms']:.1f}")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(steps):
        X, info = nn.invert(A, X=X, ws=ws, flags=nn.NN_FLAG_TIME_GEMMS, **kw)
        infos.append(info)
        log(f"step {i + 1}/{steps}: status={info['status']} iters={info['iters']} "
            f"rms={info['rms']:.3e} device_ms={info['device_ms']:.1f}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return X, infos, t1 - t0


def sampled_check(A_h, X_h, lam, Q, cols):
    """Columns of X against the known inverse Q diag(1/lam) Q^T, and the
    residual columns e_j - A x_j, in FP64 on the host."""
    import numpy as np
    errs, res = [], []
    for j in cols:
        xt = Q @ (Q[j, :] / lam)
        errs.append(float(np.linalg.norm(X_h[:, j] - xt) / np.linalg.norm(xt)))
        e = -A_h @ X_h[:, j]
        e[j] += 1.0
        res.append(float(np.linalg.norm(e)))
    return max(errs), max(res)


def host_cpu():
    """(model name, logical CPUs, BLAS threads) of the host the oracle runs on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=os.cpu_count())
    except Exception:
        threads = os.cpu_count()
    return model, os.cpu_count(), int(threads)


def cpu_baseline(A_h, depth, tol, gpu_iters):
    """The oracle as it stands, run once in full on the headline problem: the
    transpose start, then nests to rms < tol with every residual (NumPy FP64,
    OpenBLAS on all host cores)."""
    import oracle
    model, ncpu, threads = host_cpu()
    t0 = time.perf_counter()
    _, info = oracle.nn_ref(A_h, d=depth, x0=oracle.X0_TRANSPOSE, tol=tol, max_iter=100)
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "inverses/s", "cores": threads, "kind": "oracle",
            "sample": (f"one full run of the N={A_h.shape[0]} FP64 oracle to rms < {tol:g}: "
                       f"{info['iters']} nests (GPU: {gpu_iters}), status {info['status']}, "
                       f"final rms {info['rms']:.3e}, {t:.1f} s; host '{model}', {ncpu} logical "
                       f"CPUs, BLAS threads {threads}"),
            "host_cpu_model": model, "seconds": t, "iters": info["iters"]}


def leg_small(nn, torch, workloads, np, n=256, reps=200, oracle_reps=5):
    """The small single-matrix workload: dense SPD N=256, spectrum uniform in
    [1, 100] (seed 1), FP64, depths 1, 2, 3, from the transpose start and
    from I / Tr A, each to rms < 1e-12.  Per (depth, start): microseconds per
    inverse through nn_invert's tolerance mode (one host read per nest) and,
    where the device-stop mode exists, with the stopping rules on the device;
    microseconds per nest from two fixed-nest runs (no host reads); GEMMs to
    the tolerance, the measured form of the optimal-depth comparison
    (Appendix 6); the GEMM launch time against the FP64 MFMA peak; and the
    oracle on the host at one BLAS thread and at all of them."""
    import oracle
    A_h = workloads.dense_spd(n, 1.0, 100.0, 1)
    A = torch.from_numpy(A_h).cuda()
    X = torch.empty_like(A)
    out = {"workload": (f"dense SPD N={n} FP64, spectrum uniform [1,100] (seed 1), tol rms 1e-12; "
                        f"GPU: mean of {reps} inversions; oracle: mean of {oracle_reps}")}
    flop = 2.0 * n ** 3
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    dev_stop = getattr(nn, "NN_FLAG_DEVICE_STOP", None)

    def per_inverse(**kw):
        for _ in range(5):
            nn.invert(A, X=X, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            _, info = nn.invert(A, X=X, **kw)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e6, info

    for x0 in ("transpose", "identity"):
        for d in (1, 2, 3):
            kw = dict(depth=d, x0=x0, tol=1e-12, max_iter=100)
            us, info = per_inverse(**kw)
            rec = {"us_per_inverse": us, "inverses_per_s": 1e6 / us, "nests": info["iters"],
                   "gemms": info["gemms"], "rms": info["rms"], "status": info["status"],
                   "flop_to_tol": info["gemms"] * flop}
            if dev_stop is not None:
                us_d, info_d = per_inverse(flags=dev_stop, **kw)
                rec.update(us_per_inverse_device_stop=us_d, device_stop_nests=info_d["iters"],
                           device_stop_status=info_d["status"],
                           device_stop_rms=info_d["rms"])
            # per nest: two fixed-nest runs, no host reads in between
            f = {}
            for k in (2, 12):
                for _ in range(3):
                    nn.invert(A, X=X, depth=d, x0=x0, fixed_iter=k)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps // 4):
                    nn.invert(A, X=X, depth=d, x0=x0, fixed_iter=k)
                torch.cuda.synchronize()
                f[k] = (time.perf_counter() - t0) / (reps // 4) * 1e6
            rec["us_per_nest_fixed"] = (f[12] - f[2]) / 10.0
            # GEMM launch time from HIP events on the library's stream
            _, it = nn.invert(A, X=X, flags=nn.NN_FLAG_TIME_GEMMS, **kw)
            g_us = it["gemm_ms"] * 1e3 / it["gemms"]
            rec["gemm_us_per_launch"] = g_us
            rec["gemm_frac_fp64_mfma_peak"] = flop / (g_us * 1e-6) / 1e12 / PEAK_TFLOPS["f64"]
            rec["whole_job_frac_fp64_mfma_peak"] = (rec["flop_to_tol"] / (us * 1e-6) / 1e12 /
                                                    PEAK_TFLOPS["f64"])
            # the oracle on the host, one BLAS thread and all of them
            xo = oracle.X0_TRANSPOSE if x0 == "transpose" else oracle.X0_SCALED_IDENTITY
            for label, lim in (("oracle_1_thread", 1), ("oracle_all_threads", None)):
                ctxm = threadpool_limits(lim) if (threadpool_limits and lim) else None
                try:
                    if ctxm is not None:
                        ctxm.__enter__()
                    t0 = time.perf_counter()
                    for _ in range(oracle_reps):
                        _, io = oracle.nn_ref(A_h, d=d, x0=xo, tol=1e-12, max_iter=100)
                    t = (time.perf_counter() - t0) / oracle_reps
                finally:
                    if ctxm is not None:
                        ctxm.__exit__(None, None, None)
                rec[label] = {"us_per_inverse": t * 1e6, "nests": io["iters"]}
            out[f"{x0}_d{d}"] = rec
            log(f"small N={n} {x0} d={d}: {rec}")
    for x0 in ("transpose", "identity"):
        g = {d: out[f"{x0}_d{d}"]["gemms"] for d in (1, 2, 3)}
        out[f"{x0}_fewest_gemms_depth"] = min(g, key=lambda d: (g[d], d))
    _, cpu_n, threads = host_cpu()
    out["host_threads"] = threads
    return out


def leg_batched(nn, torch, workloads, np, reps=50):
    """4096 massive-MIMO Gram matrices G = H^H H + 0.1 I (H 128 x K, K in
    {8,16,32,64}), complex64, depth 2, 4 fixed nests, one graph launch."""
    packed, offsets, sizes, mats = workloads.mimo_gram_batch(batch=4096, seed=3)
    P = torch.from_numpy(packed).cuda()
    O = torch.from_numpy(offsets).cuda()
    S = torch.from_numpy(sizes).cuda()
    best_ms, wk, wg = nn.batched_autotune(P, O, S, 64, fixed_iter=4)
    log(f"batched autotune: best {best_ms:.3f} ms wave_max_k={wk} wg_per_cu={wg}")
    X = torch.empty_like(P)
    info = torch.empty(4096 * 16, dtype=torch.uint8, device="cuda")
    hold = nn.workspace(nn.nn_batched_workspace_size(4096, nn.NN_C64), P.device)
    out = {}
    for x0 in ("transpose", "identity"):
        for _ in range(3):
            nn.invert_batched(P, O, S, 64, x0=x0, fixed_iter=4, X=X, info=info, ws=hold)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            nn.invert_batched(P, O, S, 64, x0=x0, fixed_iter=4, X=X, info=info, ws=hold)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / reps
        it, st, rms = nn.decode_batched_info(info)
        K = sizes.astype(np.float64)
        flop = float(np.sum((4 * 3 + 1) * 8.0 * K ** 3))  # (k(d+1)+1) complex products
        byts = float(np.sum(2 * 8.0 * K ** 2))  # read A, write X (complex64)
        rms_by_k = {int(k): float(np.median(rms[sizes == k])) for k in (8, 16, 32, 64)}
        out[x0] = {"ms_per_batch": ms, "inverses_per_s": 4096 / (ms / 1e3),
                   "tflops": flop / (ms / 1e3) / 1e12, "gb_per_s": byts / (ms / 1e3) / 1e9,
                   "frac_fp32_mfma_peak": flop / (ms / 1e3) / 1e12 / PEAK_TFLOPS["f32"],
                   "frac_hbm_peak": byts / (ms / 1e3) / 1e9 / 8000.0,
                   "all_ok": bool(np.all(st == 0)), "median_rms_by_K": rms_by_k}
        log(f"batched {x0}: {out[x0]}")
    # the same matrices one by one through plain FP64 (complex128) nn_invert,
    # 4 fixed nests each: every 16th matrix of the batch, scaled to the batch
    sample = list(range(0, 4096, 16))
    wide = [torch.from_numpy(mats[b].astype(np.complex128)).cuda() for b in sample]
    for Mt in wide[:4]:
        nn.invert(Mt, depth=2, x0="transpose", fixed_iter=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for Mt in wide:
        nn.invert(Mt, depth=2, x0="transpose", fixed_iter=4)
    torch.cuda.synchronize()
    per = (time.perf_counter() - t0) / len(sample)
    out["plain_fp64_one_by_one"] = {"s_per_matrix": per, "inverses_per_s": 1.0 / per,
                                    "sample": f"{len(sample)} matrices (every 16th)"}
    out["batched_vs_plain_fp64"] = out["transpose"]["inverses_per_s"] * per
    log(f"batched vs plain fp64 one by one: {out['batched_vs_plain_fp64']:.0f}x")
    out["autotune"] = {"best_ms": best_ms, "wave_max_k": wk, "wg_per_cu": wg}
    out["workload"] = ("4096 complex64 MIMO Gram matrices, M=128, K uniform in {8,16,32,64}, "
                       "sigma2=0.1, depth 2, 4 fixed nests, seed 3")
    return out


def leg_mixed(nn, torch, workloads, np, n, host_input=False):
    """Dense SPD N=16384, cond 1e4 (log-uniform spectrum), depth 2, tol 1e-11:
    mixed BF16/FP32/FP64 schedule vs plain FP64, each from the scaled
    identity start I / Tr A and from Theta_2(8) I."""
    A_h, lam, Q = workloads.dense_spd(n, 1.0, 1e4, 4, log_spectrum=True,
                                      device=None if host_input else "cuda",
                                      return_factors=True)
    A = torch.from_numpy(A_h).cuda()
    torch.cuda.synchronize()
    res = {}
    Xs = {}
    runs = (("mixed", dict(prec="mixed", x0="identity")),
            ("plain_fp64", dict(prec="plain", x0="identity")),
            ("mixed_power_identity", dict(prec="mixed", x0="power_identity")),
            ("plain_fp64_power_identity", dict(prec="plain", x0="power_identity")))
    for label, kw in runs:
        X, info = nn.invert(A, depth=2, tol=1e-11, max_iter=100, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = nn.invert(A, depth=2, tol=1e-11, max_iter=100, X=X, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        Xs[label] = X
        ph = info["phase_iters"]
        flop = 2.0 * n ** 3 * info["gemms"]
        # every product against the peak of the arithmetic it ran in, with the
        # per-precision counts the library reports (BF16, FP32, FP64)
        pg = info["prec_gemms"]
        assert sum(pg) == info["gemms"], (pg, info["gemms"])
        per = 2.0 * n ** 3
        ideal = per * (pg[0] / PEAK_TFLOPS["bf16"] + pg[1] / PEAK_TFLOPS["f32"] +
                       pg[2] / PEAK_TFLOPS["f64"]) / 1e12
        res[label] = {"s": t, "inverses_per_s": 1.0 / t, "status": info["status"],
                      "iters": info["iters"], "phase_iters_bf16_fp32_fp64": ph,
                      "gemms_bf16_fp32_fp64": pg, "device_ms": info["device_ms"],
                      "rms": info["rms"], "gemms": info["gemms"],
                      "tflops": flop / t / 1e12, "roofline_frac_phase_weighted": ideal / t}
        log(f"mixed leg {label}: {res[label]}")
    diff = (torch.linalg.norm(Xs["mixed"] - Xs["plain_fp64"]) /
            torch.linalg.norm(Xs["plain_fp64"])).item()
    X_h = Xs["mixed"].cpu().numpy()
    cols = list(np.random.default_rng(1).choice(n, 4, replace=False))
    err, resid = sampled_check(A_h, X_h, lam, Q, cols)
    res["speedup_vs_plain_fp64"] = res["plain_fp64"]["s"] / res["mixed"]["s"]
    res["speedup_power_identity_vs_plain_fp64_same_start"] = (
        res["plain_fp64_power_identity"]["s"] / res["mixed_power_identity"]["s"])
    res["speedup_mixed_power_identity_vs_plain_fp64_identity"] = (
        res["plain_fp64"]["s"] / res["mixed_power_identity"]["s"])
    res["rel_fro_diff_mixed_power_identity_vs_plain_fp64"] = (
        torch.linalg.norm(Xs["mixed_power_identity"] - Xs["plain_fp64"]) /
        torch.linalg.norm(Xs["plain_fp64"])).item()
    res["rel_fro_diff_mixed_vs_plain_fp64"] = diff
    res["mixed_sampled_rel_err_vs_exact_inverse_col"] = err
    res["workload"] = (f"dense SPD N={n}, spectrum log-uniform [1,1e4] (cond 1e4), depth 2, "
                       "scaled identity start (and Theta_2(8) I), tol rms 1e-11, seed 4")
    return res


def leg_factorized(nn, torch, workloads, np, A, n):
    """A X = B for the headline matrix and 64 right-hand sides: the
    factorised series of Corollary 6 applied to B (relative residual 1e-7,
    above its FP64 floor of ~3e-8 on this matrix) against nn_solve (the NN
    inverse to rms 1e-8, then X B), both from the transpose start."""
    B = torch.from_numpy(workloads.rng(9).standard_normal((n, 64))).cuda()
    out = {}
    for label, fn in (("factorized", lambda: nn.solve_factorized(A, B, x0="transpose", tol=1e-7)),
                      ("nn_solve", lambda: nn.solve(A, B, depth=2, x0="transpose", tol=1e-8))):
        X, info = fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = fn()
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        out[label] = {"s": t, "solves_per_s": 1.0 / t, "status": info["status"],
                      "iters": info["iters"], "gemms": info["gemms"],
                      "rel_residual": info["rel_residual"]}
        log(f"factorized leg {label}: {out[label]}")
    out["speedup_vs_nn_solve"] = out["nn_solve"]["s"] / out["factorized"]["s"]
    out["workload"] = (f"dense SPD N={n} FP64 cond 1e3 (the headline matrix), 64 right-hand "
                       "sides N(0,1) seed 9, transpose start")
    return out


def leg_cns(nn, torch, workloads, np, A, n):
    """A X = B for the headline matrix and 64 right-hand sides by the
    Chebyshev-Neumann series (NN nests for phi, then the series in I - phi A
    applied to B, in refinement form) against nn_solve, all to FP64
    accuracy: CNS to relative residual 1e-12; nn_solve with the inverse to
    rms 1e-12.  Variants: plain FP64 nests (transpose start, phi to rms
    1e-2); mixed BF16/FP32 nests (identity start, phi to rms 1e-2); and a
    second right-hand-side batch against the kept phi (reuse)."""
    B = torch.from_numpy(workloads.rng(9).standard_normal((n, 64))).cuda()
    B2 = torch.from_numpy(workloads.rng(10).standard_normal((n, 64))).cuda()
    out = {}

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = fn()
        torch.cuda.synchronize()
        return X, info, time.perf_counter() - t0

    runs = (("cns_plain", lambda: nn.solve_cns(A, B, x0="transpose", precond_tol=1e-2, tol=1e-12)),
            ("cns_mixed", lambda: nn.solve_cns(A, B, x0="identity", precond_tol=1e-2,
                                               prec="mixed", tol=1e-12)),
            ("nn_solve", lambda: nn.solve(A, B, depth=2, x0="transpose", tol=1e-12)))
    for label, fn in runs:
        fn()
        X, info, t = timed(fn)
        rec = {"s": t, "solves_per_s": 1.0 / t, "status": info["status"],
               "rel_residual": info["rel_residual"], "gemms": info["gemms"]}
        if "precond" in info:
            p = info["precond"]
            rec.update(terms=info["iters"], nests=p["iters"], precond_rms=p["rms"],
                       precond_phase_iters=p["phase_iters"], precond_gemms=p["gemms"],
                       series_device_ms=info["device_ms"], precond_device_ms=p["device_ms"])
            if label == "cns_mixed":
                ws = info["ws"]
                _, i2, t2 = timed(lambda: nn.solve_cns(A, B2, x0="identity", precond_tol=1e-2,
                                                       prec="mixed", tol=1e-12, ws=ws,
                                                       reuse_phi=True))
                out["cns_reuse_phi"] = {"s": t2, "solves_per_s": 1.0 / t2,
                                        "status": i2["status"], "terms": i2["iters"],
                                        "rel_residual": i2["rel_residual"]}
                log(f"cns leg cns_reuse_phi: {out['cns_reuse_phi']}")
        else:
            rec["nests"] = info["iters"]
        out[label] = rec
        log(f"cns leg {label}: {rec}")
    for label in ("cns_plain", "cns_mixed"):
        out[f"speedup_{label}_vs_nn_solve"] = out["nn_solve"]["s"] / out[label]["s"]
    out["workload"] = (f"dense SPD N={n} FP64 cond 1e3 (the headline matrix), 64 right-hand "
                       "sides N(0,1) seeds 9 and 10")
    return out


def leg_starts(nn, torch, workloads, np, A, n):
    """The other normalisations (start iterates) on the headline matrix, each
    to rms 1e-12: the ||A||_1 ||A||_inf and ||A||_F^2 transpose scales,
    Theta_2(8) A^H (power iteration on A A^H), I / Tr A and Theta_2(8) I.
    Then a massive-MIMO Gram matrix (1024 users, 8192 antennas, complex128,
    sigma^2 0.1) with the Jacobi start diag(G)^-1 against I / Tr G and
    Theta_2(8) I."""
    def run(M, x0, **kw):
        nn.invert(M, x0=x0, tol=1e-12, max_iter=100, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info = nn.invert(M, x0=x0, tol=1e-12, max_iter=100, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        return {"s": t, "inverses_per_s": 1.0 / t, "nests": info["iters"], "gemms": info["gemms"],
                "rms": info["rms"], "status": info["status"]}

    out = {"headline": {}, "mimo_gram": {}}
    for x0, kw in (("transpose", {}), ("transpose_frob", {}), ("power_transpose", {"power_k": 8}),
                   ("identity", {}), ("power_identity", {"power_k": 8})):
        out["headline"][x0] = run(A, x0, **kw)
        log(f"starts leg headline {x0}: {out['headline'][x0]}")
    G = torch.from_numpy(workloads.mimo_gram(8192, 1024, 11)).cuda()
    for x0, kw in (("identity", {}), ("power_identity", {"power_k": 8}), ("jacobi", {})):
        out["mimo_gram"][x0] = run(G, x0, **kw)
        log(f"starts leg mimo_gram {x0}: {out['mimo_gram'][x0]}")
    out["workload"] = (f"headline: dense SPD N={n} FP64 cond 1e3 seed 2, d=2, tol rms 1e-12; "
                       "mimo_gram: G = H^H H + 0.1 I, H 8192 x 1024 CN(0,1) seed 11, complex128")
    return out


def leg_sparse(nn, torch, workloads, np, grid=2048, nrhs=16, shift=0.5):
    """W X = B for the 5-point Laplacian on a grid x grid mesh + shift I
    (CSR, FP64; cond (8 + shift) / shift) and nrhs right-hand sides N(0,1)
    by the sparse series (Algorithm 2, Horner form on the device) with the
    Jacobi start, to control residual 1e-10.  The per-term time is the
    difference of two fixed-term runs; its bytes are the algorithmic ones:
    the CSR arrays, phi and its weights, x and B read once, x' written."""
    ip, ix, v = workloads.laplacian_2d(grid, grid, shift)
    n = grid * grid
    nnz = int(ix.size)
    B = workloads.rng(12).standard_normal((n, nrhs))
    ipd, ixd, vd = (torch.from_numpy(a).cuda() for a in (ip, ix, v))
    Bd = torch.from_numpy(B).cuda()
    torch.cuda.synchronize()

    def timed(**kw):
        nn.solve_sparse(ipd, ixd, vd, Bd, x0="jacobi", **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X, info = nn.solve_sparse(ipd, ixd, vd, Bd, x0="jacobi", **kw)
        torch.cuda.synchronize()
        return X, info, time.perf_counter() - t0

    X, info, t = timed(tol=1e-10, check_every=64)
    _, i1, t1 = timed(fixed_terms=50)
    _, i2, t2 = timed(fixed_terms=550)
    per_term = (i2["device_ms"] - i1["device_ms"]) / 500.0 / 1e3
    bytes_term = nnz * (8 + 4) + (n + 1) * 4 + 2 * n * 8 + 3 * n * nrhs * 8
    achieved = bytes_term / per_term / 1e9
    out = {"s": t, "solves_per_s": 1.0 / t, "status": info["status"], "terms": info["iters"],
           "control_residual": info["rms"], "rel_residual": info["rel_residual"],
           "per_term_ms": per_term * 1e3, "algorithmic_bytes_per_term": bytes_term,
           "roofline": {"bound": "hbm", "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                        "frac": achieved / 8000.0},
           "workload": (f"5-point Laplacian {grid}x{grid} + {shift} I (n={n}, nnz={nnz}), FP64, "
                        f"{nrhs} right-hand sides N(0,1) seed 12, Jacobi start, tol 1e-10")}
    log(f"sparse leg: {out}")
    return out


def leg_serving(nn, torch, workloads, np, pool_size, n_req, window_s=30.0, overload_s=5.0):
    """The serving workload over a pool of FP32 SPD / complex64 HPD matrices,
    N log-uniform in [32, 4096], cond log-uniform in [10, 1e4], tol 1e-4 or
    1e-8: closed-loop capacity on n_req requests; sustained Poisson streams
    of window_s seconds at 0.5 and 0.9 of that capacity (every arrival served
    to the end); a bounded overload window of overload_s seconds at the
    2000 req/s of the workload's definition (queue length over time, the rate
    served; unfinished requests are dropped at the window's end); and the
    capacity requests one by one through plain FP64 nn_invert.  Requests are
    drawn uniformly from the pool; latency is arrival to result in host
    memory."""
    t_build = time.perf_counter()
    pool = workloads.serving_pool(pool_size, seed=5)
    mats = []
    for e in pool:
        mats.append(torch.from_numpy(workloads.build_request(
            e, device="cuda" if e["n"] >= 512 else None)).cuda())
    torch.cuda.synchronize()
    log(f"serving pool of {pool_size} built in {time.perf_counter() - t_build:.1f} s")
    g = workloads.rng(55)
    d = 2

    def flop_of(entry, iters):
        f = (iters * (d + 1) + 1) * 2.0 * entry["n"] ** 3
        return f * (4 if entry["complex"] else 1)

    def run(arrivals, picks, x0="power_identity", stop_s=None):
        """Serve requests i = 0.. arriving at arrivals[i] (seconds) with pool
        entry picks[i].  stop_s: stop at that time (overload), else drain."""
        n_req = len(picks)
        srv = nn.Server(96 << 30, depth=d, x0=x0, max_active=512, n_streams=4)
        srv.submit(-1, mats[0], 1e-4)
        srv.run_until_idle()
        srv.release(-1)
        t0 = time.perf_counter()
        nxt, lat, recs, queue = 0, {}, [], []
        next_sample = 0.0
        while len(lat) < n_req:
            now = time.perf_counter() - t0
            if stop_s is not None and now >= stop_s:
                break
            while nxt < n_req and arrivals[nxt] <= now:
                e = pool[picks[nxt]]
                srv.submit(nxt, mats[picks[nxt]], e["tol"], 100)
                nxt += 1
            s = srv.tick()
            for r in srv.poll():
                if r["status"] >= 0:
                    srv.fetch(r["id"], r["n"], r["out_dtype"], out_device="cpu")
                else:
                    srv.release(r["id"])
                lat[r["id"]] = time.perf_counter() - t0 - arrivals[r["id"]]
                recs.append(r)
            now = time.perf_counter() - t0
            if now >= next_sample:
                queue.append([round(now, 2), int(s.queued), int(s.active), len(lat), nxt])
                next_sample += 1.0 if stop_s is None else 0.5
            if s.active == 0 and s.queued == 0 and nxt < n_req:
                time.sleep(max(0.0, min(arrivals[nxt] - (time.perf_counter() - t0), 1e-3)))
        wall = time.perf_counter() - t0
        srv.close()
        L = np.array(list(lat.values())) if lat else np.zeros(1)
        ok = sum(1 for r in recs if r["status"] == 0)
        return {"requests_arrived": nxt, "requests_done": len(lat), "wall_s": wall,
                "inverses_per_s": len(lat) / wall,
                "p50_ms": 1e3 * float(np.percentile(L, 50)),
                "p99_ms": 1e3 * float(np.percentile(L, 99)),
                "tflops": sum(flop_of(pool[picks[r["id"]]], r["iters"]) for r in recs) / wall / 1e12,
                "ok": ok, "promoted_to_fp64": sum(1 for r in recs if r["wide_iters"] > 0),
                "max_rms_over_tol_ok": max([r["rms"] / pool[picks[r["id"]]]["tol"] for r in recs
                                            if r["status"] == 0], default=None),
                "queue_over_time_s_queued_active_done_arrived": queue}

    out = {}
    cap_picks = g.integers(0, pool_size, n_req)
    out["capacity_closed_loop"] = run(np.zeros(n_req), cap_picks)
    cap = out["capacity_closed_loop"]["inverses_per_s"]
    log(f"serving capacity: {cap:.1f} inverses/s")
    out["capacity_identity_start"] = run(np.zeros(n_req), cap_picks, "identity")
    log(f"serving capacity, I / Tr A start: "
        f"{out['capacity_identity_start']['inverses_per_s']:.1f} inverses/s")
    for frac in (0.5, 0.9):
        rate = frac * cap
        m = int(rate * window_s * 1.5) + 16
        arr = np.cumsum(g.exponential(1.0 / rate, m))
        arr = arr[arr < window_s]
        picks = g.integers(0, pool_size, arr.size)
        rec = run(arr, picks)
        rec.update(offered_req_per_s=rate, window_s=window_s, frac_of_capacity=frac)
        out[f"stream_{frac:g}x_capacity"] = rec
        log(f"serving stream {frac:g}x capacity ({rate:.1f} req/s, {arr.size} requests over "
            f"{window_s:g} s): p50 {rec['p50_ms']:.1f} ms, p99 {rec['p99_ms']:.1f} ms, "
            f"{rec['inverses_per_s']:.1f} inverses/s")
    rate = 2000.0
    arr = np.cumsum(g.exponential(1.0 / rate, int(rate * overload_s * 1.5)))
    arr = arr[arr < overload_s]
    picks = g.integers(0, pool_size, arr.size)
    rec = run(arr, picks, stop_s=overload_s)
    rec.update(offered_req_per_s=rate, window_s=overload_s,
               note=("overload: the offered rate exceeds capacity; the window stops at "
                     f"{overload_s:g} s and unfinished requests are dropped, so p50/p99 cover "
                     "only the requests that finished inside it"))
    out["overload_2000_req_per_s"] = rec
    log(f"serving overload 2000 req/s: {rec['requests_arrived']} arrived, "
        f"{rec['requests_done']} done in {overload_s:g} s")
    # the capacity requests one by one through plain FP64 nn_invert, same start
    wide = {}
    for i in set(int(x) for x in cap_picks):
        wide[i] = mats[i].to(torch.complex128 if mats[i].is_complex() else torch.float64)
    for x0 in ("power_identity", "identity"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in cap_picks:
            nn.invert(wide[int(i)], depth=d, x0=x0, tol=pool[int(i)]["tol"], max_iter=100)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        key = "plain_fp64_sequential" + ("" if x0 == "power_identity" else "_identity_start")
        out[key] = {"wall_s": t, "inverses_per_s": n_req / t}
        log(f"serving {key}: {out[key]}")
    out["served_vs_plain_fp64"] = (out["capacity_closed_loop"]["inverses_per_s"] /
                                   out["plain_fp64_sequential"]["inverses_per_s"])
    out["workload"] = (f"pool of {pool_size} (seed 5): FP32 SPD or complex64 HPD 50/50, N "
                       "log-uniform [32,4096], cond log-uniform [10,1e4], tol 1e-4 or 1e-8 50/50; "
                       f"capacity on {n_req} requests; Poisson streams of {window_s:g} s at 0.5x "
                       f"and 0.9x capacity; {overload_s:g} s at 2000 req/s; depth 2, "
                       "Theta_2(8) I start (I / Tr A for the *_identity_start entries); latency "
                       "= arrival to result in host memory")
    return out


def main():
    args = parse()
    if args.profile_report:
        profile_report(args.profile_report, args.n)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU: --gpus must be 1; "
                                   "more GPUs are not supported"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2212_02406_amd import nn, workloads

    n, d = args.n, args.depth
    log(f"generating dense SPD n={n} (cond 1e3, log-uniform spectrum, seed 2)")
    gen_dev = "cuda" if n >= 2048 and not args.host_input else None
    A_h, lam, Q = workloads.dense_spd(n, 1.0, 1e3, 2, log_spectrum=True, device=gen_dev,
                                      return_factors=True)
    A = torch.from_numpy(A_h).to("cuda:0")
    torch.cuda.synchronize()
    log("input resident in HBM")

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x 1 GiB device copies done")

    X, infos, secs = time_inversions(nn, torch, A, args.steps, args.warmup, depth=d,
                                     x0="transpose", tol=1e-12, max_iter=100)
    info = infos[-1]
    gemms = sum(i["gemms"] for i in infos)
    gemm_ms = sum(i["gemm_ms"] for i in infos)
    flop_gemm = 2.0 * n ** 3
    avg_gemm_s = gemm_ms / 1e3 / gemms
    achieved = flop_gemm / avg_gemm_s / 1e12
    value = args.steps / secs
    tflops = gemms * flop_gemm / secs / 1e12
    X_h = X.cpu().numpy()
    cols = list(np.random.default_rng(0).choice(n, 8, replace=False))
    err, res = sampled_check(A_h, X_h, lam, Q, cols)
    log(f"fp64: {value:.3f} inv/s, {tflops:.1f} TFLOP/s whole job, GEMM {achieved:.1f} TFLOP/s "
        f"({avg_gemm_s * 1e3:.2f} ms/launch), sampled rel err {err:.2e}")

    out = {
        "metric": METRIC, "value": value, "unit": "inverses/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"dense SPD N={n} FP64, spectrum log-uniform [1,1e3] (cond 1e3), "
                               f"depth {d}, transpose start, tol rms 1e-12, plain NN",
                   "n": n, "depth": d, "x0": "transpose", "tol": 1e-12, "seed": 2},
        "tflops": tflops, "iters": info["iters"], "rms": info["rms"], "status": info["status"],
        "gemms_per_inverse": info["gemms"],
        "check": {"sampled_cols": len(cols), "max_rel_err_vs_exact_inverse_col": err,
                  "max_residual_col_norm": res},
        "roofline": {"bound": "mfma", "kernel": "gemm_kernel<double,128,128,16,2,4,2,2,false,true>",
                     "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["f64"], "traffic": traffic_per_launch(n),
                     "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-scaled)",
                     "algorithmic_bytes_per_launch": 3 * 8 * n * n,
                     "per_launch_flop": flop_gemm, "avg_launch_ms": avg_gemm_s * 1e3},
    }

    extra = {}
    legs = set() if args.no_extras else set(args.legs.split(","))
    if "small" in legs:
        extra["small"] = leg_small(nn, torch, workloads, np)
    if "fp32" in legs:
        A32 = A.to(torch.float32)
        X32, i32, s32 = time_inversions(nn, torch, A32, 1, 1, depth=d, x0="transpose", tol=1e-6,
                                        max_iter=100)
        g32 = i32[-1]
        avg32 = g32["gemm_ms"] / 1e3 / g32["gemms"]
        extra["fp32"] = {"n": n, "inverses_per_s": 1.0 / s32, "status": g32["status"],
                         "iters": g32["iters"], "rms": g32["rms"],
                         "tflops": g32["gemms"] * flop_gemm / s32 / 1e12,
                         "gemm_tflops": flop_gemm / avg32 / 1e12,
                         "gemm_frac_of_fp32_peak": flop_gemm / avg32 / 1e12 / PEAK_TFLOPS["f32"],
                         "note": "tol 1e-6 is below the FP32 rounding floor; runs to STAGNATED"}
        log(f"fp32: {extra['fp32']}")
        del A32, X32
    if "factorized" in legs:
        extra["factorized"] = leg_factorized(nn, torch, workloads, np, A, n)
    if "cns" in legs:
        extra["cns"] = leg_cns(nn, torch, workloads, np, A, n)
        torch.cuda.empty_cache()
    if "sparse" in legs:
        extra["sparse"] = leg_sparse(nn, torch, workloads, np)
        torch.cuda.empty_cache()
    if "starts" in legs:
        extra["starts"] = leg_starts(nn, torch, workloads, np, A, n)
        torch.cuda.empty_cache()
    if legs & {"batched", "mixed", "serving"}:
        del X
        torch.cuda.empty_cache()
    if "batched" in legs:
        extra["batched"] = leg_batched(nn, torch, workloads, np, args.batched_reps)
    if "mixed" in legs:
        extra["mixed"] = leg_mixed(nn, torch, workloads, np, args.mixed_n, args.host_input)
        torch.cuda.empty_cache()
    if "serving" in legs:
        extra["serving"] = leg_serving(nn, torch, workloads, np, args.serve_pool,
                                       args.serve_requests, args.serve_window,
                                       args.serve_overload)
    out["extra"] = extra

    if not args.no_cpu:
        log("timing the oracle on the host (one full inversion)")
        out["cpu_baseline"] = cpu_baseline(A_h, d, 1e-12, info["iters"])
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
