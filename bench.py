"""Benchmark of the NN inversion on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 8192] [--no-cpu] [--no-extras]

A step is one whole inversion through the C ABI: start-iterate prologue, then
nests of d + 1 GEMMs until rms = ||I - A X||_F / sqrt(N) < tol.  The headline
workload is a dense SPD A of size 8192 in FP64, spectrum log-uniform in
[1, 1e3] (cond 1e3), depth 2, transpose start, tol 1e-12.  Inputs are
synthetic and seeded, resident in HBM before the timed region.

The JSON line carries the whole-job rate (inverses/s), the GEMM roofline
(average GEMM launch duration from HIP events recorded by the library on its
stream during the timed steps, against the FP64 MFMA peak), the oracle timed
on the host on a bounded sample, and extra workloads under "extra".
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
    return ap.parse_args()


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


def cpu_baseline(A_h, depth, iters):
    """The oracle as it stands, timed on one nest of the full problem and
    scaled to iters nests plus the final residual."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max((p.get("num_threads", 1) for p in threadpool_info()), default=os.cpu_count())
    except Exception:
        threads = os.cpu_count()
    _, X0 = oracle.initial_guess(A_h, oracle.X0_TRANSPOSE)
    t0 = time.perf_counter()
    R = oracle.residual(A_h, X0)
    t1 = time.perf_counter()
    X1 = oracle.nn_step(X0, R, depth)
    t2 = time.perf_counter()
    del X1, R
    t_res, t_nest = t1 - t0, (t2 - t0)
    per_inverse = iters * t_nest + t_res
    return {"value": 1.0 / per_inverse, "unit": "inverses/s", "cores": int(threads),
            "kind": "oracle",
            "sample": (f"one nest ({depth + 1} products, {t_nest:.2f} s) of the N={A_h.shape[0]} FP64 "
                       f"oracle on the host, scaled to {iters} nests + final residual "
                       f"({per_inverse:.1f} s per inverse)")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU: --gpus must be 1; "
                                   "more GPUs are not supported"}))
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2212_02406_amd import nn, workloads

    n, d = args.n, args.depth
    log(f"generating dense SPD n={n} (cond 1e3, log-uniform spectrum, seed 2)")
    A_h, lam, Q = workloads.dense_spd(n, 1.0, 1e3, 2, log_spectrum=True,
                                      device="cuda" if n >= 2048 else None, return_factors=True)
    A = torch.from_numpy(A_h).to("cuda:0")
    torch.cuda.synchronize()
    log("input resident in HBM")

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
        "roofline": {"bound": "mfma", "kernel": "gemm_kernel<double,128,128,8,2,4,2,2,false>",
                     "achieved": achieved, "peak": PEAK_TFLOPS["f64"], "unit": "TFLOP/s",
                     "frac": achieved / PEAK_TFLOPS["f64"], "traffic": None,
                     "per_launch_flop": flop_gemm, "avg_launch_ms": avg_gemm_s * 1e3},
    }

    extra = {}
    if not args.no_extras:
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
    out["extra"] = extra

    if not args.no_cpu:
        log("timing the oracle on the host (one nest)")
        out["cpu_baseline"] = cpu_baseline(A_h, d, info["iters"])
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
