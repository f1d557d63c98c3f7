"""ctypes binding of libnn.so (include/nn.h) — argument marshalling only.

Every step of the NN iteration runs in the HIP library.  PyTorch is used here
for device memory (tensors, workspace) and streams only.  If libnn.so has not
been built this module raises ImportError: there is no fallback path.

Low level: ``lib`` exposes the C entry points with the same names
(``nn_create``, ``nn_invert``, ``nn_solve``, ``nn_invert_batched``, ...).
High level: ``invert``, ``solve``, ``invert_batched`` take torch tensors.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("NN_LIBRARY") or os.path.join(_HERE, "libnn.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "nn.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_02406_amd.build`")

# torch first: its HIP runtime is then the one libnn.so binds to, so both
# share one runtime instance (streams, device memory).  Loading libnn.so
# first brings in a second runtime, and nn_create then fails on the device.
import torch  # noqa: E402,F401

lib = ctypes.CDLL(LIB_PATH)

# ---- enums (values from include/nn.h) --------------------------------------
NN_OK, NN_NOT_CONVERGED, NN_STAGNATED = 0, 1, 2
NN_ERR_ARG, NN_ERR_DIVERGED, NN_ERR_NONFINITE = -1, -2, -3
NN_ERR_HIP, NN_ERR_WORKSPACE, NN_ERR_UNSUPPORTED = -4, -5, -6
NN_F64, NN_F32, NN_C64, NN_C128 = 0, 1, 2, 3
NN_X0_TRANSPOSE, NN_X0_SCALED_IDENTITY, NN_X0_GIVEN = 0, 1, 2
NN_X0_TRANSPOSE_FROB, NN_X0_POWER_IDENTITY, NN_X0_POWER_TRANSPOSE, NN_X0_JACOBI = 3, 4, 5, 6
NN_POWER_MAX_K = 64
NN_PREC_PLAIN, NN_PREC_MIXED = 0, 1
NN_MAX_DEPTH = 8
NN_TRACE_MAX = 128
NN_FLAG_TIME_GEMMS = 1
NN_FLAG_DEVICE_STOP = 2
NN_NOALLOC_SCRATCH_BYTES = 32 << 20
NN_CNS_MAX_TERMS = 1000000
NN_SPARSE_MAX_TERMS = 100000000

X0_NAMES = {"transpose": NN_X0_TRANSPOSE, "identity": NN_X0_SCALED_IDENTITY,
            "scaled_identity": NN_X0_SCALED_IDENTITY, "given": NN_X0_GIVEN,
            "transpose_frob": NN_X0_TRANSPOSE_FROB, "power_identity": NN_X0_POWER_IDENTITY,
            "power_transpose": NN_X0_POWER_TRANSPOSE, "jacobi": NN_X0_JACOBI}


class nn_params(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("x0", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("fixed_iter", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("power_k", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class nn_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rms", ctypes.c_double),
                ("device_ms", ctypes.c_float), ("gemm_ms", ctypes.c_float),
                ("gemms", ctypes.c_int32),
                ("n_trace", ctypes.c_int32), ("phase_iters", ctypes.c_int32 * 3),
                ("prec_gemms", ctypes.c_int32 * 3),
                ("rms_trace", ctypes.c_double * NN_TRACE_MAX)]

    def as_dict(self):
        return {"iters": self.iters, "status": self.status, "rms": self.rms,
                "device_ms": self.device_ms, "gemm_ms": self.gemm_ms, "gemms": self.gemms,
                "phase_iters": list(self.phase_iters), "prec_gemms": list(self.prec_gemms),
                "trace": [self.rms_trace[i] for i in range(self.n_trace)]}


class nn_cns_params(ctypes.Structure):
    _fields_ = [("precond", nn_params), ("tol", ctypes.c_double), ("max_terms", ctypes.c_int32),
                ("fixed_terms", ctypes.c_int32), ("reuse_phi", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class nn_sparse_params(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_int32), ("power_k", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_terms", ctypes.c_int32), ("fixed_terms", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class nn_info_dev(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rms", ctypes.c_double)]


class nn_server_params(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("x0", ctypes.c_int32), ("max_active", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("wide_tol", ctypes.c_double),
                ("power_k", ctypes.c_int32), ("batch_max_n", ctypes.c_int32)]


class nn_request_info(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("wide_iters", ctypes.c_int32), ("out_dtype", ctypes.c_int32),
                ("n", ctypes.c_int64), ("rms", ctypes.c_double), ("t_submit", ctypes.c_double),
                ("t_admit", ctypes.c_double), ("t_finish", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class nn_server_stats(ctypes.Structure):
    _fields_ = [("finished", ctypes.c_int32), ("active", ctypes.c_int32),
                ("queued", ctypes.c_int32), ("ready", ctypes.c_int32),
                ("pool_used", ctypes.c_size_t)]


_p, _i64, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
_PP = ctypes.POINTER(nn_params)
_SIGS = {
    "nn_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, _p]),
    "nn_destroy": (None, [_p]),
    "nn_set_stream": (ctypes.c_int, [_p, _p]),
    "nn_workspace_size": (_sz, [_i64, ctypes.c_int, _PP]),
    "nn_invert": (ctypes.c_int, [_p, _p, _i64, _p, _i64, _i64, ctypes.c_int, _PP, _p, _sz,
                                 ctypes.POINTER(nn_info)]),
    "nn_invert_noalloc": (ctypes.c_int, [_p, _p, _i64, _p, _i64, _i64, ctypes.c_int, _PP,
                                         ctypes.POINTER(nn_info)]),
    "nn_solve_workspace_size": (_sz, [_i64, _i64, ctypes.c_int, _PP]),
    "nn_solve": (ctypes.c_int, [_p, _p, _i64, _p, _i64, _p, _i64, _i64, _i64, ctypes.c_int, _PP,
                                _p, _sz, ctypes.POINTER(nn_info), ctypes.POINTER(ctypes.c_double)]),
    "nn_solve_factorized_workspace_size": (_sz, [_i64, _i64, ctypes.c_int, _PP]),
    "nn_solve_factorized": (ctypes.c_int, [_p, _p, _i64, _p, _i64, _p, _i64, _i64, _i64,
                                           ctypes.c_int, _PP, _p, _sz, ctypes.POINTER(nn_info),
                                           ctypes.POINTER(ctypes.c_double)]),
    "nn_solve_cns_workspace_size": (_sz, [_i64, _i64, ctypes.c_int,
                                          ctypes.POINTER(nn_cns_params)]),
    "nn_solve_cns": (ctypes.c_int, [_p, _p, _i64, _p, _i64, _p, _i64, _i64, _i64, ctypes.c_int,
                                    ctypes.POINTER(nn_cns_params), _p, _sz,
                                    ctypes.POINTER(nn_info), ctypes.POINTER(nn_info),
                                    ctypes.POINTER(ctypes.c_double)]),
    "nn_solve_sparse_workspace_size": (_sz, [_i64, _i64, ctypes.c_int,
                                             ctypes.POINTER(nn_sparse_params)]),
    "nn_solve_sparse": (ctypes.c_int, [_p, _p, _p, _p, _i64, _i64, _p, _i64, _p, _i64, _i64,
                                       ctypes.c_int, ctypes.POINTER(nn_sparse_params), _p, _sz,
                                       ctypes.POINTER(nn_info), ctypes.POINTER(ctypes.c_double)]),
    "nn_batched_workspace_size": (_sz, [_i32, ctypes.c_int]),
    "nn_invert_batched": (ctypes.c_int, [_p, _p, _p, _p, _p, _i32, _i32, ctypes.c_int, _PP, _p,
                                         _sz, _p]),
    "nn_batched_autotune": (ctypes.c_int, [_p, _p, _p, _p, _p, _i32, _i32, ctypes.c_int, _PP, _p,
                                           _sz, ctypes.POINTER(ctypes.c_float),
                                           ctypes.POINTER(_i32)]),
    "nn_batched_fit_config": (_i32, [ctypes.c_int, _i32, _i32, _i32]),
    "nn_batched_get_config": (ctypes.c_int, [_p, ctypes.c_int, _i32, ctypes.POINTER(_i32),
                                             ctypes.POINTER(_i32)]),
    "nn_batched_set_config": (ctypes.c_int, [_p, ctypes.c_int, _i32, _i32, _i32]),
    "nn_server_create": (ctypes.c_int, [_p, _p, _sz, ctypes.POINTER(nn_server_params),
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "nn_server_destroy": (None, [_p]),
    "nn_server_footprint": (_sz, [_p, _i64, ctypes.c_int, ctypes.c_double]),
    "nn_server_submit": (ctypes.c_int, [_p, _i64, _p, _i64, _i64, ctypes.c_int, ctypes.c_double,
                                        _i32]),
    "nn_server_tick": (ctypes.c_int, [_p, ctypes.POINTER(nn_server_stats)]),
    "nn_server_poll": (_i32, [_p, ctypes.POINTER(nn_request_info), _i32]),
    "nn_server_fetch": (ctypes.c_int, [_p, _i64, _p, _i64]),
    "nn_server_release": (ctypes.c_int, [_p, _i64]),
    "nn_status_string": (ctypes.c_char_p, [ctypes.c_int]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


def header_functions(path: str = HEADER_PATH):
    """Names of the functions include/nn.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nn_[a-z_]+)\s*\(", text)))


def status_string(st: int) -> str:
    return nn_status_string(st).decode()


class NNError(RuntimeError):
    def __init__(self, status: int, where: str = ""):
        super().__init__(f"{where}: {status_string(status)} ({status})")
        self.status = status


def make_params(depth=2, x0="transpose", tol=1e-12, max_iter=100, fixed_iter=0, prec="plain",
                flags=0, power_k=8):
    if isinstance(x0, str):
        x0 = X0_NAMES[x0]
    p = nn_params()
    p.depth, p.x0, p.tol, p.max_iter = int(depth), int(x0), float(tol), int(max_iter)
    p.fixed_iter = int(fixed_iter)
    p.prec = NN_PREC_MIXED if prec in ("mixed", NN_PREC_MIXED) else NN_PREC_PLAIN
    p.flags = int(flags)
    p.power_k = int(power_k)
    p.reserved = 0
    return p


# ---- torch-facing helpers (plumbing) ----------------------------------------

def _torch():
    import torch
    return torch


def dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float64: NN_F64, torch.float32: NN_F32, torch.complex64: NN_C64,
         torch.complex128: NN_C128}
    if t.dtype not in m:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return m[t.dtype]


class Context:
    """An nn_ctx bound to a device and a stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream or 0)
        self._ptr = ctypes.c_void_p()
        st = nn_create(ctypes.byref(self._ptr), int(device), ctypes.c_void_p(handle))
        if st != NN_OK:
            raise NNError(st, "nn_create")
        self.device = device
        self.stream = stream

    @property
    def ptr(self):
        return self._ptr

    def close(self):
        if self._ptr:
            nn_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_CTX = {}


def default_context(device: int = 0) -> Context:
    torch = _torch()
    key = (device, torch.cuda.current_stream(device).cuda_stream)
    if key not in _CTX:
        _CTX[key] = Context(device)
    return _CTX[key]


def workspace(nbytes: int, device) :
    """A 256-byte aligned device byte buffer of at least nbytes (torch-owned)."""
    torch = _torch()
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf, buf.data_ptr() + off, int(nbytes)


def invert(A, depth=2, x0="transpose", tol=1e-12, max_iter=100, fixed_iter=0, prec="plain",
           X=None, ctx: Context | None = None, ws=None, check=True, flags=0, power_k=8):
    """X ~ A^-1 by nn_invert.  Returns (X, info dict).

    A: square CUDA tensor (float64, float32, complex64, complex128), row-major
    with any leading dimension (stride(1) must be 1).  With x0="given", X
    holds the start iterate.
    """
    torch = _torch()
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("A must be a square row-major matrix")
    n = A.shape[0]
    dt = dtype_code(A)
    prm = make_params(depth, x0, tol, max_iter, fixed_iter, prec, flags, power_k)
    if X is None:
        X = torch.empty((n, n), dtype=A.dtype, device=A.device)
    elif X.shape != A.shape or X.dtype != A.dtype or X.stride(1) != 1:
        raise ValueError("X must be a row-major matrix of A's shape and dtype")
    ctx = ctx or default_context(A.device.index or 0)
    need = nn_workspace_size(n, dt, ctypes.byref(prm))
    if need == 0:
        raise NNError(NN_ERR_ARG, "nn_workspace_size")
    hold = None
    if ws is None:
        hold, ws_ptr, ws_bytes = workspace(need, A.device)
    else:
        hold, ws_ptr, ws_bytes = ws
    info = nn_info()
    st = nn_invert(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.stride(0),
                   ctypes.c_void_p(X.data_ptr()), X.stride(0), n, dt, ctypes.byref(prm),
                   ctypes.c_void_p(ws_ptr), ws_bytes, ctypes.byref(info))
    del hold
    d = info.as_dict()
    d["status"] = st
    if check and st < 0 and st not in (NN_ERR_DIVERGED, NN_ERR_NONFINITE):
        raise NNError(st, "nn_invert")
    return X, d


def invert_noalloc(A, X, depth=2, x0="transpose", tol=1e-12, max_iter=100, fixed_iter=0,
                   prec="plain", ctx: Context | None = None, flags=0, power_k=8):
    """nn_invert_noalloc: X ~ A^-1 with the library's static device scratch
    (no workspace, no allocation; X must be given).  Returns (status, info)."""
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("A must be a square row-major matrix")
    if X.shape != A.shape or X.dtype != A.dtype or X.stride(1) != 1:
        raise ValueError("X must be a row-major matrix of A's shape and dtype")
    prm = make_params(depth, x0, tol, max_iter, fixed_iter, prec, flags, power_k)
    ctx = ctx or default_context(A.device.index or 0)
    info = nn_info()
    st = nn_invert_noalloc(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.stride(0),
                           ctypes.c_void_p(X.data_ptr()), X.stride(0), A.shape[0],
                           dtype_code(A), ctypes.byref(prm), ctypes.byref(info))
    d = info.as_dict()
    d["status"] = st
    return st, d


def solve(A, B, depth=2, x0="transpose", tol=1e-12, max_iter=100, fixed_iter=0,
          ctx: Context | None = None, check=True, power_k=8):
    """Xsol with A Xsol = B by nn_solve (Corollary 3).  Returns (Xsol, info)."""
    torch = _torch()
    n, nrhs = B.shape
    dt = dtype_code(A)
    prm = make_params(depth, x0, tol, max_iter, fixed_iter, power_k=power_k)
    Xs = torch.empty((n, nrhs), dtype=A.dtype, device=A.device)
    ctx = ctx or default_context(A.device.index or 0)
    need = nn_solve_workspace_size(n, nrhs, dt, ctypes.byref(prm))
    if need == 0:
        raise NNError(NN_ERR_ARG, "nn_solve_workspace_size")
    hold, ws_ptr, ws_bytes = workspace(need, A.device)
    info = nn_info()
    rel = ctypes.c_double(0.0)
    st = nn_solve(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.stride(0),
                  ctypes.c_void_p(B.data_ptr()), B.stride(0), ctypes.c_void_p(Xs.data_ptr()),
                  Xs.stride(0), n, nrhs, dt, ctypes.byref(prm), ctypes.c_void_p(ws_ptr),
                  ws_bytes, ctypes.byref(info), ctypes.byref(rel))
    del hold
    d = info.as_dict()
    d["status"] = st
    d["rel_residual"] = rel.value
    if check and st < 0 and st not in (NN_ERR_DIVERGED, NN_ERR_NONFINITE):
        raise NNError(st, "nn_solve")
    return Xs, d


def solve_factorized(A, B, x0="transpose", tol=1e-10, max_factors=60, fixed_factors=0,
                     ctx: Context | None = None, check=True, power_k=8):
    """Xsol with A Xsol = B by nn_solve_factorized (Corollary 6 applied to B).
    Returns (Xsol, info); info["iters"] is the number of factors and
    info["rms"] the relative residual ||B - A Xsol||_F / ||B||_F."""
    torch = _torch()
    n, nrhs = B.shape
    dt = dtype_code(A)
    prm = make_params(1, x0, tol, max_factors, fixed_factors, power_k=power_k)
    Xs = torch.empty((n, nrhs), dtype=A.dtype, device=A.device)
    ctx = ctx or default_context(A.device.index or 0)
    need = nn_solve_factorized_workspace_size(n, nrhs, dt, ctypes.byref(prm))
    if need == 0:
        raise NNError(NN_ERR_ARG, "nn_solve_factorized_workspace_size")
    hold, ws_ptr, ws_bytes = workspace(need, A.device)
    info = nn_info()
    rel = ctypes.c_double(0.0)
    st = nn_solve_factorized(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.stride(0),
                             ctypes.c_void_p(B.data_ptr()), B.stride(0),
                             ctypes.c_void_p(Xs.data_ptr()), Xs.stride(0), n, nrhs, dt,
                             ctypes.byref(prm), ctypes.c_void_p(ws_ptr), ws_bytes,
                             ctypes.byref(info), ctypes.byref(rel))
    del hold
    d = info.as_dict()
    d["status"] = st
    d["rel_residual"] = rel.value
    if check and st < 0 and st not in (NN_ERR_DIVERGED, NN_ERR_NONFINITE):
        raise NNError(st, "nn_solve_factorized")
    return Xs, d


def make_cns_params(depth=2, x0="transpose", nests=0, precond_tol=1e-2, max_nests=100,
                    prec="plain", tol=1e-12, max_terms=100, fixed_terms=None, reuse_phi=False,
                    power_k=8):
    c = nn_cns_params()
    c.precond = make_params(depth, x0, precond_tol, max_nests, nests, prec, power_k=power_k)
    c.tol = float(tol)
    c.max_terms = int(max_terms)
    c.fixed_terms = -1 if fixed_terms is None else int(fixed_terms)
    c.reuse_phi = 1 if reuse_phi else 0
    c.reserved = 0
    return c


def solve_cns(A, B, depth=2, x0="transpose", nests=0, precond_tol=1e-2, max_nests=100,
              prec="plain", tol=1e-12, max_terms=100, fixed_terms=None, ws=None,
              reuse_phi=False, ctx: Context | None = None, check=True, power_k=8):
    """Xsol with A Xsol = B by nn_solve_cns: NN nests for phi (``nests`` > 0
    fixed, else down to rms < precond_tol), then the Neumann series in
    I - phi A applied to B (``fixed_terms`` terms, else down to the relative
    residual ``tol``).  Returns (Xsol, info): info["iters"] = terms,
    info["rms"] = info["rel_residual"] = ||B - A Xsol||_F / ||B||_F,
    info["precond"] = the nests' record, info["ws"] = the workspace, whose
    head holds phi: pass it back as ``ws`` with ``reuse_phi=True`` to solve
    further right-hand sides against the same A without new nests."""
    torch = _torch()
    if B.dim() != 2 or B.stride(1) != 1 or A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A and B must be row-major matrices")
    n, nrhs = B.shape
    dt = dtype_code(A)
    prm = make_cns_params(depth, x0, nests, precond_tol, max_nests, prec, tol, max_terms,
                          fixed_terms, reuse_phi, power_k)
    Xs = torch.empty((n, nrhs), dtype=A.dtype, device=A.device)
    ctx = ctx or default_context(A.device.index or 0)
    need = nn_solve_cns_workspace_size(n, nrhs, dt, ctypes.byref(prm))
    if need == 0:
        raise NNError(NN_ERR_ARG, "nn_solve_cns_workspace_size")
    if ws is None:
        if reuse_phi:
            raise ValueError("reuse_phi needs the workspace of an earlier call")
        ws = workspace(need, A.device)
    _, ws_ptr, ws_bytes = ws
    pinfo, info = nn_info(), nn_info()
    rel = ctypes.c_double(0.0)
    st = nn_solve_cns(ctx.ptr, ctypes.c_void_p(A.data_ptr()), A.stride(0),
                      ctypes.c_void_p(B.data_ptr()), B.stride(0), ctypes.c_void_p(Xs.data_ptr()),
                      Xs.stride(0), n, nrhs, dt, ctypes.byref(prm), ctypes.c_void_p(ws_ptr),
                      ws_bytes, ctypes.byref(pinfo), ctypes.byref(info), ctypes.byref(rel))
    d = info.as_dict()
    d["status"] = st
    d["rel_residual"] = rel.value
    d["precond"] = pinfo.as_dict()
    d["ws"] = ws
    if check and st < 0 and st not in (NN_ERR_DIVERGED, NN_ERR_NONFINITE):
        raise NNError(st, "nn_solve_cns")
    return Xs, d


def make_sparse_params(x0="identity", power_k=8, tol=1e-10, max_terms=100000,
                       fixed_terms=None, check_every=16):
    if isinstance(x0, str):
        x0 = X0_NAMES[x0]
    p = nn_sparse_params()
    p.x0, p.power_k, p.tol = int(x0), int(power_k), float(tol)
    p.max_terms = int(max_terms)
    p.fixed_terms = -1 if fixed_terms is None else int(fixed_terms)
    p.check_every = int(check_every)
    p.reserved = 0
    return p


def solve_sparse(indptr, indices, values, B, x0="identity", power_k=8, tol=1e-10,
                 max_terms=100000, fixed_terms=None, check_every=16, ctx: Context | None = None,
                 ws=None, check=True):
    """Xsol with W Xsol = B for a CSR matrix W by nn_solve_sparse (the
    Neumann series in I - phi W applied to phi B, Algorithm 2).  indptr and
    indices: int32 CUDA tensors; values and B: CUDA tensors of one dtype.
    Returns (Xsol, info): info["iters"] = terms, info["rms"] = control
    residual, info["rel_residual"] = plain ||B - W Xsol||_F / ||B||_F."""
    torch = _torch()
    if indptr.dtype != torch.int32 or indices.dtype != torch.int32:
        raise TypeError("indptr and indices must be int32")
    if values.dtype != B.dtype:
        raise TypeError("values and B must share a dtype")
    if B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major matrix")
    n, nrhs = B.shape
    if indptr.numel() != n + 1:
        raise ValueError("indptr must have n + 1 entries")
    nnz = indices.numel()
    if values.numel() != nnz:
        raise ValueError("values and indices must have nnz entries")
    dt = dtype_code(B)
    prm = make_sparse_params(x0, power_k, tol, max_terms, fixed_terms, check_every)
    Xs = torch.empty((n, nrhs), dtype=B.dtype, device=B.device)
    ctx = ctx or default_context(B.device.index or 0)
    need = nn_solve_sparse_workspace_size(n, nrhs, dt, ctypes.byref(prm))
    if need == 0:
        raise NNError(NN_ERR_ARG, "nn_solve_sparse_workspace_size")
    hold = None
    if ws is None:
        hold, ws_ptr, ws_bytes = workspace(need, B.device)
    else:
        hold, ws_ptr, ws_bytes = ws
    info = nn_info()
    rel = ctypes.c_double(0.0)
    st = nn_solve_sparse(ctx.ptr, ctypes.c_void_p(indptr.data_ptr()),
                         ctypes.c_void_p(indices.data_ptr() if nnz else 0),
                         ctypes.c_void_p(values.data_ptr() if nnz else 0), n, nnz,
                         ctypes.c_void_p(B.data_ptr()), B.stride(0),
                         ctypes.c_void_p(Xs.data_ptr()), Xs.stride(0), nrhs, dt,
                         ctypes.byref(prm), ctypes.c_void_p(ws_ptr), ws_bytes,
                         ctypes.byref(info), ctypes.byref(rel))
    del hold
    d = info.as_dict()
    d["status"] = st
    d["rel_residual"] = rel.value
    if check and st < 0 and st not in (NN_ERR_DIVERGED, NN_ERR_NONFINITE):
        raise NNError(st, "nn_solve_sparse")
    return Xs, d


def invert_batched(packed, offsets, sizes, max_n, depth=2, x0="transpose", fixed_iter=4,
                   X=None, info=None, ctx: Context | None = None, ws=None, check=True,
                   tol=0.0, max_iter=1):
    """nn_invert_batched on packed device buffers.  Returns (X_packed, info tensor).

    packed: 1-D complex64/float32 CUDA tensor; offsets int64 and sizes int32
    CUDA tensors.  info: (batch, 2) int32 + rms as a (batch,) float64 view of
    an nn_info_dev array (returned as a raw uint8 tensor of batch*16 bytes).
    fixed_iter=0 selects the tolerance mode (tol, max_iter per matrix); with
    x0="given", X (required) holds the start iterates on entry.
    """
    torch = _torch()
    batch = int(sizes.numel())
    dt = dtype_code(packed)
    prm = make_params(depth, x0, float(tol), int(max_iter), fixed_iter)
    if X is None:
        if prm.x0 == NN_X0_GIVEN:
            raise ValueError("x0='given' needs X holding the start iterates")
        X = torch.empty_like(packed)
    if info is None:
        info = torch.empty(batch * ctypes.sizeof(nn_info_dev), dtype=torch.uint8, device=packed.device)
    ctx = ctx or default_context(packed.device.index or 0)
    need = nn_batched_workspace_size(batch, dt)
    hold = None
    if ws is None:
        hold, ws_ptr, ws_bytes = workspace(max(need, 1), packed.device)
    else:
        hold, ws_ptr, ws_bytes = ws
    st = nn_invert_batched(ctx.ptr, ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                           ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(sizes.data_ptr()),
                           batch, int(max_n), dt, ctypes.byref(prm), ctypes.c_void_p(ws_ptr),
                           ws_bytes, ctypes.c_void_p(info.data_ptr()))
    if check and st != NN_OK:
        raise NNError(st, "nn_invert_batched")
    X._nn_ws_hold = hold  # keep the workspace alive until the caller syncs
    return X, info


def batched_autotune(packed, offsets, sizes, max_n, depth=2, x0="transpose", fixed_iter=4,
                     ctx: Context | None = None, with_source=False):
    """nn_batched_autotune; returns (best_ms, wave_max_k, wg_per_cu), plus
    whether the configuration came from the NN_AUTOTUNE_CACHE file when
    with_source is set."""
    torch = _torch()
    batch = int(sizes.numel())
    dt = dtype_code(packed)
    prm = make_params(depth, x0, 0.0, 1, fixed_iter)
    X = torch.empty_like(packed)
    ctx = ctx or default_context(packed.device.index or 0)
    hold, ws_ptr, ws_bytes = workspace(nn_batched_workspace_size(batch, dt), packed.device)
    best = ctypes.c_float(0.0)
    cached = ctypes.c_int32(0)
    st = nn_batched_autotune(ctx.ptr, ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                             ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(sizes.data_ptr()),
                             batch, int(max_n), dt, ctypes.byref(prm), ctypes.c_void_p(ws_ptr),
                             ws_bytes, ctypes.byref(best), ctypes.byref(cached))
    if st != NN_OK:
        raise NNError(st, "nn_batched_autotune")
    wk, wg = ctypes.c_int32(), ctypes.c_int32()
    nn_batched_get_config(ctx.ptr, dt, int(max_n), ctypes.byref(wk), ctypes.byref(wg))
    del hold
    if with_source:
        return best.value, wk.value, wg.value, bool(cached.value)
    return best.value, wk.value, wg.value


def batched_set_config(dtype_code_, max_n, wave_max_k, wg_per_cu, ctx: Context | None = None,
                       device: int = 0):
    ctx = ctx or default_context(device)
    st = nn_batched_set_config(ctx.ptr, int(dtype_code_), int(max_n), int(wave_max_k), int(wg_per_cu))
    if st != NN_OK:
        raise NNError(st, "nn_batched_set_config")


def decode_batched_info(info_bytes):
    """(iters int32[], status int32[], rms float64[]) from an nn_info_dev buffer."""
    import numpy as np
    raw = info_bytes.cpu().numpy().view(np.uint8)
    rec = np.frombuffer(raw.tobytes(), dtype=np.dtype([("iters", "<i4"), ("status", "<i4"),
                                                        ("rms", "<f8")]))
    return rec["iters"].copy(), rec["status"].copy(), rec["rms"].copy()


# ---- continuous-batching server ----------------------------------------------

_TORCH_OF = {NN_F64: "float64", NN_F32: "float32", NN_C64: "complex64", NN_C128: "complex128"}


class Server:
    """nn_server over a torch-owned device pool of ``pool_bytes``.

    submit(id, A, tol, max_iter) queues a device (or host) matrix; tick()
    advances every active request by one nest; poll() returns the records of
    retired requests; fetch(id) returns the result as a new tensor (on
    ``out_device``) and frees its pool memory.  Source tensors are kept
    referenced until their request is polled.
    """

    def __init__(self, pool_bytes, depth=2, x0="identity", max_active=1024, n_streams=4,
                 wide_tol=1e-6, device=0, ctx: Context | None = None, power_k=8,
                 batch_max_n=64):
        torch = _torch()
        self.ctx = ctx or default_context(device)
        self.device = torch.device("cuda", device)
        self._pool = workspace(int(pool_bytes), self.device)
        p = nn_server_params()
        p.depth, p.x0 = int(depth), X0_NAMES[x0] if isinstance(x0, str) else int(x0)
        p.max_active, p.n_streams, p.wide_tol = int(max_active), int(n_streams), float(wide_tol)
        p.power_k, p.batch_max_n = int(power_k), int(batch_max_n)
        self.params = p
        self._ptr = ctypes.c_void_p()
        st = nn_server_create(self.ctx.ptr, ctypes.c_void_p(self._pool[1]), self._pool[2],
                              ctypes.byref(p), ctypes.byref(self._ptr))
        if st != NN_OK:
            raise NNError(st, "nn_server_create")
        self._src = {}
        self.stats = nn_server_stats()
        self._rec = (nn_request_info * 256)()

    def footprint(self, n, dtype, tol):
        return nn_server_footprint(self._ptr, int(n), int(dtype), float(tol))

    def submit(self, rid, A, tol, max_iter=100):
        if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
            raise ValueError("A must be a square row-major matrix")
        st = nn_server_submit(self._ptr, int(rid), ctypes.c_void_p(A.data_ptr()), A.stride(0),
                              A.shape[0], dtype_code(A), float(tol), int(max_iter))
        if st != NN_OK:
            raise NNError(st, "nn_server_submit")
        self._src[int(rid)] = A

    def tick(self):
        st = nn_server_tick(self._ptr, ctypes.byref(self.stats))
        if st != NN_OK:
            raise NNError(st, "nn_server_tick")
        return self.stats

    def poll(self):
        out = []
        while True:
            k = nn_server_poll(self._ptr, self._rec, len(self._rec))
            for i in range(k):
                d = self._rec[i].as_dict()
                self._src.pop(d["id"], None)
                out.append(d)
            if k < len(self._rec):
                return out

    def fetch(self, rid, n, out_dtype, out_device=None):
        torch = _torch()
        dev = self.device if out_device is None else torch.device(out_device)
        X = torch.empty((int(n), int(n)), dtype=getattr(torch, _TORCH_OF[int(out_dtype)]),
                        device=dev, pin_memory=(dev.type == "cpu"))
        st = nn_server_fetch(self._ptr, int(rid), ctypes.c_void_p(X.data_ptr()), int(n))
        if st != NN_OK:
            raise NNError(st, "nn_server_fetch")
        return X

    def release(self, rid):
        st = nn_server_release(self._ptr, int(rid))
        if st != NN_OK:
            raise NNError(st, "nn_server_release")

    def run_until_idle(self, max_ticks=100000):
        """Tick until nothing is queued or active; returns the polled records."""
        recs = []
        for _ in range(max_ticks):
            s = self.tick()
            recs += self.poll()
            if s.active == 0 and s.queued == 0:
                return recs
        raise RuntimeError("server did not drain")

    def close(self):
        if self._ptr:
            nn_server_destroy(self._ptr)
            self._ptr = ctypes.c_void_p()
        self._src.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
