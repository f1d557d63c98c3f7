"""C-ABI checks that need no GPU: the library loads, exports every function
include/nn.h declares, its structs have the sizes the binding assumes, and
argument errors are reported before anything touches the device."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2212_02406_amd", "libnn.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libnn.so not built")


def _nn():
    from paper_2212_02406_amd import nn
    return nn


def test_exports_every_declared_symbol():
    nn = _nn()
    names = nn.header_functions()
    assert {"nn_create", "nn_destroy", "nn_invert", "nn_solve", "nn_invert_batched",
            "nn_workspace_size", "nn_status_string"} <= set(names)
    raw = ctypes.CDLL(LIB)
    for name in names:
        assert hasattr(raw, name), name


def test_struct_layout_matches_c_compiler():
    """Every field offset and struct size of the binding equals what gcc
    computes from include/nn.h (offsetof / sizeof in a generated C file)."""
    import shutil
    import subprocess
    import tempfile
    nn = _nn()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = [nn.nn_params, nn.nn_info, nn.nn_info_dev, nn.nn_cns_params, nn.nn_sparse_params,
               nn.nn_server_params, nn.nn_request_info, nn.nn_server_stats]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "nn.h"', "int main(void) {"]
    expect = []
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("%zu\\n", sizeof({name}));')
        expect.append(ctypes.sizeof(st))
        for field, _ in st._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({name}, {field}));')
            expect.append(getattr(st, field).offset)
    lines += ["  return 0;", "}"]
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "layout.c"), os.path.join(td, "layout")
        open(src, "w").write("\n".join(lines) + "\n")
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                       check=True)
        got = [int(x) for x in subprocess.run([exe], check=True, capture_output=True,
                                               text=True).stdout.split()]
    assert got == expect


def test_struct_layout():
    nn = _nn()
    assert ctypes.sizeof(nn.nn_params) == 40 and nn.nn_params.power_k.offset == 32
    assert nn.nn_info.prec_gemms.offset == 44 and nn.nn_info.rms_trace.offset == 56
    assert ctypes.sizeof(nn.nn_info) == 56 + 8 * nn.NN_TRACE_MAX
    assert ctypes.sizeof(nn.nn_info_dev) == 16
    assert ctypes.sizeof(nn.nn_server_params) == 32 and nn.nn_server_params.power_k.offset == 24
    assert ctypes.sizeof(nn.nn_request_info) == 64
    assert nn.nn_request_info.rms.offset == 32
    assert ctypes.sizeof(nn.nn_server_stats) == 24
    assert ctypes.sizeof(nn.nn_sparse_params) == 32 and nn.nn_sparse_params.tol.offset == 8
    assert ctypes.sizeof(nn.nn_cns_params) == 64
    assert nn.nn_cns_params.tol.offset == 40 and nn.nn_cns_params.reuse_phi.offset == 56


def test_server_argument_errors_before_device_work():
    nn = _nn()
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert nn.nn_server_create(None, fake, 1 << 20, None, ctypes.byref(out)) == nn.NN_ERR_ARG
    assert nn.nn_server_footprint(None, 64, nn.NN_F32, 1e-4) == 0
    assert nn.nn_server_submit(None, 1, fake, 4, 4, nn.NN_F32, 1e-4, 10) == nn.NN_ERR_ARG
    assert nn.nn_server_tick(None, None) == nn.NN_ERR_ARG
    assert nn.nn_server_fetch(None, 1, fake, 4) == nn.NN_ERR_ARG
    assert nn.nn_server_release(None, 1) == nn.NN_ERR_ARG
    nn.nn_server_destroy(None)


def test_status_strings():
    nn = _nn()
    for st in range(-6, 3):
        assert nn.status_string(st)
    assert "unknown" in nn.status_string(42)


def test_argument_errors_before_launch():
    nn = _nn()
    p = nn.make_params()
    info = nn.nn_info()
    fake = ctypes.c_void_p(0x1000)
    # null context / pointers, bad n, bad lda, bad depth: all NN_ERR_ARG
    assert nn.nn_invert(None, fake, 4, fake, 4, 4, nn.NN_F64, ctypes.byref(p), fake, 1 << 20,
                        ctypes.byref(info)) == nn.NN_ERR_ARG
    bad = nn.make_params(depth=0)
    assert nn.nn_workspace_size(16, nn.NN_F64, ctypes.byref(bad)) == 0
    bad = nn.make_params(depth=nn.NN_MAX_DEPTH + 1)
    assert nn.nn_workspace_size(16, nn.NN_F64, ctypes.byref(bad)) == 0
    bad = nn.make_params(tol=-1.0)
    assert nn.nn_workspace_size(16, nn.NN_F64, ctypes.byref(bad)) == 0
    assert nn.nn_workspace_size(0, nn.NN_F64, ctypes.byref(p)) == 0
    assert nn.nn_workspace_size(16, 9, ctypes.byref(p)) == 0
    bad = nn.make_params(flags=4)
    assert nn.nn_workspace_size(16, nn.NN_F64, ctypes.byref(bad)) == 0
    assert nn.nn_invert_noalloc(None, fake, 4, fake, 4, 4, nn.NN_F64, ctypes.byref(p),
                                ctypes.byref(info)) == nn.NN_ERR_ARG


def test_noalloc_scratch_limits():
    """The largest sizes whose workspace fits nn_invert_noalloc's static
    scratch, as include/nn.h states them."""
    nn = _nn()
    L = nn.NN_NOALLOC_SCRATCH_BYTES
    assert L == 32 << 20
    stated = {nn.NN_F64: (1437, 1176, 1013), nn.NN_C64: (1437, 1176, 1013),
              nn.NN_F32: (2019, 1656, 1437), nn.NN_C128: (1013, 830, 720)}
    for dt, ns in stated.items():
        for d, n in zip((1, 2, 3), ns):
            p = nn.make_params(depth=d)
            assert 0 < nn.nn_workspace_size(n, dt, ctypes.byref(p)) <= L
            assert nn.nn_workspace_size(n + 1, dt, ctypes.byref(p)) > L
    p = nn.make_params(depth=2, prec="mixed", x0="identity")
    assert 0 < nn.nn_workspace_size(698, nn.NN_F64, ctypes.byref(p)) <= L
    assert nn.nn_workspace_size(699, nn.NN_F64, ctypes.byref(p)) > L


def test_cns_argument_errors_and_workspace():
    nn = _nn()
    fake = ctypes.c_void_p(0x1000)
    pi, inf = nn.nn_info(), nn.nn_info()
    ok = nn.make_cns_params()
    assert nn.nn_solve_cns(None, fake, 4, fake, 1, fake, 1, 4, 1, nn.NN_F64, ctypes.byref(ok),
                           fake, 1 << 20, ctypes.byref(pi), ctypes.byref(inf), None) == nn.NN_ERR_ARG
    sz = lambda c, n=256, r=8, dt=nn.NN_F64: nn.nn_solve_cns_workspace_size(n, r, dt, ctypes.byref(c))
    base = sz(ok)
    # phi + nn_invert's workspace + two n x nrhs buffers at least
    inv = nn.nn_workspace_size(256, nn.NN_F64, ctypes.byref(ok.precond))
    assert base >= 256 * 256 * 8 + inv + 2 * 256 * 8 * 8
    assert sz(nn.make_cns_params(depth=1)) < base
    assert sz(nn.make_cns_params(fixed_terms=0)) == base
    for bad in (nn.make_cns_params(depth=0), nn.make_cns_params(tol=-1.0),
                nn.make_cns_params(max_terms=0), nn.make_cns_params(fixed_terms=-2),
                nn.make_cns_params(max_terms=nn.NN_CNS_MAX_TERMS + 1)):
        assert sz(bad) == 0
    c = nn.make_cns_params()
    c.reserved = 1
    assert sz(c) == 0
    c = nn.make_cns_params()
    c.reuse_phi = 2
    assert sz(c) == 0
    # the mixed preconditioner exists for FP64 only
    assert sz(nn.make_cns_params(prec="mixed", x0="identity")) > 0
    assert sz(nn.make_cns_params(prec="mixed", x0="identity"), dt=nn.NN_F32) == 0
    assert sz(ok, n=0) == 0 and sz(ok, r=0) == 0 and sz(ok, dt=7) == 0


def test_sparse_argument_errors_and_workspace():
    nn = _nn()
    fake = ctypes.c_void_p(0x1000)
    inf = nn.nn_info()
    ok = nn.make_sparse_params()
    assert nn.nn_solve_sparse(None, fake, fake, fake, 4, 4, fake, 1, fake, 1, 1, nn.NN_F64,
                              ctypes.byref(ok), fake, 1 << 20, ctypes.byref(inf),
                              None) == nn.NN_ERR_ARG
    sz = lambda c, n=1000, r=16, dt=nn.NN_F64: nn.nn_solve_sparse_workspace_size(
        n, r, dt, ctypes.byref(c))
    base = sz(ok)
    assert base >= 2 * 1000 * 16 * 8
    assert sz(ok, r=32) > base and sz(ok, dt=nn.NN_C128) > base
    for bad in (nn.make_sparse_params(x0="transpose"), nn.make_sparse_params(x0="given"),
                nn.make_sparse_params(tol=-1.0), nn.make_sparse_params(max_terms=0),
                nn.make_sparse_params(check_every=0), nn.make_sparse_params(check_every=1025),
                nn.make_sparse_params(fixed_terms=-2),
                nn.make_sparse_params(x0="power_identity", power_k=0)):
        assert sz(bad) == 0
    c = nn.make_sparse_params()
    c.reserved = 3
    assert sz(c) == 0
    assert sz(nn.make_sparse_params(x0="jacobi", fixed_terms=0, check_every=0)) > 0


def test_workspace_sizes_grow_with_depth_and_n():
    nn = _nn()
    sizes = [nn.nn_workspace_size(512, nn.NN_F64, ctypes.byref(nn.make_params(depth=d)))
             for d in (1, 2, 3, 4)]
    assert sizes[0] < sizes[1] < sizes[2] == sizes[3]
    mat = 512 * 512 * 8
    assert sizes[0] >= 2 * mat and sizes[2] >= 4 * mat
    f32 = nn.nn_workspace_size(512, nn.NN_F32, ctypes.byref(nn.make_params()))
    c128 = nn.nn_workspace_size(512, nn.NN_C128, ctypes.byref(nn.make_params()))
    assert f32 < sizes[1] < c128


def test_create_without_gpu_reports_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    nn = _nn()
    c = ctypes.c_void_p()
    assert nn.nn_create(ctypes.byref(c), 0, None) in (nn.NN_ERR_HIP, nn.NN_ERR_ARG)
    assert nn.nn_create(None, 0, None) == nn.NN_ERR_ARG


def test_batched_one_wave_limit_fits_lds():
    """nn_batched_fit_config lowers the one-wave size limit until the LDS of
    one workgroup holds the matrices at the given depth.  The expected value
    is recomputed here from the layout the batched kernel documents: a K x K
    matrix buffer has pad16(K) rows of pad16(K or 2K real columns) + 4 floats;
    two buffers per matrix (three from depth 3); a workgroup holds one matrix
    of max_n or eight one-wave matrices; the kernel's static LDS is 8720
    bytes; limits 150 KB dynamic, 160 KB per CU."""
    nn = _nn()

    def pad(x):
        return (x + 15) // 16 * 16

    def lds(cplx, max_n, wk, depth):
        buf = lambda k: pad(k) * (pad(2 * k if cplx else k) + 4)  # noqa: E731
        nb = 3 if depth >= 3 else 2
        return 4 * max(nb * buf(max_n), 8 * nb * buf(max(wk, 1)))

    lim = min(150 * 1024, 160 * 1024 - 8720)
    for dt, cplx in ((nn.NN_C64, True), (nn.NN_F32, False)):
        for depth in (1, 2, 3, 5, 8):
            for max_n in (1, 8, 16, 33, 64):
                for wk in (0, 5, 8, 16, 24, 32):
                    w = min(wk, max_n)
                    while w > 0 and lds(cplx, max_n, w, depth) > lim:
                        w = 16 if w > 16 else 8 if w > 8 else 0
                    assert nn.nn_batched_fit_config(dt, max_n, wk, depth) == w, (dt, depth, max_n, wk)
    assert nn.nn_batched_fit_config(nn.NN_C64, 64, 32, 3) == 16   # 204 KB would not fit
    assert nn.nn_batched_fit_config(nn.NN_C64, 64, 32, 2) == 32
    assert nn.nn_batched_fit_config(nn.NN_F32, 64, 32, 8) == 32
    assert nn.nn_batched_fit_config(nn.NN_F64, 64, 32, 2) == -1
    assert nn.nn_batched_fit_config(nn.NN_C64, 65, 32, 2) == -1
    assert nn.nn_batched_fit_config(nn.NN_C64, 64, 33, 2) == -1
    assert nn.nn_batched_fit_config(nn.NN_C64, 64, 16, 0) == -1
