"""Split-K thin products (n x n times n x nrhs) used by nn_solve,
nn_solve_factorized and nn_solve_cns.  NN_GEMM_SPLIT forces the split on
small sizes, ragged and exact tilings, every dtype; results against the
unsplit run (the same sums in another order: relative 1e-13 in double,
64 u32 in single) and against the oracle (the usual parity bars)."""
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


def _relF(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


@pytest.mark.parametrize("n,nrhs", [(197, 7), (256, 64), (300, 33), (64, 1)])
@pytest.mark.parametrize("dtype", [np.float64, np.complex128, np.float32, np.complex64])
@pytest.mark.parametrize("split", [2, 4, 8])
def test_forced_split_matches_unsplit_and_oracle(n, nrhs, dtype, split, monkeypatch):
    _say(f"splitk n={n} nrhs={nrhs} {np.dtype(dtype).name} split={split}")
    cplx = np.dtype(dtype).kind == "c"
    single = np.dtype(dtype) in (np.dtype(np.float32), np.dtype(np.complex64))
    A = W.dense_spd(n, 1.0, 20.0, 1000 + n, complex_=cplx, dtype=dtype)
    g = W.rng(1001 + n)
    B = (g.standard_normal((n, nrhs)) + (1j * g.standard_normal((n, nrhs)) if cplx else 0.0)
         ).astype(dtype)
    At, Bt = torch.from_numpy(A).to(DEV), torch.from_numpy(B).to(DEV)
    ref_dt = np.complex128 if cplx else np.float64
    runs = {
        "cns": lambda: nn.solve_cns(At, Bt, nests=3, fixed_terms=4)[0],
        "factorized": lambda: nn.solve_factorized(At, Bt, fixed_factors=6)[0],
        "solve": lambda: nn.solve(At, Bt, fixed_iter=5)[0],
    }
    refs = {
        "cns": lambda: oracle.nn_cns_solve_ref(A.astype(ref_dt), B.astype(ref_dt), nests=3,
                                               fixed_terms=4)[0],
        "factorized": lambda: oracle.nn_factorized_solve_ref(A.astype(ref_dt), B.astype(ref_dt),
                                                             fixed_factors=6)[0],
        "solve": lambda: oracle.nn_solve_ref(A.astype(ref_dt), B.astype(ref_dt),
                                             fixed_iter=5)[0],
    }
    kappa = np.linalg.cond(A.astype(ref_dt))
    for name, fn in runs.items():
        monkeypatch.setenv("NN_GEMM_SPLIT", "1")
        X1 = fn().cpu().numpy()
        monkeypatch.setenv("NN_GEMM_SPLIT", str(split))
        Xs = fn().cpu().numpy()
        torch.cuda.synchronize()
        bar = 64 * U32 * kappa if single else 1e-13
        assert _relF(Xs.astype(ref_dt), X1.astype(ref_dt)) < bar, name
        xo = refs[name]()
        assert _relF(Xs.astype(ref_dt), xo) < (64 * U32 * kappa if single else 1e-10), name
