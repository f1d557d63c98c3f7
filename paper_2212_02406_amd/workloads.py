"""Seeded synthetic inputs for the NN library, its tests and its benchmark.

This module builds matrices only; it holds none of the NN method's
arithmetic, and it is the one piece of code that both the HIP path's callers
and the oracle's tests use, so both sides see the same input bits.

Workloads (the paper runs none; these are synthetic stand-ins with the shape
of its intended uses — dense positive definite inversion, Sec. II-D, and the
massive-MIMO Gram matrices of Corollary 4's discussion):

* dense SPD / HPD:  A = Q diag(lam) Q^H with Q the orthogonal (unitary) factor
  of the QR of an iid N(0,1) (CN(0,1)) matrix, sign-fixed so the factorisation
  is unique, and lam drawn uniform or log-uniform in [lo, hi] with both
  endpoints pinned so cond(A) = hi/lo exactly.  A is symmetrised
  ((A + A^H)/2) in FP64 and rounded once to the run dtype.
* massive-MIMO Gram batch: G = H^H H + sigma^2 I, H of shape M x K with iid
  CN(0,1) entries, K drawn uniformly from a set per matrix; packed row-major,
  back to back, with int64 element offsets and int32 sizes.

Random numbers come from NumPy's PCG64 with an explicit seed.  For N >= 4096
the QR and the product Q diag(lam) Q^H may run on a torch device (plumbing
only: the random draws are still the host PCG64 ones); the result is then
copied back to the host so the oracle sees the same bits.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "spectrum_uniform", "spectrum_loguniform", "haar_unitary",
    "dense_spd", "mimo_gram_batch", "pack_batch", "serving_pool",
    "ragged_batch", "mimo_gram", "diag_dominant", "laplacian_2d", "random_sparse_hpd",
    "csr_to_dense",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def spectrum_uniform(n: int, lo: float, hi: float, g: np.random.Generator) -> np.ndarray:
    lam = g.uniform(lo, hi, n)
    lam[0] = lo
    if n > 1:
        lam[-1] = hi
    return lam


def spectrum_loguniform(n: int, lo: float, hi: float, g: np.random.Generator) -> np.ndarray:
    lam = np.exp(g.uniform(np.log(lo), np.log(hi), n))
    lam[0] = lo
    if n > 1:
        lam[-1] = hi
    return lam


def _gaussian(n: int, m: int, g: np.random.Generator, complex_: bool) -> np.ndarray:
    if complex_:
        return (g.standard_normal((n, m)) + 1j * g.standard_normal((n, m))) / np.sqrt(2.0)
    return g.standard_normal((n, m))


def haar_unitary(n: int, g: np.random.Generator, complex_: bool = False, device=None):
    """Q of the QR of an iid Gaussian matrix, columns sign/phase fixed."""
    Gm = _gaussian(n, n, g, complex_)
    if device is None:
        Q, R = np.linalg.qr(Gm)
        d = np.diag(R)
        ph = d / np.abs(d)
        return Q * ph[None, :]
    import torch  # plumbing for large N only
    Gt = torch.from_numpy(Gm).to(device)
    Q, R = torch.linalg.qr(Gt)
    d = torch.diagonal(R)
    ph = d / d.abs()
    return Q * ph[None, :]


def dense_spd(n: int, lo: float, hi: float, seed: int, *, log_spectrum: bool = False,
              complex_: bool = False, dtype=None, device=None, return_factors: bool = False):
    """Dense SPD (or HPD) A = Q diag(lam) Q^H, rounded once to ``dtype``.

    Returns A as a host NumPy array (and (lam, Q) in FP64/complex128 when
    ``return_factors``; Q is returned on the host).
    """
    g = rng(seed)
    lam = (spectrum_loguniform if log_spectrum else spectrum_uniform)(n, lo, hi, g)
    if dtype is None:
        dtype = np.complex128 if complex_ else np.float64
    if device is None:
        Q = haar_unitary(n, g, complex_)
        A = (Q * lam[None, :]) @ Q.conj().T
        A = 0.5 * (A + A.conj().T)
        Ah = A.astype(dtype)
        return (Ah, lam, Q) if return_factors else Ah
    import torch
    Q = haar_unitary(n, g, complex_, device=device)
    lam_t = torch.from_numpy(lam).to(device=device, dtype=Q.dtype)
    A = (Q * lam_t[None, :]) @ Q.conj().T
    A = 0.5 * (A + A.conj().T)
    Ah = A.cpu().numpy().astype(dtype)
    if return_factors:
        return Ah, lam, Q.cpu().numpy()
    return Ah


def pack_batch(mats, dtype) -> tuple:
    """Pack square matrices back to back, row-major.

    Returns (packed 1-D array of ``dtype``, offsets int64 element offsets,
    sizes int32).
    """
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    offsets = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        offsets[1:] = np.cumsum(sizes.astype(np.int64) ** 2)[:-1]
    total = int(np.sum(sizes.astype(np.int64) ** 2))
    packed = np.empty(total, dtype=dtype)
    for m, o in zip(mats, offsets):
        k = m.shape[0]
        packed[o:o + k * k] = np.asarray(m, dtype=dtype).reshape(-1)
    return packed, offsets, sizes


def mimo_gram_batch(batch: int = 4096, M: int = 128, Ks=(8, 16, 32, 64),
                    sigma2: float = 0.1, seed: int = 3, dtype=np.complex64):
    """Massive-MIMO regularised Gram matrices G = H^H H + sigma^2 I.

    H is M x K with iid CN(0,1) entries; K is drawn uniformly from ``Ks`` per
    matrix.  Returns (packed, offsets, sizes, mats) where ``mats`` holds the
    dtype-rounded matrices (as ``dtype``) for the oracle.
    """
    g = rng(seed)
    Kdraw = g.choice(np.asarray(Ks), size=batch)
    mats = []
    for K in Kdraw:
        H = _gaussian(M, int(K), g, True)
        G = H.conj().T @ H + sigma2 * np.eye(int(K))
        G = 0.5 * (G + G.conj().T)
        mats.append(G.astype(dtype))
    packed, offsets, sizes = pack_batch(mats, dtype)
    return packed, offsets, sizes, mats


def mimo_gram(M: int, K: int, seed: int, sigma2: float = 0.1, complex_: bool = True,
              dtype=np.complex128):
    """One massive-MIMO regularised Gram matrix G = H^H H + sigma^2 I, H of
    shape M x K with iid CN(0,1) (N(0,1) if not complex_) entries.  With
    M >> K its spectrum over diag(G) lies near [(1 - sqrt(K/M))^2,
    (1 + sqrt(K/M))^2]."""
    g = rng(seed)
    H = _gaussian(M, K, g, complex_)
    G = H.conj().T @ H + sigma2 * np.eye(K)
    G = 0.5 * (G + G.conj().T)
    return G.astype(dtype)


def diag_dominant(n: int, seed: int, complex_: bool = False, dtype=None, margin: float = 1.0):
    """Hermitian, strictly diagonally dominant, positive diagonal: off-diagonal
    entries uniform in [-1, 1) (real and imaginary parts), a_ii = sum_j |a_ij|
    + margin.  Such a matrix is positive definite."""
    g = rng(seed)
    E = g.uniform(-1.0, 1.0, (n, n))
    if complex_:
        E = E + 1j * g.uniform(-1.0, 1.0, (n, n))
    E = 0.5 * (E + E.conj().T)
    np.fill_diagonal(E, 0.0)
    A = E + np.diag(np.abs(E).sum(axis=1) + margin)
    if dtype is None:
        dtype = np.complex128 if complex_ else np.float64
    return A.astype(dtype)


def ragged_batch(sizes, seed: int, lo: float = 1.0, hi: float = 100.0,
                 complex_: bool = True, dtype=np.complex64):
    """A batch of HPD/SPD matrices of the given sizes (test helper)."""
    mats = [dense_spd(int(k), lo, hi, seed * 1000 + i, complex_=complex_, dtype=dtype)
            for i, k in enumerate(sizes)]
    packed, offsets, sizes_a = pack_batch(mats, dtype)
    return packed, offsets, sizes_a, mats


def serving_pool(count: int, seed: int = 5, n_lo: int = 32, n_hi: int = 4096,
                 cond_lo: float = 10.0, cond_hi: float = 1e4):
    """Request pool for the serving stream.

    Each entry: N = round(exp U[ln n_lo, ln n_hi]), cond = exp U[ln cond_lo,
    ln cond_hi], real FP32 SPD or complex64 HPD with probability 1/2,
    tolerance 1e-4 or 1e-8 with probability 1/2 (the split is not given
    anywhere; 50/50 is our choice).  Matrices are built lazily: the pool
    holds their parameters and seeds, ``build`` materialises one.
    """
    g = rng(seed)
    ns = np.rint(np.exp(g.uniform(np.log(n_lo), np.log(n_hi), count))).astype(np.int64)
    conds = np.exp(g.uniform(np.log(cond_lo), np.log(cond_hi), count))
    cplx = g.uniform(size=count) < 0.5
    tols = np.where(g.uniform(size=count) < 0.5, 1e-4, 1e-8)
    seeds = g.integers(1, 2**31 - 1, size=count)
    pool = []
    for i in range(count):
        pool.append({"n": int(ns[i]), "cond": float(conds[i]), "complex": bool(cplx[i]),
                     "tol": float(tols[i]), "seed": int(seeds[i])})
    return pool


def build_request(entry, device=None):
    """Materialise one serving-pool entry: log-uniform spectrum in [1, cond]."""
    dtype = np.complex64 if entry["complex"] else np.float32
    return dense_spd(entry["n"], 1.0, entry["cond"], entry["seed"], log_spectrum=True,
                     complex_=entry["complex"], dtype=dtype, device=device)


def laplacian_2d(nx: int, ny: int, shift: float = 0.5, dtype=np.float64):
    """CSR arrays of the 5-point Laplacian on an nx x ny grid (Dirichlet
    boundary, natural row-major ordering: node (i, j) is row i * ny + j) plus
    shift * I: diagonal 4 + shift, -1 for each grid neighbour.  Its
    eigenvalues are 4 + shift - 2 cos(pi p / (nx + 1)) - 2 cos(pi q / (ny + 1)),
    p = 1..nx, q = 1..ny, with eigenvectors sin(pi p (i+1) / (nx+1))
    sin(pi q (j+1) / (ny+1)).  Returns (indptr int32, indices int32, values)."""
    n = nx * ny
    i, j = np.divmod(np.arange(n, dtype=np.int64), ny)
    cols, vals = [], []
    for di, dj, v in ((-1, 0, -1.0), (0, -1, -1.0), (0, 0, 4.0 + shift), (0, 1, -1.0),
                      (1, 0, -1.0)):
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny)
        c = np.where(ok, ii * ny + jj, -1)
        cols.append(c)
        vals.append(np.where(ok, v, 0.0))
    C = np.stack(cols, axis=1)          # n x 5, columns already ascending
    V = np.stack(vals, axis=1)
    keep = C >= 0
    counts = keep.sum(axis=1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    indices = C[keep].astype(np.int32)
    values = V[keep].astype(dtype)
    return indptr.astype(np.int32), indices, values


def random_sparse_hpd(n: int, seed: int, deg_lo: int = 1, deg_hi: int = 32,
                      complex_: bool = False, dtype=None, margin: float = 1.0):
    """CSR arrays of a random Hermitian, strictly diagonally dominant sparse
    matrix with an uneven row-length mix: row r draws an off-diagonal count
    uniform in [deg_lo, deg_hi] and that many random columns with values
    uniform in [-1, 1) (+ i [-1, 1)); the pattern is symmetrised (conjugate
    values), and a_rr = sum of the row's |a_rc| + margin."""
    g = rng(seed)
    deg = g.integers(deg_lo, deg_hi + 1, size=n)
    rows = np.repeat(np.arange(n), deg)
    cols = g.integers(0, n, size=rows.size)
    v = g.uniform(-1.0, 1.0, rows.size)
    if complex_:
        v = v + 1j * g.uniform(-1.0, 1.0, rows.size)
    off = rows != cols
    rows, cols, v = rows[off], cols[off], v[off]
    # symmetrise: (r, c, v) and (c, r, conj v); duplicates are summed
    R = np.concatenate([rows, cols])
    Cc = np.concatenate([cols, rows])
    Vv = np.concatenate([v, np.conj(v)]) * 0.5
    key = R.astype(np.int64) * n + Cc
    order = np.argsort(key, kind="stable")
    key, Vv = key[order], Vv[order]
    uniq, start = np.unique(key, return_index=True)
    vals = np.add.reduceat(Vv, start) if key.size else Vv
    R, Cc = np.divmod(uniq, n)
    rowabs = np.zeros(n)
    np.add.at(rowabs, R, np.abs(vals))
    # insert the diagonal
    R = np.concatenate([R, np.arange(n)])
    Cc = np.concatenate([Cc, np.arange(n)])
    vals = np.concatenate([vals, (rowabs + margin).astype(vals.dtype)])
    key = R * n + Cc
    order = np.argsort(key, kind="stable")
    R, Cc, vals = R[order], Cc[order], vals[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, R + 1, 1)
    np.cumsum(indptr, out=indptr)
    if dtype is None:
        dtype = np.complex128 if complex_ else np.float64
    return indptr.astype(np.int32), Cc.astype(np.int32), vals.astype(dtype)


def csr_to_dense(indptr, indices, values, n: int) -> np.ndarray:
    """The dense n x n matrix of CSR arrays (duplicates summed)."""
    A = np.zeros((n, n), dtype=values.dtype)
    rows = np.repeat(np.arange(n), np.diff(indptr.astype(np.int64)))
    np.add.at(A, (rows, indices.astype(np.int64)), values)
    return A
