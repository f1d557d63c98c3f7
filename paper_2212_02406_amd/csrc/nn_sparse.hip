// nn_sparse.hip — sparse form of the Neumann / NN series applied to B
// (declared in nn.h as nn_solve_sparse).
//
// Algorithm 2 of the paper (arXiv 2212.02406), with Corollary 6 and the
// sparse-system passage after it, approximates the solution of W x = B by
// the Neumann series sum_{m<=T} P^m phi B, P = I - phi W, without storing
// any power of P; T = (L+1)^i - 1 terms are i NN nests of depth L applied to
// B (Corollary 2).  phi is a scalar (1 / Re Tr W, or Theta_2(k)) or the
// diagonal diag(W)^-1, so every application of P keeps W's sparsity.
//
// Device design: one fused kernel per term evaluates the series in Horner
// form, r_t = B - W x_t and x_{t+1} = x_t + phi r_t (CSR rows, dense
// row-major multi-vectors; G lanes per row, one lane per right-hand-side
// column), with the sums of w_r |r|^2 (w_r = |phi_r|) and |r|^2 fused as
// per-block partials.  A one-block check kernel turns the partials into the
// control residual in a fixed order and applies the stopping rules on the
// device; later steps see the stop flag and do nothing, and three rotating
// iterate buffers keep x_{t-1} and x_t intact, so the host only reads the
// control block every check_every terms.  The CSR structure is checked on the
// device before the first product.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr int kSpBlocks = 4096;  // most blocks of a step launch (grid-stride beyond)
// Rows a lane group of the step kernel carries at once: two for
// multi-vectors (measured 23-26% faster than one at 16 and 64 right-hand
// sides; four raised the VGPR count to 100 and lost occupancy), one for a
// single vector (one lane per row: more rows per lane cost occupancy).
constexpr int rows_in_flight(int g) { return g == 1 ? 1 : 2; }
constexpr size_t kAlign = 256;

struct SparseCtl {
  int32_t done, status, terms, result;  // result: buffer index of the returned x
  int32_t fixed, max_terms, steps, pad;
  double tol, c_prev, p_prev, c_ret, p_ret, bw, bp, pad2;
  double trace[NN_TRACE_MAX];
};

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

__device__ __forceinline__ void block_sum2(double& a, double& b, double* sa, double* sb) {
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sa[threadIdx.x] += sa[threadIdx.x + w];
      sb[threadIdx.x] += sb[threadIdx.x + w];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
}

// ---- CSR structure checks (per-block counts of violations) -----------------
__global__ void __launch_bounds__(256) csr_check_ptr(const int32_t* rp, int64_t n, int64_t nnz,
                                                     double* part) {
  __shared__ double sa[256], sb[256];
  double bad = 0.0, dummy = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r <= n;
       r += (int64_t)gridDim.x * 256) {
    const int64_t a = rp[r];
    if (a < 0 || a > nnz) bad += 1.0;
    if (r == 0 && a != 0) bad += 1.0;
    if (r == n && a != nnz) bad += 1.0;
    if (r < n && (int64_t)rp[r + 1] < a) bad += 1.0;
  }
  block_sum2(bad, dummy, sa, sb);
  if (threadIdx.x == 0) part[blockIdx.x] = bad;
}

__global__ void __launch_bounds__(256) csr_check_cols(const int32_t* ci, int64_t nnz, int64_t n,
                                                      double* part) {
  __shared__ double sa[256], sb[256];
  double bad = 0.0, dummy = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * 256) {
    const int64_t c = ci[j];
    if (c < 0 || c >= n) bad += 1.0;
  }
  block_sum2(bad, dummy, sa, sb);
  if (threadIdx.x == 0) part[blockIdx.x] = bad;
}

// out[b] = sum (op 0) or NaN-propagating min (op 1) of the values a block
// strides over (block b of the grid, fixed order): the first level of a
// reduction over long vectors, or the whole of it with one block.
__global__ void __launch_bounds__(256) reduce_one(const double* vals, int64_t count, int op,
                                                  double* out) {
  __shared__ double red[256];
  double acc = op == 0 ? 0.0 : INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const double v = vals[i];
    if (op == 0) acc += v;
    else acc = (isnan(acc) || isnan(v)) ? NAN : (v < acc ? v : acc);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = red[threadIdx.x], b = red[threadIdx.x + w];
      red[threadIdx.x] = op == 0 ? a + b : ((isnan(a) || isnan(b)) ? NAN : (a < b ? a : b));
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void norm_finish(const double* sumsq, double mult, double* out) {
  if (threadIdx.x == 0) out[0] = mult * sqrt(sumsq[0]);
}

// Two-level reduction of a long vector into out[0] (part: kSpBlocks scratch).
hipError_t reduce_long(const double* vals, int64_t count, int op, double* part, double* out,
                       hipStream_t s) {
  const int nb = (int)std::min<int64_t>((count + 255) / 256, kSpBlocks);
  hipLaunchKernelGGL(reduce_one, dim3(nb), dim3(256), 0, s, vals, count, op, part);
  hipLaunchKernelGGL(reduce_one, dim3(1), dim3(256), 0, s, part, (int64_t)nb, op, out);
  return hipGetLastError();
}

// Diagonal of W (duplicates summed): dre[r] = Re d_r, dab[r] = |d_r| (NaN if
// not finite); with dinv: dinv_r = 1 / d_r and wdiag_r = |1 / d_r|.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) csr_diag(const int32_t* rp, const int32_t* ci,
                                                const T* val, int64_t n, double* dre,
                                                double* dab, T* dinv, double* wdiag) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  double re = 0.0, im = 0.0;
  for (int64_t j = rp[r]; j < rp[r + 1]; ++j) {
    if ((int64_t)ci[j] == r) {
      if constexpr (CPLX) {
        re += (double)val[2 * j];
        im += (double)val[2 * j + 1];
      } else {
        re += (double)val[j];
      }
    }
  }
  dre[r] = re;
  const bool fin = isfinite(re) && isfinite(im);
  dab[r] = fin ? sqrt(re * re + im * im) : NAN;
  if (dinv) {
    const double m2 = re * re + im * im;
    if constexpr (CPLX) {
      dinv[2 * r] = (T)(re / m2);
      dinv[2 * r + 1] = (T)(-im / m2);
    } else {
      dinv[r] = (T)(1.0 / re);
    }
    wdiag[r] = 1.0 / sqrt(m2);
  }
}

// One power step on CSR: y = W (x / ||x||), rowsq[r] = |y_r|^2 (x, y FP64).
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) csr_power_step(const int32_t* rp, const int32_t* ci,
                                                      const T* val, int64_t n, const double* x,
                                                      const double* xnorm, double* y,
                                                      double* rowsq) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const double nv = xnorm[0];
  const double inv = nv > 0.0 ? 1.0 / nv : (nv == 0.0 ? 0.0 : NAN);
  double sr = 0.0, si = 0.0;
  for (int64_t j = rp[r]; j < rp[r + 1]; ++j) {
    const int64_t c = ci[j];
    if constexpr (CPLX) {
      const double ar = (double)val[2 * j], ai = (double)val[2 * j + 1];
      const double br = x[2 * c], bi = x[2 * c + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    } else {
      sr += (double)val[j] * x[c];
    }
  }
  sr *= inv;
  si *= inv;
  if constexpr (CPLX) {
    y[2 * r] = sr;
    y[2 * r + 1] = si;
  } else {
    y[r] = sr;
  }
  rowsq[r] = sr * sr + si * si;
}

__global__ void scal_ops(double* scal, int op, double k) {
  if (threadIdx.x != 0) return;
  if (op == 1) scal[0] = (k + 1.0) / k * scal[0];  // power: den = (k+1)/k ||W u_k||
  scal[1] = 1.0 / scal[0];                         // theta = 1 / den
}

// phi_r r for one element, phi a scalar (theta) or a per-row value (dinv).
template <typename T, bool CPLX>
__device__ __forceinline__ void phi_mul(const double* theta, const T* dinv, int64_t r, T ar,
                                        T ai, T& outr, T& outi) {
  if (dinv) {
    if constexpr (CPLX) {
      const T pr = dinv[2 * r], pi = dinv[2 * r + 1];
      outr = pr * ar - pi * ai;
      outi = pr * ai + pi * ar;
    } else {
      outr = dinv[r] * ar;
      outi = T(0);
    }
  } else {
    const T t = (T)theta[0];
    outr = t * ar;
    outi = t * ai;
  }
}

// x0 = phi B; per-block partials of sum w |B|^2 and sum |B|^2.
template <typename T, bool CPLX, int G>
__global__ void __launch_bounds__(256) sparse_init(int64_t n, int64_t nrhs, const T* B,
                                                   int64_t ldb, T* x0, int64_t ldx,
                                                   const double* theta, const T* dinv,
                                                   const double* wdiag, double* part) {
  __shared__ double sa[256], sb[256];
  constexpr int RPB = 256 / G;
  constexpr int C = CPLX ? 2 : 1;
  const int lane = threadIdx.x % G;
  double accw = 0.0, accp = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * RPB + threadIdx.x / G; r < n;
       r += (int64_t)gridDim.x * RPB) {
    const double w = wdiag ? wdiag[r] : 1.0;
    for (int64_t c = lane; c < nrhs; c += G) {
      const T br = B[(r * ldb + c) * C];
      const T bi = CPLX ? B[(r * ldb + c) * C + 1] : T(0);
      T xr, xi;
      phi_mul<T, CPLX>(theta, dinv, r, br, bi, xr, xi);
      x0[(r * ldx + c) * C] = xr;
      if constexpr (CPLX) x0[(r * ldx + c) * C + 1] = xi;
      const double m2 = (double)br * (double)br + (double)bi * (double)bi;
      accw += w * m2;
      accp += m2;
    }
  }
  block_sum2(accw, accp, sa, sb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = accw;
    part[2 * blockIdx.x + 1] = accp;
  }
}

__global__ void __launch_bounds__(256) ctl_init(SparseCtl* ctl, const double* part, int nblocks,
                                                int32_t fixed, int32_t max_terms, double tol) {
  __shared__ double sa[256], sb[256];
  double w = 0.0, p = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    w += part[2 * i];
    p += part[2 * i + 1];
  }
  block_sum2(w, p, sa, sb);
  if (threadIdx.x == 0) {
    ctl->done = 0;
    ctl->status = NN_OK;
    ctl->terms = 0;
    ctl->result = 0;
    ctl->fixed = fixed;
    ctl->max_terms = max_terms;
    ctl->steps = 0;
    ctl->tol = tol;
    ctl->c_prev = NAN;
    ctl->p_prev = NAN;
    ctl->c_ret = NAN;
    ctl->p_ret = NAN;
    ctl->bw = sqrt(w);
    ctl->bp = sqrt(p);
  }
}

// One term: r = B - W x (x = xin), xout = x + phi r (if update); partials of
// sum w |r|^2 and sum |r|^2.  Does nothing once the control block says done.
// A lane group of G lanes (one lane per right-hand-side column) carries U
// rows at once.  Every load is unconditional (rows past the end and entries
// past a row's end re-read an in-range entry with weight 0): with a select
// on a loaded value the compiler branches around the load and waits inside
// each branch, which serialises the gathers; branch-free, the U index/value
// loads and then the U x gathers are in flight together.
template <typename T, bool CPLX, int G>
__global__ void __launch_bounds__(256) sparse_step(const int32_t* rp, const int32_t* ci,
                                                   const T* val, int64_t n, int64_t nrhs,
                                                   const T* B, int64_t ldb, const T* xin,
                                                   int64_t ldxi, T* xout, int64_t ldxo,
                                                   const double* theta, const T* dinv,
                                                   const double* wdiag, double* part,
                                                   const SparseCtl* ctl, int update) {
  if (ctl->done) return;
  __shared__ double sa[256], sb[256];
  constexpr int RPB = 256 / G;
  constexpr int U = rows_in_flight(G);
  constexpr int C = CPLX ? 2 : 1;
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int32_t nlast = (int32_t)(n - 1);
  double accw = 0.0, accp = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * RPB * U; base < n;
       base += (int64_t)gridDim.x * RPB * U) {
    // rows past the end are clamped to the last row (loads stay in range and
    // unconditional) and masked out of the stores and sums
    int32_t j0[U], len[U];
    int maxlen = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = base + u * RPB + grp;
      const int32_t rc = r < n ? (int32_t)r : nlast;
      const int32_t a = rp[rc], b = rp[rc + 1];
      j0[u] = a;
      len[u] = r < n ? b - a : 0;
      maxlen = len[u] > maxlen ? len[u] : maxlen;
    }
    for (int64_t c = lane; c < nrhs; c += G) {
      T sr[U], si[U];
#pragma unroll
      for (int u = 0; u < U; ++u) sr[u] = si[u] = T(0);
      for (int k = 0; k < maxlen; ++k) {
        // a row shorter than k re-reads its own last entry, an empty row entry
        // 0 (maxlen > 0 implies nnz > 0) with weight 0
        int32_t col[U];
        T ar[U], ai[U], m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // an empty row reads entry 0 (its row_ptr may equal nnz)
          const int32_t j = len[u] > 0 ? j0[u] + (k < len[u] ? k : len[u] - 1) : 0;
          m[u] = k < len[u] ? T(1) : T(0);
          col[u] = ci[j];
          ar[u] = val[(int64_t)j * C];
          ai[u] = CPLX ? val[(int64_t)j * C + 1] : T(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t xo = ((int64_t)col[u] * ldxi + c) * C;
          const T xr = xin[xo];
          const T xi = CPLX ? xin[xo + 1] : T(0);
          const T a = m[u] * ar[u], b = m[u] * ai[u];
          sr[u] += a * xr - (CPLX ? b * xi : T(0));
          if constexpr (CPLX) si[u] += a * xi + b * xr;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = base + u * RPB + grp;
        const int64_t rc = r < n ? r : n - 1;
        const T rr = B[(rc * ldb + c) * C] - sr[u];
        const T ri = CPLX ? B[(rc * ldb + c) * C + 1] - si[u] : T(0);
        const double wr = wdiag ? wdiag[rc] : 1.0;
        if (r < n) {
          if (update) {
            T pr, pi;
            phi_mul<T, CPLX>(theta, dinv, r, rr, ri, pr, pi);
            xout[(r * ldxo + c) * C] = xin[(r * ldxi + c) * C] + pr;
            if constexpr (CPLX) xout[(r * ldxo + c) * C + 1] = xin[(r * ldxi + c) * C + 1] + pi;
          }
          const double m2 = (double)rr * (double)rr + (double)ri * (double)ri;
          accw += wr * m2;
          accp += m2;
        }
      }
    }
  }
  block_sum2(accw, accp, sa, sb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = accw;
    part[2 * blockIdx.x + 1] = accp;
  }
}

// The same term with V = 2 or 4 adjacent right-hand-side columns per lane
// (real types; nrhs and leading dimensions multiples of V, rows aligned to V
// elements): every x gather, B read and x store is one V-element vector
// access, so a wave moves V times the bytes per load instruction and the
// index and value loads are shared by V columns.  Loads stay unconditional
// as above.
template <typename T, int G, int V>
__global__ void __launch_bounds__(256) sparse_step2(const int32_t* rp, const int32_t* ci,
                                                    const T* val, int64_t n, int64_t nrhs,
                                                    const T* B, int64_t ldb, const T* xin,
                                                    int64_t ldxi, T* xout, int64_t ldxo,
                                                    const double* theta, const T* dinv,
                                                    const double* wdiag, double* part,
                                                    const SparseCtl* ctl, int update) {
  typedef T T2 __attribute__((ext_vector_type(V)));
  if (ctl->done) return;
  __shared__ double sa[256], sb[256];
  constexpr int RPB = 256 / G;
  constexpr int U = rows_in_flight(G);
  const int lane = threadIdx.x % G;
  const int grp = threadIdx.x / G;
  const int32_t nlast = (int32_t)(n - 1);
  double accw = 0.0, accp = 0.0;
  for (int64_t base = (int64_t)blockIdx.x * RPB * U; base < n;
       base += (int64_t)gridDim.x * RPB * U) {
    int32_t j0[U], len[U];
    int maxlen = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = base + u * RPB + grp;
      const int32_t rc = r < n ? (int32_t)r : nlast;
      const int32_t a = rp[rc], b = rp[rc + 1];
      j0[u] = a;
      len[u] = r < n ? b - a : 0;
      maxlen = len[u] > maxlen ? len[u] : maxlen;
    }
    for (int64_t c = V * lane; c < nrhs; c += V * G) {
      T2 sr[U];
#pragma unroll
      for (int u = 0; u < U; ++u) sr[u] = T2(T(0));
      for (int k = 0; k < maxlen; ++k) {
        int32_t col[U];
        T a[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // an empty row reads entry 0 (its row_ptr may equal nnz)
          const int32_t j = len[u] > 0 ? j0[u] + (k < len[u] ? k : len[u] - 1) : 0;
          col[u] = ci[j];
          a[u] = (k < len[u] ? T(1) : T(0)) * val[j];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const T2 x = *reinterpret_cast<const T2*>(&xin[(int64_t)col[u] * ldxi + c]);
          sr[u] += a[u] * x;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t r = base + u * RPB + grp;
        const int64_t rc = r < n ? r : n - 1;
        const T2 rr = *reinterpret_cast<const T2*>(&B[rc * ldb + c]) - sr[u];
        const double wr = wdiag ? wdiag[rc] : 1.0;
        if (r < n) {
          if (update) {
            T2 pv;
#pragma unroll
            for (int q = 0; q < V; ++q) {
              T pq, unused;
              phi_mul<T, false>(theta, dinv, r, rr[q], T(0), pq, unused);
              pv[q] = pq;
            }
            const T2 xv = *reinterpret_cast<const T2*>(&xin[r * ldxi + c]);
            *reinterpret_cast<T2*>(&xout[r * ldxo + c]) = xv + pv;
          }
#pragma unroll
          for (int q = 0; q < V; ++q) {
            const double mq = (double)rr[q] * (double)rr[q];
            accw += wr * mq;
            accp += mq;
          }
        }
      }
    }
  }
  block_sum2(accw, accp, sa, sb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = accw;
    part[2 * blockIdx.x + 1] = accp;
  }
}

// The stopping rules for term t, on the device (fixed order sums).
__global__ void __launch_bounds__(256) sparse_check(SparseCtl* ctl, const double* part,
                                                    int nblocks, int32_t t) {
  if (ctl->done) return;
  __shared__ double sa[256], sb[256];
  double w = 0.0, p = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) {
    w += part[2 * i];
    p += part[2 * i + 1];
  }
  block_sum2(w, p, sa, sb);
  if (threadIdx.x != 0) return;
  const double c = ctl->bw > 0.0 ? sqrt(w) / ctl->bw : 0.0;
  const double pl = ctl->bp > 0.0 ? sqrt(p) / ctl->bp : 0.0;
  if (t < NN_TRACE_MAX) ctl->trace[t] = c;
  ctl->steps = t + 1;
  int st = -100, terms = t, res = t % 3;
  double cr = c, pr = pl;
  if (ctl->fixed >= 0) {
    if (t == ctl->fixed) st = isfinite(c) ? NN_OK : NN_ERR_NONFINITE;
  } else if (!isfinite(c)) {
    st = NN_ERR_NONFINITE;
  } else if (c < ctl->tol) {
    st = NN_OK;
  } else if (t > 0 && c >= 1.0 && c > ctl->c_prev) {
    st = NN_ERR_DIVERGED;
  } else if (t > 0 && ctl->c_prev < 0.1 && c >= ctl->c_prev) {
    st = NN_STAGNATED;
    terms = t - 1;
    res = (t + 2) % 3;
    cr = ctl->c_prev;
    pr = ctl->p_prev;
  } else if (t == ctl->max_terms) {
    st = NN_NOT_CONVERGED;
  }
  if (st != -100) {
    ctl->status = st;
    ctl->terms = terms;
    ctl->result = res;
    ctl->c_ret = cr;
    ctl->p_ret = pr;
    ctl->done = 1;
  } else {
    ctl->c_prev = c;
    ctl->p_prev = pl;
  }
}

int lanes_for(int64_t nrhs) {
  int g = 1;
  while (g < 64 && g < nrhs) g <<= 1;
  return g;
}

struct SparseWs {
  SparseCtl* ctl;
  void* buf[2];
  void* dinv;
  double* wdiag;
  double* part;
  double* dre;
  double* dab;
  double* pa;
  double* pb;
  double* scal;  // [0] den, [1] theta, [8..] power norms
  size_t bytes;
};

SparseWs carve(void* base, int64_t n, int64_t nrhs, nn_dtype dt) {
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off += up(bytes);
    return p;
  };
  const size_t e = elem_size(dt);
  const int C = is_complex(dt) ? 2 : 1;
  SparseWs w;
  w.ctl = static_cast<SparseCtl*>(take(sizeof(SparseCtl)));
  w.buf[0] = take((size_t)n * nrhs * e);
  w.buf[1] = take((size_t)n * nrhs * e);
  w.dinv = take((size_t)n * e);
  w.wdiag = static_cast<double*>(take(sizeof(double) * n));
  w.part = static_cast<double*>(take(sizeof(double) * 2 * kSpBlocks));
  w.dre = static_cast<double*>(take(sizeof(double) * n));
  w.dab = static_cast<double*>(take(sizeof(double) * n));
  w.pa = static_cast<double*>(take(sizeof(double) * C * n));
  w.pb = static_cast<double*>(take(sizeof(double) * C * n));
  w.scal = static_cast<double*>(take(sizeof(double) * (8 + kPowerMaxK + 8)));
  w.bytes = off;
  return w;
}

bool valid_params(const nn_sparse_params* p) {
  if (!p || p->reserved != 0) return false;
  if (p->x0 != NN_X0_SCALED_IDENTITY && p->x0 != NN_X0_POWER_IDENTITY && p->x0 != NN_X0_JACOBI)
    return false;
  if (p->x0 == NN_X0_POWER_IDENTITY && (p->power_k < 1 || p->power_k > NN_POWER_MAX_K))
    return false;
  if (p->fixed_terms < -1 || p->fixed_terms > NN_SPARSE_MAX_TERMS) return false;
  if (p->fixed_terms == -1 &&
      (!(p->tol >= 0.0) || p->max_terms < 1 || p->max_terms > NN_SPARSE_MAX_TERMS ||
       p->check_every < 1 || p->check_every > 1024))
    return false;
  return true;
}

template <typename T, bool CPLX>
struct Launch {
  static hipError_t diag(const int32_t* rp, const int32_t* ci, const void* v, int64_t n,
                         const SparseWs& w, bool jacobi, hipStream_t s) {
    hipLaunchKernelGGL((csr_diag<T, CPLX>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       rp, ci, static_cast<const T*>(v), n, w.dre, w.dab,
                       jacobi ? static_cast<T*>(w.dinv) : nullptr, jacobi ? w.wdiag : nullptr);
    return hipGetLastError();
  }
  static hipError_t power(const int32_t* rp, const int32_t* ci, const void* v, int64_t n, int k,
                          const SparseWs& w, hipStream_t s) {
    double* xa = w.pa;
    double* xb = w.pb;
    double* nrm = w.scal + 8;
    // ||.|| of an n-vector of squares: two-level sum, then the root
    auto norm = [&](double* out) {
      hipError_t e = reduce_long(w.dre, n, 0, w.part, w.scal + 2, s);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(norm_finish, dim3(1), dim3(64), 0, s, w.scal + 2, 1.0, out);
        e = hipGetLastError();
      }
      return e;
    };
    hipError_t e = launch_power_vector(CPLX, xa, w.dre, n, s);
    if (e == hipSuccess) e = norm(nrm);
    for (int j = 0; j <= k && e == hipSuccess; ++j) {
      hipLaunchKernelGGL((csr_power_step<T, CPLX>), dim3((unsigned)((n + 255) / 256)), dim3(256),
                         0, s, rp, ci, static_cast<const T*>(v), n, xa, nrm + j, xb, w.dre);
      e = norm(j == k ? w.scal : nrm + j + 1);
      std::swap(xa, xb);
    }
    return e;
  }
  template <int G>
  static hipError_t init_g(int64_t n, int64_t nrhs, const void* B, int64_t ldb, void* x0,
                           int64_t ldx, const double* theta, const void* dinv,
                           const double* wdiag, double* part, int nb, hipStream_t s) {
    hipLaunchKernelGGL((sparse_init<T, CPLX, G>), dim3(nb), dim3(256), 0, s, n, nrhs,
                       static_cast<const T*>(B), ldb, static_cast<T*>(x0), ldx, theta,
                       static_cast<const T*>(dinv), wdiag, part);
    return hipGetLastError();
  }
  template <int G>
  static hipError_t step_g(const int32_t* rp, const int32_t* ci, const void* v, int64_t n,
                           int64_t nrhs, const void* B, int64_t ldb, const void* xin,
                           int64_t ldxi, void* xout, int64_t ldxo, const double* theta,
                           const void* dinv, const double* wdiag, double* part,
                           const SparseCtl* ctl, int update, int nb, hipStream_t s) {
    hipLaunchKernelGGL((sparse_step<T, CPLX, G>), dim3(nb), dim3(256), 0, s, rp, ci,
                       static_cast<const T*>(v), n, nrhs, static_cast<const T*>(B), ldb,
                       static_cast<const T*>(xin), ldxi, static_cast<T*>(xout), ldxo, theta,
                       static_cast<const T*>(dinv), wdiag, part, ctl, update);
    return hipGetLastError();
  }
  template <int G, int V>
  static hipError_t step2_g(const int32_t* rp, const int32_t* ci, const void* v, int64_t n,
                            int64_t nrhs, const void* B, int64_t ldb, const void* xin,
                            int64_t ldxi, void* xout, int64_t ldxo, const double* theta,
                            const void* dinv, const double* wdiag, double* part,
                            const SparseCtl* ctl, int update, int nb, hipStream_t s) {
    hipLaunchKernelGGL((sparse_step2<T, G, V>), dim3(nb), dim3(256), 0, s, rp, ci,
                       static_cast<const T*>(v), n, nrhs, static_cast<const T*>(B), ldb,
                       static_cast<const T*>(xin), ldxi, static_cast<T*>(xout), ldxo, theta,
                       static_cast<const T*>(dinv), wdiag, part, ctl, update);
    return hipGetLastError();
  }
};

#define NN_SP_G(G_, CALL) \
  case G_:                \
    return CALL<G_>

template <typename T, bool CPLX>
hipError_t launch_init(int g, int64_t n, int64_t nrhs, const void* B, int64_t ldb, void* x0,
                       int64_t ldx, const double* theta, const void* dinv, const double* wdiag,
                       double* part, int nb, hipStream_t s) {
  using L = Launch<T, CPLX>;
  switch (g) {
    NN_SP_G(1, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(2, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(4, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(8, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(16, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(32, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
    NN_SP_G(64, L::template init_g)(n, nrhs, B, ldb, x0, ldx, theta, dinv, wdiag, part, nb, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, bool CPLX>
hipError_t launch_step(int vec, int g, const int32_t* rp, const int32_t* ci, const void* v,
                       int64_t n, int64_t nrhs, const void* B, int64_t ldb, const void* xin,
                       int64_t ldxi, void* xout, int64_t ldxo, const double* theta,
                       const void* dinv, const double* wdiag, double* part,
                       const SparseCtl* ctl, int update, int nb, hipStream_t s) {
  using L = Launch<T, CPLX>;
#define NN_SP_STEP_ARGS \
  rp, ci, v, n, nrhs, B, ldb, xin, ldxi, xout, ldxo, theta, dinv, wdiag, part, ctl, update, nb, s
#define NN_SP_GV(G_, V_) \
  case G_:               \
    return L::template step2_g<G_, V_>(NN_SP_STEP_ARGS)
  if constexpr (!CPLX) {
    if (vec == 2) {
      switch (g) {
        NN_SP_GV(1, 2); NN_SP_GV(2, 2); NN_SP_GV(4, 2); NN_SP_GV(8, 2);
        NN_SP_GV(16, 2); NN_SP_GV(32, 2); NN_SP_GV(64, 2);
      }
      return hipErrorInvalidValue;
    }
    if (vec == 4) {
      switch (g) {
        NN_SP_GV(1, 4); NN_SP_GV(2, 4); NN_SP_GV(4, 4); NN_SP_GV(8, 4);
        NN_SP_GV(16, 4); NN_SP_GV(32, 4); NN_SP_GV(64, 4);
      }
      return hipErrorInvalidValue;
    }
  }
#undef NN_SP_GV
  if (vec != 1) return hipErrorInvalidValue;
  switch (g) {
    NN_SP_G(1, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(2, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(4, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(8, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(16, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(32, L::template step_g)(NN_SP_STEP_ARGS);
    NN_SP_G(64, L::template step_g)(NN_SP_STEP_ARGS);
  }
#undef NN_SP_STEP_ARGS
  return hipErrorInvalidValue;
}

// Type dispatch of the three pieces.
struct Ops {
  nn_dtype dt;
  hipError_t diag(const int32_t* rp, const int32_t* ci, const void* v, int64_t n,
                  const SparseWs& w, bool jac, hipStream_t s) const {
    switch (dt) {
      case NN_F64: return Launch<double, false>::diag(rp, ci, v, n, w, jac, s);
      case NN_F32: return Launch<float, false>::diag(rp, ci, v, n, w, jac, s);
      case NN_C128: return Launch<double, true>::diag(rp, ci, v, n, w, jac, s);
      case NN_C64: return Launch<float, true>::diag(rp, ci, v, n, w, jac, s);
    }
    return hipErrorInvalidValue;
  }
  hipError_t power(const int32_t* rp, const int32_t* ci, const void* v, int64_t n, int k,
                   const SparseWs& w, hipStream_t s) const {
    switch (dt) {
      case NN_F64: return Launch<double, false>::power(rp, ci, v, n, k, w, s);
      case NN_F32: return Launch<float, false>::power(rp, ci, v, n, k, w, s);
      case NN_C128: return Launch<double, true>::power(rp, ci, v, n, k, w, s);
      case NN_C64: return Launch<float, true>::power(rp, ci, v, n, k, w, s);
    }
    return hipErrorInvalidValue;
  }
  template <typename... A>
  hipError_t init(A... a) const {
    switch (dt) {
      case NN_F64: return launch_init<double, false>(a...);
      case NN_F32: return launch_init<float, false>(a...);
      case NN_C128: return launch_init<double, true>(a...);
      case NN_C64: return launch_init<float, true>(a...);
    }
    return hipErrorInvalidValue;
  }
  template <typename... A>
  hipError_t step(A... a) const {
    switch (dt) {
      case NN_F64: return launch_step<double, false>(a...);
      case NN_F32: return launch_step<float, false>(a...);
      case NN_C128: return launch_step<double, true>(a...);
      case NN_C64: return launch_step<float, true>(a...);
    }
    return hipErrorInvalidValue;
  }
};

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return NN_ERR_HIP; \
  } while (0)

}  // namespace
}  // namespace nn

using namespace nn;

extern "C" {

size_t nn_solve_sparse_workspace_size(int64_t n, int64_t nrhs, nn_dtype dt,
                                      const nn_sparse_params* prm) {
  if (n < 1 || nrhs < 1 || dt < NN_F64 || dt > NN_C128 || !valid_params(prm)) return 0;
  return carve(nullptr, n, nrhs, dt).bytes;
}

nn_status nn_solve_sparse(nn_ctx* ctx, const int32_t* row_ptr, const int32_t* col_idx,
                          const void* values, int64_t n, int64_t nnz, const void* B, int64_t ldb,
                          void* Xsol, int64_t ldx, int64_t nrhs, nn_dtype dt,
                          const nn_sparse_params* prm, void* ws, size_t ws_bytes, nn_info* info,
                          double* rel_residual) {
  if (!ctx || !row_ptr || !B || !Xsol || n < 1 || nrhs < 1 || ldb < nrhs || ldx < nrhs)
    return NN_ERR_ARG;
  if (nnz < 0 || nnz > INT32_MAX || n > INT32_MAX || (nnz > 0 && (!col_idx || !values)))
    return NN_ERR_ARG;
  if (dt < NN_F64 || dt > NN_C128 || !valid_params(prm)) return NN_ERR_ARG;
  if (Xsol == B) return NN_ERR_ARG;
  const SparseWs w0 = carve(nullptr, n, nrhs, dt);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) || ws_bytes < w0.bytes)
    return NN_ERR_WORKSPACE;
  {
    const uintptr_t x = reinterpret_cast<uintptr_t>(Xsol), wb = reinterpret_cast<uintptr_t>(ws);
    const uintptr_t span = (uintptr_t)(((n - 1) * ldx + nrhs) * (int64_t)elem_size(dt));
    if (x < wb + w0.bytes && wb < x + span) return NN_ERR_ARG;
  }
  const uintptr_t addr = reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(Xsol) |
                         reinterpret_cast<uintptr_t>(values);
  if (addr % (elem_size(dt) / (is_complex(dt) ? 2 : 1))) return NN_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(row_ptr) | reinterpret_cast<uintptr_t>(col_idx)) & 3u)
    return NN_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  if (info) memset(info, 0, sizeof(*info));
  const SparseWs w = carve(ws, n, nrhs, dt);
  hipStream_t s = ctx->stream;
  const Ops ops{dt};
  // V = 2 columns per lane for real types when every row of B and of the
  // three iterate buffers starts on a two-element boundary, else 1.  V = 4
  // (NN_SPARSE_VEC=4) measured slower on the 2048^2 Laplacian with 16
  // right-hand sides: 0.564 against 0.522 ms per term.
  const size_t esz = (dt == NN_F64) ? 8 : 4;
  auto fits = [&](int v) {
    return (dt == NN_F64 || dt == NN_F32) && nrhs % v == 0 && ldb % v == 0 && ldx % v == 0 &&
           reinterpret_cast<uintptr_t>(B) % (v * esz) == 0 &&
           reinterpret_cast<uintptr_t>(Xsol) % (v * esz) == 0;
  };
  const char* vv = getenv("NN_SPARSE_VEC");  // 1, 2 or 4: the largest width tried
  const int vmax = vv ? atoi(vv) : 2;
  const int vec = (vmax >= 4 && fits(4)) ? 4 : (vmax >= 2 && fits(2)) ? 2 : 1;
  const int g = lanes_for(nrhs / vec);
  const int64_t rpb = 256 / g * rows_in_flight(g);  // rows per block and step iteration
  const int nb = (int)std::min<int64_t>((n + rpb - 1) / rpb, kSpBlocks);

  HIP_TRY(hipEventRecord(ctx->ev_start, s));
  // ---- CSR structure check (before any product reads through it) ----------
  {
    const int g1 = (int)std::min<int64_t>((n + 1 + 255) / 256, kSpBlocks);
    hipLaunchKernelGGL(csr_check_ptr, dim3(g1), dim3(256), 0, s, row_ptr, n, nnz, w.part);
    hipLaunchKernelGGL(reduce_one, dim3(1), dim3(256), 0, s, w.part, (int64_t)g1, 0, w.scal + 2);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(ctx->host, w.scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ctx->host[0] != 0.0) return NN_ERR_ARG;
    if (nnz > 0) {
      const int g2 = (int)std::min<int64_t>((nnz + 255) / 256, kSpBlocks);
      hipLaunchKernelGGL(csr_check_cols, dim3(g2), dim3(256), 0, s, col_idx, nnz, n, w.part);
      hipLaunchKernelGGL(reduce_one, dim3(1), dim3(256), 0, s, w.part, (int64_t)g2, 0,
                         w.scal + 2);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(ctx->host, w.scal + 2, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (ctx->host[0] != 0.0) return NN_ERR_ARG;
    }
  }
  // ---- phi: den in scal[0], theta = 1 / den in scal[1] (scalar starts) -----
  const bool jac = prm->x0 == NN_X0_JACOBI;
  if (prm->x0 == NN_X0_POWER_IDENTITY) {
    HIP_TRY(ops.power(row_ptr, col_idx, values, n, prm->power_k, w, s));
    hipLaunchKernelGGL(scal_ops, dim3(1), dim3(64), 0, s, w.scal, 1, (double)prm->power_k);
  } else {
    HIP_TRY(ops.diag(row_ptr, col_idx, values, n, w, jac, s));
    HIP_TRY(reduce_long(jac ? w.dab : w.dre, n, jac ? 1 : 0, w.part, w.scal, s));
    if (!jac) hipLaunchKernelGGL(scal_ops, dim3(1), dim3(64), 0, s, w.scal, 0, 0.0);
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(ctx->host, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double den = ctx->host[0];
  auto fail = [&](nn_status st) {
    (void)hipEventRecord(ctx->ev_stop, s);
    (void)hipEventSynchronize(ctx->ev_stop);
    if (info) info->status = st;
    if (rel_residual) *rel_residual = NAN;
    return st;
  };
  if (!isfinite(den)) return fail(NN_ERR_NONFINITE);
  if (den <= 0.0) return fail(NN_ERR_DIVERGED);
  const double* theta = jac ? nullptr : w.scal + 1;
  const void* dinv = jac ? w.dinv : nullptr;
  const double* wdiag = jac ? w.wdiag : nullptr;

  // ---- x_0 = phi B, ||B|| (weighted and plain), control block --------------
  void* buf[3] = {Xsol, w.buf[0], w.buf[1]};
  const int64_t ld[3] = {ldx, nrhs, nrhs};
  HIP_TRY(ops.init(g, n, nrhs, B, ldb, Xsol, ldx, theta, dinv, wdiag, w.part, nb, s));
  const bool fixed = prm->fixed_terms >= 0;
  hipLaunchKernelGGL(ctl_init, dim3(1), dim3(256), 0, s, w.ctl, w.part, nb,
                     fixed ? prm->fixed_terms : -1, prm->max_terms, prm->tol);
  HIP_TRY(hipGetLastError());

  // ---- the series, one fused step and one device-side check per term -------
  const int64_t last = fixed ? prm->fixed_terms : prm->max_terms;
  const int every = fixed ? INT32_MAX : prm->check_every;
  int64_t t = 0;
  for (;;) {
    int enq = 0;
    for (; t <= last && enq < every; ++t, ++enq) {
      const int i = (int)(t % 3), o = (int)((t + 1) % 3);
      HIP_TRY(ops.step(vec, g, row_ptr, col_idx, values, n, nrhs, B, ldb, buf[i], ld[i], buf[o],
                       ld[o], theta, dinv, wdiag, w.part, w.ctl, t < last ? 1 : 0, nb, s));
      hipLaunchKernelGGL(sparse_check, dim3(1), dim3(256), 0, s, w.ctl, w.part, nb, (int32_t)t);
      HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipMemcpyAsync(ctx->host, w.ctl, 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int32_t head[4];
    memcpy(head, ctx->host, sizeof(head));
    if (head[0] || t > last) break;
  }
  // ---- outcome --------------------------------------------------------------
  SparseCtl* hc = reinterpret_cast<SparseCtl*>(ctx->host);  // pinned slots: >= sizeof header
  static_assert(sizeof(SparseCtl) <= sizeof(double) * (NN_TRACE_MAX + 16),
                "control block must fit the context's read-back slots");
  HIP_TRY(hipMemcpyAsync(hc, w.ctl, sizeof(SparseCtl), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int res = hc->result;
  if (res != 0 && hc->done)
    HIP_TRY(hipMemcpy2DAsync(Xsol, (size_t)ldx * elem_size(dt), buf[res],
                             (size_t)ld[res] * elem_size(dt), (size_t)nrhs * elem_size(dt),
                             (size_t)n, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipEventRecord(ctx->ev_stop, s));
  HIP_TRY(hipEventSynchronize(ctx->ev_stop));
  const nn_status st = hc->done ? (nn_status)hc->status : NN_ERR_HIP;
  if (info) {
    info->status = st;
    info->iters = hc->terms;
    info->rms = hc->c_ret;
    info->gemms = hc->steps;
    const int nt = std::min<int>(hc->steps, NN_TRACE_MAX);
    info->n_trace = nt;
    for (int i = 0; i < nt; ++i) info->rms_trace[i] = hc->trace[i];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop) == hipSuccess) info->device_ms = ms;
  }
  if (rel_residual) *rel_residual = hc->p_ret;
  return st;
}

}  // extern "C"
