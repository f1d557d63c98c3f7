// nn_start.hip — start iterates X_0 of the NN iteration (gfx950).
//
// The normalisation of Sec. II-A asks for X_0 with ||I - A X_0||_2 < 1.
// Starts built here (den is the scale X_0 = M / den, left in scal[0]):
//   TRANSPOSE        M = A^H, den = ||A||_1 ||A||_inf
//   SCALED_IDENTITY  M = I,   den = Re Tr(A)                 (Theta_1)
//   TRANSPOSE_FROB   M = A^H, den = ||A||_F^2 = Tr(A^H A)    (the Theta of
//                    the normal-equation solve, Sec. II-D)
//   POWER_IDENTITY   M = I,   den = 1 / Theta_2(k) of W = A
//   POWER_TRANSPOSE  M = A^H, den = 1 / Theta_2(k) of W = A A^H
//   JACOBI           X_0 = diag(A)^-1; den = min_i |a_ii| flags a zero or
//                    non-finite diagonal (the diagonal preconditioner of the
//                    CNS discussion, Sec. II-D)
// Theta_2(k) = k ||W^k v|| / ((k + 1) ||W^(k+1) v||) (Sec. II-A, read with
// plain norms): k + 1 power steps u <- W u / ||W u|| from v / ||v||, the last
// norm being ||W^(k+1) v|| / ||W^k v||.  Each step is one or two HBM-bound
// matrix-vector products (one wave per row for A u; column sums over row
// chunks for A^H u) in FP64 accumulation, norms by fixed-order reductions.
// The vector v is drawn from SplitMix64 (Steele, Lea and Flood, 2014),
// entry i being the (i+1)-th output from seed 0, top 53 bits mapped to
// [-1, 1): a counter-based draw any implementation reproduces.
#include <math.h>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr int kChunk = 256;  // rows per column-sum chunk

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ uint64_t splitmix64_out(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// 1 / ||u|| for a stored norm: 0 for a zero vector (the estimate then
// collapses to den = 0, DIVERGED), NaN for a non-finite one.
__device__ __forceinline__ double inv_norm(const double* nrm) {
  if (!nrm) return 1.0;
  const double v = nrm[0];
  return v > 0.0 ? 1.0 / v : (v == 0.0 ? 0.0 : NAN);
}

template <bool CPLX>
__global__ void __launch_bounds__(256) power_init(double* x, double* rowsq, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const uint64_t z = splitmix64_out((uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull);
  const double v = 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
  if constexpr (CPLX) {
    x[2 * i] = v;
    x[2 * i + 1] = 0.0;
  } else {
    x[i] = v;
  }
  rowsq[i] = v * v;
}

// y = M (x / ||x||), one wave per row; rowsq[r] = |y_r|^2.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) gemv_rows(const T* M, int64_t ldm, const double* x,
                                                 const double* xnorm, double* y, double* rowsq,
                                                 int64_t n) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  double sr = 0.0, si = 0.0;
  if constexpr (CPLX) {
    const T* row = M + 2 * r * ldm;
    for (int64_t j = lane; j < n; j += 64) {
      const double ar = (double)row[2 * j], ai = (double)row[2 * j + 1];
      const double br = x[2 * j], bi = x[2 * j + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    si = wsum(si);
  } else {
    const T* row = M + r * ldm;
    for (int64_t j = lane; j < n; j += 64) sr += (double)row[j] * x[j];
  }
  sr = wsum(sr);
  const double inv = inv_norm(xnorm);
  sr *= inv;
  si *= inv;
  if (lane == 0) {
    if constexpr (CPLX) {
      y[2 * r] = sr;
      y[2 * r + 1] = si;
    } else {
      y[r] = sr;
    }
    rowsq[r] = sr * sr + si * si;
  }
}

// Column chunk sums of M^H (x / ||x||): colpart[chunk][c] = sum over the
// chunk's rows r of conj(M_rc) x_r / ||x||.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) gemv_cols(const T* M, int64_t ldm, const double* x,
                                                 const double* xnorm, double* colpart,
                                                 int64_t n) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * kChunk;
  if (c >= n) return;
  const int64_t r1 = r0 + kChunk < n ? r0 + kChunk : n;
  const double inv = inv_norm(xnorm);
  double sr = 0.0, si = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    if constexpr (CPLX) {
      const double ar = (double)M[2 * (r * ldm + c)], ai = -(double)M[2 * (r * ldm + c) + 1];
      const double br = x[2 * r], bi = x[2 * r + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    } else {
      sr += (double)M[r * ldm + c] * x[r];
    }
  }
  if constexpr (CPLX) {
    colpart[2 * ((int64_t)blockIdx.y * n + c)] = sr * inv;
    colpart[2 * ((int64_t)blockIdx.y * n + c) + 1] = si * inv;
  } else {
    colpart[(int64_t)blockIdx.y * n + c] = sr * inv;
  }
}

template <bool CPLX>
__global__ void __launch_bounds__(256) cols_finalize(const double* colpart, int nchunks, int64_t n,
                                                     double* y) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= n) return;
  constexpr int C = CPLX ? 2 : 1;
#pragma unroll
  for (int q = 0; q < C; ++q) {
    double s = 0.0;
    for (int k = 0; k < nchunks; ++k) s += colpart[((int64_t)k * n + c) * C + q];
    y[c * C + q] = s;
  }
}

// One block: out[0] = mult * sqrt(sum_i part[i]) in a fixed order.
__global__ void __launch_bounds__(256) norm_reduce(const double* part, int64_t count, double mult,
                                                   double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < count; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = mult * sqrt(red[0]);
}

__global__ void scal_square(double* scal) {
  if (threadIdx.x == 0) scal[0] = scal[0] * scal[0];
}

// scal[0] = min_i |a_ii|, NaN if any diagonal entry is not finite.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) diag_min_abs(const T* A, int64_t lda, int64_t n,
                                                    double* scal) {
  __shared__ double red[256];
  double m = INFINITY;
  bool bad = false;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    double a;
    if constexpr (CPLX) {
      const double re = (double)A[2 * (i * lda + i)], im = (double)A[2 * (i * lda + i) + 1];
      a = sqrt(re * re + im * im);
      if (!isfinite(re) || !isfinite(im)) bad = true;
    } else {
      a = fabs((double)A[i * lda + i]);
      if (!isfinite(a)) bad = true;
    }
    m = a < m ? a : m;
  }
  red[threadIdx.x] = bad ? NAN : m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = red[threadIdx.x], b = red[threadIdx.x + w];
      red[threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : (a < b ? a : b);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[0] = red[0];
}

// X = diag(A)^-1 (zero off the diagonal).
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) x0_jacobi_kernel(const T* A, int64_t lda, T* X,
                                                        int64_t ldx, int64_t n) {
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n;
       c += (int64_t)gridDim.x * 256) {
    if constexpr (CPLX) {
      T re = T(0), im = T(0);
      if (r == c) {
        const double ar = (double)A[2 * (r * lda + r)], ai = (double)A[2 * (r * lda + r) + 1];
        const double m2 = ar * ar + ai * ai;
        re = (T)(ar / m2);
        im = (T)(-ai / m2);
      }
      X[2 * (r * ldx + c)] = re;
      X[2 * (r * ldx + c) + 1] = im;
    } else {
      X[r * ldx + c] = (r == c) ? (T)(1.0 / (double)A[r * lda + r]) : T(0);
    }
  }
}

template <typename T, bool CPLX>
hipError_t power_den(bool transpose, int k, const void* Av, int64_t lda, int64_t n, double* pw,
                     double* scal, hipStream_t s) {
  const T* A = static_cast<const T*>(Av);
  constexpr int C = CPLX ? 2 : 1;
  const int nchunks = (int)((n + kChunk - 1) / kChunk);
  double* xa = pw;
  double* xb = pw + C * n;
  double* t = pw + 2 * C * n;
  double* rowsq = pw + 3 * C * n;
  double* nrm = rowsq + n;                   // k + 2 norms
  double* colpart = nrm + kPowerMaxK + 8;    // nchunks * C * n
  const unsigned gb = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL((power_init<CPLX>), dim3(gb), dim3(256), 0, s, xa, rowsq, n);
  hipLaunchKernelGGL(norm_reduce, dim3(1), dim3(256), 0, s, rowsq, n, 1.0, nrm);
  for (int j = 0; j <= k; ++j) {
    const double* xin = xa;
    const double* xn = nrm + j;
    if (transpose) {  // t = A^H (x / ||x||)
      hipLaunchKernelGGL((gemv_cols<T, CPLX>), dim3(gb, (unsigned)nchunks), dim3(256), 0, s, A,
                         lda, xa, nrm + j, colpart, n);
      hipLaunchKernelGGL((cols_finalize<CPLX>), dim3(gb), dim3(256), 0, s, colpart, nchunks, n, t);
      xin = t;
      xn = nullptr;
    }
    hipLaunchKernelGGL((gemv_rows<T, CPLX>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, A,
                       lda, xin, xn, xb, rowsq, n);
    // ||W u_j||; the last one becomes den = (k + 1) / k * ||W^(k+1) v|| / ||W^k v||
    const double mult = j == k ? (double)(k + 1) / (double)k : 1.0;
    hipLaunchKernelGGL(norm_reduce, dim3(1), dim3(256), 0, s, rowsq, n, mult,
                       j == k ? scal : nrm + j + 1);
    double* sw = xa;
    xa = xb;
    xb = sw;
  }
  return hipGetLastError();
}

template <typename T, bool CPLX>
hipError_t jacobi_start(const void* A, int64_t lda, void* X, int64_t ldx, int64_t n, double* scal,
                        hipStream_t s) {
  hipLaunchKernelGGL((diag_min_abs<T, CPLX>), dim3(1), dim3(256), 0, s,
                     static_cast<const T*>(A), lda, n, scal);
  const int gx = (int)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64);
  hipLaunchKernelGGL((x0_jacobi_kernel<T, CPLX>), dim3(gx, (unsigned)n), dim3(256), 0, s,
                     static_cast<const T*>(A), lda, static_cast<T*>(X), ldx, n);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_power_vector(bool cplx, double* x, double* rowsq, int64_t n, hipStream_t s) {
  const unsigned gb = (unsigned)((n + 255) / 256);
  if (cplx)
    hipLaunchKernelGGL((power_init<true>), dim3(gb), dim3(256), 0, s, x, rowsq, n);
  else
    hipLaunchKernelGGL((power_init<false>), dim3(gb), dim3(256), 0, s, x, rowsq, n);
  return hipGetLastError();
}

hipError_t launch_norm_reduce(const double* part, int64_t count, double mult, double* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(norm_reduce, dim3(1), dim3(256), 0, s, part, count, mult, out);
  return hipGetLastError();
}

size_t start_scratch_doubles(int64_t n) {
  const int64_t nchunks = (n + kChunk - 1) / kChunk;
  return (size_t)(7 * n + kPowerMaxK + 8 + nchunks * 2 * n + 256);
}

hipError_t launch_start(nn_dtype dt, int x0, int power_k, const void* A, int64_t lda, void* X,
                        int64_t ldx, int64_t n, double* denpart, double* pw, double* scal,
                        hipStream_t s) {
  const bool cplx = is_complex(dt), dbl = is_double(dt);
  hipError_t e = hipSuccess;
  switch (x0) {
    case NN_X0_TRANSPOSE:
      e = launch_den_transpose(dt, A, lda, n, denpart, scal, s);
      break;
    case NN_X0_SCALED_IDENTITY:
      e = launch_den_trace(dt, A, lda, n, scal, s);
      break;
    case NN_X0_TRANSPOSE_FROB: {
      const int64_t cm = cplx ? 2 : 1;
      e = launch_sumsq(A, dbl, cm * lda, n, cm * n, pw, scal, s);  // pw: >= 256 partials
      if (e == hipSuccess) {
        hipLaunchKernelGGL(scal_square, dim3(1), dim3(64), 0, s, scal);
        e = hipGetLastError();
      }
      break;
    }
    case NN_X0_POWER_IDENTITY:
    case NN_X0_POWER_TRANSPOSE: {
      const bool tr = x0 == NN_X0_POWER_TRANSPOSE;
      switch (dt) {
        case NN_F64: e = power_den<double, false>(tr, power_k, A, lda, n, pw, scal, s); break;
        case NN_F32: e = power_den<float, false>(tr, power_k, A, lda, n, pw, scal, s); break;
        case NN_C128: e = power_den<double, true>(tr, power_k, A, lda, n, pw, scal, s); break;
        case NN_C64: e = power_den<float, true>(tr, power_k, A, lda, n, pw, scal, s); break;
      }
      break;
    }
    case NN_X0_JACOBI:
      switch (dt) {
        case NN_F64: return jacobi_start<double, false>(A, lda, X, ldx, n, scal, s);
        case NN_F32: return jacobi_start<float, false>(A, lda, X, ldx, n, scal, s);
        case NN_C128: return jacobi_start<double, true>(A, lda, X, ldx, n, scal, s);
        case NN_C64: return jacobi_start<float, true>(A, lda, X, ldx, n, scal, s);
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  const bool transpose = x0 == NN_X0_TRANSPOSE || x0 == NN_X0_TRANSPOSE_FROB ||
                         x0 == NN_X0_POWER_TRANSPOSE;
  return transpose ? launch_x0_transpose(dt, A, lda, X, ldx, n, scal, s)
                   : launch_x0_identity(dt, X, ldx, n, scal, s);
}

}  // namespace nn
