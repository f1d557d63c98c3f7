// nn_aux.hip — O(N^2) kernels around the NN GEMM chain (gfx950).
//
//  * start-iterate prologue: den = ||A||_1 ||A||_inf (transpose start) or
//    Re Tr(A) (identity start, the trace normalisation of Sec. II-A), then
//    X_0 = A^H / den or I / den;
//  * fixed-order reduction of the residual GEMM's per-tile partials into
//    rms = ||I - A X||_F / sqrt(N);
//  * element-wise casts used by the mixed-precision schedule.
// All sums are accumulated in FP64 in an order that depends only on the
// matrix size, never on timing, so results are bitwise reproducible.
#include <math.h>

#include "nn_internal.h"

namespace nn {
namespace {

template <typename T, bool CPLX>
__device__ __forceinline__ double absval(const T* A, int64_t idx) {
  if constexpr (CPLX) {
    const double re = (double)A[2 * idx], im = (double)A[2 * idx + 1];
    return sqrt(re * re + im * im);
  } else {
    return fabs((double)A[idx]);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per row: rowsum[r] = sum_j |a_rj|.
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) row_abs_sums(const T* A, int64_t lda, int64_t n,
                                                    double* rowsum) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < n; j += 64) s += absval<T, CPLX>(A, r * lda + j);
  s = wave_sum(s);
  if (lane == 0) rowsum[r] = s;
}

// Column partial sums over row chunks of col_chunk(n) rows: short chunks for
// small n, so the launch still has enough workgroups (at n = 256 one chunk of
// 256 rows was a single workgroup walking every row: 26 us of a 0.45 ms
// inversion).
__host__ __device__ inline int64_t col_chunk(int64_t n) {
  return n < 1024 ? 16 : n < 4096 ? 64 : 256;
}
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) col_abs_sums(const T* A, int64_t lda, int64_t n,
                                                    double* colpart) {
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t chunk = col_chunk(n);
  const int64_t r0 = (int64_t)blockIdx.y * chunk;
  if (c >= n) return;
  const int64_t r1 = (r0 + chunk < n) ? r0 + chunk : n;
  double s = 0.0;
  for (int64_t r = r0; r < r1; ++r) s += absval<T, CPLX>(A, r * lda + c);
  colpart[(int64_t)blockIdx.y * n + c] = s;
}

// One block: ||A||_1 = max_c sum_chunks colpart, ||A||_inf = max_r rowsum.
__global__ void __launch_bounds__(256) norms_finalize(const double* rowsum, const double* colpart,
                                                      int64_t n, int nchunks, double* scal) {
  __shared__ double m1[256], mi[256];
  double b1 = 0.0, bi = 0.0;
  bool bad = false;
  for (int64_t c = threadIdx.x; c < n; c += 256) {
    double s = 0.0;
    for (int k = 0; k < nchunks; ++k) s += colpart[(int64_t)k * n + c];
    if (!isfinite(s)) bad = true;
    b1 = s > b1 ? s : b1;
    const double t = rowsum[c];
    if (!isfinite(t)) bad = true;
    bi = t > bi ? t : bi;
  }
  m1[threadIdx.x] = bad ? NAN : b1;
  mi[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double a = m1[threadIdx.x], b = m1[threadIdx.x + w];
      m1[threadIdx.x] = (isnan(a) || isnan(b)) ? NAN : (a > b ? a : b);
      const double c = mi[threadIdx.x], d = mi[threadIdx.x + w];
      mi[threadIdx.x] = c > d ? c : d;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[0] = m1[0] * mi[0];
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) trace_kernel(const T* A, int64_t lda, int64_t n,
                                                    double* scal) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256)
    s += CPLX ? (double)A[2 * (i * lda + i)] : (double)A[i * lda + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) scal[0] = red[0];
}

// X = A^H / den, through a 32 x 32 LDS tile (coalesced on both sides).
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) x0_transpose_kernel(const T* A, int64_t lda, T* X,
                                                           int64_t ldx, int64_t n,
                                                           const double* scal) {
  constexpr int C = CPLX ? 2 : 1;
  __shared__ T tile[32][33 * C];
  const double den = scal[0];
  const T s = (T)(1.0 / den);
  const int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = by + k, c = bx + tx;  // read A[r][c]
    if (r < n && c < n) {
#pragma unroll
      for (int q = 0; q < C; ++q) tile[k][tx * C + q] = A[(r * lda + c) * C + q];
    }
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int64_t r = bx + k, c = by + tx;  // write X[r][c] = conj(A[c][r]) * s
    if (r < n && c < n) {
      if constexpr (CPLX) {
        X[(r * ldx + c) * 2] = tile[tx][k * 2] * s;
        X[(r * ldx + c) * 2 + 1] = -tile[tx][k * 2 + 1] * s;
      } else {
        X[r * ldx + c] = tile[tx][k] * s;
      }
    }
  }
}

template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) x0_identity_kernel(T* X, int64_t ldx, int64_t n,
                                                          const double* scal) {
  const T s = (T)(1.0 / scal[0]);
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < n; c += (int64_t)gridDim.x * 256) {
    if constexpr (CPLX) {
      X[(r * ldx + c) * 2] = (r == c) ? s : T(0);
      X[(r * ldx + c) * 2 + 1] = T(0);
    } else {
      X[r * ldx + c] = (r == c) ? s : T(0);
    }
  }
}

__global__ void __launch_bounds__(256) rms_reduce_kernel(const double* part, int count,
                                                         double inv_rows, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sqrt(red[0] * inv_rows);
}

// The rms of one residual as rms_reduce_kernel computes it (same order, same
// bits), then the stopping rules of the tolerance mode for nest index k, in
// the host loop's order; a set `done` makes the whole kernel a no-op.
__global__ void __launch_bounds__(256) rms_control_kernel(const double* part, int count,
                                                          double inv_rows, double* out,
                                                          DevCtl* ctl, int k, double tol,
                                                          int max_iter, double sqrtn) {
  if (ctl->done) return;
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < count; i += 256) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double rms = sqrt(red[0] * inv_rows);
  out[0] = rms;
  const double prev = ctl->rms_prev;
  int st = -100;  // no rule fired
  int iters = k;
  double ret = rms;
  if (!isfinite(rms)) st = NN_ERR_NONFINITE;
  else if (rms < tol) st = NN_OK;
  else if (k > 0 && rms >= 1.0 && rms > prev) st = NN_ERR_DIVERGED;
  else if (k > 0 && sqrtn * prev < 0.1 && rms >= prev) {
    st = NN_STAGNATED;
    iters = k - 1;
    ret = prev;
  } else if (k == max_iter) st = NN_NOT_CONVERGED;
  ctl->last_k = k;
  if (st == -100) {
    ctl->rms_prev = rms;
    return;
  }
  ctl->status = st;
  ctl->iters = iters;
  ctl->rms_ret = ret;
  ctl->done = 1;
}

// den (may be null): the start scale; not finite -> NONFINITE, <= 0 ->
// DIVERGED before any nest, as the host loop tests it.
__global__ void ctl_init_kernel(DevCtl* ctl, const double* den) {
  int st = NN_OK, done = 0;
  if (den) {
    const double v = den[0];
    if (!isfinite(v)) st = NN_ERR_NONFINITE, done = 1;
    else if (v <= 0.0) st = NN_ERR_DIVERGED, done = 1;
  }
  ctl->done = done;
  ctl->status = st;
  ctl->iters = 0;
  ctl->last_k = -1;
  ctl->rms_prev = __builtin_nan("");
  ctl->rms_ret = __builtin_nan("");
}

constexpr int kSumsqBlocks = 256;
template <typename T>
__global__ void __launch_bounds__(256) sumsq_kernel(const T* src, int64_t ld, int64_t rows,
                                                    int64_t cols, double* part) {
  __shared__ double red[256];
  double s = 0.0;
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t r = e / cols, c = e - r * cols;
    const double v = (double)src[r * ld + c];
    s += v * v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Round to nearest even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <typename S, typename D>
__device__ __forceinline__ D convert(S v);
template <>
__device__ __forceinline__ float convert<double, float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ double convert<float, double>(float v) { return (double)v; }
template <>
__device__ __forceinline__ uint16_t convert<double, uint16_t>(double v) {
  return f32_to_bf16((float)v);
}
template <>
__device__ __forceinline__ uint16_t convert<float, uint16_t>(float v) { return f32_to_bf16(v); }

template <typename S, typename D>
__global__ void __launch_bounds__(256) cast_kernel(const S* src, int64_t lds, D* dst, int64_t ldd,
                                                   int64_t rows, int64_t cols) {
  const int64_t r = blockIdx.y;
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < cols;
       c += (int64_t)gridDim.x * 256)
    dst[r * ldd + c] = convert<S, D>(src[r * lds + c]);
}

template <typename S, typename D>
hipError_t launch_cast(const S* src, int64_t lds, D* dst, int64_t ldd, int64_t rows, int64_t cols,
                       hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const int gx = (int)((cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64);
  hipLaunchKernelGGL((cast_kernel<S, D>), dim3(gx, (unsigned)rows), dim3(256), 0, s, src, lds, dst,
                     ldd, rows, cols);
  return hipGetLastError();
}

template <typename T, bool CPLX>
hipError_t den_transpose_t(const void* A, int64_t lda, int64_t n, double* part, double* scal,
                           hipStream_t s) {
  const T* a = static_cast<const T*>(A);
  double* rowsum = part;
  double* colpart = part + n;
  const int nchunks = (int)((n + col_chunk(n) - 1) / col_chunk(n));
  hipLaunchKernelGGL((row_abs_sums<T, CPLX>), dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, a,
                     lda, n, rowsum);
  hipLaunchKernelGGL((col_abs_sums<T, CPLX>), dim3((unsigned)((n + 255) / 256), nchunks),
                     dim3(256), 0, s, a, lda, n, colpart);
  hipLaunchKernelGGL(norms_finalize, dim3(1), dim3(256), 0, s, rowsum, colpart, n, nchunks, scal);
  return hipGetLastError();
}

}  // namespace

size_t den_partials_elems(int64_t n) {
  return (size_t)n + (size_t)((n + col_chunk(n) - 1) / col_chunk(n)) * (size_t)n;
}

hipError_t launch_den_transpose(nn_dtype dt, const void* A, int64_t lda, int64_t n, double* part,
                                double* scal, hipStream_t s) {
  switch (dt) {
    case NN_F64: return den_transpose_t<double, false>(A, lda, n, part, scal, s);
    case NN_F32: return den_transpose_t<float, false>(A, lda, n, part, scal, s);
    case NN_C128: return den_transpose_t<double, true>(A, lda, n, part, scal, s);
    case NN_C64: return den_transpose_t<float, true>(A, lda, n, part, scal, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_den_trace(nn_dtype dt, const void* A, int64_t lda, int64_t n, double* scal,
                            hipStream_t s) {
  switch (dt) {
    case NN_F64:
      hipLaunchKernelGGL((trace_kernel<double, false>), dim3(1), dim3(256), 0, s,
                         static_cast<const double*>(A), lda, n, scal);
      break;
    case NN_F32:
      hipLaunchKernelGGL((trace_kernel<float, false>), dim3(1), dim3(256), 0, s,
                         static_cast<const float*>(A), lda, n, scal);
      break;
    case NN_C128:
      hipLaunchKernelGGL((trace_kernel<double, true>), dim3(1), dim3(256), 0, s,
                         static_cast<const double*>(A), lda, n, scal);
      break;
    case NN_C64:
      hipLaunchKernelGGL((trace_kernel<float, true>), dim3(1), dim3(256), 0, s,
                         static_cast<const float*>(A), lda, n, scal);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_x0_transpose(nn_dtype dt, const void* A, int64_t lda, void* X, int64_t ldx,
                               int64_t n, const double* scal, hipStream_t s) {
  const dim3 grid((unsigned)((n + 31) / 32), (unsigned)((n + 31) / 32));
  switch (dt) {
    case NN_F64:
      hipLaunchKernelGGL((x0_transpose_kernel<double, false>), grid, dim3(256), 0, s,
                         static_cast<const double*>(A), lda, static_cast<double*>(X), ldx, n, scal);
      break;
    case NN_F32:
      hipLaunchKernelGGL((x0_transpose_kernel<float, false>), grid, dim3(256), 0, s,
                         static_cast<const float*>(A), lda, static_cast<float*>(X), ldx, n, scal);
      break;
    case NN_C128:
      hipLaunchKernelGGL((x0_transpose_kernel<double, true>), grid, dim3(256), 0, s,
                         static_cast<const double*>(A), lda, static_cast<double*>(X), ldx, n, scal);
      break;
    case NN_C64:
      hipLaunchKernelGGL((x0_transpose_kernel<float, true>), grid, dim3(256), 0, s,
                         static_cast<const float*>(A), lda, static_cast<float*>(X), ldx, n, scal);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_x0_identity(nn_dtype dt, void* X, int64_t ldx, int64_t n, const double* scal,
                              hipStream_t s) {
  const int gx = (int)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64);
  const dim3 grid(gx, (unsigned)n);
  switch (dt) {
    case NN_F64:
      hipLaunchKernelGGL((x0_identity_kernel<double, false>), grid, dim3(256), 0, s,
                         static_cast<double*>(X), ldx, n, scal);
      break;
    case NN_F32:
      hipLaunchKernelGGL((x0_identity_kernel<float, false>), grid, dim3(256), 0, s,
                         static_cast<float*>(X), ldx, n, scal);
      break;
    case NN_C128:
      hipLaunchKernelGGL((x0_identity_kernel<double, true>), grid, dim3(256), 0, s,
                         static_cast<double*>(X), ldx, n, scal);
      break;
    case NN_C64:
      hipLaunchKernelGGL((x0_identity_kernel<float, true>), grid, dim3(256), 0, s,
                         static_cast<float*>(X), ldx, n, scal);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_rms_reduce(const double* partials, int count, int64_t n_rows, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(rms_reduce_kernel, dim3(1), dim3(256), 0, s, partials, count,
                     1.0 / (double)n_rows, out);
  return hipGetLastError();
}

hipError_t launch_ctl_init(DevCtl* ctl, const double* den, hipStream_t s) {
  hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(1), 0, s, ctl, den);
  return hipGetLastError();
}

hipError_t launch_rms_control(const double* partials, int count, int64_t n_rows, double* out,
                              DevCtl* ctl, int k, double tol, int max_iter, hipStream_t s) {
  hipLaunchKernelGGL(rms_control_kernel, dim3(1), dim3(256), 0, s, partials, count,
                     1.0 / (double)n_rows, out, ctl, k, tol, max_iter, sqrt((double)n_rows));
  return hipGetLastError();
}

hipError_t launch_sumsq(const void* src, bool f64, int64_t ld, int64_t rows, int64_t cols,
                        double* part, double* out, hipStream_t s) {
  if (f64)
    hipLaunchKernelGGL((sumsq_kernel<double>), dim3(kSumsqBlocks), dim3(256), 0, s,
                       static_cast<const double*>(src), ld, rows, cols, part);
  else
    hipLaunchKernelGGL((sumsq_kernel<float>), dim3(kSumsqBlocks), dim3(256), 0, s,
                       static_cast<const float*>(src), ld, rows, cols, part);
  hipLaunchKernelGGL(rms_reduce_kernel, dim3(1), dim3(256), 0, s, part, kSumsqBlocks, 1.0, out);
  return hipGetLastError();
}

hipError_t launch_cast_f64_f32(const double* src, int64_t lds, float* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s) {
  return launch_cast<double, float>(src, lds, dst, ldd, rows, cols, s);
}
hipError_t launch_cast_f32_f64(const float* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t rows, int64_t cols, hipStream_t s) {
  return launch_cast<float, double>(src, lds, dst, ldd, rows, cols, s);
}
hipError_t launch_cast_f64_bf16(const double* src, int64_t lds, uint16_t* dst, int64_t ldd,
                                int64_t rows, int64_t cols, hipStream_t s) {
  return launch_cast<double, uint16_t>(src, lds, dst, ldd, rows, cols, s);
}
hipError_t launch_cast_f32_bf16(const float* src, int64_t lds, uint16_t* dst, int64_t ldd,
                                int64_t rows, int64_t cols, hipStream_t s) {
  return launch_cast<float, uint16_t>(src, lds, dst, ldd, rows, cols, s);
}

}  // namespace nn
