// nn_factor.cpp — factorised Neumann-series solve (declared in nn.h).
//
// Corollary 6 of the paper (arXiv 2212.02406) factorises the truncated
// Neumann series sum_{n < 2^s} P^n phi, P = I - phi A, into
// prod_{n < s} (I + P^(2^n)) phi; applied to a right-hand side B it solves
// A x = B without forming the inverse:
//     y_0 = phi B,   y_{n+1} = y_n + P^(2^n) y_n,   P^(2^n) = (P^(2^(n-1)))^2.
// On the device every step is a GEMM of the NN chain (nn_gemm.hip): the
// residual B - A y with its fused per-tile sum of squares (relative residual
// from one fixed-order reduction), the n x n square when a factor is applied,
// and the n x nrhs factor with y as the epilogue addend.  Control follows the
// rules of nn_invert on the relative residual:
//   rel_s not finite                              -> NONFINITE
//   rel_s < tol                                   -> OK, y_s
//   s > 0, rel_s >= 1, rel_s > rel_{s-1}          -> DIVERGED
//   s > 0, rel_{s-1} < 0.1, rel_s >= rel_{s-1}    -> STAGNATED, y_{s-1}
//   s == max_iter                                 -> NOT_CONVERGED, y_s
#include <math.h>

#include <algorithm>
#include <utility>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxFactors = 62;
constexpr int kStats = NN_TRACE_MAX + 1;
constexpr int kSumsqParts = 256;  // partials the sum-of-squares kernel writes

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct FactorWs {
  void* phi = nullptr;
  void* p[2] = {nullptr, nullptr};  // P^(2^n) ping-pong
  void* yalt = nullptr;             // partner of Xsol
  void* r = nullptr;                // residual B - A y
  double* part = nullptr;
  double* denpart = nullptr;
  double* pw = nullptr;     // start-iterate scratch
  double* scal = nullptr;   // [0] den, [1] ||B||_F
  double* stats = nullptr;  // ||B - A y_s||_F per s
  void* work = nullptr;     // split-K partials of the thin products
  size_t bytes = 0;
};

FactorWs carve(void* base, int64_t n, int64_t nrhs, nn_dtype dt) {
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off += up(bytes);
    return p;
  };
  const size_t e = elem_size(dt);
  const int cm = is_complex(dt) ? 2 : 1;
  const Elem el = is_double(dt) ? Elem::F64 : Elem::F32;
  FactorWs w;
  w.phi = take((size_t)n * n * e);
  w.p[0] = take((size_t)n * n * e);
  w.p[1] = take((size_t)n * n * e);
  w.yalt = take((size_t)n * nrhs * e);
  w.r = take((size_t)n * nrhs * e);
  const GemmPlan pnr = plan_gemm_k(el, n, cm * nrhs, cm * n);
  const int tiles = std::max({pnr.num_tiles(), kSumsqParts, 1});
  w.part = static_cast<double*>(take(sizeof(double) * (size_t)tiles));
  w.denpart = static_cast<double*>(take(sizeof(double) * den_partials_elems(n)));
  w.pw = static_cast<double*>(take(sizeof(double) * start_scratch_doubles(n)));
  w.scal = static_cast<double*>(take(sizeof(double) * 8));
  w.stats = static_cast<double*>(take(sizeof(double) * kStats));
  const size_t wb = gemm_work_bytes(pnr, el, n, cm * nrhs);
  w.work = wb ? take(wb) : nullptr;
  w.bytes = off;
  return w;
}

nn_status check(const nn_params* p) {
  if (!p) return NN_ERR_ARG;
  if (p->x0 < NN_X0_TRANSPOSE || p->x0 > NN_X0_JACOBI) return NN_ERR_ARG;
  if (p->x0 == NN_X0_GIVEN) return NN_ERR_UNSUPPORTED;
  if ((p->x0 == NN_X0_POWER_IDENTITY || p->x0 == NN_X0_POWER_TRANSPOSE) &&
      (p->power_k < 1 || p->power_k > NN_POWER_MAX_K))
    return NN_ERR_ARG;
  if (p->fixed_iter < 0 || p->fixed_iter > kMaxFactors) return NN_ERR_ARG;
  if (p->fixed_iter == 0 && (!(p->tol >= 0.0) || p->max_iter < 1 || p->max_iter > kMaxFactors))
    return NN_ERR_ARG;
  if (p->prec != NN_PREC_PLAIN) return p->prec == NN_PREC_MIXED ? NN_ERR_UNSUPPORTED : NN_ERR_ARG;
  if (p->flags & ~NN_FLAG_TIME_GEMMS) return NN_ERR_ARG;
  return NN_OK;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return NN_ERR_HIP; \
  } while (0)

}  // namespace
}  // namespace nn

using namespace nn;

extern "C" {

size_t nn_solve_factorized_workspace_size(int64_t n, int64_t nrhs, nn_dtype dt,
                                          const nn_params* prm) {
  if (n < 1 || nrhs < 1 || dt < NN_F64 || dt > NN_C128 || check(prm) != NN_OK) return 0;
  return carve(nullptr, n, nrhs, dt).bytes;
}

nn_status nn_solve_factorized(nn_ctx* ctx, const void* A, int64_t lda, const void* B,
                              int64_t ldb, void* Xsol, int64_t ldx, int64_t n, int64_t nrhs,
                              nn_dtype dt, const nn_params* prm, void* ws, size_t ws_bytes,
                              nn_info* info, double* rel_residual) {
  if (!ctx || !A || !B || !Xsol || n < 1 || nrhs < 1 || lda < n || ldb < nrhs || ldx < nrhs)
    return NN_ERR_ARG;
  if (dt < NN_F64 || dt > NN_C128) return NN_ERR_ARG;
  const nn_status pc = check(prm);
  if (pc != NN_OK) return pc;
  if (Xsol == A || Xsol == B) return NN_ERR_ARG;
  const FactorWs w0 = carve(nullptr, n, nrhs, dt);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) || ws_bytes < w0.bytes)
    return NN_ERR_WORKSPACE;
  if (dt == NN_C128 && ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
                         reinterpret_cast<uintptr_t>(Xsol)) & 15u))
    return NN_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const FactorWs w = carve(ws, n, nrhs, dt);
  hipStream_t s = ctx->stream;
  const bool cplx = is_complex(dt);
  const Elem e = is_double(dt) ? Elem::F64 : Elem::F32;
  const int64_t cm = cplx ? 2 : 1;
  const int64_t nr = cm * n, rr = cm * nrhs;  // real extents
  const GemmPlan pnn = plan_gemm(e, n, nr), pnr = plan_gemm_k(e, n, rr, nr);
  const size_t esz = elem_size(dt);
  int gemms = 0;
  double trace[NN_TRACE_MAX];
  int n_trace = 0;
  auto finish = [&](nn_status st, int factors, double rel) {
    (void)hipEventRecord(ctx->ev_stop, s);
    (void)hipEventSynchronize(ctx->ev_stop);
    if (info) {
      info->status = st;
      info->iters = factors;
      info->rms = rel;
      info->gemms = gemms;
      for (int i = 0; i < 3; ++i) info->prec_gemms[i] = 0;
      info->prec_gemms[is_double(dt) ? 2 : 1] = gemms;
      info->gemm_ms = 0.f;
      info->n_trace = n_trace;
      for (int i = 0; i < n_trace; ++i) info->rms_trace[i] = trace[i];
      for (int i = 0; i < 3; ++i) info->phase_iters[i] = 0;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop) == hipSuccess) info->device_ms = ms;
    }
    if (rel_residual) *rel_residual = rel;
    return st;
  };

  HIP_TRY(hipEventRecord(ctx->ev_start, s));
  // phi (the start iterate) and its scale
  HIP_TRY(launch_start(dt, prm->x0, prm->power_k, A, lda, w.phi, n, n, w.denpart, w.pw, w.scal,
                       s));
  HIP_TRY(launch_sumsq(B, is_double(dt), cm * ldb, n, rr, w.part, w.scal + 1, s));
  HIP_TRY(hipMemcpyAsync(ctx->host, w.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double den = ctx->host[0], bnorm = ctx->host[1];
  if (!isfinite(den)) return finish(NN_ERR_NONFINITE, 0, NAN);
  if (den <= 0.0) return finish(NN_ERR_DIVERGED, 0, NAN);
  // P = I - phi A;  y_0 = phi B (in Xsol)
  {
    GemmArgs g{w.phi, nr, A, cm * lda, w.p[0], nr, nullptr, 0, n, nr, nr, -1.0, 1.0, nullptr};
    HIP_TRY(launch_gemm(e, cplx, pnn, g, s));
    GemmArgs h{w.phi, nr, B, cm * ldb, Xsol, cm * ldx, nullptr, 0, n, rr, nr, 1.0, 0.0, nullptr};
    h.work = w.work;
    HIP_TRY(launch_gemm(e, cplx, pnr, h, s));
    gemms += 2;
  }
  void* cur = Xsol;
  int64_t ld_cur = ldx;
  void* alt = w.yalt;
  int64_t ld_alt = nrhs;
  int pk = 0;  // P^(2^(s-1)) lives in p[pk] once a factor has been applied
  const bool fixed = prm->fixed_iter > 0;
  const double inv_b = bnorm > 0.0 ? 1.0 / bnorm : 0.0;
  nn_status st = NN_OK;
  int factors = 0;
  double rel_ret = NAN, rel_prev = NAN;
  bool use_alt = false;
  for (int k = 0;; ++k) {
    // residual of y_k: R = B - A y_k, ||R||_F into stats[k]
    GemmArgs r{A, cm * lda, cur, cm * ld_cur, w.r, rr, B, cm * ldb, n, rr, nr, -1.0, 0.0,
               w.part};
    r.work = w.work;
    HIP_TRY(launch_gemm(e, cplx, pnr, r, s));
    ++gemms;
    HIP_TRY(launch_rms_reduce(w.part, pnr.num_tiles(), 1, w.stats + std::min(k, kStats - 1), s));
    if (fixed) {
      if (k == prm->fixed_iter) {
        factors = k;
        break;
      }
    } else {
      HIP_TRY(hipMemcpyAsync(ctx->host + 2, w.stats + std::min(k, kStats - 1), sizeof(double),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double rel = ctx->host[2] * inv_b;
      if (n_trace < NN_TRACE_MAX) trace[n_trace++] = rel;
      factors = k;
      rel_ret = rel;
      if (!isfinite(rel)) { st = NN_ERR_NONFINITE; break; }
      if (rel < prm->tol) { st = NN_OK; break; }
      if (k > 0 && rel >= 1.0 && rel > rel_prev) { st = NN_ERR_DIVERGED; break; }
      if (k > 0 && rel_prev < 0.1 && rel >= rel_prev) {
        st = NN_STAGNATED;
        factors = k - 1;
        rel_ret = rel_prev;
        use_alt = true;
        break;
      }
      if (k == prm->max_iter) { st = NN_NOT_CONVERGED; break; }
      rel_prev = rel;
    }
    // factor k: P^(2^k) (a square of the previous power for k > 0), then
    // y_{k+1} = y_k + P^(2^k) y_k
    if (k > 0) {
      GemmArgs q{w.p[pk], nr, w.p[pk], nr, w.p[pk ^ 1], nr, nullptr, 0, n, nr, nr, 1.0, 0.0,
                 nullptr};
      HIP_TRY(launch_gemm(e, cplx, pnn, q, s));
      ++gemms;
      pk ^= 1;
    }
    GemmArgs u{w.p[pk], nr, cur, cm * ld_cur, alt, cm * ld_alt, cur, cm * ld_cur, n, rr, nr, 1.0,
               0.0, nullptr};
    u.work = w.work;
    HIP_TRY(launch_gemm(e, cplx, pnr, u, s));
    ++gemms;
    std::swap(cur, alt);
    std::swap(ld_cur, ld_alt);
  }
  void* res = use_alt ? alt : cur;
  const int64_t ld_res = use_alt ? ld_alt : ld_cur;
  if (res != Xsol)
    HIP_TRY(hipMemcpy2DAsync(Xsol, (size_t)ldx * esz, res, (size_t)ld_res * esz,
                             (size_t)nrhs * esz, (size_t)n, hipMemcpyDeviceToDevice, s));
  if (fixed) {
    const int cnt = std::min(prm->fixed_iter + 1, kStats);
    HIP_TRY(hipMemcpyAsync(ctx->host + 2, w.stats, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    n_trace = std::min(cnt, NN_TRACE_MAX);
    for (int i = 0; i < n_trace; ++i) trace[i] = ctx->host[2 + i] * inv_b;
    rel_ret = ctx->host[2 + cnt - 1] * inv_b;
    st = isfinite(rel_ret) ? NN_OK : NN_ERR_NONFINITE;
  }
  return finish(st, factors, rel_ret);
}

}  // extern "C"
