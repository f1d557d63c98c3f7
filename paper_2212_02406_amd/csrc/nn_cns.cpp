// nn_cns.cpp — Chebyshev-Neumann series solve (declared in nn.h).
//
// The CNS of the paper (arXiv 2212.02406, Sec. II-D, the CNS equation after
// Corollary 2) runs m NN nests for a preconditioner phi = X_m and then sums
// T + 1 terms of the Neumann series in Q = I - phi A applied to phi B:
//     x_T = sum_{k=0}^{T} Q^k phi B.
// Its Horner form x_{k+1} = Q x_k + phi B = x_k + phi (B - A x_k) is one
// refinement step per term, two n x n x nrhs products (the residual with its
// fused per-tile sum of squares, then the correction with x_k as the epilogue
// addend).  Q is never formed: every residual is recomputed from A, so the
// relative residual reaches the rounding level of one product rather than
// that of a formed Q.  The nests are nn_invert itself (plain or mixed), with
// phi kept at the head of the workspace for later calls on the same A.
// Control on rel_k = ||B - A x_k||_F / ||B||_F, tolerance mode:
//   rel_k not finite                              -> NONFINITE
//   rel_k < tol                                   -> OK, x_k
//   k > 0, rel_k >= 1, rel_k > rel_{k-1}          -> DIVERGED
//   k > 0, rel_{k-1} < 0.1, rel_k >= rel_{k-1}    -> STAGNATED, x_{k-1}
//   k == max_terms                                -> NOT_CONVERGED, x_k
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr size_t kAlign = 256;
constexpr int kStats = NN_TRACE_MAX + 1;
constexpr int kSumsqParts = 256;  // partials the sum-of-squares kernel writes

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct CnsWs {
  void* phi = nullptr;      // n x n, leading dimension n (kept across calls)
  void* inv_ws = nullptr;   // nn_invert's workspace
  size_t inv_bytes = 0;
  void* yalt = nullptr;     // partner of Xsol in the ping-pong
  void* r = nullptr;        // residual B - A y
  double* part = nullptr;   // per-tile partials
  double* scal = nullptr;   // [0] ||B||_F
  double* stats = nullptr;  // ||B - A y_k||_F per term
  void* work = nullptr;     // split-K partials of the thin products
  size_t bytes = 0;
};

bool valid_params(const nn_cns_params* p, nn_dtype dt) {
  if (!p || p->reserved != 0 || (p->reuse_phi != 0 && p->reuse_phi != 1)) return false;
  if (p->fixed_terms < -1 || p->fixed_terms > NN_CNS_MAX_TERMS) return false;
  if (p->fixed_terms == -1 &&
      (!(p->tol >= 0.0) || p->max_terms < 1 || p->max_terms > NN_CNS_MAX_TERMS))
    return false;
  if (p->precond.prec == NN_PREC_MIXED && dt != NN_F64) return false;
  return true;
}

// Layout (nullptr base: sizes only).  inv_bytes == 0 means the preconditioner
// parameters were rejected by nn_workspace_size.
CnsWs carve(void* base, int64_t n, int64_t nrhs, nn_dtype dt, const nn_params* pre) {
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
  CnsWs w;
  w.phi = take((size_t)n * n * e);
  w.inv_bytes = nn_workspace_size(n, dt, pre);
  w.inv_ws = take(w.inv_bytes);
  w.yalt = take((size_t)n * nrhs * e);
  w.r = take((size_t)n * nrhs * e);
  const GemmPlan pnr = plan_gemm_k(el, n, cm * nrhs, cm * n);
  const int tiles = std::max({pnr.num_tiles(), kSumsqParts, 1});
  w.part = static_cast<double*>(take(sizeof(double) * (size_t)tiles));
  w.scal = static_cast<double*>(take(sizeof(double) * 8));
  w.stats = static_cast<double*>(take(sizeof(double) * kStats));
  const size_t wb = gemm_work_bytes(pnr, el, n, cm * nrhs);
  w.work = wb ? take(wb) : nullptr;
  w.bytes = off;
  return w;
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

size_t nn_solve_cns_workspace_size(int64_t n, int64_t nrhs, nn_dtype dt,
                                   const nn_cns_params* prm) {
  if (n < 1 || nrhs < 1 || dt < NN_F64 || dt > NN_C128 || !valid_params(prm, dt)) return 0;
  const CnsWs w = carve(nullptr, n, nrhs, dt, &prm->precond);
  return w.inv_bytes ? w.bytes : 0;
}

nn_status nn_solve_cns(nn_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                       void* Xsol, int64_t ldx, int64_t n, int64_t nrhs, nn_dtype dt,
                       const nn_cns_params* prm, void* ws, size_t ws_bytes,
                       nn_info* precond_info, nn_info* info, double* rel_residual) {
  if (!ctx || !A || !B || !Xsol || n < 1 || nrhs < 1 || lda < n || ldb < nrhs || ldx < nrhs)
    return NN_ERR_ARG;
  if (dt < NN_F64 || dt > NN_C128) return NN_ERR_ARG;
  if (!valid_params(prm, dt)) return NN_ERR_ARG;
  if (Xsol == A || Xsol == B) return NN_ERR_ARG;
  const CnsWs w0 = carve(nullptr, n, nrhs, dt, &prm->precond);
  if (w0.inv_bytes == 0) return NN_ERR_ARG;  // preconditioner parameters rejected
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) || ws_bytes < w0.bytes)
    return NN_ERR_WORKSPACE;
  {
    // Xsol's span [x, x + ((n - 1) ldx + nrhs) elements) must miss the workspace
    const uintptr_t x = reinterpret_cast<uintptr_t>(Xsol), wb = reinterpret_cast<uintptr_t>(ws);
    const uintptr_t span = (uintptr_t)(((n - 1) * ldx + nrhs) * (int64_t)elem_size(dt));
    if (x < wb + w0.bytes && wb < x + span) return NN_ERR_ARG;
  }
  const uintptr_t addr = reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B) |
                         reinterpret_cast<uintptr_t>(Xsol);
  if (addr % (elem_size(dt) / (is_complex(dt) ? 2 : 1))) return NN_ERR_ARG;
  if (dt == NN_C128 && (addr & 15u)) return NN_ERR_ARG;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const CnsWs w = carve(ws, n, nrhs, dt, &prm->precond);
  if (precond_info) memset(precond_info, 0, sizeof(*precond_info));
  if (info) memset(info, 0, sizeof(*info));

  // ---- preconditioner: m NN nests (or phi kept from an earlier call) ------
  if (!prm->reuse_phi) {
    nn_info pi;
    const nn_status ps = nn_invert(ctx, A, lda, w.phi, n, n, dt, &prm->precond, w.inv_ws,
                                   w.inv_bytes, &pi);
    if (precond_info) *precond_info = pi;
    if (ps < 0) {
      if (info) info->status = ps;
      return ps;
    }
  }

  // ---- the series in Horner form ------------------------------------------
  hipStream_t s = ctx->stream;
  const bool cplx = is_complex(dt);
  const Elem e = is_double(dt) ? Elem::F64 : Elem::F32;
  const int64_t cm = cplx ? 2 : 1;
  const int64_t nr = cm * n, rr = cm * nrhs;  // real extents
  const GemmPlan pnr = plan_gemm_k(e, n, rr, nr);
  const size_t esz = elem_size(dt);
  int gemms = 0;
  double trace[NN_TRACE_MAX];
  int n_trace = 0;
  auto finish = [&](nn_status st, int terms, double rel) {
    (void)hipEventRecord(ctx->ev_stop, s);
    (void)hipEventSynchronize(ctx->ev_stop);
    if (info) {
      info->status = st;
      info->iters = terms;
      info->rms = rel;
      info->gemms = gemms;
      for (int i = 0; i < 3; ++i) info->prec_gemms[i] = 0;
      info->prec_gemms[is_double(dt) ? 2 : 1] = gemms;
      info->n_trace = n_trace;
      for (int i = 0; i < n_trace; ++i) info->rms_trace[i] = trace[i];
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop) == hipSuccess) info->device_ms = ms;
    }
    if (rel_residual) *rel_residual = rel;
    return st;
  };

  HIP_TRY(hipEventRecord(ctx->ev_start, s));
  HIP_TRY(launch_sumsq(B, is_double(dt), cm * ldb, n, rr, w.part, w.scal, s));
  // y_0 = phi B (in Xsol)
  {
    GemmArgs g{w.phi, nr, B, cm * ldb, Xsol, cm * ldx, nullptr, 0, n, rr, nr, 1.0, 0.0, nullptr};
    g.work = w.work;
    HIP_TRY(launch_gemm(e, cplx, pnr, g, s));
    ++gemms;
  }
  HIP_TRY(hipMemcpyAsync(ctx->host, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double bnorm = ctx->host[0];
  const double inv_b = bnorm > 0.0 ? 1.0 / bnorm : 0.0;

  void* cur = Xsol;
  int64_t ld_cur = ldx;
  void* alt = w.yalt;
  int64_t ld_alt = nrhs;
  const bool fixed = prm->fixed_terms >= 0;
  nn_status st = NN_OK;
  int terms = 0;
  double rel_ret = NAN, rel_prev = NAN;
  bool use_alt = false;
  for (int k = 0;; ++k) {
    // r = B - A y_k, ||r||_F into stats[k]
    GemmArgs r{A, cm * lda, cur, cm * ld_cur, w.r, rr, B, cm * ldb, n, rr, nr, -1.0, 0.0,
               w.part};
    r.work = w.work;
    HIP_TRY(launch_gemm(e, cplx, pnr, r, s));
    ++gemms;
    HIP_TRY(launch_rms_reduce(w.part, pnr.num_tiles(), 1, w.stats + std::min(k, kStats - 1), s));
    if (fixed) {
      if (k == prm->fixed_terms) {
        terms = k;
        break;
      }
    } else {
      HIP_TRY(hipMemcpyAsync(ctx->host + 1, w.stats + std::min(k, kStats - 1), sizeof(double),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double rel = ctx->host[1] * inv_b;
      if (n_trace < NN_TRACE_MAX) trace[n_trace++] = rel;
      terms = k;
      rel_ret = rel;
      if (!isfinite(rel)) { st = NN_ERR_NONFINITE; break; }
      if (rel < prm->tol) { st = NN_OK; break; }
      if (k > 0 && rel >= 1.0 && rel > rel_prev) { st = NN_ERR_DIVERGED; break; }
      if (k > 0 && rel_prev < 0.1 && rel >= rel_prev) {
        st = NN_STAGNATED;
        terms = k - 1;
        rel_ret = rel_prev;
        use_alt = true;
        break;
      }
      if (k == prm->max_terms) { st = NN_NOT_CONVERGED; break; }
      rel_prev = rel;
    }
    // y_{k+1} = y_k + phi r
    GemmArgs u{w.phi, nr, w.r, rr, alt, cm * ld_alt, cur, cm * ld_cur, n, rr, nr, 1.0, 0.0,
               nullptr};
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
    const int cnt = std::min(prm->fixed_terms + 1, kStats);
    HIP_TRY(hipMemcpyAsync(ctx->host + 1, w.stats, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    n_trace = std::min(cnt, NN_TRACE_MAX);
    for (int i = 0; i < n_trace; ++i) trace[i] = ctx->host[1 + i] * inv_b;
    rel_ret = ctx->host[1 + cnt - 1] * inv_b;
    st = isfinite(rel_ret) ? NN_OK : NN_ERR_NONFINITE;
  }
  return finish(st, terms, rel_ret);
}

}  // extern "C"
