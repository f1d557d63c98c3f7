// nn_api.cpp — C ABI and host control of the NN library (see include/nn.h).
//
// The host side validates arguments, carves the caller's workspace, enqueues
// the kernels of each nest on the caller's stream, and applies the stopping
// rules.  The rules (the paper iterates a fixed number of nests, Algorithm 1;
// the tolerance stop and status outcomes are this library's):
//   before the loop:  den not finite -> NONFINITE, den <= 0 -> DIVERGED
//   for k = 0, 1, ... with rms_k = ||I - A X_k||_F / sqrt(N):
//     fixed mode: stop at k == fixed_iter
//     tolerance mode, in this order:
//       rms_k not finite                          -> NONFINITE
//       rms_k < tol                               -> OK, X_k
//       k > 0, rms_k >= 1, rms_k > rms_{k-1}      -> DIVERGED
//       k > 0, sqrt(N) rms_{k-1} < 0.1, rms_k >= rms_{k-1}
//                                                 -> STAGNATED, X_{k-1}
//       k == max_iter                             -> NOT_CONVERGED, X_k
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "nn_internal.h"

namespace nn {
namespace {

// Workspace of nn_invert_noalloc: a file-scope device array.  Every device
// the library runs on holds its own copy until the process ends.  In host
// code `scratch` names a host-side stand-in, not the device memory: its
// device address comes from hipGetSymbolAddress (scratch_address), once per
// device, with that device current, and only that address is ever used.
static __device__ __align__(256) unsigned char scratch[NN_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on `device` (current on entry).
hipError_t scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr int kHostSlots = NN_TRACE_MAX + 16;
constexpr int kStatSlots = NN_TRACE_MAX + 1;

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  void* take(size_t bytes) {
    void* p = base ? base + off : nullptr;
    off += up(bytes);
    return p;
  }
};

// Workspace regions of one plain inversion.
struct PlainWs {
  void* xalt = nullptr;
  void* r = nullptr;
  void* u0 = nullptr;
  void* u1 = nullptr;
  double* part = nullptr;     // per-tile partials of the residual GEMM
  double* denpart = nullptr;  // row sums / column partial sums for the norms
  double* pw = nullptr;       // start-iterate scratch (power steps)
  double* scal = nullptr;     // [0] den
  double* stats = nullptr;    // rms per nest
  DevCtl* ctl = nullptr;      // device-side stopping rules
  size_t bytes = 0;
};

PlainWs carve_plain(void* base, int64_t n, nn_dtype dt, int depth) {
  Carver c(base);
  PlainWs w;
  const size_t mat = (size_t)n * (size_t)n * elem_size(dt);
  const bool cplx = is_complex(dt);
  const GemmPlan plan = plan_gemm(is_double(dt) ? Elem::F64 : Elem::F32, n, cplx ? 2 * n : n);
  w.xalt = c.take(mat);
  w.r = c.take(mat);
  if (depth >= 2) w.u0 = c.take(mat);
  if (depth >= 3) w.u1 = c.take(mat);
  w.part = static_cast<double*>(c.take(sizeof(double) * (size_t)std::max(plan.num_tiles(), 1)));
  w.denpart = static_cast<double*>(c.take(sizeof(double) * den_partials_elems(n)));
  w.pw = static_cast<double*>(c.take(sizeof(double) * start_scratch_doubles(n)));
  w.scal = static_cast<double*>(c.take(sizeof(double) * 8));
  w.stats = static_cast<double*>(c.take(sizeof(double) * kStatSlots));
  w.ctl = static_cast<DevCtl*>(c.take(sizeof(DevCtl)));
  w.bytes = c.off;
  return w;
}

bool valid_dtype(int d) { return d >= NN_F64 && d <= NN_C128; }

nn_status check_params(const nn_params* p) {
  if (!p) return NN_ERR_ARG;
  if (p->depth < 1 || p->depth > NN_MAX_DEPTH) return NN_ERR_ARG;
  if (p->x0 < NN_X0_TRANSPOSE || p->x0 > NN_X0_JACOBI) return NN_ERR_ARG;
  if ((p->x0 == NN_X0_POWER_IDENTITY || p->x0 == NN_X0_POWER_TRANSPOSE) &&
      (p->power_k < 1 || p->power_k > NN_POWER_MAX_K))
    return NN_ERR_ARG;
  if (p->fixed_iter < 0) return NN_ERR_ARG;
  if (p->fixed_iter == 0) {
    if (!(p->tol >= 0.0) || p->max_iter < 1) return NN_ERR_ARG;
  }
  if (p->prec != NN_PREC_PLAIN && p->prec != NN_PREC_MIXED) return NN_ERR_ARG;
  if (p->flags & ~(NN_FLAG_TIME_GEMMS | NN_FLAG_DEVICE_STOP)) return NN_ERR_ARG;
  return NN_OK;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return NN_ERR_HIP; \
  } while (0)

struct Ctl {
  nn_ctx* ctx;
  nn_dtype dt;
  int64_t n;
  const nn_params* prm;
  nn_info* info;
  int gemms = 0;
  int timed = 0;  // GEMM launches bracketed by event pairs

  bool timing() const { return (prm->flags & NN_FLAG_TIME_GEMMS) && ctx->ev_gemm; }
  // Launch one GEMM, bracketed by events when timing is on.
  hipError_t gemm(Elem e, bool cplx, const GemmPlan& plan, const GemmArgs& a) {
    const bool t = timing() && timed < kTimedGemms;
    if (t) {
      hipError_t r = hipEventRecord(ctx->ev_gemm[2 * timed], ctx->stream);
      if (r != hipSuccess) return r;
    }
    hipError_t err = launch_gemm(e, cplx, plan, a, ctx->stream);
    if (err != hipSuccess) return err;
    if (t) {
      err = hipEventRecord(ctx->ev_gemm[2 * timed + 1], ctx->stream);
      ++timed;
    }
    ++gemms;
    return err;
  }
  // Summed duration of the first `limit` timed launches (all by default).
  float gemm_ms(int limit = 1 << 30) const {
    float tot = 0.f;
    for (int i = 0; i < timed && i < limit; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ctx->ev_gemm[2 * i], ctx->ev_gemm[2 * i + 1]) == hipSuccess)
        tot += ms;
    }
    return tot;
  }
};

hipError_t ensure_gemm_events(nn_ctx* ctx) {
  if (ctx->ev_gemm) return hipSuccess;
  hipEvent_t* ev = new (std::nothrow) hipEvent_t[2 * kTimedGemms];
  if (!ev) return hipErrorOutOfMemory;
  for (int i = 0; i < 2 * kTimedGemms; ++i) {
    hipError_t e = hipEventCreate(&ev[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      delete[] ev;
      return e;
    }
  }
  ctx->ev_gemm = ev;
  return hipSuccess;
}

// Residual GEMM R = I - A X with partials, then rms into stats[slot].
hipError_t residual_rms(Ctl& c, Elem e, bool cplx, const GemmPlan& plan, const void* A,
                        int64_t lda_r, const void* Xc, int64_t ldx_r, void* R, int64_t n,
                        double* part, double* rms_out) {
  const int64_t nr = cplx ? 2 * n : n;
  GemmArgs g{A, lda_r, Xc, ldx_r, R, nr, nullptr, 0, n, nr, nr, -1.0, 1.0, part};
  hipError_t err = c.gemm(e, cplx, plan, g);
  if (err != hipSuccess) return err;
  return launch_rms_reduce(part, plan.num_tiles(), n, rms_out, c.ctx->stream);
}

// gemms < 0: every launch made did work (c.gemms); else the launches that did
// work, a prefix of those made (device-side stopping).
nn_status finish_info(Ctl& c, nn_status st, int iters, double rms, int n_trace,
                      const double* trace, int gemms = -1) {
  if (gemms < 0) gemms = c.gemms;
  if (c.info) {
    c.info->status = st;
    c.info->iters = iters;
    c.info->rms = rms;
    c.info->gemms = gemms;
    for (int i = 0; i < 3; ++i) c.info->prec_gemms[i] = 0;
    c.info->prec_gemms[is_double(c.dt) ? 2 : 1] = gemms;
    c.info->n_trace = n_trace;
    for (int i = 0; i < n_trace && i < NN_TRACE_MAX; ++i) c.info->rms_trace[i] = trace[i];
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c.ctx->ev_start, c.ctx->ev_stop) == hipSuccess)
      c.info->device_ms = ms;
    c.info->gemm_ms = c.gemm_ms(gemms);
  }
  return st;
}

// Nests to enqueue before the host next reads the device control block: the
// fewest m >= 1 with rms^((d+1)^m) < tol.  A nest maps R to R^(d+1), and for
// a normal R the power-mean inequality gives rms_{k+1} >= rms_k^(d+1), so
// every one of these nests is needed; capped at kChunkMax nests (a start far
// from convergence, or a non-normal residual that falls faster).
constexpr int kChunkMax = 16;
int nests_ahead(double rms, double tol, int d) {
  if (!(rms < 1.0) || !(rms > 0.0) || !(tol > 0.0) || tol >= 1.0) return 1;
  const double need = log(tol) / log(rms);  // (d+1)^m must exceed this
  int m = 1;
  for (double p = d + 1.0; p <= need && m < kChunkMax; p *= d + 1.0) ++m;
  return m;
}

// The plain tolerance-mode loop with the stopping rules on the device
// (NN_FLAG_DEVICE_STOP).  After the residual of nest index k, one kernel
// reduces its rms and applies the rules; once they fire it sets ctl->done and
// every product enqueued after it returns at once, so X_k (X_{k-1} for
// STAGNATED) is left where the ping-pong put it: X_j is in the caller's X for
// even j and in the workspace's xalt for odd j.  The host enqueues
// nests_ahead() nests per read of the control block.
nn_status run_plain_device_stop(Ctl& c, const void* A, int64_t lda, void* X, int64_t ldx,
                                const PlainWs& w) {
  nn_ctx* ctx = c.ctx;
  const nn_params* prm = c.prm;
  const int64_t n = c.n;
  const nn_dtype dt = c.dt;
  hipStream_t s = ctx->stream;
  const bool cplx = is_complex(dt);
  const Elem e = is_double(dt) ? Elem::F64 : Elem::F32;
  const int cm = cplx ? 2 : 1;
  const int64_t nr = cm * n;
  const GemmPlan plan = plan_gemm(e, n, nr);
  const size_t esz = elem_size(dt);
  const int d = prm->depth;
  const int32_t* skip = &w.ctl->done;

  if (prm->x0 != NN_X0_GIVEN)
    HIP_TRY(launch_start(dt, prm->x0, prm->power_k, A, lda, X, ldx, n, w.denpart, w.pw, w.scal,
                         s));
  HIP_TRY(launch_ctl_init(w.ctl, prm->x0 != NN_X0_GIVEN ? w.scal : nullptr, s));

  void* buf[2] = {X, w.xalt};
  const int64_t ld[2] = {ldx, n};
  // residual of nest index k (X_k in buf[k & 1]) and the rules for k
  auto residual = [&](int k) -> hipError_t {
    const int b = k & 1;
    GemmArgs g{A, lda * cm, buf[b], ld[b] * cm, w.r, nr, nullptr, 0, n, nr, nr, -1.0, 1.0, w.part};
    g.skip = skip;
    hipError_t err = c.gemm(e, cplx, plan, g);
    if (err != hipSuccess) return err;
    return launch_rms_control(w.part, plan.num_tiles(), n, w.stats + std::min(k, kStatSlots - 1),
                              w.ctl, k, prm->tol, prm->max_iter, s);
  };
  // nest k: X_{k+1} = X_k + X_k U_d from R_k
  auto nest = [&](int k) -> hipError_t {
    const void* U = w.r;
    for (int m = 1; m < d; ++m) {
      void* Un = (m & 1) ? w.u0 : w.u1;
      GemmArgs g{w.r, nr, U, nr, Un, nr, w.r, nr, n, nr, nr, 1.0, 0.0, nullptr};
      g.skip = skip;
      hipError_t err = c.gemm(e, cplx, plan, g);
      if (err != hipSuccess) return err;
      U = Un;
    }
    const int b = k & 1;
    GemmArgs g{buf[b], ld[b] * cm, U, nr, buf[b ^ 1], ld[b ^ 1] * cm, buf[b], ld[b] * cm, n, nr,
               nr, 1.0, 0.0, nullptr};
    g.skip = skip;
    return c.gemm(e, cplx, plan, g);
  };

  HIP_TRY(residual(0));
  int k = 0;  // residuals enqueued for k = 0..this
  DevCtl hc;
  for (;;) {
    HIP_TRY(hipMemcpyAsync(ctx->host + 1, w.ctl, sizeof(DevCtl), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ctx->host + 6, w.stats + std::min(k, kStatSlots - 1), sizeof(double),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    memcpy(&hc, ctx->host + 1, sizeof(DevCtl));
    if (hc.done) break;
    // the rules let every residual up to k pass, so k < max_iter
    const int m = std::min(nests_ahead(ctx->host[6], prm->tol, d), prm->max_iter - k);
    for (int j = 0; j < m; ++j, ++k) {
      HIP_TRY(nest(k));
      HIP_TRY(residual(k + 1));
    }
  }

  const nn_status st = static_cast<nn_status>(hc.status);
  // products that did work: residuals 0..last_k and the nests between them
  const int gemms = hc.last_k < 0 ? 0 : hc.last_k * (d + 1) + 1;
  double trace[NN_TRACE_MAX];
  const int n_trace = std::min(hc.last_k + 1, NN_TRACE_MAX);
  if (n_trace > 0)
    HIP_TRY(hipMemcpyAsync(ctx->host + 8, w.stats, sizeof(double) * n_trace,
                           hipMemcpyDeviceToHost, s));
  // the returned iterate to X (for a negative status, the last one, as the
  // host loop leaves it)
  if (hc.iters & 1)
    HIP_TRY(hipMemcpy2DAsync(X, (size_t)ldx * esz, w.xalt, (size_t)n * esz, (size_t)n * esz,
                             (size_t)n, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipEventRecord(ctx->ev_stop, s));
  HIP_TRY(hipEventSynchronize(ctx->ev_stop));
  for (int i = 0; i < n_trace; ++i) trace[i] = ctx->host[8 + i];
  return finish_info(c, st, hc.iters, hc.rms_ret, n_trace, trace, gemms);
}

// The plain NN loop: every GEMM in the dtype of A.
nn_status run_plain(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx, int64_t n,
                    nn_dtype dt, const nn_params* prm, const PlainWs& w, nn_info* info) {
  hipStream_t s = ctx->stream;
  const bool cplx = is_complex(dt);
  const Elem e = is_double(dt) ? Elem::F64 : Elem::F32;
  const int cm = cplx ? 2 : 1;  // real components per element
  const int64_t nr = cm * n;
  const GemmPlan plan = plan_gemm(e, n, nr);
  const size_t esz = elem_size(dt);
  Ctl c{ctx, dt, n, prm, info};
  if (prm->flags & NN_FLAG_TIME_GEMMS) HIP_TRY(ensure_gemm_events(ctx));
  double trace[NN_TRACE_MAX];
  int n_trace = 0;

  HIP_TRY(hipEventRecord(ctx->ev_start, s));
  if (prm->fixed_iter == 0 && (prm->flags & NN_FLAG_DEVICE_STOP))
    return run_plain_device_stop(c, A, lda, X, ldx, w);
  // Start iterate X_0 in the caller's X.
  if (prm->x0 != NN_X0_GIVEN) {
    HIP_TRY(launch_start(dt, prm->x0, prm->power_k, A, lda, X, ldx, n, w.denpart, w.pw, w.scal,
                         s));
    HIP_TRY(hipMemcpyAsync(ctx->host, w.scal, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double den = ctx->host[0];
    if (!isfinite(den) || den <= 0.0) {
      HIP_TRY(hipEventRecord(ctx->ev_stop, s));
      HIP_TRY(hipEventSynchronize(ctx->ev_stop));
      return finish_info(c, isfinite(den) ? NN_ERR_DIVERGED : NN_ERR_NONFINITE, 0, NAN, 0, trace);
    }
  }

  void* cur = X;
  int64_t ld_cur = ldx;
  void* alt = w.xalt;
  int64_t ld_alt = n;
  const bool fixed = prm->fixed_iter > 0;
  const int d = prm->depth;
  double rms_prev = NAN;
  nn_status st = NN_OK;
  int iters = 0;
  double rms_ret = NAN;
  bool use_alt = false;  // result lives in `alt` (the previous iterate)

  for (int k = 0;; ++k) {
    const int slot = std::min(k, kStatSlots - 1);
    HIP_TRY(residual_rms(c, e, cplx, plan, A, lda * cm, cur, ld_cur * cm, w.r, n, w.part,
                         w.stats + slot));
    if (fixed) {
      if (k == prm->fixed_iter) {
        iters = k;
        break;
      }
    } else {
      HIP_TRY(hipMemcpyAsync(ctx->host + 1, w.stats + slot, sizeof(double),
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double rms = ctx->host[1];
      if (n_trace < NN_TRACE_MAX) trace[n_trace++] = rms;
      iters = k;
      rms_ret = rms;
      if (!isfinite(rms)) { st = NN_ERR_NONFINITE; break; }
      if (rms < prm->tol) { st = NN_OK; break; }
      if (k > 0 && rms >= 1.0 && rms > rms_prev) { st = NN_ERR_DIVERGED; break; }
      if (k > 0 && sqrt((double)n) * rms_prev < 0.1 && rms >= rms_prev) {
        st = NN_STAGNATED;
        iters = k - 1;
        rms_ret = rms_prev;
        use_alt = true;
        break;
      }
      if (k == prm->max_iter) { st = NN_NOT_CONVERGED; break; }
      rms_prev = rms;
    }
    // Horner chain U_1 = R, U_{m+1} = R + R U_m, ping-pong between u0/u1.
    const void* U = w.r;
    for (int m = 1; m < d; ++m) {
      void* Un = (m & 1) ? w.u0 : w.u1;
      GemmArgs g{w.r, nr, U, nr, Un, nr, w.r, nr, n, nr, nr, 1.0, 0.0, nullptr};
      HIP_TRY(c.gemm(e, cplx, plan, g));
      U = Un;
    }
    // Update X' = X + X U_d into the other buffer.
    GemmArgs g{cur, ld_cur * cm, U, nr, alt, ld_alt * cm, cur, ld_cur * cm, n, nr, nr, 1.0, 0.0,
               nullptr};
    HIP_TRY(c.gemm(e, cplx, plan, g));
    std::swap(cur, alt);
    std::swap(ld_cur, ld_alt);
  }

  void* res = use_alt ? alt : cur;
  const int64_t ld_res = use_alt ? ld_alt : ld_cur;
  if (res != X)
    HIP_TRY(hipMemcpy2DAsync(X, (size_t)ldx * esz, res, (size_t)ld_res * esz, (size_t)n * esz,
                             (size_t)n, hipMemcpyDeviceToDevice, s));
  if (fixed) {
    const int cnt = std::min(prm->fixed_iter + 1, kStatSlots);
    HIP_TRY(hipMemcpyAsync(ctx->host + 2, w.stats, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipEventRecord(ctx->ev_stop, s));
  HIP_TRY(hipEventSynchronize(ctx->ev_stop));
  if (fixed) {
    const int cnt = std::min(prm->fixed_iter + 1, kStatSlots);
    n_trace = std::min(cnt, NN_TRACE_MAX);
    for (int i = 0; i < n_trace; ++i) trace[i] = ctx->host[2 + i];
    rms_ret = ctx->host[2 + cnt - 1];
    st = isfinite(rms_ret) ? NN_OK : NN_ERR_NONFINITE;
  }
  return finish_info(c, st, iters, rms_ret, n_trace, trace);
}

nn_status validate_invert(nn_ctx* ctx, const void* A, int64_t lda, const void* X, int64_t ldx,
                          int64_t n, nn_dtype dt, const nn_params* prm) {
  if (!ctx || !A || !X || n < 1 || lda < n || ldx < n) return NN_ERR_ARG;
  if (!valid_dtype(dt)) return NN_ERR_ARG;
  if (check_params(prm) != NN_OK) return NN_ERR_ARG;
  if (A == X) return NN_ERR_ARG;
  if (dt == NN_C128 && ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(X)) & 15u))
    return NN_ERR_ARG;
  if ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(X)) % (elem_size(dt) / (is_complex(dt) ? 2 : 1)))
    return NN_ERR_ARG;
  return NN_OK;
}

}  // namespace

// Implemented in nn_mixed.cpp.
size_t mixed_workspace_size(int64_t n, const nn_params* prm);
nn_status run_mixed(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx, int64_t n,
                    const nn_params* prm, void* ws, size_t ws_bytes, nn_info* info);

}  // namespace nn

using namespace nn;

extern "C" {

nn_status nn_create(nn_ctx** out, int device, void* stream) {
  if (!out) return NN_ERR_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return NN_ERR_HIP;
  if (device < 0 || device >= count) return NN_ERR_ARG;
  if (hipSetDevice(device) != hipSuccess) return NN_ERR_HIP;
  nn_ctx* c = new (std::nothrow) nn_ctx();
  if (!c) return NN_ERR_HIP;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
    if (prop.multiProcessorCount > 0) c->num_cus = prop.multiProcessorCount;
    // the architecture name up to its feature suffix ("gfx950:sramecc+:xnack-")
    size_t i = 0;
    for (; i + 1 < sizeof(c->arch) && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i)
      c->arch[i] = prop.gcnArchName[i];
    c->arch[i] = 0;
  }
  if (!c->arch[0]) strcpy(c->arch, "unknown");
  if (scratch_address(device, &c->scratch) != hipSuccess) {
    nn_destroy(c);
    return NN_ERR_HIP;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->host), sizeof(double) * kHostSlots,
                    hipHostMallocDefault) != hipSuccess ||
      hipEventCreate(&c->ev_start) != hipSuccess || hipEventCreate(&c->ev_stop) != hipSuccess) {
    nn_destroy(c);
    return NN_ERR_HIP;
  }
  *out = c;
  return NN_OK;
}

void nn_destroy(nn_ctx* c) {
  if (!c) return;
  if (c->host) (void)hipHostFree(c->host);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
  if (c->ev_gemm) {
    for (int i = 0; i < 2 * kTimedGemms; ++i) (void)hipEventDestroy(c->ev_gemm[i]);
    delete[] c->ev_gemm;
  }
  if (c->bgraph.exec) (void)hipGraphExecDestroy(c->bgraph.exec);
  if (c->bgraph.graph) (void)hipGraphDestroy(c->bgraph.graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

nn_status nn_set_stream(nn_ctx* c, void* stream) {
  if (!c) return NN_ERR_ARG;
  c->stream = static_cast<hipStream_t>(stream);
  return NN_OK;
}

size_t nn_workspace_size(int64_t n, nn_dtype dt, const nn_params* prm) {
  if (n < 1 || !valid_dtype(dt) || check_params(prm) != NN_OK) return 0;
  if (prm->prec == NN_PREC_MIXED) return dt == NN_F64 ? mixed_workspace_size(n, prm) : 0;
  return carve_plain(nullptr, n, dt, prm->depth).bytes;
}

nn_status nn_invert(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx, int64_t n,
                    nn_dtype dt, const nn_params* prm, void* ws, size_t ws_bytes, nn_info* info) {
  nn_status v = validate_invert(ctx, A, lda, X, ldx, n, dt, prm);
  if (v != NN_OK) return v;
  if (info) memset(info, 0, sizeof(*info));
  if (prm->prec == NN_PREC_MIXED) {
    if (dt != NN_F64) return NN_ERR_UNSUPPORTED;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) ||
        ws_bytes < mixed_workspace_size(n, prm))
      return NN_ERR_WORKSPACE;
    if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
    return run_mixed(ctx, A, lda, X, ldx, n, prm, ws, ws_bytes, info);
  }
  const size_t need = carve_plain(nullptr, n, dt, prm->depth).bytes;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) || ws_bytes < need)
    return NN_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const PlainWs w = carve_plain(ws, n, dt, prm->depth);
  return run_plain(ctx, A, lda, X, ldx, n, dt, prm, w, info);
}

nn_status nn_invert_noalloc(nn_ctx* ctx, const void* A, int64_t lda, void* X, int64_t ldx,
                            int64_t n, nn_dtype dt, const nn_params* prm, nn_info* info) {
  nn_status v = validate_invert(ctx, A, lda, X, ldx, n, dt, prm);
  if (v != NN_OK) return v;
  // event timing would create events on first use
  if (prm->flags & NN_FLAG_TIME_GEMMS) return NN_ERR_ARG;
  if (!ctx->scratch) return NN_ERR_HIP;
  const size_t need = nn_workspace_size(n, dt, prm);
  if (need == 0) return prm->prec == NN_PREC_MIXED ? NN_ERR_UNSUPPORTED : NN_ERR_ARG;
  if (need > (size_t)NN_NOALLOC_SCRATCH_BYTES) return NN_ERR_WORKSPACE;
  return nn_invert(ctx, A, lda, X, ldx, n, dt, prm, ctx->scratch, NN_NOALLOC_SCRATCH_BYTES, info);
}

size_t nn_solve_workspace_size(int64_t n, int64_t nrhs, nn_dtype dt, const nn_params* prm) {
  if (n < 1 || nrhs < 1 || !valid_dtype(dt) || check_params(prm) != NN_OK) return 0;
  if (prm->prec != NN_PREC_PLAIN || prm->x0 == NN_X0_GIVEN) return 0;
  const size_t esz = elem_size(dt);
  const size_t inv = up((size_t)n * n * esz);
  const size_t rb = up((size_t)n * nrhs * esz);
  const int cm = is_complex(dt) ? 2 : 1;
  const Elem el = is_double(dt) ? Elem::F64 : Elem::F32;
  const GemmPlan plan = plan_gemm_k(el, n, (int64_t)cm * nrhs, (int64_t)cm * n);
  const size_t part = up(sizeof(double) * std::max(plan.num_tiles(), 256)) + up(sizeof(double) * 8);
  return inv + rb + part + up(gemm_work_bytes(plan, el, n, (int64_t)cm * nrhs)) +
         carve_plain(nullptr, n, dt, prm->depth).bytes;
}

nn_status nn_solve(nn_ctx* ctx, const void* A, int64_t lda, const void* B, int64_t ldb,
                   void* Xsol, int64_t ldx, int64_t n, int64_t nrhs, nn_dtype dt,
                   const nn_params* prm, void* ws, size_t ws_bytes, nn_info* info,
                   double* rel_residual) {
  if (!ctx || !A || !B || !Xsol || n < 1 || nrhs < 1 || lda < n || ldb < nrhs || ldx < nrhs)
    return NN_ERR_ARG;
  if (!valid_dtype(dt) || check_params(prm) != NN_OK) return NN_ERR_ARG;
  if (prm->prec != NN_PREC_PLAIN || prm->x0 == NN_X0_GIVEN) return NN_ERR_UNSUPPORTED;
  if (Xsol == B || Xsol == A) return NN_ERR_ARG;
  const size_t need = nn_solve_workspace_size(n, nrhs, dt, prm);
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1)) || ws_bytes < need)
    return NN_ERR_WORKSPACE;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const size_t esz = elem_size(dt);
  Carver c(ws);
  void* Xinv = c.take((size_t)n * n * esz);
  void* Rb = c.take((size_t)n * nrhs * esz);
  const int cm = is_complex(dt) ? 2 : 1;
  const Elem e = is_double(dt) ? Elem::F64 : Elem::F32;
  const GemmPlan plan = plan_gemm_k(e, n, (int64_t)cm * nrhs, (int64_t)cm * n);
  double* part = static_cast<double*>(c.take(sizeof(double) * std::max(plan.num_tiles(), 256)));
  double* scal = static_cast<double*>(c.take(sizeof(double) * 8));
  const size_t wb = gemm_work_bytes(plan, e, n, (int64_t)cm * nrhs);
  void* work = wb ? c.take(wb) : nullptr;
  void* rest = c.base + c.off;
  const PlainWs w = carve_plain(rest, n, dt, prm->depth);
  nn_info local;
  nn_info* inf = info ? info : &local;
  nn_status st = run_plain(ctx, A, lda, Xinv, n, n, dt, prm, w, inf);
  if (st < 0) return st;
  hipStream_t s = ctx->stream;
  const bool cplx = is_complex(dt);
  // Xsol = Xinv B  (n x n times n x nrhs).
  GemmArgs g{Xinv, (int64_t)cm * n, B, (int64_t)cm * ldb, Xsol, (int64_t)cm * ldx, nullptr, 0, n,
             (int64_t)cm * nrhs, (int64_t)cm * n, 1.0, 0.0, nullptr};
  g.work = work;
  HIP_TRY(launch_gemm(e, cplx, plan, g, s));
  if (rel_residual) {
    // Rb = B - A Xsol with partials -> ||Rb||_F; ||B||_F by a plain sum of squares.
    GemmArgs r{A, (int64_t)cm * lda, Xsol, (int64_t)cm * ldx, Rb, (int64_t)cm * nrhs, B,
               (int64_t)cm * ldb, n, (int64_t)cm * nrhs, (int64_t)cm * n, -1.0, 0.0, part};
    r.work = work;
    HIP_TRY(launch_gemm(e, cplx, plan, r, s));
    HIP_TRY(launch_rms_reduce(part, plan.num_tiles(), 1, scal, s));
    HIP_TRY(launch_sumsq(B, is_double(dt), (int64_t)cm * ldb, n, (int64_t)cm * nrhs, part,
                         scal + 1, s));
    HIP_TRY(hipMemcpyAsync(ctx->host, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));
  if (rel_residual) *rel_residual = ctx->host[1] > 0 ? ctx->host[0] / ctx->host[1] : 0.0;
  return st;
}

const char* nn_status_string(nn_status s) {
  switch (s) {
    case NN_OK: return "ok";
    case NN_NOT_CONVERGED: return "not converged: max_iter reached above tol";
    case NN_STAGNATED: return "stagnated: rounding floor reached above tol";
    case NN_ERR_ARG: return "invalid argument";
    case NN_ERR_DIVERGED: return "diverged: start iterate violates ||I - A X0||_2 < 1";
    case NN_ERR_NONFINITE: return "non-finite value in A, the start scale or a residual";
    case NN_ERR_HIP: return "HIP runtime error";
    case NN_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case NN_ERR_UNSUPPORTED: return "unsupported combination";
  }
  return "unknown status";
}

}  // extern "C"
