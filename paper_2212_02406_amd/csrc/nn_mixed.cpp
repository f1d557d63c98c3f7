// nn_mixed.cpp — mixed-precision NN schedule for FP64 Hermitian PD input.
//
// The nests of the NN iteration (arXiv 2212.02406, Sec. II-D Theorem) are run
// in three phases, each continuing from the previous phase's iterate (any X
// with ||I - A X||_2 < 1 is a valid start, Appendix 2):
//
//   B  BF16 products with FP32 accumulation, FP32 master iterate.  The
//      start is the paper's own X_0 = I / Tr(A) (Sec. II-A, Sec. II-D), or
//      Theta_2(k) I, whose iterate norm stays small for many nests.  BF16 rounding perturbs A X by
//      about u_bf16 ||A|| ||X||; the phase ends while that is still small:
//      when u_bf16 ||A||_F ||X||_F / N > 0.1, or when the rms stops decreasing.
//   F  FP32 products and residual, while one more FP32 nest is predicted to
//      save an FP64 nest (an exact nest raises the residual to the power d+1,
//      Appendix 2; the rms, a mean dominated by the slowest modes, falls with
//      a smaller effective order p, measured from the last two FP32 nests, and
//      the FP64 nests needed from rms r are ceil(log_p(log tol / log r))), or
//      until an FP32 nest no longer takes 5% off the rms, or lands more than
//      twice above what the previous nest's order predicts (once the rms is
//      below 0.05), or the rms stagnates in the asymptotic regime (sqrt(N)
//      rms_{k-1} < 0.1 and rms_k >= rms_{k-1} / 2) — the FP32 rounding floor.  A loose tolerance (tol >= 1e-4, far above that floor:
//      a preconditioner) is met by the FP32 iterate itself: the phase then
//      runs until the FP32 rms is below tol, and phase D only confirms it.
//   D  FP64 residual and FP64 refinement nests until rms < tol.  A nest
//      may be deeper or shallower than d when one nest of that depth is
//      predicted to finish (fp64_nest_depth): from the FP32 floor one depth-3
//      nest replaces two depth-2 nests.
//
// The transpose start squares the condition number (A X_0 = s A A^H); with
// cond(A) = 1e4 neither the BF16 nor the FP32 phase stays inside the
// convergence region, so this schedule requires the identity start.
// n not a multiple of 8 skips phase B (BF16 rows are read as 16-byte runs).
#include <math.h>
#include <string.h>

#include <algorithm>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr size_t kAlign = 256;
constexpr double kUbf16 = 1.0 / 256.0;  // BF16 unit roundoff 2^-8
constexpr double kTauB = 0.1;
constexpr double kLooseTol = 1e-4;  // tolerances the FP32 iterate can meet

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct MixedWs {
  float* A32;
  uint16_t* Abf;
  float* X32[2];
  uint16_t* Xbf[2];
  uint16_t* XbfT[2];
  float* R32;
  uint16_t* Rbf;
  uint16_t* RbfT;
  uint16_t* UbfT[2];
  float* U32[2];
  double* X64alt;
  double* R64;
  double* U64[2];
  double* part;
  double* scal;   // [0] den, [1] ||A||_F, [2] rms, [3] ||X||_F
  double* spart;  // sum-of-squares partials
  double* denpart;  // start-iterate scratch (power steps)
  double* pw;
  size_t bytes;
  int64_t ldb;    // leading dimension of the BF16 buffers
};

MixedWs carve(void* base, int64_t n, int depth) {
  char* b = static_cast<char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = b ? b + off : nullptr;
    off += up(bytes);
    return p;
  };
  MixedWs w;
  w.ldb = (n + 7) / 8 * 8;
  const size_t nn = (size_t)n * (size_t)n, nb = (size_t)n * (size_t)w.ldb;
  w.A32 = static_cast<float*>(take(4 * nn));
  w.Abf = static_cast<uint16_t*>(take(2 * nb));
  for (int i = 0; i < 2; ++i) {
    w.X32[i] = static_cast<float*>(take(4 * nn));
    w.Xbf[i] = static_cast<uint16_t*>(take(2 * nb));
    w.XbfT[i] = static_cast<uint16_t*>(take(2 * nb));
  }
  w.R32 = static_cast<float*>(take(4 * nn));
  w.Rbf = static_cast<uint16_t*>(take(2 * nb));
  w.RbfT = static_cast<uint16_t*>(take(2 * nb));
  w.UbfT[0] = static_cast<uint16_t*>(take(2 * nb));
  w.UbfT[1] = depth >= 3 ? static_cast<uint16_t*>(take(2 * nb)) : nullptr;
  w.U32[0] = static_cast<float*>(take(4 * nn));
  w.U32[1] = depth >= 3 ? static_cast<float*>(take(4 * nn)) : nullptr;
  w.X64alt = static_cast<double*>(take(8 * nn));
  w.R64 = static_cast<double*>(take(8 * nn));
  w.U64[0] = static_cast<double*>(take(8 * nn));
  w.U64[1] = static_cast<double*>(take(8 * nn));  // FP64 nests may run deeper than d
  const GemmPlan p64 = plan_gemm(Elem::F64, n, n), p32 = plan_gemm(Elem::F32, n, n),
                 pb = plan_gemm_bf16(n, n);
  const int tiles = std::max({p64.num_tiles(), p32.num_tiles(), pb.num_tiles(), 1});
  w.part = static_cast<double*>(take(sizeof(double) * tiles));
  w.spart = static_cast<double*>(take(sizeof(double) * 256));
  w.denpart = static_cast<double*>(take(sizeof(double) * den_partials_elems(n)));
  w.pw = static_cast<double*>(take(sizeof(double) * start_scratch_doubles(n)));
  w.scal = static_cast<double*>(take(sizeof(double) * 16));
  w.bytes = off;
  return w;
}

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return NN_ERR_HIP; \
  } while (0)

// FP64 nests predicted to take the rms r below tol at effective order p.
int fp64_nests(double r, double p, double tol) {
  if (!(r >= tol)) return 0;
  if (r >= 1.0) return 1 << 20;
  return (int)ceil(log(log(tol) / log(r)) / log(p));
}

// Depth of the next FP64 nest from residual rms r.  A nest of any depth q
// leaves the residual R^(q+1) (I - A X sum_{i<=q} R^i = R^(q+1)), and from an
// FP32 iterate the FP64 residual falls at that full order (its error is
// rounding spread over all modes, not a few slow ones).  So in the asymptotic
// regime (sqrt(N) r < 0.1) the nest takes the smallest q with r^(q+1) <
// tol / 10, which finishes in one nest at q + 1 products (Horner, update,
// final residual), when that is no more than the (d+1)-product nests of
// depth d predicted at full order; otherwise depth d.  If the prediction
// falls short, the loop simply runs another nest.
int fp64_nest_depth(double r, int d, int64_t n, double tol) {
  if (!(sqrt((double)n) * r < 0.1) || !(r > 0.0) || !(tol > 0.0)) return d;
  const int q = std::max(1, (int)ceil(log(0.1 * tol) / log(r)) - 1);
  if (q > NN_MAX_DEPTH) return d;
  return q + 1 <= fp64_nests(r, d + 1, tol) * (d + 1) ? q : d;
}

struct Run {
  nn_ctx* ctx;
  int64_t n;
  int d;
  int gemms = 0;
  int prec_gemms[3] = {0, 0, 0};  // BF16, FP32, FP64 products
  int n_trace = 0;
  double trace[NN_TRACE_MAX];
  hipStream_t s() const { return ctx->stream; }
  void push(double r) {
    if (n_trace < NN_TRACE_MAX) trace[n_trace++] = r;
  }
  // Read `count` doubles from device into ctx->host after all queued work.
  hipError_t fetch(const double* dev, int count) {
    hipError_t e = hipMemcpyAsync(ctx->host, dev, sizeof(double) * count, hipMemcpyDeviceToHost, s());
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s());
  }
};

// One plain nest of depth `depth` (FP32 or FP64) after its residual R is
// known: Horner chain and update X' = X + X U into Xn.
template <typename T>
hipError_t plain_update(Run& r, Elem e, const GemmPlan& plan, const T* X, int64_t ldx, T* Xn,
                        int64_t ldxn, const T* R, T* const U[2], int depth) {
  const int64_t n = r.n;
  const T* Ucur = R;
  for (int m = 1; m < depth; ++m) {
    T* Un = U[(m - 1) & 1];
    GemmArgs g{R, n, Ucur, n, Un, n, R, n, n, n, n, 1.0, 0.0, nullptr};
    hipError_t err = launch_gemm(e, false, plan, g, r.s());
    if (err != hipSuccess) return err;
    ++r.gemms;
    ++r.prec_gemms[sizeof(T) == 8 ? 2 : 1];
    Ucur = Un;
  }
  GemmArgs g{X, ldx, Ucur, n, Xn, ldxn, X, ldx, n, n, n, 1.0, 0.0, nullptr};
  ++r.gemms;
  ++r.prec_gemms[sizeof(T) == 8 ? 2 : 1];
  return launch_gemm(e, false, plan, g, r.s());
}

}  // namespace

size_t mixed_workspace_size(int64_t n, const nn_params* prm) {
  return carve(nullptr, n, prm->depth).bytes;
}

nn_status run_mixed(nn_ctx* ctx, const void* Av, int64_t lda, void* Xv, int64_t ldx, int64_t n,
                    const nn_params* prm, void* ws, size_t ws_bytes, nn_info* info) {
  (void)ws_bytes;
  if ((prm->x0 != NN_X0_SCALED_IDENTITY && prm->x0 != NN_X0_POWER_IDENTITY) ||
      prm->fixed_iter != 0)
    return NN_ERR_UNSUPPORTED;
  const double* A = static_cast<const double*>(Av);
  double* X = static_cast<double*>(Xv);
  const MixedWs w = carve(ws, n, prm->depth);
  Run r{ctx, n, prm->depth};
  hipStream_t s = ctx->stream;
  const GemmPlan p64 = plan_gemm(Elem::F64, n, n), p32 = plan_gemm(Elem::F32, n, n),
                 pb = plan_gemm_bf16(n, n);
  int phase_it[3] = {0, 0, 0};
  nn_status st = NN_OK;
  double rms_ret = NAN;
  int iters = 0;

  HIP_TRY(hipEventRecord(ctx->ev_start, s));
  // Start: den = Tr A or 1 / Theta_2(k) of A (FP64; the caller's X serves as
  // the scratch FP64 start), X_0 = I / den in FP32; copies of A in FP32, BF16.
  if (prm->x0 == NN_X0_POWER_IDENTITY)
    HIP_TRY(launch_start(NN_F64, NN_X0_POWER_IDENTITY, prm->power_k, A, lda, X, ldx, n, w.denpart,
                         w.pw, w.scal, s));
  else
    HIP_TRY(launch_den_trace(NN_F64, A, lda, n, w.scal, s));
  HIP_TRY(launch_sumsq(A, true, lda, n, n, w.spart, w.scal + 1, s));
  HIP_TRY(r.fetch(w.scal, 2));
  const double den = ctx->host[0], normA = ctx->host[1];
  auto finish = [&](nn_status status, double rms) {
    (void)hipEventRecord(ctx->ev_stop, s);
    (void)hipEventSynchronize(ctx->ev_stop);
    if (info) {
      info->status = status;
      info->iters = iters;
      info->rms = rms;
      info->gemms = r.gemms;
      info->n_trace = r.n_trace;
      for (int i = 0; i < r.n_trace; ++i) info->rms_trace[i] = r.trace[i];
      for (int i = 0; i < 3; ++i) info->phase_iters[i] = phase_it[i];
      for (int i = 0; i < 3; ++i) info->prec_gemms[i] = r.prec_gemms[i];
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop) == hipSuccess) info->device_ms = ms;
    }
    return status;
  };
  if (!isfinite(den) || !isfinite(normA)) return finish(NN_ERR_NONFINITE, NAN);
  if (den <= 0.0) return finish(NN_ERR_DIVERGED, NAN);
  HIP_TRY(launch_cast_f64_f32(A, lda, w.A32, n, n, n, s));
  HIP_TRY(launch_x0_identity(NN_F32, w.X32[0], n, n, w.scal, s));
  int cur = 0;
  const int max_iter = prm->max_iter;
  double rms_prev = INFINITY;

  // ---- phase B: BF16 products, FP32 accumulation and master iterate ----------
  if (n % 8 == 0) {
    HIP_TRY(launch_cast_bf16(true, A, lda, w.Abf, w.ldb, nullptr, 0, n, n, s));
    HIP_TRY(launch_cast_bf16(false, w.X32[0], n, w.Xbf[0], w.ldb, w.XbfT[0], w.ldb, n, n, s));
    double xnorm = sqrt((double)n) / den;  // ||X_0||_F
    for (;;) {
      if (kUbf16 * normA * xnorm / (double)n > kTauB || iters >= max_iter) break;
      // R = I - A X (BF16 inputs); R in FP32, BF16 and BF16^T; rms partials
      Bf16GemmArgs g{w.Abf, w.ldb, w.XbfT[cur], w.ldb, n, n, n, -1.0, 1.0, nullptr, 0,
                     w.R32, n, w.Rbf, w.ldb, w.RbfT, w.ldb, w.part};
      HIP_TRY(launch_gemm_bf16(pb, g, s));
      ++r.gemms;
      ++r.prec_gemms[0];
      HIP_TRY(launch_rms_reduce(w.part, pb.num_tiles(), n, w.scal + 2, s));
      HIP_TRY(r.fetch(w.scal + 2, 1));
      const double rms = ctx->host[0];
      r.push(rms);
      if (!isfinite(rms) || rms >= rms_prev) break;  // leave the iterate to phase F
      rms_prev = rms;
      // Horner chain on BF16 operands: U_{m+1} = R + R U_m (E = R in FP32)
      const uint16_t* UT = w.RbfT;
      for (int m = 1; m < r.d; ++m) {
        uint16_t* UTn = w.UbfT[(m - 1) & 1];
        Bf16GemmArgs h{w.Rbf, w.ldb, UT, w.ldb, n, n, n, 1.0, 0.0, w.R32, n,
                       nullptr, 0, nullptr, 0, UTn, w.ldb, nullptr};
        HIP_TRY(launch_gemm_bf16(pb, h, s));
        ++r.gemms;
        ++r.prec_gemms[0];
        UT = UTn;
      }
      // X' = X + X U (FP32 master), BF16 copies of X' for the next nest, ||X'||_F
      const int nx = cur ^ 1;
      Bf16GemmArgs u{w.Xbf[cur], w.ldb, UT, w.ldb, n, n, n, 1.0, 0.0, w.X32[cur], n,
                     w.X32[nx], n, w.Xbf[nx], w.ldb, w.XbfT[nx], w.ldb, w.part};
      HIP_TRY(launch_gemm_bf16(pb, u, s));
      ++r.gemms;
      ++r.prec_gemms[0];
      HIP_TRY(launch_rms_reduce(w.part, pb.num_tiles(), 1, w.scal + 3, s));
      HIP_TRY(r.fetch(w.scal + 3, 1));
      xnorm = ctx->host[0];
      cur = nx;
      ++iters;
      ++phase_it[0];
      if (!isfinite(xnorm)) return finish(NN_ERR_NONFINITE, rms);
    }
  }

  // ---- phase F: FP32 products until the FP32 rounding floor -------------------
  rms_prev = INFINITY;
  double p_last = NAN;  // effective order measured on the previous FP32 nest
  for (;;) {
    GemmArgs g{w.A32, n, w.X32[cur], n, w.R32, n, nullptr, 0, n, n, n, -1.0, 1.0, w.part};
    HIP_TRY(launch_gemm(Elem::F32, false, p32, g, s));
    ++r.gemms;
    ++r.prec_gemms[1];
    HIP_TRY(launch_rms_reduce(w.part, p32.num_tiles(), n, w.scal + 2, s));
    HIP_TRY(r.fetch(w.scal + 2, 1));
    const double rms = ctx->host[0];
    r.push(rms);
    if (!isfinite(rms)) return finish(NN_ERR_NONFINITE, rms);
    if (rms >= 1.0 && rms > rms_prev) return finish(NN_ERR_DIVERGED, rms);
    if (iters >= max_iter) break;
    // no progress (rms at least 0.95 of the previous one): the FP32 floor,
    // wherever it lies (the floor rule below needs sqrt(N) rms < 0.1)
    if (isfinite(rms_prev) && rms >= 0.95 * rms_prev) break;
    if (prm->tol >= kLooseTol) {
      if (rms < prm->tol) break;  // the FP32 iterate meets a loose tolerance
    } else {
      // Another FP32 nest (half the cost of an FP64 one) is taken while it is
      // predicted to save an FP64 nest.  The rms falls per nest with an
      // effective order p below d + 1 (the slowest modes dominate the mean),
      // measured on the previous FP32 nest.
      double p = (double)(r.d + 1);
      if (isfinite(rms_prev) && rms_prev < 1.0 && rms < rms_prev && rms > 0.0)
        p = std::min(std::max(log(rms) / log(rms_prev), 1.5), (double)(r.d + 1));
      // FP32 floor: near convergence (previous rms < 0.05) a nest that lands
      // more than twice above what the previous nest's order predicts has run
      // into the rounding of the FP32 residual; the next one would not help.
      if (isfinite(p_last) && rms_prev < 0.05 && rms > 2.0 * pow(rms_prev, p_last)) break;
      if (fp64_nests(pow(rms, p), p, prm->tol) >= fp64_nests(rms, p, prm->tol)) break;
      p_last = p;
    }
    if (sqrt((double)n) * rms_prev < 0.1 && rms >= 0.5 * rms_prev) break;  // FP32 floor
    rms_prev = rms;
    float* U[2] = {w.U32[0], w.U32[1]};
    HIP_TRY(plain_update<float>(r, Elem::F32, p32, w.X32[cur], n, w.X32[cur ^ 1], n, w.R32, U,
                                r.d));
    cur ^= 1;
    ++iters;
    ++phase_it[1];
  }

  // ---- phase D: FP64 residual and refinement nests ----------------------------
  HIP_TRY(launch_cast_f32_f64(w.X32[cur], n, X, ldx, n, n, s));
  double* Xc = X;
  int64_t ldc = ldx;
  double* Xo = w.X64alt;
  int64_t ldo = n;
  rms_prev = INFINITY;
  bool use_prev = false;
  for (;;) {
    GemmArgs g{A, lda, Xc, ldc, w.R64, n, nullptr, 0, n, n, n, -1.0, 1.0, w.part};
    HIP_TRY(launch_gemm(Elem::F64, false, p64, g, s));
    ++r.gemms;
    ++r.prec_gemms[2];
    HIP_TRY(launch_rms_reduce(w.part, p64.num_tiles(), n, w.scal + 2, s));
    HIP_TRY(r.fetch(w.scal + 2, 1));
    const double rms = ctx->host[0];
    r.push(rms);
    rms_ret = rms;
    if (!isfinite(rms)) { st = NN_ERR_NONFINITE; break; }
    if (rms < prm->tol) { st = NN_OK; break; }
    if (rms >= 1.0 && rms > rms_prev) { st = NN_ERR_DIVERGED; break; }
    if (sqrt((double)n) * rms_prev < 0.1 && rms >= rms_prev) {
      st = NN_STAGNATED;
      rms_ret = rms_prev;
      use_prev = true;
      --iters;
      break;
    }
    if (iters >= max_iter) { st = NN_NOT_CONVERGED; break; }
    rms_prev = rms;
    double* U[2] = {w.U64[0], w.U64[1]};
    HIP_TRY(plain_update<double>(r, Elem::F64, p64, Xc, ldc, Xo, ldo, w.R64, U,
                                 fp64_nest_depth(rms, r.d, n, prm->tol)));
    std::swap(Xc, Xo);
    std::swap(ldc, ldo);
    ++iters;
    ++phase_it[2];
  }
  double* res = use_prev ? Xo : Xc;
  const int64_t ldr = use_prev ? ldo : ldc;
  if (res != X)
    HIP_TRY(hipMemcpy2DAsync(X, (size_t)ldx * 8, res, (size_t)ldr * 8, (size_t)n * 8, (size_t)n,
                             hipMemcpyDeviceToDevice, s));
  if (use_prev) --phase_it[2];
  return finish(st, rms_ret);
}

}  // namespace nn
