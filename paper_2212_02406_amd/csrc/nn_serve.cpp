// nn_serve.cpp — continuous-batching inversion server (declared in nn.h).
//
// Every active request advances by one NN nest per tick (Sec. II-D Theorem),
// so a request that arrives while others are on the device starts at the next
// tick instead of waiting for the running ones to finish.  Per tick the host
// synchronises once: the residual rms of every active request's iterate is
// written to its slot of a device array at the head of the pool, the array is
// read back in one copy, each request's rules are applied on the host, and the
// next nest and residual of every continuing request are enqueued at once.
//
// Per request the rules are nn_invert's tolerance-mode rules, applied per
// precision phase, plus the promotion rules of the narrow (FP32 / complex64)
// phase:
//   rms not finite                              -> NONFINITE
//   rms < tol                                   -> OK, current iterate
//   phase nests > 0, rms >= 1, rms > previous   -> DIVERGED
//   narrow, wide phase reserved, previous rms below the promotion point
//     pow(1e-9, 1/(d+1)) or stagnated           -> promote (better iterate)
//   stagnated (sqrt(N) prev < 0.1, rms >= prev) -> narrow: promote if the wide
//                                                  buffers fit, else STAGNATED;
//                                                  wide: STAGNATED, previous X
//   nests == max_iter                           -> NOT_CONVERGED
// The promotion point is one narrow nest past the rms at which the next nest
// of order d+1 would reach about 1e-9: the narrow iterate then sits at its
// rounding floor, and one or two wide nests finish it.
//
// Small requests (FP32 / complex64, n <= batch_max_n <= 64) skip the per-nest
// ticks of their narrow phase: the tick that admits them forms their X_0 like
// any other request's, then runs all of them, one launch per dtype, through
// the batched persistent kernel in its tolerance mode (each matrix applies the
// rules above on the device, with X, R and U in LDS).  A request that must
// finish wide stops there at the promotion point instead of its tolerance and
// is promoted; a stagnated one is promoted if the wide buffers fit.  The
// batched kernel's result does not depend on the rest of the batch, so the
// co-runner independence of results holds for this path too.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <functional>
#include <map>
#include <new>
#include <queue>
#include <unordered_map>
#include <vector>

#include "nn_internal.h"
#include "nn_sched.h"

namespace nn {
namespace {

using sched::PoolAlloc;
using sched::RState;
using sched::single_dtype;
using sched::widen;
using sched::up;

constexpr size_t kAlign = sched::kAlign;
constexpr int kMaxStreams = 8;
constexpr int kMaxActiveLimit = 65536;
constexpr int kBatchMaxN = 64;  // the batched kernel's largest size

// Matrices of one precision phase of a request.
struct PhaseBufs {
  nn_dtype dt = NN_F32;
  void* A = nullptr;
  void* X[2] = {nullptr, nullptr};
  void* R = nullptr;
  void* U[2] = {nullptr, nullptr};
};

struct Block {
  size_t off = 0, bytes = 0;
  bool held = false;
};

// A request: its scheduling state (sched::Req) plus what the device work
// needs.
struct Request : sched::Req {
  const void* src = nullptr;
  int64_t src_ld = 0;
  Block narrow, wide;
  PhaseBufs ph[2];            // [0] narrow (single precision), [1] wide
  double* part = nullptr;     // residual GEMM tile partials
  double* denpart = nullptr;  // norm partials of the transpose start
  double* pw = nullptr;       // power-step scratch of the Theta_2 starts
  double* scal = nullptr;     // [0] den
  int slot = -1;
  int stream = 0;
  int bidx = -1;          // index in this tick's batched launch (small path)
  bool polled = false;    // its record has been handed out by nn_server_poll
  bool dropped = false;   // fetched or released before it was polled
  double t_submit = 0, t_admit = 0, t_finish = 0;
};

Elem elem_of(nn_dtype d) { return is_double(d) ? Elem::F64 : Elem::F32; }

// The sizes that fix a request's pool block (tile partials enough for either
// precision's plan).
sched::ReqSizes sizes_of(int64_t n, nn_dtype dt, int depth) {
  const int cm = is_complex(dt) ? 2 : 1;
  const int t64 = plan_gemm(Elem::F64, n, cm * n).num_tiles();
  const int t32 = plan_gemm(Elem::F32, n, cm * n).num_tiles();
  sched::ReqSizes z;
  z.part = sizeof(double) * (size_t)std::max({t64, t32, 1});
  z.denpart = sizeof(double) * den_partials_elems(n);
  z.pw = sizeof(double) * start_scratch_doubles(n);
  z.narrow_mat = single_dtype(dt) ? (size_t)n * (size_t)n * elem_size(dt) : 0;
  z.wide_mat = (size_t)n * (size_t)n * elem_size(widen(dt));
  z.depth = depth;
  return z;
}

}  // namespace
}  // namespace nn

using namespace nn;

struct nn_server {
  nn_ctx* ctx = nullptr;
  char* pool = nullptr;  // start of the allocatable region
  nn_server_params prm{};
  int n_streams = 1;
  PoolAlloc alloc;
  size_t pool_bytes = 0;  // allocatable bytes
  double* slots_dev = nullptr;   // 2 doubles per slot: rms, den
  double* slots_host = nullptr;  // pinned
  std::priority_queue<int, std::vector<int>, std::greater<int>> free_slots;
  std::deque<sched::Req*> queued;  // Request objects, in arrival order
  std::vector<Request*> active;
  std::unordered_map<int64_t, Request*> by_id;  // queued, active or retired (not fetched)
  std::deque<Request*> unpolled;
  size_t ready = 0;
  hipStream_t streams[kMaxStreams] = {};
  hipEvent_t done[kMaxStreams] = {};
  hipStream_t ctl = nullptr;
  hipEvent_t entry = nullptr;  // orders the server's streams after the context stream
  // Batched narrow phase: argument arrays (max_active entries each) and the
  // plan workspace after the slots; pinned staging of the arrays (same
  // layout) followed by the per-matrix records read back.
  char* bdev = nullptr;
  char* bhost = nullptr;
  size_t barg_bytes = 0;
  std::vector<Request*> small_new;  // admitted this tick, small path
  int rr = 0;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace nn {
namespace {

#define HIP_TRY(expr)                         \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return NN_ERR_HIP; \
  } while (0)

// Layout of the batched argument block for m entries (device and host).
struct BatchLayout {
  size_t off, xoff, tols, sizes, maxits, bytes;  // argument arrays
  size_t info, ws, total;                         // device: + records, plan workspace
};
BatchLayout batch_layout(int m) {
  BatchLayout L;
  L.off = 0;
  L.xoff = L.off + up(8 * (size_t)m);
  L.tols = L.xoff + up(8 * (size_t)m);
  L.sizes = L.tols + up(8 * (size_t)m);
  L.maxits = L.sizes + up(4 * (size_t)m);
  L.bytes = L.maxits + up(4 * (size_t)m);
  L.info = L.bytes;
  L.ws = L.info + up(sizeof(nn_info_dev) * (size_t)m);
  L.total = L.ws + up(batched_ws_bytes(m));
  return L;
}

bool small_path(const nn_server* s, int64_t n, nn_dtype dt, int32_t max_iter) {
  return single_dtype(dt) && n <= s->prm.batch_max_n && max_iter <= kBatchedMaxIter;
}

size_t footprint_of(const nn_server* s, int64_t n, nn_dtype dt, double tol, bool* reserve_wide) {
  const bool rw = single_dtype(dt) && tol < s->prm.wide_tol;
  if (reserve_wide) *reserve_wide = rw;
  return sched::admission_bytes(sizes_of(n, dt, s->prm.depth), rw);
}

void set_phase(char* base, const sched::PhaseLayout& L, nn_dtype dt, PhaseBufs* out) {
  out->dt = dt;
  out->A = base + L.A;
  out->X[0] = base + L.X0;
  out->X[1] = base + L.X1;
  out->R = base + L.R;
  out->U[0] = L.U0 ? base + L.U0 : nullptr;
  out->U[1] = L.U1 ? base + L.U1 : nullptr;
}

// Lay out an admitted request's first block: control region, then the start
// phase (narrow for single-precision dtypes, else wide), then the reserved
// wide phase if any.
void carve_request(nn_server* s, Request* q) {
  char* b = s->pool + q->narrow.off;
  const sched::ReqLayout L = sched::carve_block(sizes_of(q->n, q->dt, s->prm.depth),
                                                q->reserve_wide);
  q->part = reinterpret_cast<double*>(b + L.part);
  q->denpart = reinterpret_cast<double*>(b + L.denpart);
  q->pw = reinterpret_cast<double*>(b + L.pw);
  q->scal = reinterpret_cast<double*>(b + L.scal);
  if (L.narrow.used) set_phase(b, L.narrow, q->dt, &q->ph[0]);
  if (L.wide.used) set_phase(b, L.wide, widen(q->dt), &q->ph[1]);
  q->has_wide = L.wide.used;
  q->cur_ph = L.narrow.used ? 0 : 1;
}

// Residual of the current iterate, rms into the request's slot.
hipError_t enqueue_residual(nn_server* s, Request* q) {
  hipStream_t st = s->streams[q->stream];
  const PhaseBufs& P = q->ph[q->cur_ph];
  const bool cplx = is_complex(P.dt);
  const int64_t n = q->n, nr = (cplx ? 2 : 1) * n;
  const GemmPlan plan = plan_gemm(elem_of(P.dt), n, nr);
  GemmArgs g{P.A, nr, P.X[q->cur], nr, P.R, nr, nullptr, 0, n, nr, nr, -1.0, 1.0, q->part};
  hipError_t err = launch_gemm(elem_of(P.dt), cplx, plan, g, st);
  if (err != hipSuccess) return err;
  return launch_rms_reduce(q->part, plan.num_tiles(), n, s->slots_dev + 2 * q->slot, st);
}

// Horner chain U_1 = R, U_{m+1} = R + R U_m, then X[from^1] = X + X U_d.
hipError_t enqueue_nest(nn_server* s, Request* q, int from) {
  hipStream_t st = s->streams[q->stream];
  const PhaseBufs& P = q->ph[q->cur_ph];
  const bool cplx = is_complex(P.dt);
  const int64_t n = q->n, nr = (cplx ? 2 : 1) * n;
  const Elem e = elem_of(P.dt);
  const GemmPlan plan = plan_gemm(e, n, nr);
  const void* U = P.R;
  for (int m = 1; m < s->prm.depth; ++m) {
    void* Un = P.U[(m - 1) & 1];
    GemmArgs g{P.R, nr, U, nr, Un, nr, P.R, nr, n, nr, nr, 1.0, 0.0, nullptr};
    hipError_t err = launch_gemm(e, cplx, plan, g, st);
    if (err != hipSuccess) return err;
    U = Un;
  }
  GemmArgs g{P.X[from], nr, U, nr, P.X[from ^ 1], nr, P.X[from], nr, n, nr, nr, 1.0, 0.0,
             nullptr};
  return launch_gemm(e, cplx, plan, g, st);
}

// Copy A into the pool, form den and X_0, copy den to the slot, then the
// residual (not for the small path, whose residuals run in the batched launch).
hipError_t enqueue_start(nn_server* s, Request* q) {
  hipStream_t st = s->streams[q->stream];
  const PhaseBufs& P = q->ph[q->cur_ph];
  const size_t e = elem_size(q->dt);
  hipError_t err = hipMemcpy2DAsync(P.A, (size_t)q->n * e, q->src, (size_t)q->src_ld * e,
                                    (size_t)q->n * e, (size_t)q->n, hipMemcpyDefault, st);
  if (err != hipSuccess) return err;
  err = launch_start(q->dt, s->prm.x0, s->prm.power_k, P.A, q->n, P.X[0], q->n, q->n, q->denpart,
                     q->pw, q->scal, st);
  if (err != hipSuccess) return err;
  err = hipMemcpyAsync(s->slots_dev + 2 * q->slot + 1, q->scal, sizeof(double),
                       hipMemcpyDeviceToDevice, st);
  if (err != hipSuccess) return err;
  q->cur = 0;
  return q->small ? hipSuccess : enqueue_residual(s, q);
}

// Widen A and the narrow iterate X[from] into the wide phase's X[0] (the
// policy has already switched q to the wide phase), then its residual.
hipError_t enqueue_promote(nn_server* s, Request* q, int from) {
  hipStream_t st = s->streams[q->stream];
  const PhaseBufs& N = q->ph[0];
  const PhaseBufs& W = q->ph[1];
  const int64_t n = q->n, nr = (is_complex(q->dt) ? 2 : 1) * n;
  hipError_t err = launch_cast_f32_f64(static_cast<const float*>(N.A), nr,
                                       static_cast<double*>(W.A), nr, n, nr, st);
  if (err != hipSuccess) return err;
  err = launch_cast_f32_f64(static_cast<const float*>(N.X[from]), nr,
                            static_cast<double*>(W.X[0]), nr, n, nr, st);
  if (err != hipSuccess) return err;
  return enqueue_residual(s, q);
}

void release_blocks(nn_server* s, Request* q) {
  if (q->narrow.held) s->alloc.release(q->narrow.off, q->narrow.bytes);
  if (q->wide.held) s->alloc.release(q->wide.off, q->wide.bytes);
  q->narrow.held = q->wide.held = false;
}

// Bookkeeping of a request the policy retired (status, rms and result_buf
// are set on it).
void retire(nn_server* s, Request* q) {
  q->state = RState::Retired;
  q->t_finish = s->now();
  s->free_slots.push(q->slot);
  q->slot = -1;
  s->unpolled.push_back(q);
  ++s->ready;
}

// Try to reserve the wide block of a request that did not reserve it.
bool reserve_wide_late(nn_server* s, Request* q) {
  if (q->has_wide) return true;
  const size_t mat = (size_t)q->n * (size_t)q->n * elem_size(widen(q->dt));
  const size_t b = up(sched::phase_bytes(mat, s->prm.depth));
  size_t off;
  if (!s->alloc.alloc(b, &off)) return false;
  q->wide = {off, b, true};
  set_phase(s->pool + off, sched::carve_phase(mat, s->prm.depth, 0), widen(q->dt), &q->ph[1]);
  q->has_wide = true;
  return true;
}

nn_status admit(nn_server* s) {
  hipError_t err = hipSuccess;
  auto try_alloc = [&](sched::Req* r) {
    if (err != hipSuccess) return false;  // stop admitting after a failed launch
    Request* q = static_cast<Request*>(r);
    size_t off;
    const size_t b = footprint_of(s, q->n, q->dt, q->tol, &q->reserve_wide);
    if (!s->alloc.alloc(b, &off)) return false;
    q->narrow = {off, b, true};
    return true;
  };
  auto on_admit = [&](sched::Req* r) {
    Request* q = static_cast<Request*>(r);
    carve_request(s, q);
    q->slot = s->free_slots.top();
    s->free_slots.pop();
    q->stream = s->rr++ % s->n_streams;
    q->small = small_path(s, q->n, q->dt, q->max_iter);
    q->t_admit = s->now();
    if (q->small) s->small_new.push_back(q);
    s->active.push_back(q);
    const hipError_t e = enqueue_start(s, q);
    if (err == hipSuccess) err = e;
  };
  sched::admit_scan(s->queued, s->active.size(), s->prm.max_active, try_alloc, on_admit);
  return err == hipSuccess ? NN_OK : NN_ERR_HIP;
}

// One batched launch per dtype over the requests admitted to the small path
// this tick, after their starts (on every stream) and before the tick's
// read-back, which then holds their records.  A request that finishes wide
// stops at the promotion point.
nn_status launch_small(nn_server* s) {
  if (s->small_new.empty()) return NN_OK;
  hipStream_t st = s->streams[0];
  for (int i = 1; i < s->n_streams; ++i) {
    HIP_TRY(hipEventRecord(s->done[i], s->streams[i]));
    HIP_TRY(hipStreamWaitEvent(st, s->done[i], 0));
  }
  const int m = s->prm.max_active;
  const BatchLayout L = batch_layout(m);
  int64_t* off = reinterpret_cast<int64_t*>(s->bhost + L.off);
  int64_t* xoff = reinterpret_cast<int64_t*>(s->bhost + L.xoff);
  double* tols = reinterpret_cast<double*>(s->bhost + L.tols);
  int32_t* sizes = reinterpret_cast<int32_t*>(s->bhost + L.sizes);
  int32_t* maxits = reinterpret_cast<int32_t*>(s->bhost + L.maxits);
  const double point = sched::promotion_point(s->prm.depth);
  int j = 0;
  int first[2] = {0, 0}, count[2] = {0, 0}, maxn[2] = {0, 0};
  const nn_dtype dts[2] = {NN_F32, NN_C64};
  for (int g = 0; g < 2; ++g) {
    first[g] = j;
    for (Request* q : s->small_new) {
      if (q->dt != dts[g]) continue;
      const PhaseBufs& P = q->ph[0];
      const size_t e = elem_size(q->dt);
      q->bidx = j;
      off[j] = (int64_t)((static_cast<char*>(P.A) - s->pool) / e);
      xoff[j] = (int64_t)((static_cast<char*>(P.X[0]) - s->pool) / e);
      sizes[j] = (int32_t)q->n;
      tols[j] = q->reserve_wide ? std::max(q->tol, point) : q->tol;
      maxits[j] = q->max_iter;
      maxn[g] = std::max(maxn[g], (int)q->n);
      ++j;
    }
    count[g] = j - first[g];
  }
  HIP_TRY(hipMemcpyAsync(s->bdev, s->bhost, L.bytes, hipMemcpyHostToDevice, st));
  nn_info_dev* info = reinterpret_cast<nn_info_dev*>(s->bdev + L.info);
  for (int g = 0; g < 2; ++g) {
    if (!count[g]) continue;
    const int f = first[g];
    BatchedArgs a;
    a.dt = dts[g];
    a.A = s->pool;
    a.X = s->pool;
    a.offsets = reinterpret_cast<const int64_t*>(s->bdev + L.off) + f;
    a.xoffsets = reinterpret_cast<const int64_t*>(s->bdev + L.xoff) + f;
    a.sizes = reinterpret_cast<const int32_t*>(s->bdev + L.sizes) + f;
    a.tols = reinterpret_cast<const double*>(s->bdev + L.tols) + f;
    a.maxits = reinterpret_cast<const int32_t*>(s->bdev + L.maxits) + f;
    a.batch = count[g];
    a.max_n = maxn[g];
    a.depth = s->prm.depth;
    a.x0 = NN_X0_GIVEN;
    a.iters = 0;
    a.ws = s->bdev + L.ws;
    a.info = info + f;
    HIP_TRY(launch_batched_direct(s->ctx, a, st));
  }
  HIP_TRY(hipMemcpyAsync(s->bhost + L.info, info, sizeof(nn_info_dev) * (size_t)j,
                         hipMemcpyDeviceToHost, st));
  s->small_new.clear();
  return NN_OK;
}

// Apply the policy to one active request whose rms (and den, if fresh) or
// batched record are in the read-back, and enqueue what it decided.
nn_status step_request(nn_server* s, Request* q, bool* keep) {
  const double* h = s->slots_host + 2 * q->slot;
  const nn_info_dev* rec = nullptr;
  if (q->small) {
    const BatchLayout L = batch_layout(s->prm.max_active);
    rec = reinterpret_cast<const nn_info_dev*>(s->bhost + L.info) + q->bidx;
    q->bidx = -1;
  }
  auto try_wide = [s](sched::Req& r) { return reserve_wide_late(s, static_cast<Request*>(&r)); };
  const sched::Decision dd = sched::decide(*q, h[0], h[1], s->prm.depth, try_wide, rec);
  *keep = dd.act != sched::Act::Retire;
  switch (dd.act) {
    case sched::Act::Retire:
      retire(s, q);
      break;
    case sched::Act::Promote:
      HIP_TRY(enqueue_promote(s, q, dd.from));
      break;
    case sched::Act::Nest:
      HIP_TRY(enqueue_nest(s, q, dd.from));
      HIP_TRY(enqueue_residual(s, q));
      break;
  }
  return NN_OK;
}

void fill_stats(const nn_server* s, int fin, nn_server_stats* st) {
  if (!st) return;
  st->finished = fin;
  st->active = (int32_t)s->active.size();
  st->queued = (int32_t)s->queued.size();
  st->ready = (int32_t)s->ready;
  st->pool_used = s->alloc.used();
}

Request* find_retired(nn_server* s, int64_t id) {
  auto it = s->by_id.find(id);
  if (it == s->by_id.end() || it->second->state != RState::Retired) return nullptr;
  return it->second;
}

// Release a retired request; its record is freed now if it was polled, else
// by the poll that skips it.
void drop(nn_server* s, Request* q) {
  release_blocks(s, q);
  s->by_id.erase(q->id);
  --s->ready;
  if (q->polled)
    delete q;
  else
    q->dropped = true;
}

}  // namespace
}  // namespace nn

extern "C" {

nn_status nn_server_create(nn_ctx* ctx, void* pool, size_t pool_bytes,
                           const nn_server_params* params, nn_server** out) {
  if (!ctx || !pool || !out) return NN_ERR_ARG;
  nn_server_params p{2, NN_X0_SCALED_IDENTITY, 1024, 4, 1e-6, 8, kBatchMaxN};
  if (params) p = *params;
  if (p.depth < 1 || p.depth > NN_MAX_DEPTH) return NN_ERR_ARG;
  if (p.x0 < NN_X0_TRANSPOSE || p.x0 > NN_X0_JACOBI || p.x0 == NN_X0_GIVEN) return NN_ERR_ARG;
  if ((p.x0 == NN_X0_POWER_IDENTITY || p.x0 == NN_X0_POWER_TRANSPOSE) &&
      (p.power_k < 1 || p.power_k > NN_POWER_MAX_K))
    return NN_ERR_ARG;
  if (p.max_active < 1 || p.max_active > kMaxActiveLimit) return NN_ERR_ARG;
  if (p.n_streams < 1 || p.n_streams > kMaxStreams) return NN_ERR_ARG;
  if (!(p.wide_tol >= 0.0)) return NN_ERR_ARG;
  if (p.batch_max_n < 0 || p.batch_max_n > kBatchMaxN) return NN_ERR_ARG;
  const size_t slots = up(2 * sizeof(double) * (size_t)p.max_active);
  const BatchLayout L = batch_layout(p.max_active);
  const size_t head = slots + L.total;
  if ((reinterpret_cast<uintptr_t>(pool) & (kAlign - 1)) || pool_bytes <= head)
    return NN_ERR_WORKSPACE;
  nn_server* s = new (std::nothrow) nn_server();
  if (!s) return NN_ERR_HIP;
  s->ctx = ctx;
  s->prm = p;
  s->n_streams = p.n_streams;
  s->slots_dev = static_cast<double*>(pool);
  s->bdev = static_cast<char*>(pool) + slots;
  s->pool = static_cast<char*>(pool) + head;
  s->pool_bytes = (pool_bytes - head) / kAlign * kAlign;
  s->alloc.reset(s->pool_bytes);
  for (int i = 0; i < p.max_active; ++i) s->free_slots.push(i);
  s->t0 = std::chrono::steady_clock::now();
  bool ok = hipSetDevice(ctx->device) == hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&s->slots_host),
                          2 * sizeof(double) * (size_t)p.max_active, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostMalloc(reinterpret_cast<void**>(&s->bhost), L.ws, hipHostMallocDefault) ==
                hipSuccess &&
            hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&s->entry, hipEventDisableTiming) == hipSuccess &&
            (p.batch_max_n == 0 || batched_allow_lds() == hipSuccess);
  for (int i = 0; ok && i < s->n_streams; ++i)
    ok = hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    nn_server_destroy(s);
    return NN_ERR_HIP;
  }
  *out = s;
  return NN_OK;
}

void nn_server_destroy(nn_server* s) {
  if (!s) return;
  (void)hipSetDevice(s->ctx->device);
  for (int i = 0; i < kMaxStreams; ++i) {
    if (s->streams[i]) {
      (void)hipStreamSynchronize(s->streams[i]);
      (void)hipStreamDestroy(s->streams[i]);
    }
    if (s->done[i]) (void)hipEventDestroy(s->done[i]);
  }
  if (s->ctl) {
    (void)hipStreamSynchronize(s->ctl);
    (void)hipStreamDestroy(s->ctl);
  }
  if (s->entry) (void)hipEventDestroy(s->entry);
  if (s->slots_host) (void)hipHostFree(s->slots_host);
  if (s->bhost) (void)hipHostFree(s->bhost);
  std::vector<Request*> all;
  for (auto& kv : s->by_id) all.push_back(kv.second);
  for (Request* q : s->unpolled)
    if (q->dropped) all.push_back(q);  // released before it was polled
  for (Request* q : all) delete q;
  delete s;
}

size_t nn_server_footprint(const nn_server* s, int64_t n, nn_dtype dtype, double tol) {
  if (!s || n < 1 || dtype < NN_F64 || dtype > NN_C128 || !(tol >= 0.0)) return 0;
  return footprint_of(s, n, dtype, tol, nullptr);
}

nn_status nn_server_submit(nn_server* s, int64_t id, const void* A, int64_t lda, int64_t n,
                           nn_dtype dtype, double tol, int32_t max_iter) {
  if (!s || !A || n < 1 || lda < n || !(tol >= 0.0) || max_iter < 1) return NN_ERR_ARG;
  if (dtype < NN_F64 || dtype > NN_C128) return NN_ERR_ARG;
  if (s->by_id.count(id)) return NN_ERR_ARG;
  if (footprint_of(s, n, dtype, tol, nullptr) > s->pool_bytes) return NN_ERR_WORKSPACE;
  Request* q = new (std::nothrow) Request();
  if (!q) return NN_ERR_HIP;
  q->id = id;
  q->n = n;
  q->dt = dtype;
  q->tol = tol;
  q->max_iter = max_iter;
  q->src = A;
  q->src_ld = lda;
  q->t_submit = s->now();
  s->queued.push_back(q);
  s->by_id[id] = q;
  return NN_OK;
}

nn_status nn_server_tick(nn_server* s, nn_server_stats* stats) {
  if (!s) return NN_ERR_ARG;
  if (hipSetDevice(s->ctx->device) != hipSuccess) return NN_ERR_HIP;
  // Work the caller enqueued on the context stream (e.g. producing A) comes first.
  HIP_TRY(hipEventRecord(s->entry, s->ctx->stream));
  for (int i = 0; i < s->n_streams; ++i) HIP_TRY(hipStreamWaitEvent(s->streams[i], s->entry, 0));
  nn_status st = admit(s);
  if (st != NN_OK) return st;
  st = launch_small(s);
  if (st != NN_OK) return st;
  if (s->active.empty()) {
    fill_stats(s, 0, stats);
    return NN_OK;
  }
  int hi = 0;
  for (Request* q : s->active) hi = std::max(hi, q->slot + 1);
  for (int i = 0; i < s->n_streams; ++i) {
    HIP_TRY(hipEventRecord(s->done[i], s->streams[i]));
    HIP_TRY(hipStreamWaitEvent(s->ctl, s->done[i], 0));
  }
  HIP_TRY(hipMemcpyAsync(s->slots_host, s->slots_dev, 2 * sizeof(double) * (size_t)hi,
                         hipMemcpyDeviceToHost, s->ctl));
  HIP_TRY(hipStreamSynchronize(s->ctl));
  int fin = 0;
  std::vector<Request*> still;
  still.reserve(s->active.size());
  for (Request* q : s->active) {
    bool keep = false;
    st = step_request(s, q, &keep);
    if (st != NN_OK) return st;
    if (keep)
      still.push_back(q);
    else
      ++fin;
  }
  s->active.swap(still);
  fill_stats(s, fin, stats);
  return NN_OK;
}

int32_t nn_server_poll(nn_server* s, nn_request_info* out, int32_t max) {
  if (!s || !out || max < 1) return 0;
  int32_t k = 0;
  while (k < max && !s->unpolled.empty()) {
    Request* q = s->unpolled.front();
    s->unpolled.pop_front();
    if (q->dropped) {
      delete q;
      continue;
    }
    q->polled = true;
    nn_request_info& r = out[k++];
    r.id = q->id;
    r.status = q->status;
    r.iters = q->iters;
    r.wide_iters = q->wide_iters;
    r.out_dtype = q->ph[q->cur_ph].dt;
    r.n = q->n;
    r.rms = q->rms;
    r.t_submit = q->t_submit;
    r.t_admit = q->t_admit;
    r.t_finish = q->t_finish;
  }
  return k;
}

nn_status nn_server_fetch(nn_server* s, int64_t id, void* dst, int64_t ldd) {
  if (!s || !dst) return NN_ERR_ARG;
  Request* q = find_retired(s, id);
  if (!q || ldd < q->n) return NN_ERR_ARG;
  if (q->status >= 0) {
    const PhaseBufs& P = q->ph[q->cur_ph];
    const size_t e = elem_size(P.dt);
    hipStream_t st = s->streams[q->stream];
    HIP_TRY(hipMemcpy2DAsync(dst, (size_t)ldd * e, P.X[q->result_buf], (size_t)q->n * e,
                             (size_t)q->n * e, (size_t)q->n, hipMemcpyDefault, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  drop(s, q);
  return NN_OK;
}

nn_status nn_server_release(nn_server* s, int64_t id) {
  if (!s) return NN_ERR_ARG;
  Request* q = find_retired(s, id);
  if (!q) return NN_ERR_ARG;
  drop(s, q);
  return NN_OK;
}

}  // extern "C"
