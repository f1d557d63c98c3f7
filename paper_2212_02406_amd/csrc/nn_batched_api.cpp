// nn_batched.cpp — C ABI of the batched persistent inversion (see include/nn.h).
//
// A call enqueues two kernels (plan, persistent) that are captured once into
// a HIP graph on a private stream and replayed on the caller's stream while
// the arguments stay the same; the graph holds no memset node (the plan
// kernel resets the work counter itself).  The kernel configuration
// (matrices per wave threshold, workgroups per CU) comes from the context's
// autotune table, filled by nn_batched_autotune, else from a default.
#include <math.h>
#include <string.h>

#include <algorithm>

#include "nn_internal.h"

namespace nn {
namespace {

constexpr size_t kLdsPerCu = 160 * 1024;

nn_status check_batched(nn_ctx* ctx, const void* A, const void* X, const int64_t* offsets,
                        const int32_t* sizes, int32_t batch, int32_t max_n, nn_dtype dt,
                        const nn_params* p, void* ws, size_t ws_bytes) {
  if (!ctx || !A || !X || !offsets || !sizes || batch < 1 || max_n < 1 || max_n > 64 || !p)
    return NN_ERR_ARG;
  if (A == X) return NN_ERR_ARG;
  if (dt != NN_C64 && dt != NN_F32) return NN_ERR_UNSUPPORTED;
  if (p->depth < 1 || p->depth > NN_MAX_DEPTH || p->flags != 0) return NN_ERR_ARG;
  if (p->x0 != NN_X0_TRANSPOSE && p->x0 != NN_X0_SCALED_IDENTITY && p->x0 != NN_X0_GIVEN)
    return NN_ERR_UNSUPPORTED;
  if (p->fixed_iter < 0) return NN_ERR_ARG;
  if (p->fixed_iter == 0 &&
      (!(p->tol >= 0.0) || p->max_iter < 1 || p->max_iter > kBatchedMaxIter))
    return NN_ERR_ARG;
  if (p->prec != NN_PREC_PLAIN) return NN_ERR_UNSUPPORTED;
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255u) || ws_bytes < batched_ws_bytes(batch))
    return NN_ERR_WORKSPACE;
  return NN_OK;
}

BatchedTune lookup(nn_ctx* ctx, nn_dtype dt, int max_n) {
  for (const BatchedTune& t : ctx->tune)
    if (t.dtype == (int)dt && t.max_n == max_n) return t;
  BatchedTune d;
  d.dtype = dt;
  d.max_n = max_n;
  d.wave_max_k = std::min(16, max_n);
  d.wg_per_cu = 1;
  return d;
}

void store(nn_ctx* ctx, const BatchedTune& t) {
  for (BatchedTune& s : ctx->tune)
    if (s.dtype == t.dtype && s.max_n == t.max_n) {
      s = t;
      return;
    }
  for (BatchedTune& s : ctx->tune)
    if (s.dtype < 0) {
      s = t;
      return;
    }
  ctx->tune[0] = t;
}

int max_wg_per_cu(nn_dtype dt, int max_n, int wave_max_k, int depth) {
  const size_t lds = batched_lds_bytes(dt, max_n, wave_max_k, depth) + 4 * 1024;  // + static LDS
  return std::max(1, (int)std::min<size_t>(8, kLdsPerCu / lds));
}

void drop_graph(nn_ctx* ctx) {
  if (ctx->bgraph.exec) (void)hipGraphExecDestroy(ctx->bgraph.exec);
  if (ctx->bgraph.graph) (void)hipGraphDestroy(ctx->bgraph.graph);
  ctx->bgraph = BatchedGraph();
}

bool same(const BatchedGraph& g, const BatchedGraph& k) {
  return g.exec && g.A == k.A && g.X == k.X && g.offsets == k.offsets && g.sizes == k.sizes &&
         g.ws == k.ws && g.info == k.info && g.batch == k.batch && g.max_n == k.max_n &&
         g.dtype == k.dtype && g.depth == k.depth && g.x0 == k.x0 && g.iters == k.iters &&
         g.wave_max_k == k.wave_max_k && g.grid == k.grid && g.tol == k.tol &&
         g.max_iter == k.max_iter;
}

BatchedArgs args_of(const BatchedGraph& k) {
  BatchedArgs a;
  a.dt = (nn_dtype)k.dtype;
  a.A = k.A;
  a.X = k.X;
  a.offsets = k.offsets;
  a.sizes = k.sizes;
  a.batch = k.batch;
  a.max_n = k.max_n;
  a.depth = k.depth;
  a.x0 = k.x0;
  a.iters = k.iters;
  a.tol = k.tol;
  a.max_iter = k.max_iter;
  a.wave_max_k = k.wave_max_k;
  a.ws = k.ws;
  a.info = k.info;
  a.grid = k.grid;
  return a;
}

// Launch through the cached graph (capturing it first if the key changed).
nn_status run_graph(nn_ctx* ctx, const BatchedGraph& key) {
#ifdef NN_DIAG_NOGRAPH
  if (!ctx->cap_stream) {
    if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess) return NN_ERR_HIP;
    if (batched_allow_lds() != hipSuccess) return NN_ERR_HIP;
  }
  return launch_batched(args_of(key), ctx->stream) == hipSuccess ? NN_OK : NN_ERR_HIP;
#endif
  if (!same(ctx->bgraph, key)) {
    drop_graph(ctx);
    if (!ctx->cap_stream) {
      if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return NN_ERR_HIP;
      if (batched_allow_lds() != hipSuccess) return NN_ERR_HIP;
    }
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return NN_ERR_HIP;
    hipError_t le = launch_batched(args_of(key), ctx->cap_stream);
    hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (le != hipSuccess || ce != hipSuccess || !graph) {
      if (graph) (void)hipGraphDestroy(graph);
      return NN_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return NN_ERR_HIP;
    }
    ctx->bgraph = key;
    ctx->bgraph.graph = graph;
    ctx->bgraph.exec = exec;
  }
  if (hipGraphLaunch(ctx->bgraph.exec, ctx->stream) != hipSuccess) return NN_ERR_HIP;
  return NN_OK;
}

BatchedGraph make_key(nn_ctx* ctx, const void* A, void* X, const int64_t* offsets,
                      const int32_t* sizes, int32_t batch, int32_t max_n, nn_dtype dt,
                      const nn_params* p, void* ws, nn_info_dev* info, const BatchedTune& t) {
  BatchedGraph k;
  k.A = A;
  k.X = X;
  k.offsets = offsets;
  k.sizes = sizes;
  k.ws = ws;
  k.info = info;
  k.batch = batch;
  k.max_n = max_n;
  k.dtype = dt;
  k.depth = p->depth;
  k.x0 = p->x0;
  k.iters = p->fixed_iter;
  k.tol = p->fixed_iter > 0 ? 0.0 : p->tol;
  k.max_iter = p->fixed_iter > 0 ? 0 : p->max_iter;
  k.wave_max_k = std::min({t.wave_max_k, max_n, 32});
  const int per_cu = std::min(t.wg_per_cu, max_wg_per_cu(dt, max_n, k.wave_max_k, p->depth));
  k.grid = std::max(1, std::min(batch, ctx->num_cus * per_cu));
#ifdef NN_DIAG_GRID
  k.grid = NN_DIAG_GRID;
#endif
  return k;
}

}  // namespace

// Uncaptured launch for callers whose arguments change on every call.  The
// configuration is the context's entry for (dtype, 64) whatever the batch's
// largest size, so a matrix's path (one wave or a group) depends on its own
// size only; the arithmetic is the same on either path.
hipError_t launch_batched_direct(nn_ctx* ctx, BatchedArgs a, hipStream_t s) {
  const BatchedTune t = lookup(ctx, a.dt, 64);
  a.wave_max_k = std::min({t.wave_max_k, a.max_n, 32});
  const int per_cu = std::min(t.wg_per_cu, max_wg_per_cu(a.dt, a.max_n, a.wave_max_k, a.depth));
  a.grid = std::max(1, std::min(a.batch, ctx->num_cus * per_cu));
  return launch_batched(a, s);
}

}  // namespace nn

using namespace nn;

extern "C" {

size_t nn_batched_workspace_size(int32_t batch, nn_dtype dtype) {
  if (batch < 1 || (dtype != NN_C64 && dtype != NN_F32)) return 0;
  return batched_ws_bytes(batch);
}

nn_status nn_invert_batched(nn_ctx* ctx, const void* A_packed, void* X_packed,
                            const int64_t* offsets, const int32_t* sizes, int32_t batch,
                            int32_t max_n, nn_dtype dtype, const nn_params* params, void* ws,
                            size_t ws_bytes, nn_info_dev* per_matrix) {
  nn_status v = check_batched(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype, params,
                              ws, ws_bytes);
  if (v != NN_OK) return v;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const BatchedTune t = lookup(ctx, dtype, max_n);
  return run_graph(ctx, make_key(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype,
                                 params, ws, per_matrix, t));
}

nn_status nn_batched_autotune(nn_ctx* ctx, const void* A_packed, void* X_packed,
                              const int64_t* offsets, const int32_t* sizes, int32_t batch,
                              int32_t max_n, nn_dtype dtype, const nn_params* params, void* ws,
                              size_t ws_bytes, float* best_ms) {
  nn_status v = check_batched(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype, params,
                              ws, ws_bytes);
  if (v != NN_OK) return v;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const int waves[] = {0, 8, 16, 32};
  BatchedTune best = lookup(ctx, dtype, max_n);
  float best_t = INFINITY;
  for (int wk : waves) {
    if (wk > max_n) continue;
    const int cap = max_wg_per_cu(dtype, max_n, wk, params->depth);
    for (int per_cu = 1; per_cu <= cap; per_cu *= 2) {
      BatchedTune t;
      t.dtype = dtype;
      t.max_n = max_n;
      t.wave_max_k = wk;
      t.wg_per_cu = per_cu;
      const BatchedGraph key = make_key(ctx, A_packed, X_packed, offsets, sizes, batch, max_n,
                                        dtype, params, ws, nullptr, t);
      float ms_min = INFINITY;
      for (int rep = 0; rep < 3; ++rep) {
        if (hipEventRecord(ctx->ev_start, ctx->stream) != hipSuccess) return NN_ERR_HIP;
        nn_status st = run_graph(ctx, key);
        if (st != NN_OK) return st;
        if (hipEventRecord(ctx->ev_stop, ctx->stream) != hipSuccess ||
            hipEventSynchronize(ctx->ev_stop) != hipSuccess)
          return NN_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop) != hipSuccess) return NN_ERR_HIP;
        if (rep > 0) ms_min = std::min(ms_min, ms);  // the first replay includes the capture
      }
      if (ms_min < best_t) {
        best_t = ms_min;
        best = t;
      }
    }
  }
  store(ctx, best);
  if (best_ms) *best_ms = best_t;
  return NN_OK;
}

nn_status nn_batched_get_config(nn_ctx* ctx, nn_dtype dtype, int32_t max_n, int32_t* wave_max_k,
                                int32_t* wg_per_cu) {
  if (!ctx || !wave_max_k || !wg_per_cu) return NN_ERR_ARG;
  const BatchedTune t = lookup(ctx, dtype, max_n);
  *wave_max_k = t.wave_max_k;
  *wg_per_cu = t.wg_per_cu;
  return NN_OK;
}

nn_status nn_batched_set_config(nn_ctx* ctx, nn_dtype dtype, int32_t max_n, int32_t wave_max_k,
                                int32_t wg_per_cu) {
  if (!ctx || max_n < 1 || max_n > 64 || wave_max_k < 0 || wave_max_k > 32 || wg_per_cu < 1 ||
      wg_per_cu > 8)
    return NN_ERR_ARG;
  BatchedTune t;
  t.dtype = dtype;
  t.max_n = max_n;
  t.wave_max_k = wave_max_k;
  t.wg_per_cu = wg_per_cu;
  store(ctx, t);
  return NN_OK;
}

}  // extern "C"
