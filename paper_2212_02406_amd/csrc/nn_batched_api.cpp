// nn_batched_api.cpp — C ABI of the batched persistent inversion (see include/nn.h).
//
// A call enqueues two kernels (plan, persistent) that are captured once into
// a HIP graph on a private stream and replayed on the caller's stream while
// the arguments stay the same; the graph holds no memset node (the plan
// kernel resets the work counter itself).  The kernel configuration
// (matrices per wave threshold, workgroups per CU) comes from the context's
// autotune table, filled by nn_batched_autotune (or read from the autotune
// cache file named by NN_AUTOTUNE_CACHE), else from a default.  The one-wave
// size limit is always clamped to what the LDS of one workgroup holds at the
// call's depth.  NN_BATCHED_GRID (a positive integer) overrides the number of
// persistent workgroups, for tests that make one workgroup process many work
// items back to back.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "nn_internal.h"

namespace nn {
namespace {

nn_status check_batched(nn_ctx* ctx, const void* A, const void* X, const int64_t* offsets,
                        const int32_t* sizes, int32_t batch, int32_t max_n, nn_dtype dt,
                        const nn_params* p) {
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
  return NN_OK;
}

nn_status check_ws(int32_t batch, void* ws, size_t ws_bytes) {
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

// Workgroups of the persistent kernel one CU holds, from their LDS (dynamic
// buffers plus the kernel's static LDS), at most 8.
int max_wg_per_cu(nn_dtype dt, int max_n, int wave_max_k, int depth) {
  const size_t lds = batched_lds_bytes(dt, max_n, wave_max_k, depth) + batched_static_lds();
  return std::max(1, (int)std::min<size_t>(8, kBatchedLdsCu / lds));
}

// NN_BATCHED_GRID: a forced number of persistent workgroups (0: none).
int grid_override() {
  const char* v = getenv("NN_BATCHED_GRID");
  if (!v) return 0;
  const long g = strtol(v, nullptr, 10);
  return g > 0 && g <= (1 << 20) ? (int)g : 0;
}

// Kernel configuration of one launch: the one-wave size limit (fitted to the
// LDS at this depth) and the persistent grid.
void configure(nn_ctx* ctx, const BatchedTune& t, nn_dtype dt, int max_n, int depth, int batch,
               int* wave_max_k, int* grid) {
  const int wk = batched_fit_wave_max_k(dt, max_n, std::min({t.wave_max_k, max_n, 32}), depth);
  const int per_cu = std::min(t.wg_per_cu, max_wg_per_cu(dt, max_n, wk, depth));
  int g = std::max(1, std::min(batch, ctx->num_cus * per_cu));
  if (const int o = grid_override()) g = std::min(o, batch);
  *wave_max_k = wk;
  *grid = g;
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

hipError_t ensure_cap_stream(nn_ctx* ctx) {
  if (ctx->cap_stream) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  return batched_allow_lds();
}

// Launch through the cached graph (capturing it first if the key changed).
nn_status run_graph(nn_ctx* ctx, const BatchedGraph& key) {
  if (!same(ctx->bgraph, key)) {
    drop_graph(ctx);
    if (ensure_cap_stream(ctx) != hipSuccess) return NN_ERR_HIP;
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
  configure(ctx, t, dt, max_n, p->depth, batch, &k.wave_max_k, &k.grid);
  return k;
}

// ---- autotune cache file ----------------------------------------------------
// One line per entry: "<arch> <dtype> <max_n> <wave_max_k> <wg_per_cu> <ms>",
// keyed by (arch, dtype, max_n); later lines replace earlier ones.

std::mutex g_cache_mu;

const char* cache_path() {
  const char* p = getenv("NN_AUTOTUNE_CACHE");
  return p && *p ? p : nullptr;
}

bool cache_read(const char* path, const char* arch, nn_dtype dt, int max_n, BatchedTune* out,
                float* ms) {
  FILE* f = fopen(path, "r");
  if (!f) return false;
  char a[64];
  int d, mn, wk, wg;
  float t;
  bool found = false;
  while (fscanf(f, "%63s %d %d %d %d %f", a, &d, &mn, &wk, &wg, &t) == 6) {
    if (strcmp(a, arch) == 0 && d == (int)dt && mn == max_n && wk >= 0 && wk <= 32 && wg >= 1 &&
        wg <= 8) {
      out->dtype = d;
      out->max_n = mn;
      out->wave_max_k = wk;
      out->wg_per_cu = wg;
      *ms = t;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void cache_write(const char* path, const char* arch, const BatchedTune& t, float ms) {
  FILE* f = fopen(path, "a");
  if (!f) return;  // the cache is an optimisation: an unwritable path only costs a re-tune
  fprintf(f, "%s %d %d %d %d %.6f\n", arch, t.dtype, t.max_n, t.wave_max_k, t.wg_per_cu, ms);
  fclose(f);
}

}  // namespace

// Uncaptured launch for callers whose arguments change on every call.  The
// configuration is the context's entry for (dtype, 64) whatever the batch's
// largest size, so a matrix's path (one wave or a group) depends on its own
// size only; the arithmetic is the same on either path.
hipError_t launch_batched_direct(nn_ctx* ctx, BatchedArgs a, hipStream_t s) {
  const BatchedTune t = lookup(ctx, a.dt, 64);
  configure(ctx, t, a.dt, a.max_n, a.depth, a.batch, &a.wave_max_k, &a.grid);
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
  nn_status v = check_batched(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype, params);
  if (v != NN_OK) return v;
  if ((v = check_ws(batch, ws, ws_bytes)) != NN_OK) return v;
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  const BatchedTune t = lookup(ctx, dtype, max_n);
  return run_graph(ctx, make_key(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype,
                                 params, ws, per_matrix, t));
}

nn_status nn_batched_autotune(nn_ctx* ctx, const void* A_packed, void* X_packed,
                              const int64_t* offsets, const int32_t* sizes, int32_t batch,
                              int32_t max_n, nn_dtype dtype, const nn_params* params, void* ws,
                              size_t ws_bytes, float* best_ms, int32_t* from_cache) {
  nn_status v = check_batched(ctx, A_packed, X_packed, offsets, sizes, batch, max_n, dtype, params);
  if (v != NN_OK) return v;
  if ((v = check_ws(batch, ws, ws_bytes)) != NN_OK) return v;
  if (from_cache) *from_cache = 0;
  const char* path = cache_path();
  if (path) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    BatchedTune c;
    float ms = 0.f;
    if (cache_read(path, ctx->arch, dtype, max_n, &c, &ms)) {
      store(ctx, c);
      if (best_ms) *best_ms = ms;
      if (from_cache) *from_cache = 1;
      return NN_OK;
    }
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return NN_ERR_HIP;
  if (ensure_cap_stream(ctx) != hipSuccess) return NN_ERR_HIP;
  const int waves[] = {0, 8, 16, 32};
  BatchedTune best = lookup(ctx, dtype, max_n);
  float best_t = INFINITY;
  std::vector<std::pair<int, int>> seen;  // (fitted wave_max_k, grid) already timed
  for (int wk : waves) {
    if (wk > max_n) continue;
    const int fit = batched_fit_wave_max_k(dtype, max_n, wk, params->depth);
    if (fit != wk) continue;  // does not fit the LDS at this depth
    const int cap = max_wg_per_cu(dtype, max_n, wk, params->depth);
    for (int per_cu = 1; per_cu <= cap; per_cu *= 2) {
      BatchedTune t;
      t.dtype = dtype;
      t.max_n = max_n;
      t.wave_max_k = wk;
      t.wg_per_cu = per_cu;
      const BatchedGraph key = make_key(ctx, A_packed, X_packed, offsets, sizes, batch, max_n,
                                        dtype, params, ws, nullptr, t);
      if (std::find(seen.begin(), seen.end(), std::make_pair(key.wave_max_k, key.grid)) !=
          seen.end())
        continue;  // the same launch as a candidate already timed
      seen.emplace_back(key.wave_max_k, key.grid);
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
  if (path && isfinite(best_t)) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache_write(path, ctx->arch, best, best_t);
  }
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

int32_t nn_batched_fit_config(nn_dtype dtype, int32_t max_n, int32_t wave_max_k, int32_t depth) {
  if (max_n < 1 || max_n > 64 || wave_max_k < 0 || wave_max_k > 32 || depth < 1 ||
      depth > NN_MAX_DEPTH || (dtype != NN_C64 && dtype != NN_F32))
    return -1;
  return batched_fit_wave_max_k(dtype, max_n, wave_max_k, depth);
}

}  // extern "C"
