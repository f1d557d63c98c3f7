// nn_sched.h — the server's scheduling policy, host-only (no HIP).
//
// What nn_server decides, separated from what it enqueues: the pool
// allocator, the layout of a request's pool block, admission (first come
// first served with bounded bypass, by HBM footprint), and the per-request
// rules applied to each residual rms (nn_invert's tolerance-mode rules per
// precision phase, plus the promotion rules of the narrow phase).  nn_serve.cpp
// drives it with device work; the CPU tests drive the same code with rms
// sequences of their own and check the decisions, under AddressSanitizer.
#pragma once

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include <deque>
#include <functional>
#include <map>

#include "../../include/nn.h"

namespace nn {
namespace sched {

constexpr size_t kAlign = 256;
constexpr int kMaxBypassTicks = 8;  // ticks a blocked head may be passed over
constexpr int kBypassScan = 64;     // queued requests looked at per tick

inline size_t up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with a coalescing free list.
class PoolAlloc {
 public:
  void reset(size_t size);
  bool alloc(size_t bytes, size_t* off);
  void release(size_t off, size_t bytes);
  size_t used() const { return used_; }
  size_t free_ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

// Byte sizes that fix a request's block: the control region (tile partials of
// either precision's plan, norm partials, power-step scratch, scalars) and
// the matrices of one precision phase (A, two X, R, U at depth >= 2 and 3).
struct ReqSizes {
  size_t part = 0, denpart = 0, pw = 0;  // bytes of each control array
  size_t narrow_mat = 0;                 // one n x n matrix in the narrow dtype (0: none)
  size_t wide_mat = 0;                   // one n x n matrix in the wide dtype
  int depth = 2;
};
inline int mats_per_phase(int depth) { return 4 + (depth >= 2) + (depth >= 3); }
size_t control_bytes(const ReqSizes& z);
size_t phase_bytes(size_t mat, int depth);
// Bytes reserved at admission: control + start phase (+ the wide phase when
// reserve_wide, i.e. a single-precision request with tol < wide_tol).
size_t admission_bytes(const ReqSizes& z, bool reserve_wide);

// Offsets (from the block start) of a request's arrays.
struct PhaseLayout {
  size_t A = 0, X0 = 0, X1 = 0, R = 0, U0 = 0, U1 = 0;  // U* valid at depth >= 2 / 3
  bool used = false;
};
struct ReqLayout {
  size_t part = 0, denpart = 0, pw = 0, scal = 0;
  PhaseLayout narrow, wide;  // wide: only if carried in this block
  size_t end = 0;            // bytes used
};
// Layout of the admission block: control region, then the narrow phase (if
// the request has one), then the wide phase when it starts wide or reserves
// it at admission.
ReqLayout carve_block(const ReqSizes& z, bool reserve_wide);
// Layout of a late wide block (one phase at offset 0).
PhaseLayout carve_phase(size_t mat, int depth, size_t base);

enum class RState { Queued, Active, Retired };

// Scheduling state of one request.
struct Req {
  int64_t id = 0;
  int64_t n = 0;
  nn_dtype dt = NN_F32;
  double tol = 0.0;
  int32_t max_iter = 0;
  RState state = RState::Queued;
  int bypassed = 0;           // ticks in which later requests were admitted before it
  bool reserve_wide = false;  // wide phase reserved at admission
  bool has_wide = false;      // wide phase buffers exist
  int cur_ph = 0;             // 0 narrow (single precision), 1 wide
  bool fresh = false;         // admitted this tick: den not checked yet
  bool small = false;         // narrow phase in this tick's batched launch
  int cur = 0;                // X[cur] is the current iterate
  int iters = 0, wide_iters = 0, phase_k = 0;
  double rms_prev = NAN;
  // outcome once retired
  int32_t status = NN_OK;
  double rms = NAN;
  int result_buf = 0;
};

inline bool single_dtype(nn_dtype d) { return d == NN_F32 || d == NN_C64; }
inline nn_dtype widen(nn_dtype d) { return d == NN_F32 ? NN_F64 : d == NN_C64 ? NN_C128 : d; }

// The rms at which a narrow iterate is handed to the wide phase early: one
// nest of order d+1 from here would reach about 1e-9.
inline double promotion_point(int depth) { return pow(1e-9, 1.0 / (depth + 1)); }

// Admission scan over the queue, in order: a request is admitted when
// active + admitted < max_active and try_alloc(q) succeeds (it reserves the
// request's block).  The first request that does not fit is passed over at
// most kMaxBypassTicks ticks in a row; after that nothing behind it is
// admitted until it fits.  on_admit runs for each admitted request (which is
// removed from the queue).  Returns the number admitted.
int admit_scan(std::deque<Req*>& queued, size_t active, int max_active,
               const std::function<bool(Req*)>& try_alloc,
               const std::function<void(Req*)>& on_admit);

// What the executor does next for a request whose rules ran.
enum class Act {
  Retire,   // done: status, rms, result_buf set on the request
  Nest,     // enqueue the nest X[from] -> X[from ^ 1], then the residual of X[cur]
  Promote,  // widen A and the narrow X[from] into the wide phase's X[0], then its residual
};
struct Decision {
  Act act = Act::Retire;
  int from = 0;
};

// The rules for a request after a tick's read-back.  den: the start scale
// when q.fresh (not finite -> NONFINITE, <= 0 -> DIVERGED).  rms: the
// residual rms of the current iterate; for a small request (q.small) the
// batched kernel's per-matrix record `small_rec` of its narrow phase instead
// (its result is in X[0]).  try_wide reserves the wide phase of a request
// without one (setting has_wide) and reports success.  Updates q (counters,
// cur, phase, and the outcome when it retires) as the decision requires.
Decision decide(Req& q, double rms, double den, int depth,
                const std::function<bool(Req&)>& try_wide,
                const nn_info_dev* small_rec = nullptr);

}  // namespace sched
}  // namespace nn
