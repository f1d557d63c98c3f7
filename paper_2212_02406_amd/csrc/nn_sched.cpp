// nn_sched.cpp — the server's scheduling policy (see nn_sched.h).  Host-only:
// no device calls, so the CPU tests build it with g++ and AddressSanitizer.
//
// Per-request rules, applied to the rms of the current iterate (nn_invert's
// tolerance-mode rules per precision phase, Sec. II-D Theorem for the nests;
// the promotion rules are this library's):
//   den (first residual only) not finite -> NONFINITE, <= 0 -> DIVERGED
//   rms not finite                              -> NONFINITE
//   rms < tol                                   -> OK, current iterate
//   phase nests > 0, rms >= 1, rms > previous   -> DIVERGED
//   narrow, wide phase reserved, previous rms below the promotion point
//     or stagnated                              -> promote (the better of the
//                                                  last two iterates)
//   stagnated (sqrt(N) prev < 0.1, rms >= prev) -> narrow: promote if the wide
//                                                  buffers fit, else STAGNATED;
//                                                  wide: STAGNATED, previous X
//   nests == max_iter                           -> NOT_CONVERGED
#include "nn_sched.h"

#include <algorithm>
#include <iterator>

namespace nn {
namespace sched {

void PoolAlloc::reset(size_t size) {
  free_.clear();
  if (size) free_[0] = size;
  used_ = 0;
}

bool PoolAlloc::alloc(size_t bytes, size_t* off) {
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < bytes) continue;
    *off = it->first;
    const size_t rest = it->second - bytes, start = it->first + bytes;
    free_.erase(it);
    if (rest) free_[start] = rest;
    used_ += bytes;
    return true;
  }
  return false;
}

void PoolAlloc::release(size_t off, size_t bytes) {
  used_ -= bytes;
  auto it = free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}

size_t control_bytes(const ReqSizes& z) {
  return up(z.part) + up(z.denpart) + up(z.pw) + up(sizeof(double) * 8);
}

size_t phase_bytes(size_t mat, int depth) { return (size_t)mats_per_phase(depth) * up(mat); }

size_t admission_bytes(const ReqSizes& z, bool reserve_wide) {
  size_t b = control_bytes(z) + phase_bytes(z.narrow_mat ? z.narrow_mat : z.wide_mat, z.depth);
  if (z.narrow_mat && reserve_wide) b += phase_bytes(z.wide_mat, z.depth);
  return up(b);
}

PhaseLayout carve_phase(size_t mat, int depth, size_t base) {
  const size_t m = up(mat);
  PhaseLayout p;
  p.A = base;
  p.X0 = base + m;
  p.X1 = base + 2 * m;
  p.R = base + 3 * m;
  p.U0 = depth >= 2 ? base + 4 * m : 0;
  p.U1 = depth >= 3 ? base + 5 * m : 0;
  p.used = true;
  return p;
}

ReqLayout carve_block(const ReqSizes& z, bool reserve_wide) {
  ReqLayout L;
  size_t b = 0;
  L.part = b;
  b += up(z.part);
  L.denpart = b;
  b += up(z.denpart);
  L.pw = b;
  b += up(z.pw);
  L.scal = b;
  b += up(sizeof(double) * 8);
  if (z.narrow_mat) {
    L.narrow = carve_phase(z.narrow_mat, z.depth, b);
    b += phase_bytes(z.narrow_mat, z.depth);
    if (reserve_wide) {
      L.wide = carve_phase(z.wide_mat, z.depth, b);
      b += phase_bytes(z.wide_mat, z.depth);
    }
  } else {
    L.wide = carve_phase(z.wide_mat, z.depth, b);
    b += phase_bytes(z.wide_mat, z.depth);
  }
  L.end = b;
  return L;
}

int admit_scan(std::deque<Req*>& queued, size_t active, int max_active,
               const std::function<bool(Req*)>& try_alloc,
               const std::function<void(Req*)>& on_admit) {
  int scanned = 0, admitted = 0;
  bool head_blocked = false;
  for (auto it = queued.begin(); it != queued.end() && scanned < kBypassScan;) {
    if (active + (size_t)admitted >= (size_t)max_active) break;
    Req* q = *it;
    ++scanned;
    if (!try_alloc(q)) {
      if (!head_blocked) {
        head_blocked = true;
        // A request passed over too often holds the line: admit nothing after it.
        if (q->bypassed >= kMaxBypassTicks) break;
        ++q->bypassed;
      }
      ++it;
      continue;
    }
    q->state = RState::Active;
    q->fresh = true;
    ++admitted;
    it = queued.erase(it);
    on_admit(q);
  }
  return admitted;
}

namespace {

Decision retire(Req& q, int32_t status, double rms, int result_buf) {
  q.status = status;
  q.rms = rms;
  q.result_buf = result_buf;
  return Decision{Act::Retire, result_buf};
}

Decision promote(Req& q, int from) {
  q.cur_ph = 1;
  q.cur = 0;
  q.phase_k = 0;
  q.rms_prev = NAN;
  return Decision{Act::Promote, from};
}

bool wide_ready(Req& q, const std::function<bool(Req&)>& try_wide) {
  return q.has_wide || try_wide(q);
}

// The outcome of a small request's batched narrow phase.
Decision decide_small(Req& q, const nn_info_dev& r, const std::function<bool(Req&)>& try_wide) {
  q.small = false;
  q.iters = r.iters;
  q.phase_k = r.iters;
  q.cur = 0;  // the batched launch leaves its result in X[0]
  const bool ok_narrow = r.status == NN_OK && r.rms < q.tol;
  const bool to_wide = (r.status == NN_OK && !ok_narrow) || r.status == NN_STAGNATED;
  if (to_wide && wide_ready(q, try_wide)) return promote(q, 0);
  // OK, an error, or a stagnation that cannot be promoted (the
  // OK-above-tolerance case always has its wide buffers, reserved at
  // admission).
  return retire(q, r.status, r.rms, 0);
}

}  // namespace

Decision decide(Req& q, double rms, double den, int depth,
                const std::function<bool(Req&)>& try_wide, const nn_info_dev* small_rec) {
  if (q.fresh) {
    q.fresh = false;
    if (!isfinite(den) || den <= 0.0) {
      q.small = false;
      return retire(q, isfinite(den) ? NN_ERR_DIVERGED : NN_ERR_NONFINITE, NAN, q.cur);
    }
  }
  if (q.small) {
    if (!small_rec) {  // no record: the launch did not run for it
      q.small = false;
      return retire(q, NN_ERR_HIP, NAN, 0);
    }
    return decide_small(q, *small_rec, try_wide);
  }
  const bool narrow = q.cur_ph == 0;
  const double sqn = sqrt((double)q.n);
  if (!isfinite(rms)) return retire(q, NN_ERR_NONFINITE, rms, q.cur);
  if (rms < q.tol) return retire(q, NN_OK, rms, q.cur);
  if (q.phase_k > 0 && rms >= 1.0 && rms > q.rms_prev)
    return retire(q, NN_ERR_DIVERGED, rms, q.cur);
  const bool stagnated = q.phase_k > 0 && sqn * q.rms_prev < 0.1 && rms >= q.rms_prev;
  if (narrow) {
    const bool early = q.reserve_wide && q.phase_k > 0 && q.rms_prev < promotion_point(depth);
    if (early || stagnated) {
      if (wide_ready(q, try_wide)) {
        const bool back = q.phase_k > 0 && q.rms_prev <= rms;  // continue from X_{k-1}
        if (back) --q.iters;
        return promote(q, back ? q.cur ^ 1 : q.cur);
      }
      if (stagnated) {
        --q.iters;
        return retire(q, NN_STAGNATED, q.rms_prev, q.cur ^ 1);
      }
    }
  } else if (stagnated) {
    --q.iters;
    --q.wide_iters;
    return retire(q, NN_STAGNATED, q.rms_prev, q.cur ^ 1);
  }
  if (q.iters >= q.max_iter) return retire(q, NN_NOT_CONVERGED, rms, q.cur);
  q.rms_prev = rms;
  const int from = q.cur;
  q.cur ^= 1;
  ++q.iters;
  ++q.phase_k;
  if (!narrow) ++q.wide_iters;
  return Decision{Act::Nest, from};
}

}  // namespace sched
}  // namespace nn
