// Host-only driver of the server's scheduling policy (nn_sched.cpp) for the
// CPU tests: a fake device that answers each residual with the next value of
// a per-request rms sequence given by the test, a tick counter for a clock,
// and host buffers standing in for the pool blocks.  Built by the tests with
// g++ and AddressSanitizer / UndefinedBehaviorSanitizer.
//
// Input (stdin, whitespace separated):
//   depth max_active wide_tol pool_bytes batch_max_n ticks_max
//   count
//   then per request:
//     id n dtype tol max_iter arrival_tick den
//     nn v_0 .. v_{nn-1}     rms of the narrow iterates X_0, X_1, ... (nn may be 0)
//     nw w_0 .. w_{nw-1}     rms of the wide iterates
//     has_rec [iters status rms]   the batched record of a small request
// A phase reads its sequence at index phase_k (the last value past its end).
// Output: one line per request in id order
//   id status iters wide_iters rms result_buf admit_tick finish_tick bypassed
//   promoted small
// then "max_used <bytes>", "max_active <count>", "ticks <count>",
// "end_used <bytes> <free ranges>", and "violation <text>" for every broken
// invariant (none expected).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <deque>
#include <map>
#include <string>
#include <vector>

#include "../paper_2212_02406_amd/csrc/nn_sched.h"

using namespace nn::sched;

namespace {

struct Held {
  size_t off = 0, bytes = 0;
  unsigned char* host = nullptr;  // a buffer of exactly `bytes`
};

struct SimReq : Req {
  int arrival = 0;
  double den = 1.0;
  std::vector<double> seq[2];
  bool has_rec = false;
  nn_info_dev rec{};
  Held narrow, wide;
  int admit_tick = -1, finish_tick = -1;
  bool promoted = false, was_small = false;
  size_t wide_mat = 0;
};

std::vector<std::string> violations;
void violate(const std::string& s) { violations.push_back(s); }

size_t esize(int dt) { return dt == NN_F64 || dt == NN_C64 ? 8 : dt == NN_F32 ? 4 : 16; }

ReqSizes sizes(const SimReq& q, int depth) {
  ReqSizes z;
  const size_t t = (size_t)((q.n + 31) / 32) * (size_t)((q.n + 31) / 32);
  z.part = 8 * t;
  z.denpart = 8 * (size_t)(q.n + 2);
  z.pw = 8 * (size_t)(2 * q.n + 4);
  const size_t nn = (size_t)q.n * (size_t)q.n;
  z.narrow_mat = single_dtype(q.dt) ? nn * esize(q.dt) : 0;
  z.wide_mat = nn * esize(widen(q.dt));
  z.depth = depth;
  return z;
}

// Fill a block's host buffer region by region: every carved array must lie
// inside the block (ASan reports a write past the buffer), be aligned, and
// no two arrays may overlap.
void touch_layout(SimReq& q, const ReqLayout& L, const ReqSizes& z, int depth) {
  unsigned char* b = q.narrow.host;
  std::vector<std::pair<size_t, size_t>> used;  // (offset, length)
  auto put = [&](size_t off, size_t len, const char* what) {
    if (off + len > q.narrow.bytes) {
      violate(std::string("carve past block: ") + what);
      return;
    }
    if (off % kAlign) violate(std::string("misaligned: ") + what);
    used.push_back({off, len});
    memset(b + off, 0xA5, len);
  };
  put(L.part, z.part, "part");
  put(L.denpart, z.denpart, "denpart");
  put(L.pw, z.pw, "pw");
  put(L.scal, 64, "scal");
  auto phase = [&](const PhaseLayout& P, size_t mat, const char* nm) {
    if (!P.used) return;
    put(P.A, mat, nm);
    put(P.X0, mat, nm);
    put(P.X1, mat, nm);
    put(P.R, mat, nm);
    if (depth >= 2) put(P.U0, mat, nm);
    if (depth >= 3) put(P.U1, mat, nm);
  };
  phase(L.narrow, z.narrow_mat, "narrow");
  phase(L.wide, z.wide_mat, "wide");
  std::sort(used.begin(), used.end());
  for (size_t i = 1; i < used.size(); ++i)
    if (used[i - 1].first + used[i - 1].second > used[i].first) violate("overlapping arrays");
  if (L.end > q.narrow.bytes) violate("layout end past block");
}

}  // namespace

int main() {
  int depth, max_active, batch_max_n, ticks_max, count;
  double wide_tol;
  size_t pool_bytes;
  if (scanf("%d %d %lf %zu %d %d %d", &depth, &max_active, &wide_tol, &pool_bytes, &batch_max_n,
            &ticks_max, &count) != 7)
    return 2;
  std::vector<SimReq*> reqs;
  for (int i = 0; i < count; ++i) {
    SimReq* q = new SimReq();
    int dt;
    if (scanf("%ld %ld %d %lf %d %d %lf", &q->id, &q->n, &dt, &q->tol, &q->max_iter, &q->arrival,
              &q->den) != 7)
      return 2;
    q->dt = static_cast<nn_dtype>(dt);
    for (int ph = 0; ph < 2; ++ph) {
      int m;
      if (scanf("%d", &m) != 1) return 2;
      q->seq[ph].resize(m);
      for (int j = 0; j < m; ++j)
        if (scanf("%lf", &q->seq[ph][j]) != 1) return 2;
    }
    int hr;
    if (scanf("%d", &hr) != 1) return 2;
    if (hr) {
      q->has_rec = true;
      if (scanf("%d %d %lf", &q->rec.iters, &q->rec.status, &q->rec.rms) != 3) return 2;
    }
    reqs.push_back(q);
  }

  PoolAlloc alloc;
  alloc.reset(pool_bytes);
  std::deque<Req*> queued;
  std::vector<SimReq*> active;
  size_t max_used = 0, max_act = 0, held_bytes = 0;
  int done = 0, tick = 0;
  size_t next = 0;
  std::vector<SimReq*> by_arrival(reqs);
  std::stable_sort(by_arrival.begin(), by_arrival.end(),
                   [](const SimReq* a, const SimReq* b) { return a->arrival < b->arrival; });

  auto release = [&](Held& h) {
    if (!h.host) return;
    alloc.release(h.off, h.bytes);
    held_bytes -= h.bytes;
    free(h.host);
    h.host = nullptr;
  };

  for (tick = 0; done < count && tick < ticks_max; ++tick) {
    while (next < by_arrival.size() && by_arrival[next]->arrival <= tick)
      queued.push_back(by_arrival[next++]);
    // admission
    auto try_alloc = [&](Req* r) {
      SimReq* q = static_cast<SimReq*>(r);
      q->reserve_wide = single_dtype(q->dt) && q->tol < wide_tol;
      const size_t b = admission_bytes(sizes(*q, depth), q->reserve_wide);
      size_t off;
      if (!alloc.alloc(b, &off)) return false;
      q->narrow = {off, b, static_cast<unsigned char*>(malloc(b))};
      held_bytes += b;
      return true;
    };
    auto on_admit = [&](Req* r) {
      SimReq* q = static_cast<SimReq*>(r);
      const ReqSizes z = sizes(*q, depth);
      const ReqLayout L = carve_block(z, q->reserve_wide);
      touch_layout(*q, L, z, depth);
      q->has_wide = L.wide.used;
      q->cur_ph = L.narrow.used ? 0 : 1;
      q->wide_mat = z.wide_mat;
      q->small = single_dtype(q->dt) && q->n <= batch_max_n && q->max_iter <= 4096;
      q->was_small = q->small;
      q->admit_tick = tick;
      q->cur = 0;
      active.push_back(q);
    };
    // a request passed over kMaxBypassTicks times holds the line: when the
    // first request of the queue left waiting had been passed over that
    // often before this tick, nothing behind it may be admitted this tick
    std::vector<std::pair<Req*, int>> before;
    for (Req* r : queued) before.push_back({r, r->bypassed});
    admit_scan(queued, active.size(), max_active, try_alloc, on_admit);
    size_t i = 0;
    while (i < before.size() && before[i].first->state != RState::Queued) ++i;
    if (i < before.size() && before[i].second >= kMaxBypassTicks)
      for (size_t j = i + 1; j < before.size(); ++j)
        if (before[j].first->state != RState::Queued)
          violate("request admitted behind a request passed over too often");
    if (alloc.used() != held_bytes) violate("allocator used != held bytes");
    if (alloc.used() > pool_bytes) violate("pool overcommitted");
    max_used = std::max(max_used, alloc.used());
    max_act = std::max(max_act, active.size());
    if ((int)active.size() > max_active) violate("more than max_active requests active");
    // the fake device's read-back, then the rules
    std::vector<SimReq*> still;
    for (SimReq* q : active) {
      const std::vector<double>& sq = q->seq[q->cur_ph];
      double rms = NAN;
      if (!sq.empty()) rms = sq[std::min((size_t)q->phase_k, sq.size() - 1)];
      auto try_wide = [&](Req& r) {
        SimReq* w = static_cast<SimReq*>(&r);
        if (w->has_wide) return true;
        const size_t b = up(phase_bytes(w->wide_mat, depth));
        size_t off;
        if (!alloc.alloc(b, &off)) return false;
        w->wide = {off, b, static_cast<unsigned char*>(malloc(b))};
        held_bytes += b;
        const PhaseLayout P = carve_phase(w->wide_mat, depth, 0);
        const size_t last = depth >= 3 ? P.U1 : depth >= 2 ? P.U0 : P.R;
        if (last + w->wide_mat > b) violate("late wide phase past its block");
        memset(w->wide.host, 0x5A, b);
        w->has_wide = true;
        return true;
      };
      const nn_info_dev* rec = q->small ? (q->has_rec ? &q->rec : nullptr) : nullptr;
      const Decision d = decide(*q, rms, q->den, depth, try_wide, rec);
      if (d.act == Act::Promote) q->promoted = true;
      if (d.act == Act::Retire) {
        q->state = RState::Retired;
        q->finish_tick = tick;
        release(q->narrow);
        release(q->wide);
        ++done;
      } else {
        if (d.act == Act::Nest && (d.from ^ 1) != q->cur) violate("nest target is not cur");
        still.push_back(q);
      }
    }
    active.swap(still);
    if (alloc.used() != held_bytes) violate("allocator used != held bytes after rules");
  }

  std::sort(reqs.begin(), reqs.end(), [](const SimReq* a, const SimReq* b) { return a->id < b->id; });
  for (SimReq* q : reqs) {
    printf("%ld %d %d %d %.17g %d %d %d %d %d %d\n", q->id, q->state == RState::Retired ? q->status : 99,
           q->iters, q->wide_iters, q->rms, q->result_buf, q->admit_tick, q->finish_tick,
           q->bypassed, (int)q->promoted, (int)q->was_small);
  }
  printf("max_used %zu\nmax_active %zu\nticks %d\n", max_used, max_act, tick);
  for (SimReq* q : reqs) {
    release(q->narrow);
    release(q->wide);
  }
  printf("end_used %zu %zu\n", alloc.used(), alloc.free_ranges());
  for (auto& v : violations) printf("violation %s\n", v.c_str());
  for (SimReq* q : reqs) delete q;
  return 0;
}
