// Continuous-batching request scheduler over step-wise solvers.
//
// Each admitted request owns a solver and one of `max_slots` HIP streams.  Every poll()
// retires finished requests (freeing their slot and memory), admits queued requests in
// arrival order while a slot is free and their solver state fits the device-memory budget,
// and gives every resident request one more tick of iterations on its own stream, so the
// work of all resident requests is in flight on the device at once.  With a large-request
// threshold set, at most one request whose work reaches it is resident: a large request that
// would be the second waits at its place in the queue, and the requests behind it that are
// not large may be admitted past it, or, with `large_alone`, nothing is admitted while a large
// request is resident (it then shares the device only with requests admitted before it).  At most two ticks per
// request are queued ahead; a request's kernels and their order are the same whether it runs
// alone or among others, so its result is too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <deque>
#include <new>
#include <vector>

#include "internal.h"

namespace aroam {

namespace {

struct Req {
  long long id = 0;
  const Model* m = nullptr;
  int kind = 0;
  aroam_solve_opts o{};
  const void* s = nullptr;
  void* x = nullptr;
  size_t foot = 0;
  double work = 0;  // multiply-accumulates of the whole solve (the policy's size measure)
  bool large = false;
  Solver* sv = nullptr;
  int slot = -1;
  hipEvent_t ev[2] = {nullptr, nullptr};
  int ev_head = 0, ev_count = 0;  // ring of outstanding tick events
  aroam_solve_info info{};
};

}  // namespace

struct Server {
  size_t budget = 0, used = 0;
  int max_slots = 0, tick = 1;
  double large_work = 0;  // 0: no large-request policy
  bool large_alone = false;
  int large_resident = 0;
  // polls after which a request waited although a slot was free, because of the budget or of
  // the large-request policy
  long long held_budget = 0, held_large = 0;
  long long next_id = 1;
  std::vector<hipStream_t> streams;
  std::vector<char> busy;
  std::deque<Req*> queue;
  std::vector<Req*> resident;
  std::deque<Req*> done;
};

namespace {

int retire(Server& sv, Req* r) {
  r->sv->finish(&r->info);  // synchronises the request's stream; info carries the status
  delete r->sv;
  r->sv = nullptr;
  for (auto& e : r->ev)
    if (e) (void)hipEventDestroy(e);
  sv.busy[r->slot] = 0;
  sv.used -= r->foot;
  if (r->large) --sv.large_resident;
  sv.done.push_back(r);
  return AROAM_OK;
}

bool tick_done(Req* r) {
  while (r->ev_count > 0) {
    const hipError_t q = hipEventQuery(r->ev[r->ev_head]);
    if (q == hipErrorNotReady) return false;
    r->ev_head = (r->ev_head + 1) % 2;
    --r->ev_count;
  }
  return true;
}

}  // namespace

int server_create(size_t budget, int max_slots, int tick, Server** out) {
  AROAM_CHECK(out && max_slots >= 1 && max_slots <= 64 && tick >= 1, AROAM_EINVAL,
              "bad server parameters");
  Server* sv = new (std::nothrow) Server();
  AROAM_CHECK(sv, AROAM_ENOMEM, "host allocation failed");
  sv->budget = budget;
  sv->max_slots = max_slots;
  sv->tick = tick;
  sv->busy.assign(max_slots, 0);
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
      delete sv;
      set_error("stream creation failed");
      return AROAM_EDEVICE;
    }
    sv->streams.push_back(st);
  }
  *out = sv;
  return AROAM_OK;
}

int server_set_large(Server& sv, double large_work, int large_alone) {
  AROAM_CHECK(large_work >= 0, AROAM_EINVAL, "negative large-request threshold");
  AROAM_CHECK(sv.queue.empty() && sv.resident.empty(), AROAM_EINVAL,
              "the large-request threshold is set before the first submission");
  sv.large_work = large_work;
  sv.large_alone = large_alone != 0;
  return AROAM_OK;
}

int server_held(const Server& sv, long long* by_budget, long long* by_large) {
  if (by_budget) *by_budget = sv.held_budget;
  if (by_large) *by_large = sv.held_large;
  return AROAM_OK;
}

int server_submit(Server& sv, const Model& m, int kind, const aroam_solve_opts& o, const void* s,
                  void* x, long long* id) {
  AROAM_CHECK(kind == 0 || kind == 1, AROAM_EINVAL, "bad solver kind");
  AROAM_CHECK(s && x, AROAM_EINVAL, "NULL vector");
  Req* r = new (std::nothrow) Req();
  AROAM_CHECK(r, AROAM_ENOMEM, "host allocation failed");
  r->id = sv.next_id++;
  r->m = &m;
  r->kind = kind;
  r->o = o;
  r->s = s;
  r->x = x;
  r->foot = solver_footprint(m, kind, o);
  r->work = solver_work(m, kind, o);
  r->large = sv.large_work > 0 && r->work >= sv.large_work;
  sv.queue.push_back(r);
  if (id) *id = r->id;
  return AROAM_OK;
}

int server_poll(Server& sv, int* n_resident, int* n_queued) {
  // 1. retire requests whose work has all been enqueued and has completed
  for (size_t i = 0; i < sv.resident.size();) {
    Req* r = sv.resident[i];
    if (r->sv->all_enqueued() && tick_done(r)) {
      retire(sv, r);
      sv.resident.erase(sv.resident.begin() + i);
    } else {
      ++i;
    }
  }
  // 2. admit in arrival order while a slot is free and the solver state fits the budget; a
  //    large request that would be the second resident one keeps its place and is passed
  bool by_budget = false, by_large = false;
  for (auto it = sv.queue.begin(); it != sv.queue.end();) {
    Req* r = *it;
    if (r->foot > sv.budget) {  // can never fit: reject
      r->info.status = AROAM_ENOMEM;
      sv.done.push_back(r);
      it = sv.queue.erase(it);
      continue;
    }
    if (sv.large_alone && sv.large_resident > 0) {
      by_large = true;
      break;
    }
    if (r->large && sv.large_resident > 0) {
      by_large = true;
      ++it;
      continue;
    }
    int slot = -1;
    for (int k = 0; k < sv.max_slots; ++k)
      if (!sv.busy[k]) {
        slot = k;
        break;
      }
    if (slot < 0) break;
    if (sv.used + r->foot > sv.budget) {
      by_budget = true;
      break;
    }
    it = sv.queue.erase(it);
    r->slot = slot;
    int rc = solver_create(*r->m, r->kind, r->o, r->s, r->x, sv.streams[slot], &r->sv);
    if (rc == AROAM_OK) {
      for (auto& e : r->ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = AROAM_EDEVICE;
    }
    if (rc != AROAM_OK) {
      delete r->sv;
      r->sv = nullptr;
      r->info.status = rc;
      sv.done.push_back(r);
      continue;
    }
    sv.busy[slot] = 1;
    sv.used += r->foot;
    if (r->large) ++sv.large_resident;
    sv.resident.push_back(r);
  }
  if (!sv.queue.empty() && (int)sv.resident.size() < sv.max_slots) {
    if (by_budget) ++sv.held_budget;
    if (by_large) ++sv.held_large;
  }
  // 3. one more tick for every resident request with fewer than two ticks in flight
  for (Req* r : sv.resident) {
    if (r->sv->all_enqueued()) continue;
    tick_done(r);
    if (r->ev_count >= 2) continue;
    AROAM_TRY(r->sv->step(sv.tick));
    const int k = (r->ev_head + r->ev_count) % 2;
    AROAM_HIP(hipEventRecord(r->ev[k], r->sv->stream));
    ++r->ev_count;
  }
  if (n_resident) *n_resident = (int)sv.resident.size();
  if (n_queued) *n_queued = (int)sv.queue.size();
  return AROAM_OK;
}

int server_collect(Server& sv, int max, long long* ids, aroam_solve_info* infos, int* n) {
  AROAM_CHECK(n && max >= 0 && (max == 0 || ids), AROAM_EINVAL, "bad collect arguments");
  int k = 0;
  while (k < max && !sv.done.empty()) {
    Req* r = sv.done.front();
    sv.done.pop_front();
    ids[k] = r->id;
    if (infos) infos[k] = r->info;
    delete r;
    ++k;
  }
  *n = k;
  return AROAM_OK;
}

void server_destroy(Server* sv) {
  if (!sv) return;
  for (Req* r : sv->resident) {
    if (r->sv) {
      (void)hipStreamSynchronize(r->sv->stream);
      delete r->sv;
    }
    for (auto& e : r->ev)
      if (e) (void)hipEventDestroy(e);
    delete r;
  }
  for (Req* r : sv->queue) delete r;
  for (Req* r : sv->done) delete r;
  for (hipStream_t s : sv->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  delete sv;
}

}  // namespace aroam
