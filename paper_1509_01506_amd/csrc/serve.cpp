// libcoex serving loop: scan requests (a host sequence of ASCII bases and the
// index of a resident automaton) arrive one at a time; a worker thread
//   - admits them in arrival order into a device arena bounded by an HBM
//     budget;
//   - copies admitted requests to the device in pieces on a copy stream, with
//     at most three pieces' worth of bytes queued at a time, the request with
//     the fewest bytes left first, so a small request never waits behind the
//     whole copy of a large one;
//   - launches every admitted request whose copy has finished as one batch
//     over the resident automaton set (continuous batching: requests that
//     arrive while a batch runs join the next one);
//   - keeps up to two batches queued on the compute stream, so copies,
//     descriptor uploads and the next launch overlap the running batch;
//   - returns each request's count with its queue, copy, device and total
//     latency, and releases its arena space.
// Each request is one (sequence, automaton) pair of a batch, so its count is
// the same alone or in any mix (tests check both against the CPU oracle).
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "coex.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

// First-fit allocator over one device buffer (offsets aligned to 256 bytes).
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes
  void init(char* b, size_t n) {
    base = b;
    size = n;
    free_.clear();
    free_[0] = n;
  }
  bool alloc(size_t n, size_t& off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        off = it->first;
        const size_t rest = it->second - n;
        free_.erase(it);
        if (rest) free_[off + n] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    used -= n;
    auto it = free_.emplace(off, n).first;
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
};

struct Req {
  const void* host = nullptr;
  uint64_t n = 0;
  uint32_t dfa = 0;
  Clock::time_point t_submit, t_admit, t_launch, t_done;
  size_t off = 0, bytes = 0;
  uint64_t copied = 0;                    // bytes whose copy has been queued
  hipEvent_t c0 = nullptr, c1 = nullptr;  // before the first and after the last piece of its copy
  float device_ms = 0.f, h2d_ms = 0.f;
  uint64_t count = 0;
  uint32_t batch_size = 0;
  int status = COEX_OK;
  bool done = false;
};

struct Slot {  // one batch in flight, on a compute stream of its own (two batches can overlap)
  hipStream_t st = nullptr;
  coex_batch* batch = nullptr;
  uint64_t* counts_dev = nullptr;
  uint64_t* counts_host = nullptr;  // pinned
  uint32_t cap = 0;
  hipEvent_t start = nullptr, done = nullptr;
  std::vector<Req*> reqs;
  bool busy = false;
};

constexpr size_t kAlign = 256;

}  // namespace

struct coex_server {
  int device = 0;
  coex_dfa_set* set = nullptr;
  uint32_t n_dfa = 0;
  hipStream_t copy_st = nullptr;
  char* arena_buf = nullptr;
  Arena arena;
  uint32_t max_batch = 1024;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> pending;
  std::vector<Req*> copying;   // admitted, copy not fully queued
  std::vector<Req*> resident;  // copy fully queued (launched once it has finished)
  uint64_t piece = 16ull << 20;  // bytes per copy piece
  std::deque<std::pair<hipEvent_t, uint64_t>> inflight;  // event after each queued piece, its bytes
  std::deque<hipEvent_t> spare;
  uint64_t inflight_bytes = 0;
  uint64_t inflight_cap = 48ull << 20;  // bytes of queued pieces before the next is queued
  std::map<uint64_t, Req*> reqs;
  Slot slots[2];
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  int fatal = COEX_OK;
  coex_server_stats_t stats{};
  ~coex_server();
};

namespace {

int grow_slot(Slot& sl, uint32_t n) {
  if (sl.cap >= n) return COEX_OK;
  const uint32_t cap = std::max<uint32_t>(n, 256);
  if (sl.counts_dev) (void)hipFree(sl.counts_dev);
  if (sl.counts_host) (void)hipHostFree(sl.counts_host);
  sl.counts_dev = nullptr;
  sl.counts_host = nullptr;
  sl.cap = 0;
  if (hipMalloc(&sl.counts_dev, (size_t)cap * 8) != hipSuccess) return COEX_ENOMEM;
  if (hipHostMalloc(&sl.counts_host, (size_t)cap * 8, hipHostMallocDefault) != hipSuccess) return COEX_ENOMEM;
  sl.cap = cap;
  return COEX_OK;
}

void finish(coex_server* S, Req* r, int status) {
  r->status = status;
  r->done = true;
  r->t_done = Clock::now();
}

// Retires finished batches; returns whether anything changed.
bool retire(coex_server* S) {
  bool any = false;
  for (Slot& sl : S->slots) {
    if (!sl.busy) continue;
    const hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    float dev_ms = 0.f;
    const int st = (q == hipSuccess && hipEventElapsedTime(&dev_ms, sl.start, sl.done) == hipSuccess)
                       ? COEX_OK : COEX_EDEVICE;
    for (size_t i = 0; i < sl.reqs.size(); ++i) {
      Req* r = sl.reqs[i];
      r->count = sl.counts_host[i];
      r->device_ms = dev_ms;
      r->batch_size = (uint32_t)sl.reqs.size();
      if (r->c0) (void)hipEventElapsedTime(&r->h2d_ms, r->c0, r->c1);
      S->arena.release(r->off, r->bytes);
      finish(S, r, st);
      S->stats.n_done += 1;
      S->stats.bases_done += r->n;
    }
    S->stats.device_ms += dev_ms;
    sl.reqs.clear();
    sl.busy = false;
    any = true;
  }
  if (any) S->cv_done.notify_all();
  return any;
}

// Admits waiting requests in arrival order while the arena has room.
bool admit(coex_server* S) {
  bool any = false;
  while (!S->pending.empty()) {
    Req* r = S->pending.front();
    const size_t need = (std::max<uint64_t>(r->n, 1) + kAlign - 1) / kAlign * kAlign;
    if (need > S->arena.size) {  // can never fit
      S->pending.pop_front();
      finish(S, r, COEX_ENOMEM);
      S->cv_done.notify_all();
      continue;
    }
    size_t off = 0;
    if (!S->arena.alloc(need, off)) break;
    r->off = off;
    r->bytes = need;
    r->t_admit = Clock::now();
    S->pending.pop_front();
    if (hipEventCreate(&r->c0) != hipSuccess || hipEventCreate(&r->c1) != hipSuccess) {
      S->arena.release(off, need);
      finish(S, r, COEX_EDEVICE);
      S->cv_done.notify_all();
      continue;
    }
    S->copying.push_back(r);
    S->stats.max_arena_bytes = std::max<uint64_t>(S->stats.max_arena_bytes, S->arena.used);
    any = true;
  }
  return any;
}

// Queues copy pieces while less than three pieces' worth of bytes is in
// flight: the next piece of the admitted request with the fewest bytes left
// (the earliest admitted among equals).  A request whose last piece is
// queued becomes resident.  Pieces trade copy efficiency (each copy has a
// fixed cost) for the wait of a small request behind a large one.
constexpr size_t kMaxInflightPieces = 64;

bool feed(coex_server* S) {
  bool any = false;
  while (!S->inflight.empty() && hipEventQuery(S->inflight.front().first) != hipErrorNotReady) {
    S->spare.push_back(S->inflight.front().first);
    S->inflight_bytes -= S->inflight.front().second;
    S->inflight.pop_front();
  }
  while (!S->copying.empty() && S->inflight.size() < kMaxInflightPieces && S->inflight_bytes < S->inflight_cap) {
    size_t best = 0;
    for (size_t i = 1; i < S->copying.size(); ++i)
      if (S->copying[i]->n - S->copying[i]->copied < S->copying[best]->n - S->copying[best]->copied) best = i;
    Req* r = S->copying[best];
    const uint64_t len = std::min<uint64_t>(r->n - r->copied, S->piece);
    int st = COEX_OK;
    if (r->copied == 0 && hipEventRecord(r->c0, S->copy_st) != hipSuccess) st = COEX_EDEVICE;
    if (st == COEX_OK && len &&
        hipMemcpyAsync(S->arena.base + r->off + r->copied, static_cast<const char*>(r->host) + r->copied, len,
                       hipMemcpyHostToDevice, S->copy_st) != hipSuccess)
      st = COEX_EDEVICE;
    hipEvent_t ev = nullptr;
    if (st == COEX_OK) {
      if (!S->spare.empty()) {
        ev = S->spare.front();
        S->spare.pop_front();
      } else if (hipEventCreate(&ev) != hipSuccess) {
        ev = nullptr;
        st = COEX_EDEVICE;
      }
    }
    if (st == COEX_OK && hipEventRecord(ev, S->copy_st) != hipSuccess) st = COEX_EDEVICE;
    if (ev && st == COEX_OK) {
      S->inflight.emplace_back(ev, len);
      S->inflight_bytes += len;
    } else if (ev) {
      S->spare.push_back(ev);
    }
    r->copied += len;
    const bool last = r->copied == r->n;
    if (st == COEX_OK && last && hipEventRecord(r->c1, S->copy_st) != hipSuccess) st = COEX_EDEVICE;
    if (st != COEX_OK || last) S->copying.erase(S->copying.begin() + (std::ptrdiff_t)best);
    if (st != COEX_OK) {
      // queued pieces may still be writing the request's arena range: wait
      // for the copy stream before the range can be reused
      (void)hipStreamSynchronize(S->copy_st);
      S->arena.release(r->off, r->bytes);
      finish(S, r, st);
      S->cv_done.notify_all();
    } else if (last) {
      S->resident.push_back(r);
    }
    any = true;
  }
  return any;
}

// Launches the resident requests whose copies are done, if a slot is free.
bool launch(coex_server* S) {
  Slot* sl = nullptr;
  for (Slot& s : S->slots)
    if (!s.busy) { sl = &s; break; }
  if (!sl || S->resident.empty()) return false;
  std::vector<Req*> ready, wait;
  for (Req* r : S->resident) {
    if (ready.size() < S->max_batch && hipEventQuery(r->c1) == hipSuccess) ready.push_back(r);
    else wait.push_back(r);
  }
  if (ready.empty()) return false;
  const uint32_t n = (uint32_t)ready.size();
  std::vector<coex_seq> seqs(n);
  std::vector<uint32_t> ps(n), pd(n);
  for (uint32_t i = 0; i < n; ++i) {
    seqs[i] = coex_seq{S->arena.base + ready[i]->off, nullptr, ready[i]->n, COEX_ENC_BYTE, 0};
    ps[i] = i;
    pd[i] = ready[i]->dfa;
  }
  int st = grow_slot(*sl, n);
  if (st == COEX_OK) st = coex_batch_update(sl->batch, seqs.data(), n, ps.data(), pd.data(), n);
  if (st == COEX_OK && hipEventRecord(sl->start, sl->st) != hipSuccess) st = COEX_EDEVICE;
  if (st == COEX_OK) st = coex_batch_run(sl->batch, sl->counts_dev, sl->st);
  if (st == COEX_OK &&
      hipMemcpyAsync(sl->counts_host, sl->counts_dev, (size_t)n * 8, hipMemcpyDeviceToHost, sl->st) != hipSuccess)
    st = COEX_EDEVICE;
  if (st == COEX_OK && hipEventRecord(sl->done, sl->st) != hipSuccess) st = COEX_EDEVICE;
  S->resident.swap(wait);
  const auto now = Clock::now();
  if (st != COEX_OK) {
    for (Req* r : ready) {
      S->arena.release(r->off, r->bytes);
      finish(S, r, st);
    }
    S->cv_done.notify_all();
    return true;
  }
  for (Req* r : ready) r->t_launch = now;
  sl->reqs = std::move(ready);
  sl->busy = true;
  S->stats.n_batches += 1;
  return true;
}

void loop(coex_server* S) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool any = retire(S);
    any |= admit(S);
    any |= feed(S);
    any |= launch(S);
    const bool idle = S->pending.empty() && S->copying.empty() && S->resident.empty() && S->inflight.empty() &&
                      !S->slots[0].busy && !S->slots[1].busy;
    if (S->stop && idle) break;
    if (!any) {
      if (idle) S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
      else S->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

}  // namespace

coex_server::~coex_server() {
  if (worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv_work.notify_all();
    worker.join();
  }
  for (auto& kv : reqs) {
    Req* r = kv.second;
    if (r->c0) (void)hipEventDestroy(r->c0);
    if (r->c1) (void)hipEventDestroy(r->c1);
    delete r;
  }
  for (auto& e : inflight) (void)hipEventDestroy(e.first);
  for (hipEvent_t e : spare) (void)hipEventDestroy(e);
  for (Slot& sl : slots) {
    if (sl.batch) coex_batch_free(sl.batch);
    if (sl.counts_dev) (void)hipFree(sl.counts_dev);
    if (sl.counts_host) (void)hipHostFree(sl.counts_host);
    if (sl.start) (void)hipEventDestroy(sl.start);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.st) (void)hipStreamDestroy(sl.st);
  }
  if (arena_buf) (void)hipFree(arena_buf);
  if (copy_st) (void)hipStreamDestroy(copy_st);
  if (set) coex_dfa_set_free(set);
}

extern "C" {

int coex_server_create(const coex_dfa* const* dfas, uint32_t n_dfa, const coex_server_opts* o, coex_server** out) {
  if (!out || !dfas || !n_dfa) return COEX_EINVAL;
  try {
    auto* S = new coex_server();
    std::unique_ptr<coex_server> guard(S);
    if (hipGetDevice(&S->device) != hipSuccess) return COEX_EDEVICE;
    coex_opts so{};
    if (o) so.width = o->width;
    int rc = coex_dfa_set_create(dfas, n_dfa, &so, &S->set);
    if (rc) return rc;
    S->n_dfa = n_dfa;
    const uint64_t budget = (o && o->hbm_budget) ? o->hbm_budget : (4ull << 30);
    if (o && o->max_batch) S->max_batch = o->max_batch;
    if (o && o->copy_piece) S->piece = o->copy_piece;
    S->inflight_cap = 3 * S->piece;
    if (hipStreamCreateWithFlags(&S->copy_st, hipStreamNonBlocking) != hipSuccess) return COEX_EDEVICE;
    if (hipMalloc(&S->arena_buf, budget) != hipSuccess) return COEX_ENOMEM;
    S->arena.init(S->arena_buf, budget);
    coex_opts bo{};
    if (o) bo.chunk = o->chunk;
    for (Slot& sl : S->slots) {
      if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess) return COEX_EDEVICE;
      rc = coex_batch_create(S->set, nullptr, 0, nullptr, nullptr, 0, &bo, &sl.batch);
      if (rc) return rc;
      if (hipEventCreate(&sl.start) != hipSuccess || hipEventCreate(&sl.done) != hipSuccess) return COEX_EDEVICE;
      rc = grow_slot(sl, 256);
      if (rc) return rc;
    }
    S->worker = std::thread(loop, S);
    *out = guard.release();
    return COEX_OK;
  } catch (const std::bad_alloc&) {
    return COEX_ENOMEM;
  } catch (...) {
    return COEX_EINTERNAL;
  }
}

int coex_server_submit(coex_server* S, const void* host_bases, uint64_t n_bases, uint32_t dfa, uint64_t* ticket) {
  if (!S || !ticket || (n_bases && !host_bases) || dfa >= S->n_dfa) return COEX_EINVAL;
  try {
    Req* r = new Req();
    r->host = host_bases;
    r->n = n_bases;
    r->dfa = dfa;
    r->t_submit = Clock::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      *ticket = S->next_ticket++;
      S->reqs[*ticket] = r;
      S->pending.push_back(r);
      S->stats.n_submitted += 1;
    }
    S->cv_work.notify_all();
    return COEX_OK;
  } catch (...) {
    return COEX_ENOMEM;
  }
}

int coex_server_wait(coex_server* S, uint64_t ticket, uint64_t* count, coex_request_stats_t* st) {
  if (!S || !count) return COEX_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  if (it == S->reqs.end()) return COEX_EINVAL;
  Req* r = it->second;
  S->cv_done.wait(lk, [&] { return r->done; });
  const int status = r->status;
  *count = r->count;
  if (st) {
    st->queue_ms = r->t_admit.time_since_epoch().count() ? ms_between(r->t_submit, r->t_admit) : 0.0;
    st->h2d_ms = r->h2d_ms;
    st->device_ms = r->device_ms;
    st->total_ms = ms_between(r->t_submit, r->t_done);
    st->launch_to_done_ms = r->t_launch.time_since_epoch().count() ? ms_between(r->t_launch, r->t_done) : 0.0;
    st->batch_size = r->batch_size;
  }
  S->reqs.erase(it);
  lk.unlock();
  if (r->c0) (void)hipEventDestroy(r->c0);
  if (r->c1) (void)hipEventDestroy(r->c1);
  delete r;
  return status;
}

int coex_server_stats(coex_server* S, coex_server_stats_t* st) {
  if (!S || !st) return COEX_EINVAL;
  std::lock_guard<std::mutex> lk(S->mu);
  *st = S->stats;
  st->arena_bytes = S->arena.size;
  return COEX_OK;
}

void coex_server_free(coex_server* S) { delete S; }

}  // extern "C"
