// Serving: continuous batching of independent farPCA solves on one GPU.
//
// A server owns one device pool (allocated once, at creation), `slots`
// streams, one scheduler thread and one finisher thread per stream.  Requests arrive
// with their A already resident.  The scheduler keeps up to `slots` solves in
// flight and advances each one block at a time (farpca_step_async enqueues a
// block on the solve's stream, farpca_step_poll examines its error indicator
// once the block has run), so the blocks of all admitted solves interleave on
// the device and a request that arrives while others run is admitted as soon
// as a stream and memory are free.
//
// Memory is granted by blocks, not by the worst case: a solve is admitted with
// a loop part (farpca_loop_bytes) for its first four blocks and moved to
// one twice as large whenever its next block needs room (farpca_grow, the old
// range released once the copies have run); the final step's part is sized for
// the basis the solve reached (farpca_final_bytes) and granted when its block
// loop ends, with the outputs U, S, V sized for the columns it returns.  A
// finisher thread runs the final step (which waits for the eigensolver's
// sweeps on the host) and keeps U, S, V in the pool until the caller releases
// them.  If every solve in flight waits for memory and nothing else can free
// any, the solve admitted last is put back at the head of the queue (its
// memory released, its blocks run again later from the start: the results are
// the same).  Requests are admitted in arrival order, first fit (a request
// that does not fit does not hold back smaller ones), unless one has waited
// longer than the starvation bound (then nothing overtakes it).
//
// The kernels of a solve and their order do not depend on what else is
// served or on how its memory was granted, and every reduction has a fixed
// order, so each result is bitwise the same alone, in a mix, and from
// farpca_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <vector>

#include "../../include/farpca.h"
#include "internal.h"

using farpca_int::plan_max_blocks;
using farpca_int::plan_rank_out;

namespace {

constexpr size_t kGranule = 256;
constexpr int64_t kInitBlocks = 4;    // loop part granted at admission, in blocks

size_t round_up(size_t x) { return (x + kGranule - 1) / kGranule * kGranule; }

// First-fit allocator over [0, size): free ranges keyed by offset, merged on
// release.  Host-side bookkeeping only (the caller holds the server lock).
class Pool {
 public:
  explicit Pool(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t *off) {
    bytes = round_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
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
  // Last fit: the free range with the highest address that holds `bytes`,
  // taken from its top end (grown loop parts alternate between the two ends
  // of the pool, so the part they leave behind joins the free space).
  bool alloc_high(size_t bytes, size_t *off) {
    bytes = round_up(bytes);
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second >= bytes) {
        const size_t start = it->first + it->second - bytes;
        *off = start;
        if (it->second == bytes) free_.erase(it->first);
        else it->second -= bytes;
        return true;
      }
    }
    return false;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  std::map<size_t, size_t> free_;
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

struct Range {
  size_t off = 0, bytes = 0;
};

struct Request {
  uint64_t tag = 0;
  farpca_params prm;
  const void *dA = nullptr;
  double t_submit = 0.0;
  farpca_plan_t *plan = nullptr;
  int64_t lmax = 0, maxblk = 0;
  size_t footprint = 0;     // the worst case: every block, final part for l_max, outputs
  int64_t cap0 = 0;         // loop part at admission, in blocks (0: kInitBlocks)
};

enum class Phase { Run, NeedFinal };

// A solve in flight (scheduler thread only).
struct Active {
  Request r;
  int slot = 0;
  double t_admit = 0.0;
  uint64_t seq = 0;         // admission order
  Range loop;
  int64_t cap = 0;          // blocks the loop part has room for
  bool pending = false;     // a block enqueued and not yet examined
  bool waiting = false;     // waiting for memory (growth or final part)
  int err = FARPCA_OK;      // an error on the way (the solve ends with it)
  Phase phase = Phase::Run;
};

struct FinishJob {
  Active a;
  Range fin, out;
};

size_t outputs_bytes(int64_t m, int64_t n, int64_t k) {
  return round_up((size_t)m * k * 4) + round_up((size_t)k * 8) + round_up((size_t)n * k * 4);
}

}  // namespace

struct farpca_server_s {
  int device = 0;
  char *pool_base = nullptr;
  size_t pool_bytes = 0;
  double starve_s = 0.0;
  Pool *pool = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_fin;
  std::deque<Request> queue;
  std::vector<farpca_result> done;
  // tag -> pool range of a finished request's outputs until released, with
  // the events recorded after the caller's fetch copies (the range is reused
  // only once they have completed)
  struct Held { Range r; std::vector<hipEvent_t> fetches; };
  std::map<uint64_t, Held> held;
  // tags from submit to release: queued, running, finished or failed
  std::set<uint64_t> live;
  std::vector<hipStream_t> streams;
  std::vector<int> free_slots;
  std::deque<FinishJob> fin_jobs;
  int finishing = 0;        // jobs queued or running on the finishers
  int active = 0;           // solves between admission and the end of their final step
  std::thread scheduler;
  std::vector<std::thread> finishers;
  bool stop = false;
  size_t in_use = 0, peak = 0;
  int64_t grows = 0, preemptions = 0;
};

namespace {

bool grab(farpca_server_s *s, size_t bytes, Range *r, bool high = false) {   // lock held
  size_t off = 0;
  if (!(high ? s->pool->alloc_high(bytes, &off) : s->pool->alloc(bytes, &off))) return false;
  r->off = off;
  r->bytes = round_up(bytes);
  s->in_use += r->bytes;
  if (s->in_use > s->peak) s->peak = s->in_use;
  return true;
}

void give_back(farpca_server_s *s, const Range &r) {      // lock held
  if (!r.bytes) return;
  s->pool->release(r.off, r.bytes);
  s->in_use -= r.bytes;
}

// Next admissible request (arrival order, first that fits; no overtaking of
// a request that has waited past the starvation bound).  Lock held.
bool take_request(farpca_server_s *s, Request *out, Range *loop, int64_t *cap) {
  const double t = now_s(s->t0);
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    const int64_t c = std::min<int64_t>(it->cap0 ? it->cap0 : kInitBlocks, it->maxblk);
    const size_t bytes = farpca_loop_bytes(it->plan, c);
    if (bytes && grab(s, bytes, loop)) {
      *out = *it;
      *cap = c;
      s->queue.erase(it);
      return true;
    }
    if (t - it->t_submit > s->starve_s) return false;
  }
  return false;
}

void publish_error(farpca_server_s *s, const Active &a, int rc) {   // lock held
  farpca_result res;
  std::memset(&res, 0, sizeof(res));
  res.tag = a.r.tag;
  res.status = rc;
  res.t_submit = a.r.t_submit;
  res.t_admit = a.t_admit;
  res.t_done = now_s(s->t0);
  res.m = a.r.prm.m;
  res.n = a.r.prm.n;
  s->held[a.r.tag] = farpca_server_s::Held();
  s->done.push_back(res);
}

// The solve's loop part to the next size (double, else one block more).
// Returns false if the pool has no room now.
bool try_grow(farpca_server_s *s, Active &a, std::vector<std::pair<hipEvent_t, Range>> &deferred,
              int *err) {
  *err = FARPCA_OK;
  const int64_t want[2] = {std::min(a.r.maxblk, std::max(a.cap + 1, 2 * a.cap)),
                           std::min(a.r.maxblk, a.cap + 1)};
  Range nr;
  int64_t ncap = 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    // the new part from the end of the pool away from the current one
    const bool high = a.loop.off < s->pool_bytes / 2;
    for (int64_t c : want) {
      if (c <= a.cap) continue;
      const size_t bytes = farpca_loop_bytes(a.r.plan, c);
      if (bytes && grab(s, bytes, &nr, high)) { ncap = c; break; }
    }
  }
  if (!ncap) return false;
  hipStream_t st = s->streams[a.slot];
  int rc = farpca_grow(a.r.plan, s->pool_base + nr.off, nr.bytes, ncap, st);
  hipEvent_t ev = nullptr;
  if (rc == FARPCA_OK && (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess ||
                          hipEventRecord(ev, st) != hipSuccess))
    rc = FARPCA_E_DEVICE;
  if (rc != FARPCA_OK) {
    if (ev) hipEventDestroy(ev);
    hipStreamSynchronize(st);
    std::lock_guard<std::mutex> lk(s->mu);
    give_back(s, nr);
    *err = rc;
    return false;
  }
  deferred.emplace_back(ev, a.loop);     // released once the copies have run
  a.loop = nr;
  a.cap = ncap;
  std::lock_guard<std::mutex> lk(s->mu);
  s->grows += 1;
  return true;
}

void scheduler_main(farpca_server_s *s) {
  if (hipSetDevice(s->device) != hipSuccess) return;
  std::vector<Active> act;
  std::vector<std::pair<hipEvent_t, Range>> deferred;
  uint64_t seq = 0;
  for (;;) {
    bool progress = false;
    // ranges left by growth, once their copies have run
    for (size_t i = 0; i < deferred.size();) {
      if (hipEventQuery(deferred[i].first) != hipErrorNotReady) {
        hipEventDestroy(deferred[i].first);
        {
          std::lock_guard<std::mutex> lk(s->mu);
          give_back(s, deferred[i].second);
        }
        deferred.erase(deferred.begin() + i);
        progress = true;
      } else {
        ++i;
      }
    }
    // admission (not while a solve in flight waits for memory: memory that
    // frees up goes to the solves already running first, so that a solve put
    // back in the queue cannot take it straight back)
    bool someone_waits = false;
    for (const auto &a : act) someone_waits = someone_waits || a.waiting;
    std::vector<Active> admitted;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (s->stop) break;
      while (!someone_waits && !s->free_slots.empty()) {
        Active a;
        if (!take_request(s, &a.r, &a.loop, &a.cap)) break;
        a.slot = s->free_slots.back();
        s->free_slots.pop_back();
        a.t_admit = now_s(s->t0);
        a.seq = seq++;
        s->active += 1;
        admitted.push_back(a);
      }
    }
    for (auto &a : admitted) {
      progress = true;
      const int rc = farpca_begin_loop(a.r.plan, a.r.dA, s->pool_base + a.loop.off, a.loop.bytes,
                                       a.cap, nullptr, s->streams[a.slot]);
      if (rc != FARPCA_OK) {
        hipStreamSynchronize(s->streams[a.slot]);
        farpca_free(a.r.plan);
        std::lock_guard<std::mutex> lk(s->mu);
        give_back(s, a.loop);
        publish_error(s, a, rc);
        s->free_slots.push_back(a.slot);
        s->active -= 1;
        s->cv_done.notify_all();
        continue;
      }
      act.push_back(a);
    }
    // advance every solve in flight by a block
    for (auto &a : act) {
      if (a.phase != Phase::Run) continue;
      if (a.pending) {
        const int rc = farpca_step_poll(a.r.plan, 0);
        if (rc == 2) continue;
        a.pending = false;
        progress = true;
        if (rc == 0) { a.phase = Phase::NeedFinal; continue; }
        if (rc < 0) { a.phase = Phase::NeedFinal; a.err = rc; continue; }
      }
      int rc = farpca_step_async(a.r.plan, s->streams[a.slot]);
      if (rc == FARPCA_E_NOMEM) {
        int err = FARPCA_OK;
        if (try_grow(s, a, deferred, &err)) {
          progress = true;
          rc = farpca_step_async(a.r.plan, s->streams[a.slot]);
        } else if (err != FARPCA_OK) {
          rc = err;
        } else {
          a.waiting = true;
          continue;
        }
      }
      a.waiting = false;
      progress = true;
      if (rc == 1) {
        a.pending = true;
      } else {
        a.phase = Phase::NeedFinal;
        if (rc < 0) a.err = rc;
      }
    }
    // solves whose block loop ended: final part and outputs, then a finisher
    for (size_t i = 0; i < act.size();) {
      Active &a = act[i];
      if (a.phase != Phase::NeedFinal) { ++i; continue; }
      const size_t fb = a.err == FARPCA_OK ? farpca_final_bytes(a.r.plan) : 0;
      if (a.err != FARPCA_OK || fb == 0) {
        hipStreamSynchronize(s->streams[a.slot]);
        const int rc = a.err != FARPCA_OK ? a.err : FARPCA_E_INVALID;
        farpca_free(a.r.plan);
        std::lock_guard<std::mutex> lk(s->mu);
        give_back(s, a.loop);
        publish_error(s, a, rc);
        s->free_slots.push_back(a.slot);
        s->active -= 1;
        s->cv_done.notify_all();
        act.erase(act.begin() + i);
        progress = true;
        continue;
      }
      const int64_t k = plan_rank_out(a.r.plan);
      bool ok = false;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        Range fin, out;
        if (grab(s, fb, &fin)) {
          if (grab(s, outputs_bytes(a.r.prm.m, a.r.prm.n, k), &out)) {
            FinishJob job;
            job.a = a;
            job.fin = fin;
            job.out = out;
            s->fin_jobs.push_back(job);
            s->finishing += 1;
            ok = true;
          } else {
            give_back(s, fin);
          }
        }
      }
      if (ok) {
        s->cv_fin.notify_one();
        act.erase(act.begin() + i);
        progress = true;
      } else {
        a.waiting = true;
        ++i;
      }
    }
    // every solve waits for memory and nothing in flight can free any: the
    // solve admitted last goes back to the head of the queue; a solve that waits
    // alone (its worst case fits the pool, but not next to what it holds) starts
    // again with room for every block
    if (!progress && deferred.empty() && act.size() == 1 && act[0].waiting && !act[0].pending &&
        act[0].phase == Phase::Run && act[0].cap < act[0].r.maxblk) {
      int fin_busy = 0;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        fin_busy = s->finishing;
      }
      if (fin_busy == 0) {
        Active self = act[0];
        act.clear();
        hipStreamSynchronize(s->streams[self.slot]);
        std::lock_guard<std::mutex> lk(s->mu);
        give_back(s, self.loop);
        self.r.cap0 = self.r.maxblk;
        s->queue.push_front(self.r);
        s->free_slots.push_back(self.slot);
        s->active -= 1;
        s->preemptions += 1;
        progress = true;
      }
    }
    if (!progress && deferred.empty() && act.size() > 1) {
      bool all_wait = true;
      for (const auto &a : act) all_wait = all_wait && a.waiting && !a.pending;
      int fin_busy = 0;
      {
        std::lock_guard<std::mutex> lk(s->mu);
        fin_busy = s->finishing;
      }
      if (all_wait && fin_busy == 0) {
        size_t v = 0;
        for (size_t i = 1; i < act.size(); ++i)
          if (act[i].seq > act[v].seq) v = i;
        Active victim = act[v];
        act.erase(act.begin() + v);
        hipStreamSynchronize(s->streams[victim.slot]);
        std::lock_guard<std::mutex> lk(s->mu);
        give_back(s, victim.loop);
        s->queue.push_front(victim.r);
        s->free_slots.push_back(victim.slot);
        s->active -= 1;
        s->preemptions += 1;
        progress = true;
      }
    }
    if (!progress) {
      bool any_pending = false;
      for (const auto &a : act) any_pending = any_pending || a.pending;
      if (any_pending || !deferred.empty()) {
        std::this_thread::yield();     // blocks in flight: poll again
      } else {
        std::unique_lock<std::mutex> lk(s->mu);
        s->cv_work.wait_for(lk, std::chrono::milliseconds(2));
      }
    }
  }
  // shutdown: let in-flight work end, release what the solves hold
  for (auto &a : act) {
    hipStreamSynchronize(s->streams[a.slot]);
    farpca_free(a.r.plan);
  }
  for (auto &d : deferred) {
    hipEventSynchronize(d.first);
    hipEventDestroy(d.first);
  }
}

void finisher_main(farpca_server_s *s) {
  if (hipSetDevice(s->device) != hipSuccess) return;
  for (;;) {
    FinishJob j;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_fin.wait(lk, [&] { return s->stop || !s->fin_jobs.empty(); });
      if (s->fin_jobs.empty()) return;     // stop requested and nothing left
      j = s->fin_jobs.front();
      s->fin_jobs.pop_front();
    }
    const Active &a = j.a;
    const farpca_params &q = a.r.prm;
    const int64_t k = plan_rank_out(a.r.plan);
    char *out = s->pool_base + j.out.off;
    float *dU = reinterpret_cast<float *>(out);
    double *dS = reinterpret_cast<double *>(out + round_up((size_t)q.m * k * 4));
    float *dV = reinterpret_cast<float *>(out + round_up((size_t)q.m * k * 4) + round_up((size_t)k * 8));
    farpca_info info;
    std::memset(&info, 0, sizeof(info));
    hipStream_t st = s->streams[a.slot];
    const int rc = farpca_finish_final(a.r.plan, s->pool_base + j.fin.off, j.fin.bytes, dU, k, dS,
                                       dV, k, &info, st);
    hipStreamSynchronize(st);
    farpca_free(a.r.plan);
    farpca_result res;
    std::memset(&res, 0, sizeof(res));
    res.tag = a.r.tag;
    res.status = rc;
    res.info = info;
    res.t_submit = a.r.t_submit;
    res.t_admit = a.t_admit;
    res.dU = dU;
    res.dS = dS;
    res.dV = dV;
    res.ld = k;
    res.m = q.m;
    res.n = q.n;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      give_back(s, a.loop);
      give_back(s, j.fin);
      res.t_done = now_s(s->t0);
      farpca_server_s::Held h;
      h.r = j.out;
      s->held[a.r.tag] = h;
      s->done.push_back(res);
      s->free_slots.push_back(a.slot);
      s->finishing -= 1;
      s->active -= 1;
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" size_t farpca_request_footprint(const farpca_params *prm) {
  if (!prm) return 0;
  farpca_plan_t *pl = nullptr;
  int64_t lmax = 0;
  size_t ws = 0;
  if (farpca_plan(prm, &pl, &lmax, &ws) != FARPCA_OK) return 0;
  farpca_free(pl);
  return round_up(ws) + outputs_bytes(prm->m, prm->n, lmax);
}

extern "C" int farpca_server_create(size_t pool_bytes, int slots, double starve_s,
                                    farpca_server_t **out) {
  if (!out || slots < 1 || slots > 64 || pool_bytes < kGranule || !(starve_s >= 0.0))
    return FARPCA_E_INVALID;
  *out = nullptr;
  farpca_server_s *s = new (std::nothrow) farpca_server_s();
  if (!s) return FARPCA_E_NOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return FARPCA_E_DEVICE; }
  void *p = nullptr;
  if (hipMalloc(&p, pool_bytes) != hipSuccess) { delete s; return FARPCA_E_NOMEM; }
  s->pool_base = static_cast<char *>(p);
  s->pool_bytes = pool_bytes / kGranule * kGranule;
  s->pool = new Pool(s->pool_bytes);
  s->starve_s = starve_s;
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < slots; ++i) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : s->streams) hipStreamDestroy(x);
      hipFree(s->pool_base);
      delete s->pool;
      delete s;
      return FARPCA_E_DEVICE;
    }
    s->streams.push_back(st);
    s->free_slots.push_back(slots - 1 - i);
  }
  s->scheduler = std::thread(scheduler_main, s);
  // one finisher per stream: the final step of a large basis (the eigensolver
  // of an order-2000 Gram) takes milliseconds, and as many may run as solves
  for (int i = 0; i < slots; ++i) s->finishers.emplace_back(finisher_main, s);
  *out = s;
  return FARPCA_OK;
}

extern "C" int farpca_server_submit(farpca_server_t *s, const farpca_params *prm, const void *dA,
                                    uint64_t tag) {
  if (!s || !prm || !dA) return FARPCA_E_INVALID;
  Request r;
  r.tag = tag;
  r.prm = *prm;
  r.dA = dA;
  size_t ws = 0;
  const int rc = farpca_plan(prm, &r.plan, &r.lmax, &ws);
  if (rc != FARPCA_OK) return rc;
  r.maxblk = plan_max_blocks(r.plan);
  r.footprint = round_up(ws) + outputs_bytes(prm->m, prm->n, r.lmax);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop || r.footprint > s->pool_bytes || s->live.count(tag)) {
      farpca_free(r.plan);
      return r.footprint > s->pool_bytes ? FARPCA_E_NOMEM : FARPCA_E_INVALID;
    }
    s->live.insert(tag);
    r.t_submit = now_s(s->t0);
    s->queue.push_back(r);
  }
  s->cv_work.notify_all();
  return FARPCA_OK;
}

extern "C" int farpca_server_poll(farpca_server_t *s, farpca_result *out, int max_out,
                                  int wait_ms) {
  if (!s || (!out && max_out > 0) || max_out < 0) return FARPCA_E_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && wait_ms > 0)
    s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !s->done.empty(); });
  int n = 0;
  while (n < max_out && !s->done.empty()) {
    out[n++] = s->done.front();
    s->done.erase(s->done.begin());
  }
  return n;
}

extern "C" int farpca_server_release(farpca_server_t *s, uint64_t tag) {
  if (!s) return FARPCA_E_INVALID;
  std::vector<hipEvent_t> fetches;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->held.find(tag);
    if (it == s->held.end()) return FARPCA_E_INVALID;
    fetches.swap(it->second.fetches);
  }
  // copies enqueued by farpca_server_fetch on the caller's streams finish
  // before the range can be handed to another request
  for (hipEvent_t ev : fetches) {
    hipEventSynchronize(ev);
    hipEventDestroy(ev);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->held.find(tag);
    if (it == s->held.end()) return FARPCA_E_INVALID;
    for (hipEvent_t ev : it->second.fetches) {     // a fetch that raced this release
      hipEventSynchronize(ev);
      hipEventDestroy(ev);
    }
    give_back(s, it->second.r);
    s->held.erase(it);
    s->live.erase(tag);
  }
  s->cv_work.notify_all();
  return FARPCA_OK;
}

extern "C" int farpca_server_fetch(farpca_server_t *s, const farpca_result *r, float *dU,
                                   int64_t ldu, double *dS, float *dV, int64_t ldv, void *stream) {
  if (!s || !r) return FARPCA_E_INVALID;
  const int64_t k = r->info.rank_out;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (!s->held.count(r->tag)) return FARPCA_E_INVALID;
  }
  if (k <= 0 || r->status < 0) return FARPCA_OK;
  if ((dU && ldu < k) || (dV && ldv < k)) return FARPCA_E_INVALID;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t m = r->m, n = r->n;
  if (dU && hipMemcpy2DAsync(dU, ldu * 4, r->dU, r->ld * 4, k * 4, m, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return FARPCA_E_DEVICE;
  if (dS && hipMemcpyAsync(dS, r->dS, k * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return FARPCA_E_DEVICE;
  if (dV && hipMemcpy2DAsync(dV, ldv * 4, r->dV, r->ld * 4, k * 4, n, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return FARPCA_E_DEVICE;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return FARPCA_E_DEVICE;
  if (hipEventRecord(ev, st) != hipSuccess) {
    hipEventDestroy(ev);
    return FARPCA_E_DEVICE;
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->held.find(r->tag);
    if (it == s->held.end()) {          // released meanwhile: wait here instead
      hipEventSynchronize(ev);
      hipEventDestroy(ev);
      return FARPCA_E_INVALID;
    }
    it->second.fetches.push_back(ev);
  }
  return FARPCA_OK;
}

extern "C" int farpca_server_stats(farpca_server_t *s, int *queued, int *running,
                                   size_t *largest_free) {
  if (!s) return FARPCA_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int)s->queue.size();
  if (running) *running = s->active;
  if (largest_free) *largest_free = s->pool->largest_free();
  return FARPCA_OK;
}

extern "C" int farpca_server_memory(farpca_server_t *s, size_t *in_use, size_t *peak,
                                    int64_t *grows, int64_t *preemptions) {
  if (!s) return FARPCA_E_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  if (in_use) *in_use = s->in_use;
  if (peak) *peak = s->peak;
  if (grows) *grows = s->grows;
  if (preemptions) *preemptions = s->preemptions;
  return FARPCA_OK;
}

extern "C" int farpca_server_destroy(farpca_server_t *s) {
  if (!s) return FARPCA_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_fin.notify_all();
  if (s->scheduler.joinable()) s->scheduler.join();
  for (auto &t : s->finishers) t.join();
  for (auto &r : s->queue) farpca_free(r.plan);
  for (auto &h : s->held)
    for (hipEvent_t ev : h.second.fetches) {
      hipEventSynchronize(ev);
      hipEventDestroy(ev);
    }
  for (hipStream_t st : s->streams) {
    hipStreamSynchronize(st);
    hipStreamDestroy(st);
  }
  hipFree(s->pool_base);
  delete s->pool;
  delete s;
  return FARPCA_OK;
}
