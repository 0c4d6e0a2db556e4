// Serving: continuous batching of independent farPCA solves on one GPU.
//
// A server owns one device pool (allocated once, at creation) and a fixed
// number of slots.  Each slot is a host thread with its own HIP stream.
// Requests arrive with their A already resident; a request is admitted into a
// free slot as soon as its device footprint - the plan's workspace plus its
// U, S, V outputs - fits in the pool (first fit, 256-byte granules).  The
// queue is scanned in arrival order and the first request that fits is
// admitted, so a large request waiting for memory does not hold back smaller
// ones behind it; a request that has waited longer than the starvation bound
// blocks overtaking until it is admitted.  An admitted request runs the whole
// method (farpca_run) on its slot's stream; the solves of different slots
// overlap on the device (the GPU interleaves the streams' kernels), and a
// request that arrives while others run is admitted the moment a slot and
// memory are free.  Results stay in the pool until released.
//
// The same kernels in the same order run on the request's stream whether it
// runs alone or among others, and every reduction has a fixed order, so a
// result does not depend on what else is being served.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "../../include/farpca.h"
#include "internal.h"

namespace {

constexpr size_t kGranule = 256;

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

struct Request {
  uint64_t tag;
  farpca_params prm;
  const void *dA;
  double t_submit;
  farpca_plan_t *plan = nullptr;
  int64_t lmax = 0;
  size_t ws = 0, footprint = 0, off = 0;
};

}  // namespace

struct farpca_server_s {
  int device = 0;
  char *pool_base = nullptr;
  size_t pool_bytes = 0;
  double starve_s = 0.0;
  Pool *pool = nullptr;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request> queue;
  std::vector<farpca_result> done;
  // tag -> pool range of a finished request until released, with the events
  // recorded after the caller's fetch copies (the range is reused only once
  // they have completed)
  struct Held { size_t off = 0, bytes = 0; std::vector<hipEvent_t> fetches; };
  std::map<uint64_t, Held> held;
  std::vector<std::thread> workers;
  int running = 0;
  bool stop = false;
};

namespace {

// Next admissible request (arrival order, first that fits; no overtaking of
// a request that has waited past the starvation bound).  Lock held.
bool take_request(farpca_server_s *s, Request *out) {
  const double t = now_s(s->t0);
  for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
    size_t off = 0;
    if (s->pool->alloc(it->footprint, &off)) {
      it->off = off;
      *out = *it;
      s->queue.erase(it);
      return true;
    }
    if (t - it->t_submit > s->starve_s) return false;
  }
  return false;
}

void worker_main(farpca_server_s *s) {
  if (hipSetDevice(s->device) != hipSuccess) return;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return;
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      for (;;) {
        if (s->stop) {          // requests still queued are dropped by destroy
          hipStreamDestroy(st);
          return;
        }
        if (take_request(s, &r)) break;
        s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      }
      s->running += 1;
    }
    farpca_result res;
    std::memset(&res, 0, sizeof(res));
    res.tag = r.tag;
    res.t_submit = r.t_submit;
    res.t_admit = now_s(s->t0);
    char *base = s->pool_base + r.off;
    const farpca_params &q = r.prm;
    // layout inside the request's range: workspace | U | S | V
    size_t o = round_up(r.ws);
    float *dU = reinterpret_cast<float *>(base + o);
    o += round_up((size_t)q.m * r.lmax * 4);
    double *dS = reinterpret_cast<double *>(base + o);
    o += round_up((size_t)r.lmax * 8);
    float *dV = reinterpret_cast<float *>(base + o);
    farpca_info info;
    std::memset(&info, 0, sizeof(info));
    const int rc = farpca_run(r.plan, r.dA, base, r.ws, dU, dS, dV, &info, nullptr, st);
    farpca_free(r.plan);
    res.status = rc;
    res.info = info;
    res.dU = dU;
    res.dS = dS;
    res.dV = dV;
    res.ld = r.lmax;
    res.m = q.m;
    res.n = q.n;
    res.t_done = now_s(s->t0);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->running -= 1;
      farpca_server_s::Held h;
      h.off = r.off;
      h.bytes = r.footprint;
      s->held[r.tag] = h;
      s->done.push_back(res);
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
  return round_up(ws) + round_up((size_t)prm->m * lmax * 4) + round_up((size_t)lmax * 8) +
         round_up((size_t)prm->n * lmax * 4);
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
  for (int i = 0; i < slots; ++i) s->workers.emplace_back(worker_main, s);
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
  const int rc = farpca_plan(prm, &r.plan, &r.lmax, &r.ws);
  if (rc != FARPCA_OK) return rc;
  r.footprint = round_up(r.ws) + round_up((size_t)prm->m * r.lmax * 4) +
                round_up((size_t)r.lmax * 8) + round_up((size_t)prm->n * r.lmax * 4);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop || r.footprint > s->pool_bytes || s->held.count(tag)) {
      farpca_free(r.plan);
      return r.footprint > s->pool_bytes ? FARPCA_E_NOMEM : FARPCA_E_INVALID;
    }
    for (const auto &q : s->queue)
      if (q.tag == tag) { farpca_free(r.plan); return FARPCA_E_INVALID; }
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
    s->pool->release(it->second.off, it->second.bytes);
    s->held.erase(it);
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
  if (k <= 0) return FARPCA_OK;
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
  if (running) *running = s->running;
  if (largest_free) *largest_free = s->pool->largest_free();
  return FARPCA_OK;
}

extern "C" int farpca_server_destroy(farpca_server_t *s) {
  if (!s) return FARPCA_E_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto &t : s->workers) t.join();
  for (auto &r : s->queue) farpca_free(r.plan);
  for (auto &h : s->held)
    for (hipEvent_t ev : h.second.fetches) {
      hipEventSynchronize(ev);
      hipEventDestroy(ev);
    }
  hipFree(s->pool_base);
  delete s->pool;
  delete s;
  return FARPCA_OK;
}
