// Served form: a request loop with continuous batching.
//
// Requests (host buffers of points) queue in FIFO order. A dispatcher thread
// forms device batches from the head of the queue as soon as a batch slot and
// enough pool memory are free: the batch's points are packed contiguously into
// a pinned host pool (by a few copy threads at once), copied to the same
// offsets of a device pool, mapped with one plain kernel launch over the
// concatenation, and copied back, all on one of several streams, so batches
// overlap on the device. Large pieces in page-locked caller memory skip the
// packing: they are copied by DMA straight to and from their place in the
// device pool. A batch's pool range
// also holds the mapping call's pre-sort scratch, so the memory budget bounds
// everything the server uses on the device. A completion thread retires
// whichever in-flight batch has finished, scatters results to the callers'
// buffers (with the copy threads), releases pool memory and slots, and records each request's latency.
// Requests larger than a batch are split into pieces; a request completes when
// its last piece does. Results are those of map_points on each request alone.
// After a device error the server fails every queued piece and dispatches no
// more; a request's wait returns once all its pieces have been retired, so no
// copy into its buffers is still pending.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "copy_pool.h"
#include "trace.h"

using namespace bm;
using Clock = std::chrono::steady_clock;

namespace {

constexpr int64_t kAlign = 256;

inline int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with coalescing of freed ranges.
class PoolAlloc {
 public:
  explicit PoolAlloc(int64_t size) { free_[0] = size; }
  int64_t alloc(int64_t bytes) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first, rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
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

 private:
  std::map<int64_t, int64_t> free_;
};

struct Request {
  uint64_t ticket = 0;
  const int32_t* xy = nullptr;
  int32_t* out = nullptr;
  int64_t n = 0;
  bool pinned_in = false, pinned_out = false;  // caller buffers in page-locked memory
  int64_t pieces_left = 0;
  bool done = false;
  int status = BM_OK;
  Clock::time_point t_submit;
};

struct Piece {
  Request* r;
  int64_t first;  // first point of the piece within its request
  int64_t n;
};

struct Batch {
  std::vector<Piece> pieces;
  std::vector<char> direct_out;  // per piece: result copied straight to the caller
  int64_t npts = 0;
  int64_t off = 0, bytes = 0;  // pool range: xy, out, then the mapping call's scratch
  int slot = -1;
  bool launched = false;
  int status = BM_OK;
};

bool is_pinned(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  const hipError_t e = hipPointerGetAttributes(&a, p);
  (void)hipGetLastError();  // pageable memory reports an error; do not leave it pending
  return e == hipSuccess && a.type == hipMemoryTypeHost;
}

}  // namespace

struct bm_server {
  const bm_index* index = nullptr;
  bm_server_cfg cfg{};
  Tuning tuning{};
  int device = 0;
  char* d_pool = nullptr;
  char* h_pool = nullptr;
  int64_t pool_bytes = 0;
  PoolAlloc* alloc = nullptr;
  CopyPool* copies = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;  // one per slot
  std::vector<int> free_slots;

  std::mutex mu;
  std::condition_variable cv_dispatch, cv_complete, cv_done;
  std::deque<Piece> queue;
  std::deque<Batch*> inflight;
  std::unordered_map<uint64_t, Request*> reqs;
  uint64_t next_ticket = 1;
  uint64_t frees = 0;  // pool releases so far (the dispatcher waits for a change)
  bool stop = false;
  int fatal = BM_OK;
  std::string fatal_msg;

  // statistics
  std::vector<double> lat_us;
  int64_t completed = 0, points = 0, batches = 0, batch_requests = 0, rejected = 0;
  bool have_first = false;
  Clock::time_point t_first, t_last;

  std::thread dispatcher, completer;

  void dispatch_loop();
  void complete_loop();
};

void bm_server::dispatch_loop() {
  const bool dev_ok = hipSetDevice(device) == hipSuccess;
  std::unique_lock<std::mutex> lk(mu);
  if (!dev_ok) {  // the loop below then fails every queued piece
    fatal = BM_EHIP;
    fatal_msg = "server: hipSetDevice failed";
  }
  uint64_t nbatch = 0;
  for (;;) {
    cv_dispatch.wait(lk, [&] { return stop || fatal != BM_OK || (!queue.empty() && !free_slots.empty()); });
    if (stop) break;
    if (fatal != BM_OK) {
      // a device error: fail what is queued, dispatch nothing more
      const auto now = Clock::now();
      while (!queue.empty()) {
        Request* r = queue.front().r;
        queue.pop_front();
        r->status = fatal;
        if (--r->pieces_left == 0) {
          r->done = true;
          completed++;
          lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        }
      }
      cv_done.notify_all();
      cv_dispatch.wait(lk, [&] { return stop || !queue.empty(); });
      continue;
    }
    // coalescing window: a small head batch may wait briefly for more arrivals
    if (cfg.coalesce_us > 0) {
      const auto deadline = queue.front().r->t_submit + std::chrono::microseconds(cfg.coalesce_us);
      auto queued = [&] {
        int64_t s = 0;
        for (const Piece& p : queue) s += p.n;
        return s;
      };
      while (!stop && queued() < cfg.max_batch_points && Clock::now() < deadline)
        cv_dispatch.wait_until(lk, deadline);
      if (stop) break;
    }
    Batch* b = new Batch();
    const bool one = (cfg.flags & BM_SERVER_ONE_PER_BATCH) != 0;
    while (!queue.empty() && b->npts + queue.front().n <= cfg.max_batch_points && !(one && !b->pieces.empty())) {
      b->pieces.push_back(queue.front());
      b->npts += queue.front().n;
      queue.pop_front();
    }
    const int64_t ws_bytes = align_up((int64_t)map_scratch_bytes(index->k, b->npts, tuning));
    b->bytes = align_up(8 * b->npts) + align_up(4 * b->npts) + ws_bytes;
    int64_t off = alloc->alloc(b->bytes);
    if (off < 0) {
      // not enough free pool memory: put the pieces back (FIFO order kept) and
      // wait for an in-flight batch to retire
      for (auto it = b->pieces.rbegin(); it != b->pieces.rend(); ++it) queue.push_front(*it);
      delete b;
      const uint64_t f0 = frees;
      cv_dispatch.wait(lk, [&] { return stop || frees != f0; });
      continue;
    }
    b->off = off;
    b->slot = free_slots.back();
    free_slots.pop_back();
    inflight.push_back(b);
    batches++;
    batch_requests += (int64_t)b->pieces.size();
    lk.unlock();

    // stage, copy in, map, copy out: all queued on the slot's stream
    bm::trace_push("server: dispatch batch");
    hipStream_t s = streams[nbatch++ % streams.size()];
    char* hx = h_pool + b->off;
    char* dx = d_pool + b->off;
    const int64_t out_off = b->off + align_up(8 * b->npts);
    hipError_t e = hipSuccess;
    b->direct_out.assign(b->pieces.size(), 0);
    int64_t pos = 0, run0 = -1;  // run0: first point of the current run of packed pieces
    auto flush_run = [&](int64_t end) {
      if (run0 >= 0 && e == hipSuccess)
        e = hipMemcpyAsync(dx + 8 * run0, hx + 8 * run0, 8 * (size_t)(end - run0), hipMemcpyHostToDevice, s);
      run0 = -1;
    };
    auto direct_in = [&](const Piece& p) { return p.r->pinned_in && p.n >= cfg.direct_min_points; };
    std::vector<CopyPool::Copy> pack;
    for (const Piece& p : b->pieces) {
      if (!direct_in(p)) pack.push_back(CopyPool::Copy{p.r->xy + 2 * p.first, hx + 8 * pos, 8 * (size_t)p.n});
      pos += p.n;
    }
    copies->run(pack);
    pos = 0;
    for (const Piece& p : b->pieces) {
      if (direct_in(p)) {
        flush_run(pos);
        if (e == hipSuccess)
          e = hipMemcpyAsync(dx + 8 * pos, p.r->xy + 2 * p.first, 8 * (size_t)p.n, hipMemcpyHostToDevice, s);
      } else if (run0 < 0) {
        run0 = pos;
      }
      pos += p.n;
    }
    flush_run(pos);
    if (e == hipSuccess)
      e = launch_map(index->k, reinterpret_cast<const int32_t*>(dx), b->npts,
                     reinterpret_cast<int32_t*>(d_pool + out_off), tuning, index->num_cu, s, nullptr,
                     ws_bytes ? d_pool + out_off + align_up(4 * b->npts) : nullptr, (size_t)ws_bytes);
    pos = 0;
    run0 = -1;
    auto flush_out = [&](int64_t end) {
      if (run0 >= 0 && e == hipSuccess)
        e = hipMemcpyAsync(h_pool + out_off + 4 * run0, d_pool + out_off + 4 * run0, 4 * (size_t)(end - run0),
                           hipMemcpyDeviceToHost, s);
      run0 = -1;
    };
    for (size_t k = 0; k < b->pieces.size(); ++k) {
      const Piece& p = b->pieces[k];
      if (p.r->pinned_out && p.n >= cfg.direct_min_points) {
        flush_out(pos);
        b->direct_out[k] = 1;
        if (e == hipSuccess)
          e = hipMemcpyAsync(p.r->out + p.first, d_pool + out_off + 4 * pos, 4 * (size_t)p.n, hipMemcpyDeviceToHost, s);
      } else if (run0 < 0) {
        run0 = pos;
      }
      pos += p.n;
    }
    flush_out(pos);
    if (e == hipSuccess) e = hipEventRecord(events[b->slot], s);
    // after a failed enqueue, what was queued must finish before the batch's
    // pool range and slot can be released
    if (e != hipSuccess) (void)hipStreamSynchronize(s);
    bm::trace_pop();

    lk.lock();
    if (e != hipSuccess) {
      b->status = BM_EHIP;
      fatal = BM_EHIP;
      fatal_msg = std::string("server: ") + hipGetErrorString(e);
    }
    b->launched = true;
    cv_complete.notify_all();
  }
}

void bm_server::complete_loop() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_complete.wait(lk, [&] {
      if (stop && inflight.empty()) return true;
      for (Batch* x : inflight)
        if (x->launched) return true;
      return false;
    });
    if (inflight.empty()) break;
    // retire a finished batch, whichever stream it ran on; poll if none is
    Batch* b = nullptr;
    for (Batch* x : inflight) {
      if (!x->launched) continue;
      if (x->status != BM_OK) { b = x; break; }
      const hipError_t q = hipEventQuery(events[x->slot]);
      if (q == hipSuccess) { b = x; break; }
      if (q != hipErrorNotReady) { x->status = BM_EHIP; b = x; break; }
    }
    if (!b) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(5));
      lk.lock();
      continue;
    }
    lk.unlock();
    bm::trace_push("server: retire batch");
    const int st = b->status;
    if (st == BM_OK) {
      const char* ho = h_pool + b->off + align_up(8 * b->npts);
      std::vector<CopyPool::Copy> unpack;
      int64_t pos = 0;
      for (size_t k = 0; k < b->pieces.size(); ++k) {
        const Piece& p = b->pieces[k];
        if (!b->direct_out[k]) unpack.push_back(CopyPool::Copy{ho + 4 * pos, p.r->out + p.first, 4 * (size_t)p.n});
        pos += p.n;
      }
      copies->run(unpack);
    }
    const auto now = Clock::now();
    bm::trace_pop();
    lk.lock();
    inflight.erase(std::find(inflight.begin(), inflight.end(), b));
    alloc->release(b->off, b->bytes);
    frees++;
    free_slots.push_back(b->slot);
    for (const Piece& p : b->pieces) {
      Request* r = p.r;
      if (st != BM_OK) r->status = st;
      if (--r->pieces_left == 0) {
        r->done = true;
        completed++;
        points += r->n;
        lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
        t_last = now;
      }
    }
    delete b;
    cv_dispatch.notify_all();
    cv_done.notify_all();
  }
}

extern "C" {

__attribute__((visibility("default"))) int bm_server_cfg_default(bm_server_cfg* c) {
  if (!c) return fail(BM_EINVAL, "bm_server_cfg_default: null argument");
  c->mem_budget_bytes = (int64_t)1 << 30;
  c->max_batch_points = (int64_t)1 << 22;
  c->max_slots = 4;
  c->n_streams = 4;
  c->coalesce_us = 0;
  c->queue_capacity = 1 << 20;
  c->flags = 0;
  bm_tuning_default(&c->tuning);
  c->copy_threads = 8;
  c->direct_min_points = (int64_t)1 << 16;
  return BM_OK;
}

__attribute__((visibility("default"))) int bm_server_create(const bm_index* index, const bm_server_cfg* cfg,
                                                           bm_server** out) {
  try {
    clear_error();
    if (!index || !out) return fail(BM_EINVAL, "bm_server_create: null argument");
    *out = nullptr;
    bm_server_cfg c;
    bm_server_cfg_default(&c);
    if (cfg) c = *cfg;
    if (c.max_batch_points < 64 || c.max_slots < 1 || c.max_slots > 64 || c.n_streams < 1 || c.n_streams > 16 ||
        c.queue_capacity < 1 || c.coalesce_us < 0 || c.copy_threads < 1 || c.copy_threads > 64 ||
        c.direct_min_points < 1)
      return fail(BM_EINVAL, "bm_server_create: configuration out of range");
    const int64_t full_batch = align_up(8 * c.max_batch_points) + align_up(4 * c.max_batch_points) +
                               align_up((int64_t)map_scratch_bytes(index->k, c.max_batch_points, tuning_from(&c.tuning)));
    if (c.mem_budget_bytes < full_batch)
      return fail(BM_EINVAL, "bm_server_create: memory budget below one full batch (" + std::to_string(full_batch) +
                                 " bytes: 12 per point, plus the pre-sort scratch of batches of 2^20 points or more)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != index->device)
      return fail(BM_EINVAL, "bm_server_create: the index must live on the current device");
    bm_server* s = new (std::nothrow) bm_server();
    if (!s) return fail(BM_ENOMEM, "bm_server_create: out of host memory");
    s->index = index;
    s->cfg = c;
    s->tuning = tuning_from(&c.tuning);
    s->device = dev;
    s->pool_bytes = align_up(c.mem_budget_bytes);
    hipError_t e = hipSuccess;
    if (c.flags & BM_SERVER_FAIL_ALLOC)
      e = hipErrorOutOfMemory;  // forced from the host, for failure-path tests
    if (e == hipSuccess) e = hipMalloc((void**)&s->d_pool, s->pool_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void**)&s->h_pool, s->pool_bytes, hipHostMallocDefault);
    for (int i = 0; e == hipSuccess && i < c.n_streams; ++i) {
      hipStream_t st;
      e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
      if (e == hipSuccess) s->streams.push_back(st);
    }
    for (int i = 0; e == hipSuccess && i < c.max_slots; ++i) {
      hipEvent_t ev;
      e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) {
        s->events.push_back(ev);
        s->free_slots.push_back(c.max_slots - 1 - i);
      }
    }
    if (e != hipSuccess) {
      for (auto st : s->streams) (void)hipStreamDestroy(st);
      for (auto ev : s->events) (void)hipEventDestroy(ev);
      if (s->d_pool) (void)hipFree(s->d_pool);
      if (s->h_pool) (void)hipHostFree(s->h_pool);
      delete s;
      return fail(e == hipErrorOutOfMemory ? BM_ENOMEM : BM_EHIP,
                  std::string("bm_server_create: ") + hipGetErrorString(e));
    }
    s->alloc = new PoolAlloc(s->pool_bytes);
    s->copies = new CopyPool(c.copy_threads);
    s->dispatcher = std::thread([s] { s->dispatch_loop(); });
    s->completer = std::thread([s] { s->complete_loop(); });
    *out = s;
    return BM_OK;
  } catch (...) {
    return fail(BM_ENOMEM, "bm_server_create: unexpected error");
  }
}

__attribute__((visibility("default"))) int bm_server_submit(bm_server* s, const int32_t* xy, int64_t n,
                                                           int32_t* out, uint64_t* ticket) {
  try {
    if (!s || !ticket) return fail(BM_EINVAL, "bm_server_submit: null argument");
    if (n < 0) return fail(BM_EINVAL, "bm_server_submit: n < 0");
    if (n > 0 && (!xy || !out)) return fail(BM_EINVAL, "bm_server_submit: null buffer");
    const bool pin_in = n >= s->cfg.direct_min_points && is_pinned(xy);
    const bool pin_out = n >= s->cfg.direct_min_points && is_pinned(out);
    std::lock_guard<std::mutex> g(s->mu);
    if (s->fatal != BM_OK) return fail(s->fatal, s->fatal_msg);
    const int64_t np = n == 0 ? 0 : (n + s->cfg.max_batch_points - 1) / s->cfg.max_batch_points;
    if ((int64_t)s->queue.size() + np > s->cfg.queue_capacity) {
      s->rejected++;
      return fail(BM_EBUSY, "bm_server_submit: queue full");
    }
    Request* r = new Request();
    r->ticket = s->next_ticket++;
    r->xy = xy;
    r->out = out;
    r->n = n;
    r->pinned_in = pin_in;
    r->pinned_out = pin_out;
    r->pieces_left = np;
    r->t_submit = Clock::now();
    if (!s->have_first) {
      s->have_first = true;
      s->t_first = r->t_submit;
    }
    s->reqs[r->ticket] = r;
    for (int64_t f = 0; f < n; f += s->cfg.max_batch_points)
      s->queue.push_back(Piece{r, f, std::min(s->cfg.max_batch_points, n - f)});
    if (np == 0) {
      r->done = true;
      s->completed++;
      s->lat_us.push_back(0.0);
    }
    *ticket = r->ticket;
    s->cv_dispatch.notify_one();
    return BM_OK;
  } catch (...) {
    return fail(BM_ENOMEM, "bm_server_submit: out of host memory");
  }
}

__attribute__((visibility("default"))) int bm_server_wait(bm_server* s, uint64_t ticket, int64_t timeout_us) {
  if (!s) return fail(BM_EINVAL, "bm_server_wait: null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return fail(BM_EINVAL, "bm_server_wait: unknown ticket");
  Request* r = it->second;
  auto ready = [&] { return r->done; };  // every piece retired, failed ones too
  if (timeout_us < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return fail(BM_ETIMEDOUT, "bm_server_wait: timed out");
  }
  const int st = r->status;
  s->reqs.erase(it);
  delete r;
  return st == BM_OK ? BM_OK : fail(st, "bm_server_wait: the request failed on the device");
}

__attribute__((visibility("default"))) int bm_server_get_stats(bm_server* s, bm_server_stats_t* o) {
  if (!s || !o) return fail(BM_EINVAL, "bm_server_get_stats: null argument");
  std::vector<double> v;
  {
    std::lock_guard<std::mutex> g(s->mu);
    v = s->lat_us;
    o->completed = s->completed;
    o->points = s->points;
    o->batches = s->batches;
    o->rejected = s->rejected;
    o->mean_requests_per_batch = s->batches ? (double)s->batch_requests / (double)s->batches : 0.0;
    const double span = s->have_first && s->completed
                            ? std::chrono::duration<double>(s->t_last - s->t_first).count()
                            : 0.0;
    o->points_per_s = span > 0 ? (double)s->points / span : 0.0;
  }
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::min<double>((double)v.size() - 1, q * (double)(v.size() - 1) + 0.5);
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
  };
  o->p50_us = pct(0.50);
  o->p99_us = pct(0.99);
  o->max_us = v.empty() ? 0.0 : *std::max_element(v.begin(), v.end());
  double sum = 0;
  for (double x : v) sum += x;
  o->mean_us = v.empty() ? 0.0 : sum / (double)v.size();
  return BM_OK;
}

__attribute__((visibility("default"))) int bm_server_stats(bm_server* s, bm_server_stats_t* o) {
  return bm_server_get_stats(s, o);
}

__attribute__((visibility("default"))) int bm_server_reset_stats(bm_server* s) {
  if (!s) return fail(BM_EINVAL, "bm_server_reset_stats: null server");
  std::lock_guard<std::mutex> g(s->mu);
  s->lat_us.clear();
  s->completed = s->points = s->batches = s->batch_requests = s->rejected = 0;
  s->have_first = false;
  return BM_OK;
}

__attribute__((visibility("default"))) int bm_server_run_trace(bm_server* s, const bm_request* reqs, int64_t nreq,
                                                              const double* arrival_us) {
  if (!s || (nreq > 0 && (!reqs || !arrival_us))) return fail(BM_EINVAL, "bm_server_run_trace: null argument");
  std::vector<uint64_t> tickets((size_t)std::max<int64_t>(nreq, 0));
  const auto t0 = Clock::now();
  for (int64_t i = 0; i < nreq; ++i) {
    const auto due = t0 + std::chrono::nanoseconds((int64_t)(arrival_us[i] * 1000.0));
    while (Clock::now() < due) {
    }
    int rc;
    while ((rc = bm_server_submit(s, reqs[i].xy, reqs[i].n, reqs[i].out_ids, &tickets[i])) == BM_EBUSY)
      std::this_thread::yield();
    if (rc != BM_OK) return rc;
  }
  for (int64_t i = 0; i < nreq; ++i) {
    int rc = bm_server_wait(s, tickets[i], -1);
    if (rc != BM_OK) return rc;
  }
  return BM_OK;
}

__attribute__((visibility("default"))) void bm_server_destroy(bm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_dispatch.notify_all();
  s->cv_complete.notify_all();
  if (s->dispatcher.joinable()) s->dispatcher.join();
  if (s->completer.joinable()) s->completer.join();
  for (auto st : s->streams) (void)hipStreamSynchronize(st);
  for (auto& kv : s->reqs) delete kv.second;
  for (auto st : s->streams) (void)hipStreamDestroy(st);
  for (auto ev : s->events) (void)hipEventDestroy(ev);
  (void)hipFree(s->d_pool);
  (void)hipHostFree(s->h_pool);
  delete s->alloc;
  delete s->copies;
  delete s;
}

}  // extern "C"
