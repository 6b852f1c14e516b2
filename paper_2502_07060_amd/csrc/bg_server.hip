// Serving loop: amplitude requests of mixed (field, n, d, p) arrive from host
// threads; one scheduler thread per server admits them into a device arena by
// their HBM footprint, merges the requests waiting for the same (field, n, d,
// p) into one launch, and keeps several launches in flight on separate
// streams, so that the copies of one batch overlap the kernels of others.
//
// Life of a request:  submit (validated, queued)  ->  admitted into a batch
// when the batch's region fits the arena and a launch slot is free  ->  on
// its stream: host-to-device 2-D copies of momenta and polarisations into the
// batch's columns, one kernel over the whole batch, device-to-host copies of
// its outputs  ->  done when the batch's event has completed; the region goes
// back to the arena.  Admission is first come, first served: the first batch
// that does not fit stops admission until memory frees up.
//
// The arena is one device allocation made at creation; nothing is allocated
// per request.  The plain mode (BG_SERVER_PLAIN) runs the same requests one
// launch per request, one at a time, in arrival order, on one stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bg.h"
#include "bg_registry.h"

namespace bg {
namespace {

constexpr int kMaxStreams = 8;
constexpr int64_t kAlign = 256;            // arena granularity (bytes)
constexpr int64_t kColAlign = 64;          // batch leading dimension rounded to 64 points
constexpr int64_t kMaxBatchPoints = 1 << 21;
constexpr size_t kMaxQueued = 1 << 20;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

int64_t elem_size(int field) { return field == BG_FIELD_C128 ? 16 : 4; }

// device bytes of a batch of `cols` columns: momenta and polarisations
// [n][d][cols], out [cols], status [cols], each part 256-byte aligned
int64_t batch_bytes(int field, int n, int d, int64_t cols) {
  const int64_t s = elem_size(field);
  return 2 * round_up((int64_t)n * d * cols * s, kAlign) + round_up(cols * s, kAlign) + round_up(cols, kAlign);
}

// first-fit allocator over [0, size) with coalescing frees
class Arena {
 public:
  void reset(int64_t size) {
    free_.clear();
    if (size > 0) free_[0] = size;
    size_ = size;
    used_ = peak_ = 0;
  }
  int64_t alloc(int64_t bytes) {
    bytes = round_up(bytes, kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest > 0) free_[off + bytes] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = round_up(bytes, kAlign);
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
  int64_t size() const { return size_; }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t size_ = 0, used_ = 0, peak_ = 0;
};

struct Request {
  uint64_t id = 0;
  bg_group g{};  // host pointers
  int64_t t_submit = 0, t_launch = 0, t_done = 0;
  int64_t col = 0;        // first column in its batch
  int batch_size = 0;     // requests that shared its launch
  int rc = BG_OK;
  bool done = false;
};

struct Batch {
  int field = 0, n = 0, d = 0;
  uint32_t p = 0;
  std::vector<Request*> reqs;
  int64_t npts = 0, cols = 0, off = -1, bytes = 0;
  int stream = 0;
  hipEvent_t ev = nullptr;
  int rc = BG_OK;
  bool same_key(const bg_group& g) const {
    return g.field == field && g.n == n && g.d == d && (field == BG_FIELD_C128 || g.p == p);
  }
};

}  // namespace
}  // namespace bg

struct bg_server {
  int device = 0;
  bool plain = false;
  int nstreams = 0;
  int max_inflight = 0;
  hipStream_t streams[bg::kMaxStreams] = {};
  int stream_load[bg::kMaxStreams] = {};
  char* arena_base = nullptr;
  bg::Arena arena;  // scheduler thread only (and create/destroy)
  std::vector<hipEvent_t> events;  // idle events, scheduler thread only
  std::vector<std::unique_ptr<bg::Batch>> inflight;  // scheduler thread only

  std::mutex mu;  // guards everything below
  std::condition_variable cv_work, cv_done;
  std::deque<bg::Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<bg::Request>> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  bg_server_stats st{};

  std::thread worker;
};

namespace bg {
namespace {

// Pull waiting requests (FIFO) into at most `slots` new batches whose
// regions fit the arena.  Requests of the first batch that does not fit,
// and every later one, stay queued in arrival order.
std::vector<std::unique_ptr<Batch>> form_batches(bg_server* s, int slots) {
  std::vector<std::unique_ptr<Batch>> out;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    while (!s->pending.empty()) {
      Request* r = s->pending.front();
      Batch* b = nullptr;
      if (!s->plain)
        for (auto& c : out)
          if (c->same_key(r->g) && c->npts + r->g.npts <= kMaxBatchPoints &&
              batch_bytes(c->field, c->n, c->d, round_up(c->npts + r->g.npts, kColAlign)) <= s->arena.size())
            b = c.get();
      if (!b) {
        if ((int)out.size() >= slots) break;
        out.emplace_back(new Batch);
        b = out.back().get();
        b->field = r->g.field;
        b->n = r->g.n;
        b->d = r->g.d;
        b->p = r->g.p;
      }
      r->col = b->npts;
      b->npts += r->g.npts;
      b->reqs.push_back(r);
      s->pending.pop_front();
    }
  }
  // allocate in formation order; the first failure returns its requests and
  // those of every later batch to the head of the queue
  size_t ok = 0;
  for (; ok < out.size(); ++ok) {
    Batch& b = *out[ok];
    b.cols = round_up(b.npts, kColAlign);
    b.bytes = batch_bytes(b.field, b.n, b.d, b.cols);
    b.off = s->arena.alloc(b.bytes);
    if (b.off < 0) break;
  }
  if (ok < out.size()) {
    std::vector<Request*> back;
    for (size_t i = ok; i < out.size(); ++i)
      for (Request* r : out[i]->reqs) back.push_back(r);
    std::sort(back.begin(), back.end(), [](const Request* a, const Request* b) { return a->id < b->id; });
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto it = back.rbegin(); it != back.rend(); ++it) s->pending.push_front(*it);
    out.resize(ok);
  }
  return out;
}

void launch_batch(bg_server* s, Batch& b) {
  int best = 0;
  for (int i = 1; i < s->nstreams; ++i)
    if (s->stream_load[i] < s->stream_load[best]) best = i;
  b.stream = best;
  s->stream_load[best]++;
  hipStream_t st = s->streams[best];
  const int64_t es = elem_size(b.field);
  const int64_t rows = (int64_t)b.n * b.d;
  char* mom = s->arena_base + b.off;
  char* pol = mom + round_up(rows * b.cols * es, kAlign);
  char* out = pol + round_up(rows * b.cols * es, kAlign);
  uint8_t* sts = reinterpret_cast<uint8_t*>(out + round_up(b.cols * es, kAlign));
  const int64_t t = now_ns();
  int rc = BG_OK;
  for (Request* r : b.reqs) {
    r->t_launch = t;
    r->batch_size = (int)b.reqs.size();
    if (r->g.npts == 0) continue;
    const size_t w = (size_t)(r->g.npts * es), dp = (size_t)(b.cols * es), sp = (size_t)(r->g.ld * es);
    if (hipMemcpy2DAsync(mom + r->col * es, dp, r->g.momenta, sp, w, (size_t)rows, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpy2DAsync(pol + r->col * es, dp, r->g.pols, sp, w, (size_t)rows, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = BG_EHIP;
  }
  if (rc == BG_OK && b.npts > 0) {
    LaunchSpec spec;
    FpConst k{};
    if (b.field == BG_FIELD_FP) k = make_fp_const(b.p);
    rc = prepare(b.field, b.n, b.d, b.npts, b.cols, mom, pol, out, sts, k, spec);
    if (rc == BG_OK) rc = enqueue(spec, st);
  }
  if (rc == BG_OK) {
    for (Request* r : b.reqs) {
      if (r->g.npts == 0) continue;
      if (hipMemcpyAsync(r->g.out, out + r->col * es, (size_t)(r->g.npts * es), hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = BG_EHIP;
      if (r->g.status &&
          hipMemcpyAsync(r->g.status, sts + r->col, (size_t)r->g.npts, hipMemcpyDeviceToHost, st) != hipSuccess)
        rc = BG_EHIP;
    }
  }
  b.rc = rc;
  if (s->events.empty()) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess) s->events.push_back(e);
  }
  if (!s->events.empty()) {
    b.ev = s->events.back();
    s->events.pop_back();
    if (hipEventRecord(b.ev, st) != hipSuccess) {
      s->events.push_back(b.ev);
      b.ev = nullptr;
    }
  }
  if (!b.ev) {  // no event: wait for the stream here
    (void)hipStreamSynchronize(st);
    b.rc = BG_EHIP;
  }
}

void finish_batch(bg_server* s, Batch& b, int rc) {
  s->arena.release(b.off, b.bytes);
  s->stream_load[b.stream]--;
  if (b.ev) s->events.push_back(b.ev);
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lk(s->mu);
  for (Request* r : b.reqs) {
    r->t_done = t;
    r->rc = rc;
    r->done = true;
    s->st.completed++;
    s->st.points += r->g.npts;
  }
  s->st.batches++;
  s->st.inflight_batches = (int64_t)s->inflight.size() - 1;
  s->st.arena_in_use = s->arena.used();
  s->st.arena_peak = s->arena.peak();
}

// returns true if some batch finished
bool reap(bg_server* s) {
  bool any = false;
  for (size_t i = 0; i < s->inflight.size();) {
    Batch& b = *s->inflight[i];
    int rc = b.rc;
    if (b.ev) {
      const hipError_t e = hipEventQuery(b.ev);
      if (e == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (e != hipSuccess && rc == BG_OK) rc = BG_EHIP;
    }
    finish_batch(s, b, rc);
    s->inflight.erase(s->inflight.begin() + i);
    any = true;
  }
  if (any) s->cv_done.notify_all();
  return any;
}

void run(bg_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    const bool reaped = reap(s);
    int launched = 0;
    const int slots = s->max_inflight - (int)s->inflight.size();
    if (slots > 0) {
      auto fresh = form_batches(s, slots);
      for (auto& b : fresh) {
        launch_batch(s, *b);
        s->inflight.push_back(std::move(b));
        ++launched;
      }
      if (launched) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.inflight_batches = (int64_t)s->inflight.size();
        s->st.queued = (int64_t)s->pending.size();
        s->st.arena_in_use = s->arena.used();
        s->st.arena_peak = s->arena.peak();
      }
    }
    if (reaped || launched) continue;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && s->pending.empty() && s->inflight.empty()) break;
    if (s->inflight.empty()) {
      s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
    } else {
      lk.unlock();
      std::this_thread::yield();  // work on the GPU: poll its events
    }
  }
}

}  // namespace
}  // namespace bg

extern "C" {

int bg_server_create(size_t hbm_budget_bytes, int flags, bg_server** out) {
  if (!out) return BG_EINVAL;
  *out = nullptr;
  if (hbm_budget_bytes < (size_t)bg::kAlign || (flags & ~BG_SERVER_PLAIN)) return BG_EINVAL;
  auto s = std::make_unique<bg_server>();
  if (hipGetDevice(&s->device) != hipSuccess) return BG_EHIP;
  s->plain = (flags & BG_SERVER_PLAIN) != 0;
  s->nstreams = s->plain ? 1 : 4;
  s->max_inflight = s->plain ? 1 : 2 * s->nstreams;
  const int64_t size = bg::round_up((int64_t)hbm_budget_bytes, bg::kAlign);
  if (hipMalloc(reinterpret_cast<void**>(&s->arena_base), (size_t)size) != hipSuccess) {
    (void)hipGetLastError();
    return BG_ENOMEM;
  }
  s->arena.reset(size);
  int rc = BG_OK;
  for (int i = 0; i < s->nstreams && rc == BG_OK; ++i)
    if (hipStreamCreateWithFlags(&s->streams[i], hipStreamNonBlocking) != hipSuccess) rc = BG_EHIP;
  for (int i = 0; i < 2 * s->max_inflight && rc == BG_OK; ++i) {
    hipEvent_t e;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) rc = BG_EHIP;
    else s->events.push_back(e);
  }
  s->st.arena_bytes = size;
  if (rc == BG_OK) {
    bg_server* raw = s.get();
    s->worker = std::thread([raw] { bg::run(raw); });
  }
  if (rc != BG_OK) {
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    for (int i = 0; i < s->nstreams; ++i)
      if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
    (void)hipFree(s->arena_base);
    return rc;
  }
  *out = s.release();
  return BG_OK;
}

int bg_server_submit(bg_server* s, const bg_group* req, uint64_t* id) {
  if (!s || !req || !id) return BG_EINVAL;
  int rc = bg::validate_group(*req);
  if (rc != BG_OK) return rc;
  const int64_t cols = bg::round_up(req->npts, bg::kColAlign);
  if (bg::batch_bytes(req->field, req->n, req->d, cols) > s->st.arena_bytes || req->npts > bg::kMaxBatchPoints) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.rejected++;
    return BG_ENOMEM;
  }
  auto r = std::make_unique<bg::Request>();
  r->g = *req;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return BG_EINVAL;
  if (s->pending.size() >= bg::kMaxQueued) {
    s->st.rejected++;
    return BG_EBUSY;
  }
  r->id = s->next_id++;
  r->t_submit = bg::now_ns();
  *id = r->id;
  s->st.submitted++;
  if (req->npts == 0) {
    r->t_launch = r->t_done = r->t_submit;
    r->done = true;
    s->st.completed++;
    s->reqs.emplace(r->id, std::move(r));
    return BG_OK;
  }
  s->pending.push_back(r.get());
  s->st.queued = (int64_t)s->pending.size();
  s->reqs.emplace(r->id, std::move(r));
  s->cv_work.notify_one();
  return BG_OK;
}

int bg_server_poll(bg_server* s, uint64_t id) {
  if (!s) return BG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return BG_EINVAL;
  return it->second->done ? 1 : 0;
}

int bg_server_wait(bg_server* s, uint64_t id, double timeout_s, bg_request_times* times) {
  if (!s) return BG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return BG_EINVAL;
  bg::Request* r = it->second.get();
  auto ready = [&] { return r->done; };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, ready);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready)) {
    return BG_EBUSY;
  }
  if (times) {
    times->submit_ns = r->t_submit;
    times->launch_ns = r->t_launch;
    times->done_ns = r->t_done;
    times->batch_requests = r->batch_size;
  }
  const int rc = r->rc;
  s->reqs.erase(it);
  return rc;
}

int bg_server_get_stats(bg_server* s, bg_server_stats* out) {
  if (!s || !out) return BG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->queued = (int64_t)s->pending.size();
  return BG_OK;
}

int64_t bg_server_now_ns(void) { return bg::now_ns(); }

int bg_server_destroy(bg_server* s) {
  if (!s) return BG_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
  for (int i = 0; i < s->nstreams; ++i)
    if (s->streams[i]) (void)hipStreamDestroy(s->streams[i]);
  (void)hipFree(s->arena_base);
  delete s;
  return BG_OK;
}

}  // extern "C"
