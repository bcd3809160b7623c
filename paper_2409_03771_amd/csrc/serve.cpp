// Request queue with continuous batching (host runtime of libmsc.so).
//
// A queue owns an HBM arena of `budget` bytes for request-resident buffers
// (inputs and outputs) and two library contexts, one per kind of work, each
// with its own stream.  Three host threads drive it:
//
//   dispatcher   admits pending requests in arrival order while their
//                footprint (resident buffers plus the workspace their launch
//                needs) fits the budget, places their buffers in the arena and
//                copies their inputs to the device, round-robin over a few
//                copy streams so that several DMA engines share the link;
//   seg worker   takes every admitted segmentation request whose launch slot
//                is free -- requests that arrived while the previous launch
//                ran join the next one -- and segments them in one batched
//                call after waiting for their input copies;
//   cc worker    the same for mask connected components, one request at a
//                time on its own stream, overlapping with segmentation.
//
// Results stay on the device until the client releases the request.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "msc_internal.hpp"

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// kCopying: taken from `pending`, its input copy being issued with the
// queue's lock released; from then on it can no longer be cancelled.
enum State { kPending, kCopying, kStaged, kRunning, kDone, kCanceled };

struct Request {
  uint64_t ticket = 0;
  int kind = 0;
  int64_t dims[3] = {0, 0, 0};
  int64_t n = 0;
  const void *host_in = nullptr;
  size_t in_bytes = 0, out_bytes = 0, ws_bytes = 0;
  size_t off = 0;
  char *dev = nullptr;
  State state = kPending;
  int rc = MSC_OK;
  int batch = 0;
  hipEvent_t copied = nullptr;
  int64_t t_submit = 0, t_start = 0, t_done = 0;
};

// First-fit allocator over [0, size) in 256-byte units, with coalescing.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
    used_ = 0;
  }
  bool alloc(size_t bytes, size_t *off) {
    bytes = (bytes + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
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
  size_t used() const { return used_; }

 private:
  std::map<size_t, size_t> free_;
  size_t used_ = 0;
};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

struct msc_queue {
  int device = 0;
  size_t budget = 0;
  int max_batch = 1;
  char *arena = nullptr;
  Arena alloc;
  size_t inflight_ws = 0;
  msc_ctx *ctx_seg = nullptr, *ctx_cc = nullptr;
  static constexpr int kCopyStreams = 4;  // copies spread over DMA engines
  hipStream_t s_copy[kCopyStreams] = {}, s_seg = nullptr, s_cc = nullptr;
  int next_copy = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending, ready_seg, ready_cc;
  std::map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread dispatcher, worker_seg, worker_cc;
};

namespace {

// Estimated device bytes a launch of this request needs beyond its resident
// buffers: a segmentation's local pointers (4 B/vertex) and exit lists
// (12 B per exit, at most about a third of the vertices on small tiles); a
// CC's 16-bit tile labels.
// A segmentation launch takes at most this many vertices (and at least one
// request): a batch's requests all complete when the launch does, so an
// unbounded batch would make its first requests wait for the last ones;
// 64M vertices keep a launch around a millisecond, long enough to fill the
// device.
constexpr int64_t kMaxBatchVertices = 64ll << 20;

// At most this many requests are staged (copy issued) and not yet taken by
// a worker. Copies issued far ahead of the workers share the link with the
// ones a worker waits for, so under overload every request's copy finishes
// late; a short window keeps the link on the requests next in line and
// still keeps it busy while a launch runs.
constexpr size_t kMaxStaged = 8;

size_t workspace_bytes(int kind, int64_t n) {
  if (kind == MSC_REQ_SEGMENT) return (size_t)n * 8 + (1 << 20);
  return (size_t)n * 2 + (1 << 20);
}

void dispatcher_loop(msc_queue *q) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  while (!q->stop) {
    bool progress = false;
    while (!q->pending.empty()) {
      if (q->ready_seg.size() + q->ready_cc.size() >= kMaxStaged) break;
      Request *r = q->pending.front();
      const size_t need = r->in_bytes + r->out_bytes;
      if (q->alloc.used() + round256(need) + q->inflight_ws + r->ws_bytes >
          q->budget)
        break;  // the head waits: arrival order is kept
      size_t off = 0;
      if (!q->alloc.alloc(need, &off)) break;
      q->pending.pop_front();
      r->state = kCopying;  // msc_cancel refuses it from here on
      r->off = off;
      r->dev = q->arena + off;
      q->inflight_ws += r->ws_bytes;
      hipStream_t cs = q->s_copy[q->next_copy];
      q->next_copy = (q->next_copy + 1) % msc_queue::kCopyStreams;
      lk.unlock();
      int rc = MSC_OK;
      // The input may be host or device memory (unified addressing).
      if (hipMemcpyAsync(r->dev, r->host_in, r->in_bytes, hipMemcpyDefault,
                         cs) != hipSuccess ||
          hipEventRecord(r->copied, cs) != hipSuccess)
        rc = MSC_EHIP;
      lk.lock();
      if (rc != MSC_OK) {
        r->rc = rc;
        r->state = kDone;
        r->t_done = now_ns();
        q->inflight_ws -= r->ws_bytes;
      } else {
        r->state = kStaged;
        (r->kind == MSC_REQ_SEGMENT ? q->ready_seg : q->ready_cc).push_back(r);
      }
      progress = true;
      q->cv.notify_all();
    }
    if (!progress) q->cv.wait(lk);
  }
}

msc_field seg_field(const Request *r) {
  msc_field f{};
  f.field = reinterpret_cast<const float *>(r->dev);
  for (int k = 0; k < 3; ++k) f.dims[k] = r->dims[k];
  int32_t *out = reinterpret_cast<int32_t *>(r->dev + round256(r->in_bytes));
  f.asc = out;
  f.desc = out + r->n;
  f.ms = out + 2 * r->n;
  return f;
}

void finish(msc_queue *q, std::vector<Request *> &batch,
            const std::vector<int> &rc) {
  const int64_t t = now_ns();
  std::lock_guard<std::mutex> lk(q->mu);
  for (size_t i = 0; i < batch.size(); ++i) {
    batch[i]->rc = rc[i];
    batch[i]->t_done = t;
    batch[i]->state = kDone;
    q->inflight_ws -= batch[i]->ws_bytes;
  }
  q->cv.notify_all();
}

void worker_loop(msc_queue *q, int kind) {
  (void)hipSetDevice(q->device);
  std::deque<Request *> &ready = kind == MSC_REQ_SEGMENT ? q->ready_seg
                                                          : q->ready_cc;
  hipStream_t s = kind == MSC_REQ_SEGMENT ? q->s_seg : q->s_cc;
  msc_ctx *ctx = kind == MSC_REQ_SEGMENT ? q->ctx_seg : q->ctx_cc;
  const int cap = kind == MSC_REQ_SEGMENT ? q->max_batch : 1;
  std::unique_lock<std::mutex> lk(q->mu);
  while (!q->stop) {
    if (ready.empty()) {
      q->cv.wait(lk);
      continue;
    }
    std::vector<Request *> batch;
    const int64_t t = now_ns();
    int64_t verts = 0;
    while (!ready.empty() && (int)batch.size() < cap &&
           (batch.empty() || verts + ready.front()->n <= kMaxBatchVertices)) {
      Request *r = ready.front();
      verts += r->n;
      ready.pop_front();
      r->state = kRunning;
      r->t_start = t;
      batch.push_back(r);
    }
    for (Request *r : batch) r->batch = (int)batch.size();
    q->cv.notify_all();  // the staging window has room again
    lk.unlock();
    std::vector<int> rc(batch.size(), MSC_OK);
    for (Request *r : batch)
      if (hipStreamWaitEvent(s, r->copied, 0) != hipSuccess)
        for (int &x : rc) x = MSC_EHIP;
    if (kind == MSC_REQ_SEGMENT) {
      std::vector<msc_field> fields;
      for (Request *r : batch) fields.push_back(seg_field(r));
      int all = rc[0] == MSC_OK
                    ? msc_segment_batched(ctx, (int)fields.size(),
                                          fields.data(), s)
                    : rc[0];
      if (all == MSC_OK && hipStreamSynchronize(s) != hipSuccess)
        all = MSC_EHIP;
      for (size_t i = 0; i < batch.size(); ++i) {
        // Each field's own outcome: a NaN in one request fails it alone.
        msc_stats st{};
        rc[i] = all;
        if (all == MSC_OK)
          rc[i] = msc_last_field_stats(ctx, (int)i, &st) == MSC_OK ? st.status
                                                                  : MSC_EHIP;
      }
    } else {
      Request *r = batch[0];
      if (rc[0] == MSC_OK)
        rc[0] = cc_label_grid(
            ctx, reinterpret_cast<const uint8_t *>(r->dev), r->dims,
            reinterpret_cast<int64_t *>(r->dev + round256(r->in_bytes)), s);
      if (rc[0] == MSC_OK && hipStreamSynchronize(s) != hipSuccess)
        rc[0] = MSC_EHIP;
    }
    finish(q, batch, rc);
    lk.lock();
  }
}

Request *find(msc_queue *q, uint64_t ticket) {
  auto it = q->all.find(ticket);
  return it == q->all.end() ? nullptr : it->second;
}

}  // namespace

extern "C" {

int msc_queue_create(int device, size_t hbm_budget, int max_batch,
                     msc_queue **out) {
  if (!out || hbm_budget < (1u << 20) || max_batch < 1) return MSC_EINVAL;
  *out = nullptr;
  msc_queue *q = new (std::nothrow) msc_queue();
  if (!q) return MSC_ENOMEM;
  q->device = device;
  q->budget = hbm_budget;
  q->max_batch = max_batch;
  int rc = msc_create(&q->ctx_seg, device);
  if (rc == MSC_OK) rc = msc_create(&q->ctx_cc, device);
  if (rc == MSC_OK) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    bool ok = hipSetDevice(device) == hipSuccess;
    for (int k = 0; ok && k < msc_queue::kCopyStreams; ++k)
      ok = hipStreamCreateWithFlags(&q->s_copy[k], hipStreamNonBlocking) ==
           hipSuccess;
    ok = ok &&
         hipStreamCreateWithFlags(&q->s_seg, hipStreamNonBlocking) ==
             hipSuccess &&
         hipStreamCreateWithFlags(&q->s_cc, hipStreamNonBlocking) == hipSuccess;
    if (!ok)
      rc = MSC_EHIP;
    else if (hipMalloc(&q->arena, hbm_budget) != hipSuccess)
      rc = MSC_ENOMEM;
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  if (rc != MSC_OK) {
    msc_queue_destroy(q);
    return rc;
  }
  q->alloc.reset(hbm_budget);
  q->dispatcher = std::thread(dispatcher_loop, q);
  q->worker_seg = std::thread(worker_loop, q, MSC_REQ_SEGMENT);
  q->worker_cc = std::thread(worker_loop, q, MSC_REQ_CC_GRID);
  *out = q;
  return MSC_OK;
}

void msc_queue_destroy(msc_queue *q) {
  if (!q) return;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->stop = true;
  }
  q->cv.notify_all();
  if (q->dispatcher.joinable()) q->dispatcher.join();
  if (q->worker_seg.joinable()) q->worker_seg.join();
  if (q->worker_cc.joinable()) q->worker_cc.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->device);
  (void)hipDeviceSynchronize();
  for (auto &kv : q->all) {
    if (kv.second->copied) (void)hipEventDestroy(kv.second->copied);
    delete kv.second;
  }
  if (q->arena) (void)hipFree(q->arena);
  for (hipStream_t cs : q->s_copy)
    if (cs) (void)hipStreamDestroy(cs);
  if (q->s_seg) (void)hipStreamDestroy(q->s_seg);
  if (q->s_cc) (void)hipStreamDestroy(q->s_cc);
  if (prev >= 0) (void)hipSetDevice(prev);
  msc_destroy(q->ctx_seg);
  msc_destroy(q->ctx_cc);
  delete q;
}

int msc_submit(msc_queue *q, const msc_request *req, uint64_t *ticket) {
  if (!q || !req || !ticket || !req->host_input) return MSC_EINVAL;
  if (req->kind != MSC_REQ_SEGMENT && req->kind != MSC_REQ_CC_GRID)
    return MSC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (req->dims[k] < 1 || req->dims[k] > (INT64_C(1) << 31))
      return MSC_EINVAL;
  const int64_t n = req->dims[0] * req->dims[1] * req->dims[2];
  if (n > INT32_MAX) return MSC_ERANGE;
  Request *r = new (std::nothrow) Request();
  if (!r) return MSC_ENOMEM;
  r->kind = req->kind;
  for (int k = 0; k < 3; ++k) r->dims[k] = req->dims[k];
  r->n = n;
  r->host_in = req->host_input;
  if (r->kind == MSC_REQ_SEGMENT) {
    r->in_bytes = (size_t)n * 4;
    r->out_bytes = 3 * (size_t)n * 4;
  } else {
    r->in_bytes = (size_t)n;
    r->out_bytes = (size_t)n * 8;
  }
  r->out_bytes += 256;  // outputs start on a 256-byte boundary
  r->ws_bytes = workspace_bytes(r->kind, n);
  if (round256(r->in_bytes + r->out_bytes) + r->ws_bytes > q->budget) {
    delete r;
    return MSC_EBUDGET;
  }
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->device);
  const bool ev_ok = hipEventCreateWithFlags(&r->copied,
                                             hipEventDisableTiming) ==
                     hipSuccess;
  if (prev >= 0) (void)hipSetDevice(prev);
  if (!ev_ok) {
    delete r;
    return MSC_EHIP;
  }
  r->t_submit = now_ns();
  {
    std::lock_guard<std::mutex> lk(q->mu);
    r->ticket = q->next_ticket++;
    q->all[r->ticket] = r;
    q->pending.push_back(r);
    *ticket = r->ticket;
  }
  q->cv.notify_all();
  return MSC_OK;
}

int msc_poll(msc_queue *q, uint64_t ticket, int *status) {
  if (!q || !status) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  Request *r = find(q, ticket);
  if (!r) return MSC_EINVAL;
  *status = r->state == kDone       ? r->rc
            : r->state == kCanceled ? MSC_ECANCELED
                                    : MSC_EBUSY;
  return MSC_OK;
}

int msc_wait(msc_queue *q, uint64_t ticket) {
  if (!q) return MSC_EINVAL;
  std::unique_lock<std::mutex> lk(q->mu);
  Request *r = find(q, ticket);
  if (!r) return MSC_EINVAL;
  q->cv.wait(lk, [&] { return r->state == kDone || r->state == kCanceled; });
  return r->state == kCanceled ? MSC_ECANCELED : r->rc;
}

int msc_get_result(msc_queue *q, uint64_t ticket, msc_result *out) {
  if (!q || !out) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  Request *r = find(q, ticket);
  if (!r) return MSC_EINVAL;
  if (r->state != kDone) return MSC_EBUSY;
  *out = msc_result{};
  out->kind = r->kind;
  out->status = r->rc;
  out->n = r->n;
  out->batch_size = r->batch;
  out->t_submit_ns = r->t_submit;
  out->t_start_ns = r->t_start;
  out->t_done_ns = r->t_done;
  if (r->rc == MSC_OK && r->dev) {
    char *o = r->dev + round256(r->in_bytes);
    if (r->kind == MSC_REQ_SEGMENT) {
      out->asc = reinterpret_cast<int32_t *>(o);
      out->desc = out->asc + r->n;
      out->ms = out->asc + 2 * r->n;
    } else {
      out->labels = reinterpret_cast<int64_t *>(o);
    }
  }
  return MSC_OK;
}

int msc_copy_result(msc_queue *q, uint64_t ticket, int which, void *dst) {
  if (!q || !dst || which < 0 || which > 3) return MSC_EINVAL;
  const char *src = nullptr;
  size_t bytes = 0;
  {
    std::lock_guard<std::mutex> lk(q->mu);
    Request *r = find(q, ticket);
    if (!r) return MSC_EINVAL;
    if (r->state != kDone) return MSC_EBUSY;
    if (r->rc != MSC_OK) return r->rc;
    if ((which == 3) != (r->kind == MSC_REQ_CC_GRID)) return MSC_EINVAL;
    const char *o = r->dev + round256(r->in_bytes);
    if (which == 3) {
      src = o;
      bytes = (size_t)r->n * 8;
    } else {
      src = o + (size_t)which * r->n * 4;
      bytes = (size_t)r->n * 4;
    }
  }
  // The region stays valid: only msc_release frees it, and the caller owns
  // the ticket.
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->device);
  const hipError_t e = hipMemcpy(dst, src, bytes, hipMemcpyDefault);
  if (prev >= 0) (void)hipSetDevice(prev);
  return e == hipSuccess ? MSC_OK : MSC_EHIP;
}

int msc_release(msc_queue *q, uint64_t ticket) {
  if (!q) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  Request *r = find(q, ticket);
  if (!r) return MSC_EINVAL;
  if (r->state != kDone && r->state != kCanceled) return MSC_EBUSY;
  if (r->dev) q->alloc.release(r->off, r->in_bytes + r->out_bytes);
  if (r->copied) (void)hipEventDestroy(r->copied);
  q->all.erase(ticket);
  delete r;
  q->cv.notify_all();
  return MSC_OK;
}

int msc_cancel(msc_queue *q, uint64_t ticket) {
  if (!q) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  Request *r = find(q, ticket);
  if (!r) return MSC_EINVAL;
  if (r->state != kPending) return MSC_EBUSY;
  for (auto it = q->pending.begin(); it != q->pending.end(); ++it) {
    if (*it == r) {
      q->pending.erase(it);
      break;
    }
  }
  r->state = kCanceled;
  r->t_done = now_ns();
  q->cv.notify_all();
  return MSC_OK;
}

int msc_queue_info(msc_queue *q, msc_queue_stats *out) {
  if (!q || !out) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(q->mu);
  *out = msc_queue_stats{};
  out->budget = q->budget;
  out->arena_used = q->alloc.used();
  out->workspace_reserved = q->inflight_ws;
  for (auto &kv : q->all) {
    switch (kv.second->state) {
      case kPending: ++out->pending; break;
      case kCopying:
      case kStaged:
      case kRunning: ++out->running; break;
      default: ++out->finished; break;
    }
  }
  return MSC_OK;
}

}  // extern "C"
