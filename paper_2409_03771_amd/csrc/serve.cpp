// Request queue with continuous batching (host runtime of libmsc.so).
//
// A queue takes `budget` bytes of device memory in one block and splits it:
// a workspace for each kind of work (the scratch of the library context that
// runs that kind, attached as a caller-owned workspace so that it is never
// reallocated while serving) and an arena for request-resident buffers
// (inputs and outputs).  Each kind has its own context and stream.  Five
// host threads drive it:
//
//   dispatcher   admits pending requests in arrival order (within a kind)
//                while the arena holds their buffers and their kind has room
//                in its staging window, and copies their inputs to the
//                device, round-robin over a few copy streams so that several
//                DMA engines share the link;
//   two workers  one per kind: take every staged request of the kind, up to
//                the launch limits -- requests that arrived while earlier
//                launches ran join the next one -- and enqueue one batched
//                call after their input copies, without waiting for the
//                device; at most two launches per kind are in flight;
//   two completers  one per kind: wait for each launch's completion event
//                and finish its requests (each with its own outcome).
//
// Results stay on the device until the client releases the request.
#include <algorithm>
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

struct Launch {
  std::vector<Request *> reqs;
  hipEvent_t done = nullptr;
  int rec = -1;           // call record of a segmentation launch
  int rc = MSC_OK;        // outcome of enqueuing it
  bool recorded = false;  // `done` marks the end of what it enqueued
};

struct msc_queue {
  int device = 0;
  size_t budget = 0;
  int max_batch = 1;
  char *mem = nullptr;           // the whole budget
  char *arena = nullptr;         // request-resident part of it
  size_t arena_size = 0;
  size_t ws_size[2] = {0, 0};    // workspace of each kind (seg, cc)
  Arena alloc;
  msc_ctx *ctx[2] = {nullptr, nullptr};
  static constexpr int kCopyStreams = 4;  // copies spread over DMA engines
  hipStream_t s_copy[kCopyStreams] = {}, s_run[2] = {nullptr, nullptr};
  int next_copy = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending, ready[2];
  std::deque<Launch *> inflight[2];
  std::vector<Launch *> spare[2];  // finished launches, their events reused
  std::map<uint64_t, Request *> all;
  uint64_t next_ticket = 1;
  int64_t launches = 0;
  bool stop = false;   // dispatcher and workers end
  bool drain = false;  // completers end once nothing is in flight
  std::thread dispatcher, worker[2], completer[2];
};

namespace {

int kind_index(int kind) { return kind == MSC_REQ_SEGMENT ? 0 : 1; }

// A launch takes at most this many vertices (and at least one request): a
// launch's requests all complete when it does, so an unbounded batch would
// make its first requests wait for the last ones; 64M vertices keep a
// launch around a millisecond, long enough to fill the device.
constexpr int64_t kMaxBatchVertices = 64ll << 20;

// At most this many requests of a kind are staged (copy issued) and not yet
// taken by its worker.  Copies issued far ahead of the workers share the
// link with the ones a worker waits for, so under overload every request's
// copy finishes late; a short window keeps the link on the requests next in
// line and still keeps it busy while a launch runs.
constexpr size_t kMaxStaged = 8;

// Launches of one kind enqueued and not yet completed.  Two keep the device
// fed while the host prepares the next one; the call records of a context
// (four) outlast them.
constexpr size_t kMaxInflight = 2;

// Share of the budget given to each kind's workspace, and its cap.
constexpr size_t kSegWsDiv = 4, kCcWsDiv = 16;
constexpr size_t kSegWsCap = 8ull << 30, kCcWsCap = 1ull << 30;

// Workspace one request adds to a launch of its kind (an upper bound: the
// launch's own need is at most the sum over its requests).
int request_workspace(const msc_queue *q, const Request *r, size_t *bytes) {
  if (r->kind == MSC_REQ_SEGMENT) {
    static float dummy_f;
    static int32_t dummy_i;
    msc_field f{&dummy_f, {r->dims[0], r->dims[1], r->dims[2]}, &dummy_i,
                &dummy_i, &dummy_i};
    return msc_workspace_size(q->ctx[0], MSC_REQ_SEGMENT, 1, &f, bytes);
  }
  static uint8_t dummy_m;
  static int64_t dummy_l;
  msc_mask m{&dummy_m, {r->dims[0], r->dims[1], r->dims[2]}, &dummy_l};
  return msc_workspace_size(q->ctx[1], MSC_REQ_CC_GRID, 1, &m, bytes);
}

void dispatcher_loop(msc_queue *q) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  while (!q->stop) {
    bool progress = false;
    for (;;) {
      // The oldest pending request whose kind has room in its window; a
      // request of a kind whose window is full does not hold up the other.
      auto it = q->pending.begin();
      while (it != q->pending.end() &&
             q->ready[kind_index((*it)->kind)].size() >= kMaxStaged)
        ++it;
      if (it == q->pending.end()) break;
      Request *r = *it;
      const size_t need = r->in_bytes + r->out_bytes;
      size_t off = 0;
      if (!q->alloc.alloc(need, &off)) break;  // it waits: order is kept
      q->pending.erase(it);
      r->state = kCopying;  // msc_cancel refuses it from here on
      r->off = off;
      r->dev = q->arena + off;
      hipStream_t cs = q->s_copy[q->next_copy];
      q->next_copy = (q->next_copy + 1) % msc_queue::kCopyStreams;
      lk.unlock();
      int rc = MSC_OK;
      // The input may be host or device memory (unified addressing).
      if (!msc::hip_ok(hipMemcpyAsync(r->dev, r->host_in, r->in_bytes,
                                      hipMemcpyDefault, cs)) ||
          !msc::hip_ok(hipEventRecord(r->copied, cs))) {
        rc = MSC_EHIP;
        // A copy may still be in flight into the request's arena space,
        // which the client frees once the request is finished.
        (void)hipStreamSynchronize(cs);
      }
      lk.lock();
      if (rc != MSC_OK) {
        r->rc = rc;
        r->state = kDone;
        r->t_done = now_ns();
      } else {
        r->state = kStaged;
        q->ready[kind_index(r->kind)].push_back(r);
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

msc_mask cc_mask(const Request *r) {
  msc_mask m{};
  m.mask = reinterpret_cast<const uint8_t *>(r->dev);
  for (int k = 0; k < 3; ++k) m.dims[k] = r->dims[k];
  m.labels = reinterpret_cast<int64_t *>(r->dev + round256(r->in_bytes));
  return m;
}

// Enqueue one launch on the kind's stream; never waits for the device.
int issue(msc_queue *q, int k, Launch *L) {
  hipStream_t s = q->s_run[k];
  msc_ctx *ctx = q->ctx[k];
  for (Request *r : L->reqs)
    if (!msc::hip_ok(hipStreamWaitEvent(s, r->copied, 0))) return MSC_EHIP;
  if (k == 0) {
    std::vector<msc_field> fields;
    fields.reserve(L->reqs.size());
    for (Request *r : L->reqs) fields.push_back(seg_field(r));
    MSC_TRY(msc::segment_batch_run(ctx, (int)fields.size(), fields.data(), s,
                                   nullptr, &L->rec));
  } else {
    std::vector<msc_mask> masks;
    masks.reserve(L->reqs.size());
    for (Request *r : L->reqs) masks.push_back(cc_mask(r));
    msc::stats_replaced(ctx);
    MSC_TRY(msc::begin_call(ctx, s));
    MSC_TRY(msc::cc_grid_batch_run(ctx, (int)masks.size(), masks.data(), s));
    MSC_TRY(msc::end_call(ctx, s));
  }
  return MSC_OK;
}

void worker_loop(msc_queue *q, int k) {
  (void)hipSetDevice(q->device);
  std::deque<Request *> &ready = q->ready[k];
  std::unique_lock<std::mutex> lk(q->mu);
  while (!q->stop) {
    if (ready.empty() || q->inflight[k].size() >= kMaxInflight) {
      q->cv.wait(lk);
      continue;
    }
    Launch *L = nullptr;
    if (!q->spare[k].empty()) {
      L = q->spare[k].back();
      q->spare[k].pop_back();
    } else {
      L = new (std::nothrow) Launch();
      if (L && hipEventCreateWithFlags(&L->done, hipEventDisableTiming) !=
                   hipSuccess) {
        delete L;
        L = nullptr;
      }
      if (!L) {  // retried once a launch finishes and frees its record
        q->cv.wait(lk);
        continue;
      }
    }
    L->reqs.clear();
    L->rec = -1;
    const int64_t t = now_ns();
    int64_t verts = 0;
    size_t ws = 0;
    while (!ready.empty() && (int)L->reqs.size() < q->max_batch) {
      Request *r = ready.front();
      if (!L->reqs.empty() && (verts + r->n > kMaxBatchVertices ||
                               ws + r->ws_bytes > q->ws_size[k]))
        break;
      verts += r->n;
      ws += r->ws_bytes;
      ready.pop_front();
      r->state = kRunning;
      r->t_start = t;
      L->reqs.push_back(r);
    }
    for (Request *r : L->reqs) r->batch = (int)L->reqs.size();
    q->cv.notify_all();  // the staging window has room again
    lk.unlock();
    L->rc = issue(q, k, L);
    // Recorded even after a failure: the completer waits for whatever the
    // launch did enqueue before its requests' memory can be released.
    L->recorded = hipEventRecord(L->done, q->s_run[k]) == hipSuccess;
    if (L->rc == MSC_OK && !msc::hip_ok(L->recorded ? hipSuccess
                                                    : hipErrorUnknown))
      L->rc = MSC_EHIP;
    lk.lock();
    q->inflight[k].push_back(L);
    ++q->launches;
    q->cv.notify_all();
  }
}

void completer_loop(msc_queue *q, int k) {
  (void)hipSetDevice(q->device);
  std::unique_lock<std::mutex> lk(q->mu);
  for (;;) {
    if (q->inflight[k].empty()) {
      if (q->drain) break;  // set once the worker has ended
      q->cv.wait(lk);
      continue;
    }
    Launch *L = q->inflight[k].front();
    lk.unlock();
    std::vector<int> rc(L->reqs.size(), L->rc);
    const bool ok = L->recorded
                        ? hipEventSynchronize(L->done) == hipSuccess
                        : hipStreamSynchronize(q->s_run[k]) == hipSuccess;
    for (size_t i = 0; i < L->reqs.size(); ++i) {
      if (rc[i] != MSC_OK) continue;
      rc[i] = !ok ? MSC_EHIP
              : k == 0 ? msc::call_field_status(q->ctx[0], L->rec, (int)i)
                       : MSC_OK;
    }
    const int64_t t = now_ns();
    lk.lock();
    for (size_t i = 0; i < L->reqs.size(); ++i) {
      Request *r = L->reqs[i];
      r->rc = rc[i];
      r->t_done = t;
      r->state = kDone;
    }
    L->reqs.clear();
    q->inflight[k].pop_front();
    q->spare[k].push_back(L);
    q->cv.notify_all();
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
  q->ws_size[0] = std::min(hbm_budget / kSegWsDiv, kSegWsCap) & ~size_t(255);
  q->ws_size[1] = std::min(hbm_budget / kCcWsDiv, kCcWsCap) & ~size_t(255);
  q->arena_size = hbm_budget - q->ws_size[0] - q->ws_size[1];
  int rc = msc_create(&q->ctx[0], device);
  if (rc == MSC_OK) rc = msc_create(&q->ctx[1], device);
  if (rc == MSC_OK) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    bool ok = hipSetDevice(device) == hipSuccess;
    for (int k = 0; ok && k < msc_queue::kCopyStreams; ++k)
      ok = hipStreamCreateWithFlags(&q->s_copy[k], hipStreamNonBlocking) ==
           hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
      ok = hipStreamCreateWithFlags(&q->s_run[k], hipStreamNonBlocking) ==
           hipSuccess;
    if (!ok)
      rc = MSC_EHIP;
    else if (msc::dev_malloc(reinterpret_cast<void **>(&q->mem),
                             hbm_budget) != hipSuccess)
      rc = MSC_ENOMEM;
    if (prev >= 0) (void)hipSetDevice(prev);
  }
  // The workspaces lead the block; each context carves every launch's
  // scratch from its own and never allocates while serving.
  if (rc == MSC_OK) rc = msc_set_workspace(q->ctx[0], q->mem, q->ws_size[0]);
  if (rc == MSC_OK)
    rc = msc_set_workspace(q->ctx[1], q->mem + q->ws_size[0], q->ws_size[1]);
  if (rc != MSC_OK) {
    msc_queue_destroy(q);
    return rc;
  }
  q->arena = q->mem + q->ws_size[0] + q->ws_size[1];
  q->alloc.reset(q->arena_size);
  q->dispatcher = std::thread(dispatcher_loop, q);
  for (int k = 0; k < 2; ++k) {
    q->worker[k] = std::thread(worker_loop, q, k);
    q->completer[k] = std::thread(completer_loop, q, k);
  }
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
  for (int k = 0; k < 2; ++k)
    if (q->worker[k].joinable()) q->worker[k].join();
  {
    std::lock_guard<std::mutex> lk(q->mu);
    q->drain = true;
  }
  q->cv.notify_all();
  for (int k = 0; k < 2; ++k)
    if (q->completer[k].joinable()) q->completer[k].join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(q->device);
  (void)hipDeviceSynchronize();
  for (auto &kv : q->all) {
    if (kv.second->copied) (void)hipEventDestroy(kv.second->copied);
    delete kv.second;
  }
  for (int k = 0; k < 2; ++k)
    for (Launch *L : q->spare[k]) {
      if (L->done) (void)hipEventDestroy(L->done);
      delete L;
    }
  // The contexts go first: their workspaces live in the block.
  msc_destroy(q->ctx[0]);
  msc_destroy(q->ctx[1]);
  (void)hipSetDevice(q->device);
  if (q->mem) (void)hipFree(q->mem);
  for (hipStream_t cs : q->s_copy)
    if (cs) (void)hipStreamDestroy(cs);
  for (hipStream_t rs : q->s_run)
    if (rs) (void)hipStreamDestroy(rs);
  if (prev >= 0) (void)hipSetDevice(prev);
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
  const int wrc = request_workspace(q, r, &r->ws_bytes);
  if (wrc != MSC_OK) {
    delete r;
    return wrc;
  }
  if (round256(r->in_bytes + r->out_bytes) > q->arena_size ||
      r->ws_bytes > q->ws_size[kind_index(r->kind)]) {
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
  const bool ok = msc::hip_ok(hipMemcpy(dst, src, bytes, hipMemcpyDefault));
  if (prev >= 0) (void)hipSetDevice(prev);
  return ok ? MSC_OK : MSC_EHIP;
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
  out->workspace_reserved = q->ws_size[0] + q->ws_size[1];
  out->arena_size = q->arena_size;
  out->launches = q->launches;
  for (msc_ctx *c : q->ctx) {
    out->workspace_grows += c->grows.load(std::memory_order_relaxed);
    out->host_waits += c->host_waits.load(std::memory_order_relaxed);
  }
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
