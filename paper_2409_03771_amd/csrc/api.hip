// C-ABI entry points of libmsc.so: argument checks, context and workspace.
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>

#include "msc_internal.hpp"

namespace msc {

namespace {
std::atomic<int> g_inject[3] = {{-1}, {-1}, {-1}};
}  // namespace

bool inject_fault(int what) {
  std::atomic<int> &c = g_inject[what];
  int v = c.load(std::memory_order_relaxed);
  while (v >= 0) {
    if (c.compare_exchange_weak(v, v - 1, std::memory_order_relaxed))
      return v == 0;
  }
  return false;
}

int host_wait(msc_ctx *ctx, hipEvent_t e) {
  const hipError_t q = hipEventQuery(e);
  if (q == hipSuccess) return MSC_OK;
  if (q != hipErrorNotReady) return MSC_EHIP;
  ++ctx->host_waits;
  MSC_HIP_TRY(hipEventSynchronize(e));
  return MSC_OK;
}

int reserve(msc_ctx *ctx, DevBuf &buf, size_t bytes) {
  if (bytes <= buf.bytes) return MSC_OK;
  if (buf.external) return MSC_ENOMEM;
  // The old block may still be read by this context's queued work.
  if (ctx->done_valid) MSC_TRY(host_wait(ctx, ctx->done));
  ++ctx->grows;
  if (buf.ptr) {
    MSC_HIP_TRY(hipFree(buf.ptr));
    buf.ptr = nullptr;
    buf.bytes = 0;
  }
  size_t want = bytes + bytes / 8 + (1 << 20);
  void *p = nullptr;
  if (dev_malloc(&p, want) != hipSuccess) {
    (void)hipGetLastError();
    return MSC_ENOMEM;
  }
  buf.ptr = static_cast<char *>(p);
  buf.bytes = want;
  return MSC_OK;
}

// Counters are cleared by a kernel, not a memset: a memset node captured
// into a HIP graph is not safe to replay.
__global__ void k_zero_u64(unsigned long long *p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0ull;
}

int zero_u64(unsigned long long *p, int n, hipStream_t stream) {
  k_zero_u64<<<(n + 63) / 64, 64, 0, stream>>>(p, n);
  MSC_HIP_TRY(hipGetLastError());
  return MSC_OK;
}

int clear_counters(msc_ctx *ctx, hipStream_t stream) {
  return zero_u64(ctx->dctr, kNumCounters, stream);
}

int begin_call(msc_ctx *ctx, hipStream_t s) {
  if (ctx->done_valid && ctx->last_stream != s)
    MSC_HIP_TRY(hipStreamWaitEvent(s, ctx->done, 0));
  return MSC_OK;
}

int end_call(msc_ctx *ctx, hipStream_t s) {
  MSC_HIP_TRY(hipEventRecord(ctx->done, s));
  ctx->last_stream = s;
  ctx->done_valid = true;
  return MSC_OK;
}

int pinned_slot(msc_ctx *ctx, size_t bytes, void **out, int *slot) {
  const int k = ctx->next_slot;
  ctx->next_slot = (k + 1) % kPinnedSlots;
  PinnedSlot &ps = ctx->slots[k];
  // The copy that last read this slot must have executed.
  if (ps.pending) MSC_TRY(host_wait(ctx, ps.copied));
  ps.pending = false;
  if (bytes > ps.bytes) {
    if (ps.ptr) (void)hipHostFree(ps.ptr);
    ps.ptr = nullptr;
    ps.bytes = 0;
    const size_t want = bytes + bytes / 4 + 4096;
    if (host_malloc(&ps.ptr, want) != hipSuccess)
      return MSC_ENOMEM;
    ps.bytes = want;
  }
  *out = ps.ptr;
  *slot = k;
  return MSC_OK;
}

int slot_copied(msc_ctx *ctx, int slot, hipStream_t s) {
  MSC_HIP_TRY(hipEventRecord(ctx->slots[slot].copied, s));
  ctx->slots[slot].pending = true;
  return MSC_OK;
}

int read_counters(msc_ctx *ctx, hipStream_t stream) {
  MSC_HIP_TRY(hipMemcpyAsync(ctx->hctr, ctx->dctr,
                             kNumCounters * sizeof(unsigned long long),
                             hipMemcpyDeviceToHost, stream));
  MSC_HIP_TRY(hipStreamSynchronize(stream));
  if (ctx->prof.on) ctx->prof.flush();
  return MSC_OK;
}

}  // namespace msc

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) return;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Entry of a call that synchronises: the pending counters of an earlier
// asynchronous call are folded first (this call replaces the stats), and
// the call's work is ordered after that call's.
int enter_sync(msc_ctx *ctx, hipStream_t s) {
  MSC_TRY(msc::finish_last(ctx));
  msc::stats_replaced(ctx);
  return msc::begin_call(ctx, s);
}

int check_dims(const int64_t dims[3], int64_t *n) {
  if (!dims) return MSC_EINVAL;
  for (int i = 0; i < 3; ++i)
    if (dims[i] < 1) return MSC_EINVAL;
  // Guard the product against overflow of int64.
  const int64_t lim = INT64_C(1) << 40;
  if (dims[0] > lim || dims[1] > lim || dims[2] > lim) return MSC_ERANGE;
  if (dims[0] * dims[1] > lim || dims[0] * dims[1] * dims[2] > lim)
    return MSC_ERANGE;
  *n = dims[0] * dims[1] * dims[2];
  return MSC_OK;
}

}  // namespace

extern "C" {

const char *msc_strerror(int code) {
  switch (code) {
    case MSC_OK: return "ok";
    case MSC_EINVAL: return "invalid argument";
    case MSC_ERANGE: return "size out of range for the id type";
    case MSC_ENAN: return "NaN in scalar field";
    case MSC_ENOMEM: return "device workspace allocation failed";
    case MSC_EBUDGET: return "request exceeds the memory budget";
    case MSC_EHIP: return "HIP runtime error";
    case MSC_ECANCELED: return "request cancelled";
    case MSC_EBUSY: return "request not finished";
    default: return "unknown error";
  }
}

int msc_create(msc_ctx **out, int device) {
  if (!out) return MSC_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess) return MSC_EHIP;
  if (device < 0 || device >= count) return MSC_EINVAL;
  DeviceGuard g(device);
  if (!g.ok) return MSC_EHIP;
  msc_ctx *c = new (std::nothrow) msc_ctx();
  if (!c) return MSC_ENOMEM;
  c->device = device;
  if (msc::dev_malloc(reinterpret_cast<void **>(&c->dctr),
                      msc::kNumCounters * sizeof(unsigned long long)) !=
      hipSuccess) {
    delete c;
    return MSC_ENOMEM;
  }
  if (msc::host_malloc(reinterpret_cast<void **>(&c->hctr),
                       msc::kNumCounters * sizeof(unsigned long long)) !=
      hipSuccess) {
    (void)hipFree(c->dctr);
    delete c;
    return MSC_ENOMEM;
  }
  std::memset(c->hctr, 0, msc::kNumCounters * sizeof(unsigned long long));
  bool ev_ok = hipEventCreateWithFlags(&c->done, hipEventDisableTiming) ==
               hipSuccess;
  for (int k = 0; ev_ok && k < msc::kPinnedSlots; ++k)
    ev_ok = hipEventCreateWithFlags(&c->slots[k].copied,
                                    hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ev_ok && k < msc::kCallRing; ++k)
    ev_ok = hipEventCreateWithFlags(&c->calls[k].done,
                                    hipEventDisableTiming) == hipSuccess;
  if (!ev_ok) {
    msc_destroy(c);
    return MSC_EHIP;
  }
  // Tile shape override for tuning runs, e.g. MSC_TILE=32x16x16.
  if (const char *t = std::getenv("MSC_TILE")) {
    int tx = 0, ty = 0, tz = 0;
    if (std::sscanf(t, "%dx%dx%d", &tx, &ty, &tz) == 3) {
      int k = msc::tile_index(tx, ty, tz);
      if (k >= 0) c->tile_choice = k;
    }
  }
  *out = c;
  return MSC_OK;
}

void msc_destroy(msc_ctx *ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->ws.ptr && !ctx->ws.external) (void)hipFree(ctx->ws.ptr);
  if (ctx->tab.ptr) (void)hipFree(ctx->tab.ptr);
  if (ctx->xg.ptr) (void)hipFree(ctx->xg.ptr);
  if (ctx->rk.ptr) (void)hipFree(ctx->rk.ptr);
  if (ctx->dctr) (void)hipFree(ctx->dctr);
  if (ctx->hctr) (void)hipHostFree(ctx->hctr);
  for (msc::CallRec &r : ctx->calls) {
    if (r.hctr) (void)hipHostFree(r.hctr);
    if (r.hfctr) (void)hipHostFree(r.hfctr);
    if (r.done) (void)hipEventDestroy(r.done);
  }
  for (msc::PinnedSlot &ps : ctx->slots) {
    if (ps.ptr) (void)hipHostFree(ps.ptr);
    if (ps.copied) (void)hipEventDestroy(ps.copied);
  }
  if (ctx->done) (void)hipEventDestroy(ctx->done);
  delete ctx;
}

int msc_debug_inject(int what, int after) {
  if (what != MSC_INJECT_ENOMEM && what != MSC_INJECT_EHIP) return MSC_EINVAL;
  msc::g_inject[what].store(after < 0 ? -1 : after, std::memory_order_relaxed);
  return MSC_OK;
}

int msc_set_workspace(msc_ctx *ctx, void *ptr, size_t bytes) {
  if (!ctx) return MSC_EINVAL;
  if (ptr && ((reinterpret_cast<uintptr_t>(ptr) & 255) || bytes < 4096))
    return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  // The current workspace may still be read by queued work.
  if (ctx->done_valid) MSC_HIP_TRY(hipEventSynchronize(ctx->done));
  if (ctx->ws.ptr && !ctx->ws.external) MSC_HIP_TRY(hipFree(ctx->ws.ptr));
  ctx->ws = msc::DevBuf{};
  if (ptr) {
    ctx->ws.ptr = static_cast<char *>(ptr);
    ctx->ws.bytes = bytes;
    ctx->ws.external = true;
  }
  return MSC_OK;
}

int msc_workspace_size(const msc_ctx *ctx, int kind, int n, const void *descs,
                       size_t *bytes) {
  if (!ctx || !bytes || n < 0 || (n > 0 && !descs)) return MSC_EINVAL;
  *bytes = 0;
  if (kind == MSC_REQ_SEGMENT) {
    const msc_field *f = static_cast<const msc_field *>(descs);
    for (int i = 0; i < n; ++i) {
      int64_t v = 0;
      MSC_TRY(check_dims(f[i].dims, &v));
      if (v > INT32_MAX) return MSC_ERANGE;
    }
    return n ? msc::segment_workspace(ctx, n, f, bytes) : MSC_OK;
  }
  if (kind == MSC_REQ_CC_GRID) {
    const msc_mask *m = static_cast<const msc_mask *>(descs);
    for (int i = 0; i < n; ++i) {
      int64_t v = 0;
      MSC_TRY(check_dims(m[i].dims, &v));
    }
    *bytes = msc::cc_grid_workspace(n, m);
    return MSC_OK;
  }
  return MSC_EINVAL;
}

int msc_segment(msc_ctx *ctx, const float *field, const int64_t dims[3],
                int32_t *asc, int32_t *desc, int32_t *ms, void *stream) {
  if (!ctx || !dims) return MSC_EINVAL;
  msc_field f{field, {dims[0], dims[1], dims[2]}, asc, desc, ms};
  return msc_segment_batched(ctx, 1, &f, stream);
}

int msc_segment_ranks(msc_ctx *ctx, const float *field, const int64_t dims[3],
                      int ranks, int32_t *asc, int32_t *desc, int32_t *ms,
                      void *stream) {
  if (!ctx || !dims || !field || (!asc && !desc && !ms)) return MSC_EINVAL;
  int64_t n = 0;
  MSC_TRY(check_dims(dims, &n));
  if (n > INT32_MAX) return MSC_ERANGE;
  if (ranks < 1 || ranks > dims[2]) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::segment_ranks_run(ctx, field, dims, ranks, asc, desc, ms,
                                static_cast<hipStream_t>(stream));
}

int msc_segment_csr(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                    const int32_t *col_idx, const float *field, int32_t *asc,
                    int32_t *desc, int32_t *ms, void *stream) {
  if (!ctx || n < 0) return MSC_EINVAL;
  if (n > INT32_MAX) return MSC_ERANGE;
  if (n > 0 && (!row_ptr || !field || (!asc && !desc && !ms)))
    return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::segment_csr_run(ctx, n, row_ptr, col_idx, field, asc, desc, ms,
                              static_cast<hipStream_t>(stream));
}

int msc_segment_batched(msc_ctx *ctx, int nfields, const msc_field *fields,
                        void *stream) {
  if (!ctx || nfields < 0 || (nfields > 0 && !fields)) return MSC_EINVAL;
  if (nfields == 0) return MSC_OK;
  for (int i = 0; i < nfields; ++i) {
    const msc_field &f = fields[i];
    if (!f.field || (!f.asc && !f.desc && !f.ms)) return MSC_EINVAL;
    int64_t n = 0;
    MSC_TRY(check_dims(f.dims, &n));
    if (n > INT32_MAX) return MSC_ERANGE;
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  return msc::segment_batch_run(ctx, nfields, fields,
                                static_cast<hipStream_t>(stream));
}

}  // extern "C"

struct msc_graph {
  msc_ctx *ctx = nullptr;  // the graph's own workspace, counters and records
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after each replay
  int rec = -1;               // call record the captured call writes
  bool launched = false;
};

extern "C" {

int msc_graph_create(msc_ctx *ctx, int nfields, const msc_field *fields,
                     void *stream, msc_graph **out) {
  if (!ctx || !out || nfields < 1 || !fields) return MSC_EINVAL;
  *out = nullptr;
  for (int i = 0; i < nfields; ++i) {
    const msc_field &f = fields[i];
    if (!f.field || (!f.asc && !f.desc && !f.ms)) return MSC_EINVAL;
    int64_t n = 0;
    MSC_TRY(check_dims(f.dims, &n));
    if (n > INT32_MAX) return MSC_ERANGE;
  }
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return MSC_EHIP;
  msc_graph *g = new (std::nothrow) msc_graph();
  if (!g) return MSC_ENOMEM;
  auto fail = [&](int rc) {
    msc_graph_destroy(g);
    return rc;
  };
  int rc = msc_create(&g->ctx, ctx->device);
  if (rc != MSC_OK) return fail(rc);
  g->ctx->tile_choice = ctx->tile_choice;
  g->ctx->table_first = ctx->table_first;
  if (!msc::hip_ok(hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking)) ||
      !msc::hip_ok(hipEventCreateWithFlags(&g->done, hipEventDisableTiming)))
    return fail(MSC_EHIP);
  // The fields may still be produced by work on the caller's stream.
  if (!msc::hip_ok(hipEventRecord(g->done, static_cast<hipStream_t>(stream))) ||
      !msc::hip_ok(hipStreamWaitEvent(g->cap, g->done, 0)))
    return fail(MSC_EHIP);
  // One ordinary call first: it sizes the workspace and allocates the call
  // record and the pinned descriptor slot, so that the captured call
  // allocates nothing and waits for nothing (and it leaves the outputs
  // computed).  The captured call then reuses that record and slot.
  rc = msc::segment_batch_run(g->ctx, nfields, fields, g->cap);
  if (rc != MSC_OK) return fail(rc);
  if (!msc::hip_ok(hipStreamSynchronize(g->cap))) return fail(MSC_EHIP);
  rc = msc::finish_last(g->ctx);
  if (rc != MSC_OK) return fail(rc);
  g->ctx->next_call = 0;
  g->ctx->calls[0].pending = false;
  g->ctx->next_slot = 0;
  g->ctx->slots[0].pending = false;
  if (!msc::hip_ok(
          hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal)))
    return fail(MSC_EHIP);
  rc = msc::segment_batch_run(g->ctx, nfields, fields, g->cap, nullptr,
                              &g->rec);
  hipGraph_t graph = nullptr;
  const hipError_t ec = hipStreamEndCapture(g->cap, &graph);
  g->graph = graph;
  if (rc != MSC_OK) return fail(rc);
  if (!msc::hip_ok(ec) || !graph) return fail(MSC_EHIP);
  if (!msc::hip_ok(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)))
    return fail(MSC_EHIP);
  *out = g;
  return MSC_OK;
}

int msc_graph_launch(msc_graph *g, void *stream) {
  if (!g || !g->exec) return MSC_EINVAL;
  DeviceGuard dg(g->ctx->device);
  if (!dg.ok) return MSC_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  MSC_HIP_TRY(hipGraphLaunch(g->exec, s));
  MSC_HIP_TRY(hipEventRecord(g->done, s));
  g->launched = true;
  return MSC_OK;
}

int msc_graph_field_stats(msc_graph *g, int index, msc_stats *out) {
  if (!g || !out || !g->launched) return MSC_EINVAL;
  DeviceGuard dg(g->ctx->device);
  if (!dg.ok) return MSC_EHIP;
  MSC_HIP_TRY(hipEventSynchronize(g->done));
  return msc::call_field_stats(g->ctx, g->rec, index, out);
}

void msc_graph_destroy(msc_graph *g) {
  if (!g) return;
  if (g->ctx) {
    DeviceGuard dg(g->ctx->device);
    if (g->cap) (void)hipStreamSynchronize(g->cap);
    if (g->launched && g->done) (void)hipEventSynchronize(g->done);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->done) (void)hipEventDestroy(g->done);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    msc_destroy(g->ctx);
  }
  delete g;
}

int msc_last_field_stats(const msc_ctx *ctx, int index, msc_stats *out) {
  if (!ctx || !out) return MSC_EINVAL;
  msc_ctx *c = const_cast<msc_ctx *>(ctx);
  DeviceGuard g(c->device);
  MSC_TRY(msc::finish_last(c));
  if (index < 0 || index >= (int)ctx->field_stats.size()) return MSC_EINVAL;
  *out = ctx->field_stats[index];
  return MSC_OK;
}

int msc_last_status(msc_ctx *ctx, int *status) {
  if (!ctx || !status) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  MSC_TRY(msc::finish_last(ctx));
  *status = ctx->last_status;
  return MSC_OK;
}

int msc_autotune(msc_ctx *ctx, int nfields, const msc_field *fields,
                 void *stream, msc_tune *out) {
  if (!ctx || !out) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  *out = msc_tune{};
  const int prev = ctx->tile_choice;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    if (a) (void)hipEventDestroy(a);
    return MSC_EHIP;
  }
  int best = -1, rc = MSC_OK;
  float best_ms = 0.f;
  const int nshape = msc::kNumTileShapes < 8 ? msc::kNumTileShapes : 8;
  for (int i = 0; i < nshape && rc == MSC_OK; ++i) {
    ctx->tile_choice = i;
    // One untimed run sizes the workspace; the best of two timed runs counts.
    rc = msc_segment_batched(ctx, nfields, fields, stream);
    float t_best = 0.f;
    for (int r = 0; r < 2 && rc == MSC_OK; ++r) {
      if (hipEventRecord(a, s) != hipSuccess) { rc = MSC_EHIP; break; }
      rc = msc_segment_batched(ctx, nfields, fields, stream);
      if (rc != MSC_OK) break;
      float ms = 0.f;
      if (hipEventRecord(b, s) != hipSuccess ||
          hipEventSynchronize(b) != hipSuccess ||
          hipEventElapsedTime(&ms, a, b) != hipSuccess) {
        rc = MSC_EHIP;
        break;
      }
      if (r == 0 || ms < t_best) t_best = ms;
    }
    out->ms[i] = t_best;
    if (rc == MSC_OK && (best < 0 || t_best < best_ms)) {
      best = i;
      best_ms = t_best;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (rc != MSC_OK) {
    ctx->tile_choice = prev;
    return rc;
  }
  ctx->tile_choice = best;
  out->n_shapes = nshape;
  out->best = best;
  for (int k = 0; k < 3; ++k) out->tile[k] = msc::kTileShapes[best][k];
  return MSC_OK;
}

int msc_tile_shapes(int *out, int max) {
  const int n = msc::kNumTileShapes;
  for (int i = 0; i < n && i < max && out; ++i)
    for (int k = 0; k < 3; ++k) out[3 * i + k] = msc::kTileShapes[i][k];
  return n;
}

int msc_set_tile(msc_ctx *ctx, int tx, int ty, int tz) {
  if (!ctx) return MSC_EINVAL;
  int k = msc::tile_index(tx, ty, tz);
  if (k < 0) return MSC_EINVAL;
  ctx->tile_choice = k;
  return MSC_OK;
}

int msc_set_table_capacity(msc_ctx *ctx, uint64_t first_capacity) {
  if (!ctx || first_capacity > (1ull << 32)) return MSC_EINVAL;
  ctx->table_first = first_capacity;
  return MSC_OK;
}

int msc_last_stats(const msc_ctx *ctx, msc_stats *out) {
  if (!ctx || !out) return MSC_EINVAL;
  msc_ctx *c = const_cast<msc_ctx *>(ctx);
  DeviceGuard g(c->device);
  MSC_TRY(msc::finish_last(c));
  *out = ctx->stats;
  return MSC_OK;
}

int msc_profile(msc_ctx *ctx, int enable) {
  if (!ctx) return MSC_EINVAL;
  if (enable) {
    DeviceGuard g(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->prof.pending.clear();
    ctx->prof.next = 0;
    ctx->prof.totals.clear();
  }
  ctx->prof.on = enable != 0;
  return MSC_OK;
}

int msc_profile_read(const msc_ctx *ctx, msc_phase *out, int max, int *count) {
  if (!ctx || !count || max < 0 || (max > 0 && !out)) return MSC_EINVAL;
  // Fold the recorded launches (their events must have completed).
  msc_ctx *c = const_cast<msc_ctx *>(ctx);
  if (!c->prof.pending.empty()) {
    DeviceGuard g(c->device);
    MSC_HIP_TRY(hipEventSynchronize(c->prof.pending.back().b));
    c->prof.flush();
  }
  int n = (int)ctx->prof.totals.size();
  *count = n;
  for (int i = 0; i < n && i < max; ++i) out[i] = ctx->prof.totals[i];
  return MSC_OK;
}

int cc_label_grid(msc_ctx *ctx, const uint8_t *mask, const int64_t dims[3],
                  int64_t *labels, void *stream) {
  if (!ctx || !mask || !labels) return MSC_EINVAL;
  int64_t n = 0;
  MSC_TRY(check_dims(dims, &n));
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  msc::stats_replaced(ctx);  // this call replaces the stats
  MSC_TRY(msc::begin_call(ctx, static_cast<hipStream_t>(stream)));
  MSC_TRY(msc::cc_grid_run(ctx, mask, dims[0], dims[1], dims[2], labels,
                           static_cast<hipStream_t>(stream)));
  return msc::end_call(ctx, static_cast<hipStream_t>(stream));
}

int cc_label_grid_batched(msc_ctx *ctx, int nmasks, const msc_mask *masks,
                          void *stream) {
  if (!ctx || nmasks < 0 || (nmasks > 0 && !masks)) return MSC_EINVAL;
  if (nmasks == 0) return MSC_OK;
  for (int i = 0; i < nmasks; ++i) {
    if (!masks[i].mask || !masks[i].labels) return MSC_EINVAL;
    int64_t n = 0;
    MSC_TRY(check_dims(masks[i].dims, &n));
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  msc::stats_replaced(ctx);
  hipStream_t s = static_cast<hipStream_t>(stream);
  MSC_TRY(msc::begin_call(ctx, s));
  MSC_TRY(msc::cc_grid_batch_run(ctx, nmasks, masks, s));
  return msc::end_call(ctx, s);
}

int cc_label_grid_ranks(msc_ctx *ctx, const uint8_t *mask,
                        const int64_t dims[3], int ranks, int64_t *labels,
                        void *stream) {
  if (!ctx || !mask || !labels) return MSC_EINVAL;
  int64_t n = 0;
  MSC_TRY(check_dims(dims, &n));
  if (ranks < 1 || ranks > dims[2]) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::cc_grid_ranks_run(ctx, mask, dims[0], dims[1], dims[2], ranks,
                                labels, static_cast<hipStream_t>(stream));
}

int msc_critical_points(msc_ctx *ctx, const float *field,
                        const int64_t dims[3], uint8_t *code, void *stream) {
  if (!ctx || !dims || !field || !code) return MSC_EINVAL;
  int64_t n = 0;
  MSC_TRY(check_dims(dims, &n));
  if (n > INT32_MAX) return MSC_ERANGE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::critical_points_run(ctx, field, dims, code,
                                  static_cast<hipStream_t>(stream));
}

int msc_extremum_graph(msc_ctx *ctx, const float *field, const int64_t dims[3],
                       const int32_t *asc, const int32_t *desc, int32_t *edges,
                       int64_t capacity, int64_t *count, void *stream) {
  if (!ctx || !dims || !field || !asc || !desc || !count || capacity < 0)
    return MSC_EINVAL;
  int64_t n = 0;
  MSC_TRY(check_dims(dims, &n));
  if (n > INT32_MAX) return MSC_ERANGE;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::extremum_graph_run(ctx, field, dims, asc, desc, edges, capacity,
                                 count, static_cast<hipStream_t>(stream));
}

int msc_csr_from_tets(msc_ctx *ctx, int64_t n, int64_t ntets,
                      const int32_t *tets, int64_t *row_ptr, int32_t *col_idx,
                      int64_t capacity, int64_t *nnz, void *stream) {
  if (!ctx || n < 0 || ntets < 0 || !row_ptr || !nnz) return MSC_EINVAL;
  if (n > INT32_MAX || ntets > (INT64_MAX >> 6)) return MSC_ERANGE;
  if (ntets > 0 && !tets) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::csr_from_tets_run(ctx, n, ntets, tets, row_ptr, col_idx,
                                capacity, nnz,
                                static_cast<hipStream_t>(stream));
}

int cc_label_csr(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                 const int32_t *col_idx, const uint8_t *mask, int64_t *labels,
                 void *stream) {
  if (!ctx || n < 0) return MSC_EINVAL;
  if (n == 0) return MSC_OK;
  if (n > INT32_MAX) return MSC_EINVAL;
  if (!row_ptr || !labels) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::cc_csr_run(ctx, n, row_ptr, col_idx, mask, labels,
                         static_cast<hipStream_t>(stream));
}

int msc_pointer_jump(msc_ctx *ctx, int64_t *d, int64_t n, int rounds,
                     int synchronous, void *stream) {
  if (!ctx || n < 0 || rounds < 0) return MSC_EINVAL;
  if (n == 0) return MSC_OK;
  if (!d) return MSC_EINVAL;
  DeviceGuard g(ctx->device);
  if (!g.ok) return MSC_EHIP;
  MSC_TRY(enter_sync(ctx, static_cast<hipStream_t>(stream)));
  return msc::jump_run(ctx, d, n, rounds, synchronous,
                       static_cast<hipStream_t>(stream));
}

}  // extern "C"
