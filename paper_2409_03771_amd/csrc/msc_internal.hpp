// Internal declarations shared by the translation units of libmsc.so.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/msc.h"

namespace msc {
// Host-side fault injection (msc_debug_inject): the check that takes a
// kind's countdown to zero reports a failure.
bool inject_fault(int what);
// A runtime call's result, failed by an armed MSC_INJECT_EHIP countdown.
inline bool hip_ok(hipError_t e) {
  return e == hipSuccess && !inject_fault(MSC_INJECT_EHIP);
}
// Device and pinned host allocations, failed by an armed MSC_INJECT_ENOMEM
// countdown (nothing is allocated then).
inline hipError_t dev_malloc(void **p, size_t bytes) {
  if (inject_fault(MSC_INJECT_ENOMEM)) return hipErrorOutOfMemory;
  return hipMalloc(p, bytes);
}
inline hipError_t host_malloc(void **p, size_t bytes) {
  if (inject_fault(MSC_INJECT_ENOMEM)) return hipErrorOutOfMemory;
  return hipHostMalloc(p, bytes, hipHostMallocDefault);
}
}  // namespace msc

#define MSC_HIP_TRY(expr)                                                   \
  do {                                                                      \
    if (!msc::hip_ok(expr)) return MSC_EHIP;                                \
  } while (0)

#define MSC_TRY(expr)                                                       \
  do {                                                                      \
    int s_ = (expr);                                                        \
    if (s_ != MSC_OK) return s_;                                            \
  } while (0)

namespace msc {

constexpr int kBlock = 256;

// Slots of the small device counter block each context owns.
enum Counter : int {
  kCtrChanged = 0,   // set nonzero by a round that changed something
  kCtrExits = 5,     // exits over all tiles (from the scan)
  kCtrBadIndex = 6,  // out-of-range CSR column seen
  kCtrOverflow = 7,  // pair table full (bit 0), broken exit chain (bit 1),
                     // in-tile jumping did not settle (bit 2)
  kCtrRounds = 9,    // longest exit chain walked
  kCtrSteps = 10,    // exit-graph links followed in total
  kCtrRootsMax = 11, // vertices that are their own ascent label
  kCtrRootsMin = 12, // vertices that are their own descent label
  kCtrNaN = 13,      // a NaN field value seen (CSR segmentation)
  kNumCounters = 16
};

}  // namespace msc

namespace msc {
// Grow-only device buffer.
struct DevBuf {
  char *ptr = nullptr;
  size_t bytes = 0;
  bool external = false;  // caller-owned: never freed or grown
};

// Event-bracketed per-kernel timing; see msc_profile in msc.h.
struct Profiler {
  struct Pending {
    int slot;
    hipEvent_t a, b;
    double bytes;
  };
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  std::vector<Pending> pending;
  std::vector<msc_phase> totals;

  int slot_of(const char *name) {
    for (size_t i = 0; i < totals.size(); ++i)
      if (std::strncmp(totals[i].name, name, sizeof(totals[i].name)) == 0)
        return (int)i;
    msc_phase p{};
    std::strncpy(p.name, name, sizeof(p.name) - 1);
    totals.push_back(p);
    return (int)totals.size() - 1;
  }
  hipEvent_t event() {
    if (next == pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[next++];
  }
  // Fold finished events into the totals; the stream must be complete.
  void flush() {
    for (const Pending &p : pending) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
        totals[p.slot].launches += 1;
        totals[p.slot].total_ms += ms;
        totals[p.slot].bytes += p.bytes;
      }
    }
    pending.clear();
    next = 0;
  }
  ~Profiler() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};
}  // namespace msc

namespace msc {
// Pinned host slot for a call's small host-to-device copies; reused once the
// copy that last read it has executed (its event has completed).
struct PinnedSlot {
  void *ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t copied = nullptr;
  bool pending = false;
};
constexpr int kPinnedSlots = 8;

// One asynchronous segmentation call: what the stats calls need of it.  Its
// counters arrive in the record's pinned buffers once its work completes
// (event `done`).  Records are reused round-robin; a record is taken again
// only after its call's event has completed.
struct CallRec {
  hipEvent_t done = nullptr;
  bool pending = false;                 // issued; its event not yet waited on
  unsigned long long *hctr = nullptr;   // pinned copy of the counter block
  unsigned long long *hfctr = nullptr;  // pinned per-field counters
  size_t hfctr_cap = 0;                 // entries
  int nfields = 0;
  std::vector<int64_t> n;               // vertices per field
  std::vector<char> has_ms;             // cells requested per field
  int tile[3] = {0, 0, 0};
};
// Asynchronous calls that may be in flight on one context before a new one
// waits for the oldest.
constexpr int kCallRing = 4;
}  // namespace msc

struct msc_ctx {
  int device = 0;
  // Grow-only device workspaces carved per call: `ws` for per-vertex
  // scratch, `tab` for hash tables and lists sized after a first pass.
  msc::DevBuf ws, tab, xg;  // workspace, pair tables, exit graph
  msc::DevBuf rk;           // virtual-rank path: slab labels, ghost graph
  // Device counters and a pinned host mirror.
  unsigned long long *dctr = nullptr;
  unsigned long long *hctr = nullptr;
  msc_stats stats{};
  msc::Profiler prof;
  int tile_choice = 0;         // segmentation tile shape (0 = default)
  uint64_t table_first = 0;    // first pair-table capacity (0 = automatic)
  void *pinned = nullptr;      // grow-only pinned host staging
  size_t pinned_bytes = 0;
  std::vector<msc_stats> field_stats;  // per field of the last batch
  // Calls return with their work enqueued.  `done` is recorded on the
  // call's stream after its last work; a call on another stream first
  // waits for it (the workspaces are shared), and the stats calls wait for
  // it before reading the counters.
  hipEvent_t done = nullptr;
  hipStream_t last_stream = nullptr;
  bool done_valid = false;
  msc::PinnedSlot slots[msc::kPinnedSlots];
  int next_slot = 0;
  // Records of the asynchronous segmentation calls; `last_call` is the
  // record whose stats the stats calls report (-1: the stats are those of a
  // call that set them itself).
  msc::CallRec calls[msc::kCallRing];
  int next_call = 0;
  int last_call = -1;
  bool last_folded = true;     // last_call's counters are in `stats`
  int last_status = MSC_OK;    // device-detected outcome of the last call
  // Workspace growths (each one waits for the context's earlier work), and
  // every time the host waited for the device before enqueuing work.
  std::atomic<int64_t> grows{0};
  std::atomic<int64_t> host_waits{0};
};

namespace msc {

// Make sure `buf` holds at least `bytes`.  Growing waits for the context's
// earlier work (the old block may still be in use) and discards the old
// contents; a caller-owned buffer is never grown (MSC_ENOMEM).
int reserve(msc_ctx *ctx, DevBuf &buf, size_t bytes);

// Wait for `e` on the host, counting the wait when it was not complete.
int host_wait(msc_ctx *ctx, hipEvent_t e);

// Order a call on stream `s` after the context's previous call (which may
// have run on another stream), and mark the end of a call's work.
int begin_call(msc_ctx *ctx, hipStream_t s);
int end_call(msc_ctx *ctx, hipStream_t s);

// A pinned host buffer of at least `bytes` for one host-to-device copy on
// `s`; call slot_copied after issuing the copy.
int pinned_slot(msc_ctx *ctx, size_t bytes, void **out, int *slot);
int slot_copied(msc_ctx *ctx, int slot, hipStream_t s);

// Wait for the last segmentation call and fold its counters into the stats.
int finish_last(msc_ctx *ctx);

// Mark the stats as set by a call that is not a recorded asynchronous one.
inline void stats_replaced(msc_ctx *ctx) {
  ctx->last_call = -1;
  ctx->last_folded = true;
  ctx->last_status = MSC_OK;
  ctx->field_stats.clear();
}

// A record for a new asynchronous call whose counters need `nfields`
// per-field entries; waits for the record's previous call if still pending.
int take_call(msc_ctx *ctx, int nfields, int *index);

// Outcome of field `i` of a recorded call, once its event has completed,
// and its counts.
int call_field_status(const msc_ctx *ctx, int index, int i);
int call_field_stats(const msc_ctx *ctx, int index, int i, msc_stats *st);

// Bump allocator over a DevBuf for the duration of one call.
struct Carver {
  char *base;
  size_t cap, used = 0;
  explicit Carver(const DevBuf &b) : base(b.ptr), cap(b.bytes) {}
  template <class T>
  T *take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    return reinterpret_cast<T *>(base + off);
  }
};

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Read the counter block back to the host (synchronises `stream`).
int read_counters(msc_ctx *ctx, hipStream_t stream);
int clear_counters(msc_ctx *ctx, hipStream_t stream);
// Zero n counters with a kernel on `stream`.
int zero_u64(unsigned long long *p, int n, hipStream_t stream);

// Launch `launch` (a statement) bracketed by profiling events when enabled.
#define MSC_PHASE(ctx, stream, name, bytes, launch)                         \
  do {                                                                      \
    hipEvent_t pa_ = nullptr, pb_ = nullptr;                                \
    if ((ctx)->prof.on) {                                                   \
      pa_ = (ctx)->prof.event();                                            \
      if (pa_) (void)hipEventRecord(pa_, stream);                           \
    }                                                                       \
    launch;                                                                 \
    MSC_HIP_TRY(hipGetLastError());                                         \
    if ((ctx)->prof.on && pa_) {                                            \
      pb_ = (ctx)->prof.event();                                            \
      if (pb_) {                                                            \
        (void)hipEventRecord(pb_, stream);                                  \
        (ctx)->prof.pending.push_back(                                      \
            {(ctx)->prof.slot_of(name), pa_, pb_, (double)(bytes)});        \
      }                                                                     \
    }                                                                       \
  } while (0)

inline unsigned grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// Segmentation tile shapes compiled in (index = ctx->tile_choice); the
// first is the default.
constexpr int kNumTileShapes = 5;
constexpr int kTileShapes[kNumTileShapes][3] = {
    {32, 16, 16}, {32, 8, 8}, {64, 8, 8}, {32, 8, 16}, {64, 8, 16}};
inline int tile_index(int tx, int ty, int tz) {
  for (int i = 0; i < kNumTileShapes; ++i)
    if (kTileShapes[i][0] == tx && kTileShapes[i][1] == ty &&
        kTileShapes[i][2] == tz)
      return i;
  return -1;
}

// Launchers implemented in the kernel translation units.
// Workspace bytes segment_batch_run carves for this batch (the context's
// tile shape).
int segment_workspace(const msc_ctx *ctx, int nfields, const msc_field *fields,
                      size_t *bytes);
// `rec` receives the index of the call's record (see take_call).
int segment_batch_run(msc_ctx *ctx, int nfields, const msc_field *fields,
                      hipStream_t s, const uint8_t *ghost = nullptr,
                      int *rec = nullptr);
int segment_ranks_run(msc_ctx *ctx, const float *field, const int64_t dims[3],
                      int ranks, int32_t *asc, int32_t *desc, int32_t *ms,
                      hipStream_t s);
int csr_from_tets_run(msc_ctx *ctx, int64_t n, int64_t ntets,
                      const int32_t *tets, int64_t *row_ptr, int32_t *col_idx,
                      int64_t capacity, int64_t *nnz, hipStream_t stream);
int critical_points_run(msc_ctx *ctx, const float *field, const int64_t *dims,
                        uint8_t *code, hipStream_t stream);
int extremum_graph_run(msc_ctx *ctx, const float *field, const int64_t *dims,
                       const int32_t *asc, const int32_t *desc, int32_t *edges,
                       int64_t capacity, int64_t *count, hipStream_t stream);
int segment_csr_run(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                    const int32_t *col_idx, const float *field, int32_t *asc,
                    int32_t *desc, int32_t *ms, hipStream_t stream);
// `sync` false marks a slab of a larger call (no stats of its own).
// label_off is added to every written label (a slab labelled in place
// inside a larger grid gets global ids).
int cc_grid_run(msc_ctx *ctx, const uint8_t *mask, int64_t X, int64_t Y,
                int64_t Z, int64_t *labels, hipStream_t s, bool sync = true,
                int64_t label_off = 0);
// Several masks, each labelled on its own, in launches of up to 32 masks.
int cc_grid_batch_run(msc_ctx *ctx, int n, const msc_mask *masks,
                      hipStream_t s);
// Workspace bytes cc_grid_batch_run carves for these masks.
size_t cc_grid_workspace(int n, const msc_mask *masks);
int cc_grid_ranks_run(msc_ctx *ctx, const uint8_t *mask, int64_t X,
                      int64_t Y, int64_t Z, int ranks, int64_t *labels,
                      hipStream_t stream);
int cc_csr_run(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
               const int32_t *col_idx, const uint8_t *mask, int64_t *labels,
               hipStream_t s);
int jump_run(msc_ctx *ctx, int64_t *d, int64_t n, int rounds, int sync,
             hipStream_t s);

}  // namespace msc
