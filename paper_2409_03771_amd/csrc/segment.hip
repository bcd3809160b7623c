// Morse-Smale segmentation kernels (gfx950).
//
// Steps (arXiv 2409.03771, methods "Ascending and Descending Segmentation",
// Alg. 1):
//   1. steepest: every vertex points to the (value,id)-largest and
//      (value,id)-smallest vertex of its closed Freudenthal neighbourhood;
//   2. jump: in-place pointer jumping d[v] <- d[d[v]] until every pointer
//      reaches a fixed point (an extremum);
//   3. cells: (asc, desc) pairs go into a device hash table keeping the
//      smallest vertex id per pair; a last pass writes that id per vertex.
#include <climits>

#include "msc_internal.hpp"

namespace msc {
namespace {

constexpr unsigned long long kEmptyKey = ~0ull;

// Fixed point of 32-bit division by a constant known on the host is not
// worth it here; grid coordinates come from one 32-bit divide pair.
struct Dims {
  uint32_t X, Y, Z;
  uint32_t XY;
  uint32_t N;
};

__device__ __forceinline__ void wave_count(bool pred, unsigned long long *ctr) {
  unsigned long long m = __ballot(pred);
  if (m && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1))
    atomicAdd(ctr, (unsigned long long)__popcll(m));
}

// One vertex per thread; the closed neighbourhood is scanned in increasing
// id order, so on equal values the later (larger-id) vertex wins the max and
// the earlier (smaller-id) vertex wins the min.  That is exactly the
// lexicographic (value, id) order.
__global__ void __launch_bounds__(kBlock)
k_steepest(const float *__restrict__ f, Dims d, int32_t *__restrict__ up,
           int32_t *__restrict__ dn, unsigned long long *ctr) {
  uint32_t v = blockIdx.x * kBlock + threadIdx.x;
  bool live = v < d.N;
  bool isnan_v = false, ismax = false, ismin = false;
  if (live) {
    uint32_t z = v / d.XY;
    uint32_t r = v - z * d.XY;
    uint32_t y = r / d.X;
    uint32_t x = r - y * d.X;
    const bool xm = x > 0, xp = x + 1 < d.X;
    const bool ym = y > 0, yp = y + 1 < d.Y;
    const bool zm = z > 0, zp = z + 1 < d.Z;
    const int64_t X = d.X, XY = d.XY;
    // (valid, offset) in increasing offset order; self in the middle.
    const bool ok[15] = {xm && ym && zm, ym && zm,  xm && zm, zm,
                         xm && ym,       ym,        xm,       true,
                         xp,             yp,        xp && yp, zp,
                         xp && zp,       yp && zp,  xp && yp && zp};
    const int64_t off[15] = {-XY - X - 1, -XY - X, -XY - 1, -XY, -X - 1, -X,
                             -1,          0,       1,       X,   X + 1,  XY,
                             XY + 1,      XY + X,  XY + X + 1};
    float fv = f[v];
    isnan_v = fv != fv;
    float bmax = fv, bmin = fv;
    int64_t imax = v, imin = v;
    bool first = true;
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      if (!ok[k]) continue;
      int64_t u = (int64_t)v + off[k];
      float fu = (k == 7) ? fv : f[u];
      if (first) {
        bmax = bmin = fu;
        imax = imin = u;
        first = false;
        continue;
      }
      if (fu >= bmax) { bmax = fu; imax = u; }
      if (fu < bmin) { bmin = fu; imin = u; }
    }
    if (up) up[v] = (int32_t)imax;
    if (dn) dn[v] = (int32_t)imin;
    ismax = imax == (int64_t)v;
    ismin = imin == (int64_t)v;
  }
  wave_count(isnan_v, ctr + kCtrNaN);
  wave_count(ismax, ctr + kCtrMaxima);
  wave_count(ismin, ctr + kCtrMinima);
}

// One in-place jumping round over both pointer arrays.
__global__ void __launch_bounds__(kBlock)
k_jump2(int32_t *a, int32_t *b, uint32_t n, unsigned long long *ctr) {
  uint32_t v = blockIdx.x * kBlock + threadIdx.x;
  bool changed = false;
  if (v < n) {
    int32_t u = a[v];
    if (u != (int32_t)v) {
      int32_t w = __atomic_load_n(&a[u], __ATOMIC_RELAXED);
      if (w != u) { a[v] = w; changed = true; }
    }
    u = b[v];
    if (u != (int32_t)v) {
      int32_t w = __atomic_load_n(&b[u], __ATOMIC_RELAXED);
      if (w != u) { b[v] = w; changed = true; }
    }
  }
  if (__ballot(changed) && (threadIdx.x & 63) == 0)
    atomicOr(ctr + kCtrChanged, 1ull);
}

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__global__ void k_table_clear(unsigned long long *keys, int32_t *vals,
                              uint32_t cap) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < cap) {
    keys[i] = kEmptyKey;
    vals[i] = INT32_MAX;
  }
}

__device__ __forceinline__ uint32_t table_insert(unsigned long long *keys,
                                                 int32_t *vals, uint32_t mask,
                                                 unsigned long long key,
                                                 int32_t id, bool *fresh) {
  uint32_t h = (uint32_t)mix64(key) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    unsigned long long cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
    if (cur == kEmptyKey) {
      cur = atomicCAS(&keys[h], kEmptyKey, key);
      if (cur == kEmptyKey) *fresh = true;
    }
    if (cur == kEmptyKey || cur == key) {
      atomicMin(&vals[h], id);
      return h;
    }
    h = (h + 1) & mask;
  }
  return UINT32_MAX;
}

// Insert every vertex's (asc, desc) pair, keeping the smallest id.  Lanes of
// a wave that share a pair are merged first: the lowest such lane holds the
// smallest id (ids increase with the lane), so only it touches the table.
__global__ void __launch_bounds__(kBlock)
k_pair_insert(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
              uint32_t n, unsigned long long *keys, int32_t *vals,
              uint32_t mask, unsigned long long *ctr) {
  uint32_t v = blockIdx.x * kBlock + threadIdx.x;
  bool pending = v < n;
  unsigned long long key = 0;
  if (pending) key = ((unsigned long long)(uint32_t)a[v] << 32) | (uint32_t)b[v];
  const int lane = threadIdx.x & 63;
  int fresh_count = 0;
  bool overflow = false;
  for (;;) {
    unsigned long long m = __ballot(pending);
    if (!m) break;
    int leader = __ffsll((long long)m) - 1;
    uint32_t lo = __builtin_amdgcn_readlane((uint32_t)key, leader);
    uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(key >> 32), leader);
    unsigned long long lkey = ((unsigned long long)hi << 32) | lo;
    if (lane == leader) {
      bool fresh = false;
      if (table_insert(keys, vals, mask, lkey, (int32_t)v, &fresh) ==
          UINT32_MAX)
        overflow = true;
      fresh_count += fresh;
    }
    if (pending && key == lkey) pending = false;
  }
  if (fresh_count) atomicAdd(ctr + kCtrCells, (unsigned long long)fresh_count);
  if (overflow) atomicOr(ctr + kCtrOverflow, 1ull);
}

__global__ void __launch_bounds__(kBlock)
k_ms_lookup(const int32_t *__restrict__ a, const int32_t *__restrict__ b,
            uint32_t n, const unsigned long long *__restrict__ keys,
            const int32_t *__restrict__ vals, uint32_t mask,
            int32_t *__restrict__ ms) {
  uint32_t v = blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  unsigned long long key =
      ((unsigned long long)(uint32_t)a[v] << 32) | (uint32_t)b[v];
  uint32_t h = (uint32_t)mix64(key) & mask;
  int32_t out = -1;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    unsigned long long cur = keys[h];
    if (cur == key) { out = vals[h]; break; }
    if (cur == kEmptyKey) break;
    h = (h + 1) & mask;
  }
  ms[v] = out;
}

uint32_t table_capacity(uint64_t n, uint64_t nmax, uint64_t nmin) {
  uint64_t bound = nmax * nmin;
  if (bound > n) bound = n;
  uint64_t cap = 1024;
  while (cap < 2 * bound) cap <<= 1;
  return (uint32_t)cap;
}

}  // namespace

int segment_run(msc_ctx *ctx, const float *f, int64_t X, int64_t Y, int64_t Z,
                int32_t *asc, int32_t *desc, int32_t *ms, hipStream_t s) {
  const int64_t n = X * Y * Z;
  Dims d{(uint32_t)X, (uint32_t)Y, (uint32_t)Z, (uint32_t)(X * Y), (uint32_t)n};
  // Workspace: pointer arrays the caller did not ask for.
  size_t need = 0;
  if (!asc) need += align256(n * sizeof(int32_t));
  if (!desc) need += align256(n * sizeof(int32_t));
  MSC_TRY(reserve(ctx->ws, need + 4096));
  Carver cv(ctx->ws);
  int32_t *A = asc ? asc : cv.take<int32_t>(n);
  int32_t *D = desc ? desc : cv.take<int32_t>(n);
  unsigned long long *ctr = ctx->dctr;

  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "steepest", 12.0 * n,
            (k_steepest<<<grid_for(n), kBlock, 0, s>>>(f, d, A, D, ctr)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrNaN]) return MSC_ENAN;
  const uint64_t nmax = ctx->hctr[kCtrMaxima], nmin = ctx->hctr[kCtrMinima];

  int rounds = 0;
  for (;;) {
    // Steepest paths are strictly monotone, so this cannot trigger; it keeps
    // the host loop bounded whatever the device returns.
    if (rounds == 96) return MSC_EHIP;
    MSC_HIP_TRY(hipMemsetAsync(ctr + kCtrChanged, 0, sizeof(unsigned long long),
                               s));
    MSC_PHASE(ctx, s, "jump_round", 24.0 * n,
              (k_jump2<<<grid_for(n), kBlock, 0, s>>>(A, D, (uint32_t)n, ctr)));
    ++rounds;
    MSC_TRY(read_counters(ctx, s));
    if (!ctx->hctr[kCtrChanged]) break;
  }

  uint64_t cells = 0;
  if (ms) {
    uint32_t cap = table_capacity(n, nmax, nmin);
    size_t tbytes = align256((size_t)cap * 8) + align256((size_t)cap * 4);
    MSC_TRY(reserve(ctx->tab, tbytes + 4096));
    Carver tc(ctx->tab);
    unsigned long long *keys = tc.take<unsigned long long>(cap);
    int32_t *vals = tc.take<int32_t>(cap);
    MSC_PHASE(ctx, s, "table_clear", 12.0 * cap,
              (k_table_clear<<<grid_for(cap), kBlock, 0, s>>>(keys, vals, cap)));
    MSC_PHASE(ctx, s, "pair_insert", 8.0 * n,
              (k_pair_insert<<<grid_for(n), kBlock, 0, s>>>(
                  A, D, (uint32_t)n, keys, vals, cap - 1, ctr)));
    MSC_PHASE(ctx, s, "ms_lookup", 12.0 * n,
              (k_ms_lookup<<<grid_for(n), kBlock, 0, s>>>(
                  A, D, (uint32_t)n, keys, vals, cap - 1, ms)));
    MSC_TRY(read_counters(ctx, s));
    if (ctx->hctr[kCtrOverflow]) return MSC_ENOMEM;
    cells = ctx->hctr[kCtrCells];
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  ctx->stats.n_maxima = (int64_t)nmax;
  ctx->stats.n_minima = (int64_t)nmin;
  ctx->stats.n_cells = (int64_t)cells;
  ctx->stats.n_exits = n;
  ctx->stats.jump_rounds = rounds;
  return MSC_OK;
}

}  // namespace msc
