// Connected components by hook-and-compress (gfx950).
//
// arXiv 2409.03771, Alg. 3 and methods "Connected Components": masked
// vertices first point to a masked neighbour chosen by id, pointer jumping
// compresses the resulting trees, and a stitching pass links trees that touch
// before a second compression.  Here every pointer goes to a smaller (or
// equal) id, so a component ends up named by its smallest id, and the stitch
// (hook) is an atomicMin on the root that is repeated, each time followed by
// compression, until no hook changes anything: a single stitch does not join
// every pair of touching trees in general.
#include <climits>

#include "msc_internal.hpp"

namespace msc {
namespace {

struct GridDims {
  int64_t X, Y, Z, XY, N;
};

__device__ __forceinline__ void coords(const GridDims &d, int64_t v,
                                       int64_t &x, int64_t &y, int64_t &z) {
  if (d.N <= (int64_t)UINT32_MAX) {
    uint32_t vv = (uint32_t)v, XY = (uint32_t)d.XY, X = (uint32_t)d.X;
    uint32_t zz = vv / XY, r = vv - zz * XY, yy = r / X;
    z = zz;
    y = yy;
    x = r - yy * X;
  } else {
    z = v / d.XY;
    int64_t r = v - z * d.XY;
    y = r / d.X;
    x = r - y * d.X;
  }
}

// Closed Freudenthal neighbourhood in increasing id order (self at k = 7).
struct Stencil {
  bool ok[15];
  int64_t off[15];
  __device__ __forceinline__ Stencil(const GridDims &d, int64_t x, int64_t y,
                                     int64_t z) {
    const bool xm = x > 0, xp = x + 1 < d.X;
    const bool ym = y > 0, yp = y + 1 < d.Y;
    const bool zm = z > 0, zp = z + 1 < d.Z;
    const int64_t X = d.X, XY = d.XY;
    const bool o[15] = {xm && ym && zm, ym && zm, xm && zm, zm,
                        xm && ym,       ym,       xm,       true,
                        xp,             yp,       xp && yp, zp,
                        xp && zp,       yp && zp, xp && yp && zp};
    const int64_t f[15] = {-XY - X - 1, -XY - X, -XY - 1, -XY, -X - 1, -X,
                           -1,          0,       1,       X,   X + 1,  XY,
                           XY + 1,      XY + X,  XY + X + 1};
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      ok[k] = o[k];
      off[k] = f[k];
    }
  }
};

__device__ __forceinline__ int64_t gid() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

__device__ __forceinline__ void flag_any(bool pred, unsigned long long *ctr) {
  if (__ballot(pred) && (threadIdx.x & 63) == 0) atomicOr(ctr, 1ull);
}

// L[v] = smallest masked id of the closed neighbourhood, or -1.
__global__ void __launch_bounds__(kBlock)
k_cc_init(const uint8_t *__restrict__ mask, GridDims d, int64_t *__restrict__ L) {
  int64_t v = gid();
  if (v >= d.N) return;
  if (!mask[v]) {
    L[v] = -1;
    return;
  }
  int64_t x, y, z;
  coords(d, v, x, y, z);
  Stencil s(d, x, y, z);
  int64_t best = v;
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    if (s.ok[k] && mask[v + s.off[k]]) {
      best = v + s.off[k];
      break;
    }
  }
  L[v] = best;
}

// One in-place jumping round; negative entries are not part of the forest.
__global__ void __launch_bounds__(kBlock)
k_jump64(int64_t *L, int64_t n, unsigned long long *ctr) {
  int64_t v = gid();
  bool changed = false;
  if (v < n) {
    int64_t u = L[v];
    if (u >= 0 && u != v) {
      int64_t w = __atomic_load_n(&L[u], __ATOMIC_RELAXED);
      if (w != u) {
        L[v] = w;
        changed = true;
      }
    }
  }
  flag_any(changed, ctr + kCtrChanged);
}

// Synchronous doubling: out[v] = in[in[v]].
__global__ void __launch_bounds__(kBlock)
k_double64(const int64_t *__restrict__ in, int64_t *__restrict__ out,
           int64_t n, unsigned long long *ctr) {
  int64_t v = gid();
  bool changed = false;
  if (v < n) {
    int64_t u = in[v];
    int64_t w = in[u];
    out[v] = w;
    changed = w != u;
  }
  flag_any(changed, ctr + kCtrChanged);
}

// Hook: the root of v's tree takes the smallest label among v's masked
// neighbours when that label is smaller than its own.
__global__ void __launch_bounds__(kBlock)
k_cc_hook(const uint8_t *__restrict__ mask, GridDims d, int64_t *L,
          unsigned long long *ctr) {
  int64_t v = gid();
  bool changed = false;
  if (v < d.N && mask[v]) {
    int64_t x, y, z;
    coords(d, v, x, y, z);
    Stencil s(d, x, y, z);
    int64_t lv = __atomic_load_n(&L[v], __ATOMIC_RELAXED);
    int64_t m = lv;
#pragma unroll
    for (int k = 0; k < 15; ++k) {
      if (k == 7 || !s.ok[k]) continue;
      int64_t u = v + s.off[k];
      if (!mask[u]) continue;
      int64_t lu = __atomic_load_n(&L[u], __ATOMIC_RELAXED);
      m = lu < m ? lu : m;
    }
    if (m < lv) {
      unsigned long long old = atomicMin((unsigned long long *)&L[lv],
                                         (unsigned long long)m);
      changed = (int64_t)old > m;
    }
  }
  flag_any(changed, ctr + kCtrChanged);
}

__global__ void __launch_bounds__(kBlock)
k_csr_init(int64_t n, const int64_t *__restrict__ rp,
           const int32_t *__restrict__ ci, const uint8_t *__restrict__ mask,
           int64_t *__restrict__ L, unsigned long long *ctr) {
  int64_t v = gid();
  bool bad = false;
  if (v < n) {
    if (mask && !mask[v]) {
      L[v] = -1;
    } else {
      int64_t best = v;
      for (int64_t e = rp[v], end = rp[v + 1]; e < end; ++e) {
        int64_t u = ci[e];
        if (u < 0 || u >= n) {
          bad = true;
          continue;
        }
        if (mask && !mask[u]) continue;
        best = u < best ? u : best;
      }
      L[v] = best;
    }
  }
  flag_any(bad, ctr + kCtrBadIndex);
}

// Hook over CSR rows in both directions of every listed edge, so a one-sided
// listing still joins its endpoints.
__global__ void __launch_bounds__(kBlock)
k_csr_hook(int64_t n, const int64_t *__restrict__ rp,
           const int32_t *__restrict__ ci, const uint8_t *__restrict__ mask,
           int64_t *L, unsigned long long *ctr) {
  int64_t v = gid();
  bool changed = false;
  if (v < n && (!mask || mask[v])) {
    int64_t lv = __atomic_load_n(&L[v], __ATOMIC_RELAXED);
    int64_t m = lv;
    for (int64_t e = rp[v], end = rp[v + 1]; e < end; ++e) {
      int64_t u = ci[e];
      if (u < 0 || u >= n) continue;
      if (mask && !mask[u]) continue;
      int64_t lu = __atomic_load_n(&L[u], __ATOMIC_RELAXED);
      if (lu < m) m = lu;
      if (lu > lv) {
        unsigned long long old = atomicMin((unsigned long long *)&L[lu],
                                           (unsigned long long)lv);
        changed |= (int64_t)old > lv;
      }
    }
    if (m < lv) {
      unsigned long long old = atomicMin((unsigned long long *)&L[lv],
                                         (unsigned long long)m);
      changed |= (int64_t)old > m;
    }
  }
  flag_any(changed, ctr + kCtrChanged);
}

int clear_changed(msc_ctx *ctx, hipStream_t s) {
  MSC_HIP_TRY(hipMemsetAsync(ctx->dctr + kCtrChanged, 0,
                             sizeof(unsigned long long), s));
  return MSC_OK;
}

// In-place doubling needs at most about log2(longest path) + 1 rounds; more
// than this many means the pointers hold a cycle (not a forest).
constexpr int kMaxRounds = 96;

// Jump in place until no pointer moves; returns rounds through *rounds.
int compress(msc_ctx *ctx, int64_t *L, int64_t n, hipStream_t s, int *rounds) {
  for (int r = 0;; ++r) {
    if (r == kMaxRounds) return MSC_EINVAL;
    MSC_TRY(clear_changed(ctx, s));
    MSC_PHASE(ctx, s, "cc_jump_round", 24.0 * n,
              (k_jump64<<<grid_for(n), kBlock, 0, s>>>(L, n, ctx->dctr)));
    if (rounds) ++*rounds;
    MSC_TRY(read_counters(ctx, s));
    if (!ctx->hctr[kCtrChanged]) return MSC_OK;
  }
}

}  // namespace

int cc_grid_run(msc_ctx *ctx, const uint8_t *mask, int64_t X, int64_t Y,
                int64_t Z, int64_t *labels, hipStream_t s) {
  GridDims d{X, Y, Z, X * Y, X * Y * Z};
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "cc_init", 9.0 * d.N,
            (k_cc_init<<<grid_for(d.N), kBlock, 0, s>>>(mask, d, labels)));
  int rounds = 0, hooks = 0;
  MSC_TRY(compress(ctx, labels, d.N, s, &rounds));
  for (;;) {
    MSC_TRY(clear_changed(ctx, s));
    MSC_PHASE(ctx, s, "cc_hook", 9.0 * d.N,
              (k_cc_hook<<<grid_for(d.N), kBlock, 0, s>>>(mask, d, labels,
                                                          ctx->dctr)));
    MSC_TRY(read_counters(ctx, s));
    if (!ctx->hctr[kCtrChanged]) break;
    ++hooks;
    MSC_TRY(compress(ctx, labels, d.N, s, &rounds));
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = d.N;
  ctx->stats.jump_rounds = rounds;
  ctx->stats.n_exits = hooks;
  return MSC_OK;
}

int cc_csr_run(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
               const int32_t *col_idx, const uint8_t *mask, int64_t *labels,
               hipStream_t s) {
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "csr_init", 17.0 * n,
            (k_csr_init<<<grid_for(n), kBlock, 0, s>>>(n, row_ptr, col_idx,
                                                       mask, labels,
                                                       ctx->dctr)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrBadIndex]) return MSC_EINVAL;
  int rounds = 0, hooks = 0;
  MSC_TRY(compress(ctx, labels, n, s, &rounds));
  for (;;) {
    MSC_TRY(clear_changed(ctx, s));
    MSC_PHASE(ctx, s, "csr_hook", 17.0 * n,
              (k_csr_hook<<<grid_for(n), kBlock, 0, s>>>(n, row_ptr, col_idx,
                                                         mask, labels,
                                                         ctx->dctr)));
    MSC_TRY(read_counters(ctx, s));
    if (!ctx->hctr[kCtrChanged]) break;
    ++hooks;
    MSC_TRY(compress(ctx, labels, n, s, &rounds));
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  ctx->stats.jump_rounds = rounds;
  ctx->stats.n_exits = hooks;
  return MSC_OK;
}

int jump_run(msc_ctx *ctx, int64_t *d, int64_t n, int rounds, int sync,
             hipStream_t s) {
  MSC_TRY(clear_counters(ctx, s));
  if (!sync) {
    if (rounds == 0) return compress(ctx, d, n, s, nullptr);
    for (int r = 0; r < rounds; ++r) {
      MSC_PHASE(ctx, s, "jump64_round", 24.0 * n,
                (k_jump64<<<grid_for(n), kBlock, 0, s>>>(d, n, ctx->dctr)));
    }
    return MSC_OK;
  }
  MSC_TRY(reserve(ctx->ws, align256(n * sizeof(int64_t)) + 4096));
  Carver cv(ctx->ws);
  int64_t *tmp = cv.take<int64_t>(n);
  int64_t *src = d, *dst = tmp;
  for (int r = 0; rounds == 0 || r < rounds; ++r) {
    if (rounds == 0 && r == kMaxRounds) return MSC_EINVAL;
    MSC_TRY(clear_changed(ctx, s));
    MSC_PHASE(ctx, s, "double64_round", 24.0 * n,
              (k_double64<<<grid_for(n), kBlock, 0, s>>>(src, dst, n,
                                                         ctx->dctr)));
    int64_t *t = src;
    src = dst;
    dst = t;
    if (rounds == 0) {
      MSC_TRY(read_counters(ctx, s));
      if (!ctx->hctr[kCtrChanged]) break;
    }
  }
  if (src != d)
    MSC_HIP_TRY(hipMemcpyAsync(d, src, n * sizeof(int64_t),
                               hipMemcpyDeviceToDevice, s));
  return MSC_OK;
}

}  // namespace msc
