// Morse-Smale segmentation kernels (gfx950).
//
// arXiv 2409.03771, Alg. 1 and methods "Ascending and Descending
// Segmentation": every vertex points to the (value,id)-largest vertex of its
// closed neighbourhood, pointer jumping compresses every path onto its
// maximum, the same runs downwards, and vertices with the same pair of
// extrema form one Morse-Smale cell.
//
// The paper splits the domain over ranks, compresses each rank's part with
// ghost vertices treated as maxima (Alg. 1), then resolves the pointers that
// leave a rank in one exchange step (Alg. 2).  Here the same two levels map
// onto the GPU's memory hierarchy:
//
//   tile_local   one workgroup per 32x8x8 tile: the field plus a one-vertex
//                halo is staged in LDS, both steepest pointers are computed
//                from LDS, halo vertices point to themselves (the ghost
//                rule), and pointer jumping runs in LDS until every owned
//                vertex points to a tile-local extremum or to a halo vertex
//                ("exit").  Writes one 16-bit tile-local pointer per vertex
//                and direction, and appends the distinct exits to a list.
//   exit_init    each exit gets its own tile's pointer as a global id.
//   exit_jump    in-place pointer jumping over the exit list only (the
//                paper's compression of the ghost graph after the exchange).
//   tile_pairs   decode every vertex's final extrema (local root or resolved
//                exit) and insert its (asc, desc) pair into a hash table
//                that keeps the smallest vertex id; per-tile LDS table first.
//   tile_write   decode again, write asc, desc and the cell id (table
//                lookup) per vertex (the paper's relabelling pass, Alg. 2).
#include <climits>

#include "msc_internal.hpp"

namespace msc {
namespace {

constexpr int TX = 32, TY = 8, TZ = 8;   // owned tile; one thread per column
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HXY = HX * HY;
constexpr int H = HX * HY * HZ;          // tile plus halo, in LDS
constexpr int kThreads = TX * TY;
constexpr int kPairSlots = 1024;         // per-tile LDS pair table
static_assert(H < 32768, "tile-local pointers are 16-bit");
static_assert(kThreads == kBlock, "one thread per tile column");

constexpr unsigned long long kEmptyKey = ~0ull;
constexpr uint32_t kTagDesc = 0x80000000u;

struct Geo {
  uint32_t X, Y, Z, XY, N;
  uint32_t ntx, nty, ntz, ntiles;
};

// Spread consecutive tiles over one XCD: the hardware hands workgroups to
// the 8 XCDs round-robin, so workgroup b runs on XCD b % 8; giving each XCD
// a contiguous range of tiles keeps halo rows shared by neighbouring tiles in
// the same L2.
__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / 8, rem = nb % 8, xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx
                   : rem * (per + 1) + (xcd - rem) * per + idx;
}

struct Tile {
  int x0, y0, z0;
};

__device__ __forceinline__ Tile tile_at(const Geo &g, uint32_t t) {
  uint32_t tx = t % g.ntx, r = t / g.ntx;
  uint32_t ty = r % g.nty, tz = r / g.nty;
  return Tile{(int)tx * TX, (int)ty * TY, (int)tz * TZ};
}

__device__ __forceinline__ bool halo_owned(int p) {
  int hz = p / HXY, r = p - hz * HXY, hy = r / HX, hx = r - hy * HX;
  return hx >= 1 && hx <= TX && hy >= 1 && hy <= TY && hz >= 1 && hz <= TZ;
}

// Global id of tile-local index p; p must lie inside the domain.
__device__ __forceinline__ uint32_t halo_global(const Geo &g, const Tile &t,
                                                int p) {
  int hz = p / HXY, r = p - hz * HXY, hy = r / HX, hx = r - hy * HX;
  return (uint32_t)(t.x0 - 1 + hx) + g.X * (uint32_t)(t.y0 - 1 + hy) +
         g.XY * (uint32_t)(t.z0 - 1 + hz);
}

__device__ __forceinline__ void wave_count(bool pred, unsigned long long *ctr) {
  unsigned long long m = __ballot(pred);
  if (m && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1))
    atomicAdd(ctr, (unsigned long long)__popcll(m));
}

__device__ __forceinline__ uint64_t mix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

// ---------------------------------------------------------------------------
// tile_local
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kThreads)
k_tile_local(const float *__restrict__ f, Geo g, int16_t *__restrict__ la,
             int16_t *__restrict__ ld, uint32_t *__restrict__ exits,
             uint32_t exit_cap, unsigned long long *ctr) {
  __shared__ float sf[H];
  __shared__ int16_t pa[H], pd[H];
  __shared__ uint8_t ea[H], ed[H];
  __shared__ unsigned s_cnt, s_cur;
  __shared__ unsigned long long s_base;

  const int tid = threadIdx.x;
  const Tile t = tile_at(g, tile_of_block(blockIdx.x, gridDim.x));
  if (tid == 0) {
    s_cnt = 0;
    s_cur = 0;
  }

  // Stage the tile and its halo; positions outside the domain hold NaN,
  // which loses every comparison below and so is never chosen.
  for (int i = tid; i < H; i += kThreads) {
    int hz = i / HXY, r = i - hz * HXY, hy = r / HX, hx = r - hy * HX;
    int gx = t.x0 - 1 + hx, gy = t.y0 - 1 + hy, gz = t.z0 - 1 + hz;
    bool in = gx >= 0 && gx < (int)g.X && gy >= 0 && gy < (int)g.Y &&
              gz >= 0 && gz < (int)g.Z;
    sf[i] = in ? f[(uint32_t)gx + g.X * (uint32_t)gy + g.XY * (uint32_t)gz]
               : __builtin_nanf("");
    pa[i] = (int16_t)i;   // halo vertices point to themselves
    pd[i] = (int16_t)i;
    ea[i] = 0;
    ed[i] = 0;
  }
  __syncthreads();

  const int cx = tid % TX, cy = tid / TX;
  const int gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < (int)g.X && gy < (int)g.Y;
  int nz = (int)g.Z - t.z0;
  nz = col_in ? (nz < TZ ? nz : TZ) : 0;
  const int i0 = (cx + 1) + HX * (cy + 1) + HXY;

  // Steepest ascent / descent over the closed neighbourhood, ordered by
  // (value, id).  Starting from v itself, a lower-id neighbour must be
  // strictly above to win the max and at most equal to win the min; a
  // higher-id neighbour wins the max when at least equal and the min when
  // strictly below.
  // Neighbour offsets in the LDS tile: the 7 lower-id neighbours in
  // decreasing id order and the 7 higher-id neighbours in increasing order.
  const int kLo[7] = {-1,   -HX,      -HX - 1,  -HXY,
                      -HXY - 1, -HXY - HX, -HXY - HX - 1};
  const int kHi[7] = {1, HX, HX + 1, HXY, HXY + 1, HXY + HX, HXY + HX + 1};
  bool any_nan = false;
  for (int lz = 0; lz < TZ; ++lz) {
    bool in = lz < nz;
    bool ismax = false, ismin = false;
    if (in) {
      const int i = i0 + lz * HXY;
      const float fv = sf[i];
      any_nan |= fv != fv;
      float bmax = fv, bmin = fv;
      int omax = 0, omin = 0;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const float fu = sf[i + kLo[k]];
        if (fu > bmax) { bmax = fu; omax = kLo[k]; }
        if (fu <= bmin) { bmin = fu; omin = kLo[k]; }
      }
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const float fu = sf[i + kHi[k]];
        if (fu >= bmax) { bmax = fu; omax = kHi[k]; }
        if (fu < bmin) { bmin = fu; omin = kHi[k]; }
      }
      pa[i] = (int16_t)(i + omax);
      pd[i] = (int16_t)(i + omin);
      ismax = omax == 0;
      ismin = omin == 0;
    }
    wave_count(ismax, ctr + kCtrMaxima);
    wave_count(ismin, ctr + kCtrMinima);
  }
  wave_count(any_nan, ctr + kCtrNaN);
  __syncthreads();

  // Pointer jumping inside the tile, in place.
  for (;;) {
    bool changed = false;
    for (int lz = 0; lz < nz; ++lz) {
      const int i = i0 + lz * HXY;
      int p = pa[i], q = pa[p];
      if (q != p) { pa[i] = (int16_t)q; changed = true; }
      p = pd[i];
      q = pd[p];
      if (q != p) { pd[i] = (int16_t)q; changed = true; }
    }
    if (!__syncthreads_or(changed)) break;
  }

  // Tile-local results; mark the halo vertices that are pointed to.
  for (int lz = 0; lz < nz; ++lz) {
    const int i = i0 + lz * HXY;
    const uint32_t v = (uint32_t)gx + g.X * (uint32_t)gy +
                       g.XY * (uint32_t)(t.z0 + lz);
    const int p = pa[i], q = pd[i];
    la[v] = (int16_t)p;
    ld[v] = (int16_t)q;
    if (!halo_owned(p)) ea[p] = 1;
    if (!halo_owned(q)) ed[q] = 1;
  }
  __syncthreads();

  // Append the marked halo vertices to the exit list (one global atomic per
  // tile).
  unsigned mine = 0;
  for (int i = tid; i < H; i += kThreads) mine += ea[i] + ed[i];
  if (mine) atomicAdd(&s_cnt, mine);
  __syncthreads();
  if (tid == 0 && s_cnt)
    s_base = atomicAdd(ctr + kCtrExits, (unsigned long long)s_cnt);
  __syncthreads();
  if (mine) {
    for (int i = tid; i < H; i += kThreads) {
      if (!(ea[i] | ed[i])) continue;
      const uint32_t gid = halo_global(g, t, i);
      if (ea[i]) {
        unsigned long long pos = s_base + atomicAdd(&s_cur, 1u);
        if (pos < exit_cap) exits[pos] = gid;
      }
      if (ed[i]) {
        unsigned long long pos = s_base + atomicAdd(&s_cur, 1u);
        if (pos < exit_cap) exits[pos] = gid | kTagDesc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// exit graph
// ---------------------------------------------------------------------------

__device__ __forceinline__ Tile tile_of_vertex(const Geo &g, uint32_t v) {
  uint32_t z = v / g.XY, r = v - z * g.XY, y = r / g.X, x = r - y * g.X;
  return Tile{(int)(x - x % TX), (int)(y - y % TY), (int)(z - z % TZ)};
}

// Each exit takes its own tile's pointer as a global id; a pointer to a
// tile-local root makes that root point to itself in the same array.
__global__ void __launch_bounds__(kBlock)
k_exit_init(const uint32_t *__restrict__ exits, uint32_t count, Geo g,
            const int16_t *__restrict__ la, const int16_t *__restrict__ ld,
            int32_t *A, int32_t *D) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const uint32_t e = exits[i];
  const bool desc = e & kTagDesc;
  const uint32_t v = e & ~kTagDesc;
  const int p = desc ? ld[v] : la[v];
  const uint32_t target = halo_global(g, tile_of_vertex(g, v), p);
  int32_t *arr = desc ? D : A;
  arr[v] = (int32_t)target;
  if (halo_owned(p)) arr[target] = (int32_t)target;
}

// In-place jumping over the exit list: every entry follows its chain to a
// fixed point; entries read by others only ever move further along their
// path, so any interleaving ends at the same extremum.
__global__ void __launch_bounds__(kBlock)
k_exit_jump(const uint32_t *__restrict__ exits, uint32_t count, uint32_t n,
            int32_t *A, int32_t *D, unsigned long long *ctr) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  unsigned steps = 0;
  bool bad = false;
  if (i < count) {
    const uint32_t e = exits[i];
    int32_t *arr = (e & kTagDesc) ? D : A;
    const uint32_t v = e & ~kTagDesc;
    // Every pointer is a vertex id and a chain is at most n long; the checks
    // only turn a broken invariant into an error instead of a bad access.
    for (; steps <= n; ++steps) {
      int32_t u = __atomic_load_n(&arr[v], __ATOMIC_RELAXED);
      if ((uint32_t)u >= n) { bad = true; break; }
      int32_t w = __atomic_load_n(&arr[u], __ATOMIC_RELAXED);
      if ((uint32_t)w >= n) { bad = true; break; }
      if (w == u) break;
      __atomic_store_n(&arr[v], w, __ATOMIC_RELAXED);
    }
    if (steps > n) bad = true;
  }
  if (bad) atomicOr(ctr + kCtrOverflow, 2ull);
  // Longest chain seen (reported as the jump-round count).
  for (int o = 32; o > 0; o >>= 1) {
    unsigned other = __shfl_xor(steps, o);
    steps = other > steps ? other : steps;
  }
  if ((threadIdx.x & 63) == 0 && steps)
    atomicMax(ctr + kCtrRounds, (unsigned long long)steps);
}

// ---------------------------------------------------------------------------
// pairs and output
// ---------------------------------------------------------------------------

// Final extremum of a vertex from its tile-local pointer p: a local root is
// final; otherwise p is an exit whose resolved value sits in arr.
__device__ __forceinline__ int32_t final_of(const Geo &g, const Tile &t, int p,
                                            const int32_t *arr) {
  const uint32_t target = halo_global(g, t, p);
  if (halo_owned(p)) return (int32_t)target;
  return __atomic_load_n(&arr[target], __ATOMIC_RELAXED);
}

__global__ void k_table_clear(unsigned long long *keys, int32_t *vals,
                              uint32_t cap) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < cap) {
    keys[i] = kEmptyKey;
    vals[i] = INT32_MAX;
  }
}

// Insert (key, id) keeping the smallest id; reads before each atomic so that
// the common case (key present with a smaller id) stays a plain load.
__device__ __forceinline__ bool table_insert(unsigned long long *keys,
                                             int32_t *vals, uint32_t mask,
                                             unsigned long long key,
                                             int32_t id, unsigned *fresh) {
  uint32_t h = (uint32_t)mix64(key) & mask;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    unsigned long long cur = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
    if (cur == kEmptyKey) {
      cur = atomicCAS(&keys[h], kEmptyKey, key);
      if (cur == kEmptyKey) {
        ++*fresh;
        cur = key;
      }
    }
    if (cur == key) {
      if (__atomic_load_n(&vals[h], __ATOMIC_RELAXED) > id)
        atomicMin(&vals[h], id);
      return true;
    }
    h = (h + 1) & mask;
  }
  return false;
}

__device__ __forceinline__ unsigned long long pair_key(int32_t a, int32_t d) {
  return ((unsigned long long)(uint32_t)a << 32) | (uint32_t)d;
}

__device__ __forceinline__ unsigned long long wave_bcast64(
    unsigned long long x, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, lane);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), lane);
  return ((unsigned long long)hi << 32) | lo;
}

__global__ void __launch_bounds__(kThreads)
k_tile_pairs(Geo g, const int16_t *__restrict__ la,
             const int16_t *__restrict__ ld, const int32_t *A,
             const int32_t *D, unsigned long long *keys, int32_t *vals,
             uint32_t mask, unsigned long long *ctr) {
  __shared__ unsigned long long skey[kPairSlots];
  __shared__ int32_t sval[kPairSlots];
  const int tid = threadIdx.x, lane = tid & 63;
  const Tile t = tile_at(g, tile_of_block(blockIdx.x, gridDim.x));
  for (int i = tid; i < kPairSlots; i += kThreads) {
    skey[i] = kEmptyKey;
    sval[i] = INT32_MAX;
  }
  __syncthreads();

  const int cx = tid % TX, cy = tid / TX;
  const int gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < (int)g.X && gy < (int)g.Y;
  unsigned fresh = 0;
  bool overflow = false;
  for (int lz = 0; lz < TZ; ++lz) {
    const bool in = col_in && t.z0 + lz < (int)g.Z;
    unsigned long long key = 0;
    int32_t id = 0;
    if (in) {
      const uint32_t v = (uint32_t)gx + g.X * (uint32_t)gy +
                         g.XY * (uint32_t)(t.z0 + lz);
      key = pair_key(final_of(g, t, la[v], A), final_of(g, t, ld[v], D));
      id = (int32_t)v;
    }
    // Lanes holding the same pair are merged: the lowest lane holds the
    // smallest id of them (ids grow with the lane inside a row, and the
    // second row of a wave has larger ids than the first).
    bool pending = in;
    for (;;) {
      unsigned long long m = __ballot(pending);
      if (!m) break;
      const int leader = __ffsll((long long)m) - 1;
      const unsigned long long lkey = wave_bcast64(key, leader);
      if (lane == leader) {
        uint32_t h = (uint32_t)mix64(lkey) & (kPairSlots - 1);
        bool done = false;
        for (int probe = 0; probe < 32 && !done; ++probe) {
          unsigned long long cur = skey[h];
          if (cur == kEmptyKey) cur = atomicCAS(&skey[h], kEmptyKey, lkey);
          if (cur == kEmptyKey || cur == lkey) {
            atomicMin(&sval[h], id);
            done = true;
          }
          h = (h + 1) & (kPairSlots - 1);
        }
        if (!done && !table_insert(keys, vals, mask, lkey, id, &fresh))
          overflow = true;
      }
      if (pending && key == lkey) pending = false;
    }
  }
  __syncthreads();
  for (int i = tid; i < kPairSlots; i += kThreads) {
    if (skey[i] != kEmptyKey &&
        !table_insert(keys, vals, mask, skey[i], sval[i], &fresh))
      overflow = true;
  }
  if (fresh) atomicAdd(ctr + kCtrCells, (unsigned long long)fresh);
  if (overflow) atomicOr(ctr + kCtrOverflow, 1ull);
}

__global__ void __launch_bounds__(kThreads)
k_tile_write(Geo g, const int16_t *__restrict__ la,
             const int16_t *__restrict__ ld, int32_t *A, int32_t *D,
             const unsigned long long *__restrict__ keys,
             const int32_t *__restrict__ vals, uint32_t mask,
             int32_t *__restrict__ ms) {
  const int tid = threadIdx.x, lane = tid & 63;
  const Tile t = tile_at(g, tile_of_block(blockIdx.x, gridDim.x));
  const int cx = tid % TX, cy = tid / TX;
  const int gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < (int)g.X && gy < (int)g.Y;
  for (int lz = 0; lz < TZ; ++lz) {
    const bool in = col_in && t.z0 + lz < (int)g.Z;
    uint32_t v = 0;
    int32_t a = 0, d = 0;
    if (in) {
      v = (uint32_t)gx + g.X * (uint32_t)gy + g.XY * (uint32_t)(t.z0 + lz);
      a = final_of(g, t, la[v], A);
      d = final_of(g, t, ld[v], D);
    }
    if (ms) {
      const unsigned long long key = pair_key(a, d);
      int32_t cell = -1;
      bool pending = in;
      for (;;) {
        unsigned long long m = __ballot(pending);
        if (!m) break;
        const int leader = __ffsll((long long)m) - 1;
        const unsigned long long lkey = wave_bcast64(key, leader);
        int32_t found = -1;
        if (lane == leader) {
          uint32_t h = (uint32_t)mix64(lkey) & mask;
          for (uint32_t probe = 0; probe <= mask; ++probe) {
            const unsigned long long cur = keys[h];
            if (cur == lkey) { found = vals[h]; break; }
            if (cur == kEmptyKey) break;
            h = (h + 1) & mask;
          }
        }
        found = __builtin_amdgcn_readlane(found, leader);
        if (pending && key == lkey) {
          cell = found;
          pending = false;
        }
      }
      if (in) ms[v] = cell;
    }
    if (in) {
      // Same value an exit already holds, so concurrent readers of A/D see a
      // final value either way.
      __atomic_store_n(&A[v], a, __ATOMIC_RELAXED);
      __atomic_store_n(&D[v], d, __ATOMIC_RELAXED);
    }
  }
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
  Geo g{};
  g.X = (uint32_t)X;
  g.Y = (uint32_t)Y;
  g.Z = (uint32_t)Z;
  g.XY = (uint32_t)(X * Y);
  g.N = (uint32_t)n;
  g.ntx = (uint32_t)((X + TX - 1) / TX);
  g.nty = (uint32_t)((Y + TY - 1) / TY);
  g.ntz = (uint32_t)((Z + TZ - 1) / TZ);
  const int64_t ntiles = (int64_t)g.ntx * g.nty * g.ntz;
  if (ntiles > INT32_MAX) return MSC_ERANGE;
  g.ntiles = (uint32_t)ntiles;
  unsigned long long *ctr = ctx->dctr;

  // Workspace: 16-bit tile-local pointers, full-size arrays the caller did
  // not ask for, and the exit list (grown if a run overflows it).
  uint64_t exit_cap = ctx->exit_cap_hint;
  if (exit_cap < 4096) exit_cap = 4096;
  if (exit_cap < (uint64_t)n / 16) exit_cap = (uint64_t)n / 16;
  if (exit_cap > UINT32_MAX) exit_cap = UINT32_MAX;
  uint64_t exits = 0;
  int16_t *la = nullptr, *ld = nullptr;
  int32_t *A = asc, *D = desc;
  uint32_t *list = nullptr;
  for (int attempt = 0;; ++attempt) {
    size_t need = 2 * align256(n * sizeof(int16_t)) +
                  align256(exit_cap * sizeof(uint32_t)) + 4096;
    if (!asc) need += align256(n * sizeof(int32_t));
    if (!desc) need += align256(n * sizeof(int32_t));
    MSC_TRY(reserve(ctx->ws, need));
    Carver cv(ctx->ws);
    la = cv.take<int16_t>(n);
    ld = cv.take<int16_t>(n);
    list = cv.take<uint32_t>(exit_cap);
    A = asc ? asc : cv.take<int32_t>(n);
    D = desc ? desc : cv.take<int32_t>(n);

    MSC_TRY(clear_counters(ctx, s));
    MSC_PHASE(ctx, s, "tile_local", 8.0 * n,
              (k_tile_local<<<g.ntiles, kThreads, 0, s>>>(
                  f, g, la, ld, list, (uint32_t)exit_cap, ctr)));
    MSC_TRY(read_counters(ctx, s));
    if (ctx->hctr[kCtrNaN]) return MSC_ENAN;
    exits = ctx->hctr[kCtrExits];
    if (exits <= exit_cap) break;
    if (attempt > 0 || exits > UINT32_MAX) return MSC_ENOMEM;
    exit_cap = exits + exits / 4;
  }
  ctx->exit_cap_hint = exit_cap;
  const uint64_t nmax = ctx->hctr[kCtrMaxima], nmin = ctx->hctr[kCtrMinima];

  if (exits) {
    const uint32_t ne = (uint32_t)exits;
    MSC_PHASE(ctx, s, "exit_init", 14.0 * ne,
              (k_exit_init<<<grid_for(ne), kBlock, 0, s>>>(list, ne, g, la, ld,
                                                           A, D)));
    MSC_PHASE(ctx, s, "exit_jump", 12.0 * ne,
              (k_exit_jump<<<grid_for(ne), kBlock, 0, s>>>(list, ne, g.N, A,
                                                           D, ctr)));
  }

  unsigned long long *keys = nullptr;
  int32_t *vals = nullptr;
  uint32_t cap = 0;
  if (ms) {
    cap = table_capacity(n, nmax, nmin);
    size_t tbytes = align256((size_t)cap * 8) + align256((size_t)cap * 4);
    MSC_TRY(reserve(ctx->tab, tbytes + 4096));
    Carver tc(ctx->tab);
    keys = tc.take<unsigned long long>(cap);
    vals = tc.take<int32_t>(cap);
    MSC_PHASE(ctx, s, "table_clear", 12.0 * cap,
              (k_table_clear<<<grid_for(cap), kBlock, 0, s>>>(keys, vals,
                                                              cap)));
    MSC_PHASE(ctx, s, "tile_pairs", 4.0 * n,
              (k_tile_pairs<<<g.ntiles, kThreads, 0, s>>>(
                  g, la, ld, A, D, keys, vals, cap - 1, ctr)));
  }
  MSC_PHASE(ctx, s, "tile_write", (ms ? 16.0 : 12.0) * n,
            (k_tile_write<<<g.ntiles, kThreads, 0, s>>>(
                g, la, ld, A, D, keys, vals, cap ? cap - 1 : 0, ms)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrOverflow] & 2) return MSC_EHIP;
  if (ctx->hctr[kCtrOverflow]) return MSC_ENOMEM;

  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  ctx->stats.n_maxima = (int64_t)nmax;
  ctx->stats.n_minima = (int64_t)nmin;
  ctx->stats.n_cells = ms ? (int64_t)ctx->hctr[kCtrCells] : -1;
  ctx->stats.n_exits = (int64_t)exits;
  ctx->stats.jump_rounds = (int32_t)ctx->hctr[kCtrRounds];
  ctx->stats.tile_x = TX;
  ctx->stats.tile_y = TY;
  ctx->stats.tile_z = TZ;
  return MSC_OK;
}

}  // namespace msc
