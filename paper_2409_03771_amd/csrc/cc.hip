// Connected components (gfx950) and the pointer-forest compression entry.
//
// arXiv 2409.03771, Alg. 3 and methods "Connected Components": masked
// vertices point to a masked neighbour chosen by id, path compression turns
// the pointers into per-component labels, and a stitching step merges the
// partial trees that touch before a last compression.  Every pointer here
// goes to a smaller (or equal) id, so a component ends up named by its
// smallest id.  The paper's single racy stitch does not join every pair of
// touching trees in general; here trees are joined with a lock-free union
// (compare-and-swap of the larger root onto the smaller one, retried until
// it sticks), whose result is the min-id labelling whatever the schedule.
//
// Grid masks use the same two levels as the segmentation, mirroring the
// paper's rank-local pass plus exchange:
//   cc_tile    one workgroup per tile: union-find over the tile's own edges
//              in LDS; writes each vertex's tile-local root (16-bit) and
//              makes every tile-local root its own parent in the global
//              label array;
//   cc_cross   unions across the tile faces (each cross-tile edge once, from
//              the tile holding its lower endpoint) on the global array,
//              touching tile-local roots only (the paper's ghost exchange);
//   cc_final   label = root of the vertex's tile-local root.
// CSR graphs have no locality to exploit: init to the smallest masked
// neighbour, one union per listed edge, then a final find per vertex.
#include <climits>
#include <mutex>

#include "msc_internal.hpp"

namespace msc {
namespace {

__device__ __forceinline__ int64_t gid() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

__device__ __forceinline__ void flag_any(bool pred, unsigned long long *ctr) {
  if (__ballot(pred) && (threadIdx.x & 63) == 0) atomicOr(ctr, 1ull);
}

// ---------------------------------------------------------------------------
// Lock-free union-find on a parent array whose pointers only decrease.
// ---------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T uf_find(T *par, T x) {
  for (;;) {
    T p = __atomic_load_n(&par[x], __ATOMIC_RELAXED);
    if (p == x) return x;
    T g = __atomic_load_n(&par[p], __ATOMIC_RELAXED);
    if (g == p) return p;
    // Path halving: g is an ancestor of x, so this only shortens the path.
    __atomic_store_n(&par[x], g, __ATOMIC_RELAXED);
    x = g;
  }
}

// Root of x without writing: used once no union is running, by the passes
// in which every entry is also an output that only its owner may write.
// The loads are cached (workgroup scope): a value older than another
// workgroup's write is still an ancestor on the path to the same root.
template <class T>
__device__ __forceinline__ T uf_root(const T *par, T x) {
  for (;;) {
    T p = __hip_atomic_load(&par[x], __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    x = p;
  }
}

// Join the trees of a and b: the larger root is hung under the smaller one.
template <class T>
__device__ __forceinline__ bool uf_unite(T *par, T a, T b) {
  bool changed = false;
  for (;;) {
    a = uf_find(par, a);
    b = uf_find(par, b);
    if (a == b) return changed;
    if (a > b) {
      T t = a;
      a = b;
      b = t;
    }
    T expect = b;
    if (__atomic_compare_exchange_n(&par[b], &expect, a, false,
                                    __ATOMIC_RELAXED, __ATOMIC_RELAXED))
      return true;
    changed = true;  // b moved meanwhile; retry from the new trees
  }
}

// The same on a forest in device memory, where every step of a walk is a
// round trip: the two walks of a union advance side by side (each step's
// loads for both are issued before either is used; a walk that has reached
// its root reloads it harmlessly), and the accesses are at device scope,
// which is all that one device's workgroups need.
__device__ __forceinline__ int64_t ld_dev(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void uf_find2_dev(int64_t *par, int64_t &a,
                                             int64_t &b) {
  bool ra = false, rb = false;
  while (!(ra && rb)) {
    const int64_t pa = ld_dev(&par[a]), pb = ld_dev(&par[b]);
    const int64_t ga = ld_dev(&par[pa]), gb = ld_dev(&par[pb]);
    if (!ra) {
      if (pa == a) {
        ra = true;
      } else if (ga == pa) {
        a = pa;
        ra = true;
      } else {
        // Path halving: ga is an ancestor of a, so this only shortens it.
        __hip_atomic_store(&par[a], ga, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        a = ga;
      }
    }
    if (!rb) {
      if (pb == b) {
        rb = true;
      } else if (gb == pb) {
        b = pb;
        rb = true;
      } else {
        __hip_atomic_store(&par[b], gb, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        b = gb;
      }
    }
  }
}

__device__ __forceinline__ bool uf_unite_dev(int64_t *par, int64_t a,
                                             int64_t b) {
  bool changed = false;
  for (;;) {
    uf_find2_dev(par, a, b);
    if (a == b) return changed;
    if (a > b) {
      const int64_t t = a;
      a = b;
      b = t;
    }
    int64_t expect = b;
    if (__hip_atomic_compare_exchange_strong(
            &par[b], &expect, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
            __HIP_MEMORY_SCOPE_AGENT))
      return true;
    changed = true;  // b moved meanwhile; retry from the new trees
  }
}

// ---------------------------------------------------------------------------
// Grid masks
// ---------------------------------------------------------------------------

constexpr int CTX = 32, CTY = 16, CTZ = 16;      // tile; one thread per column
constexpr int kCThreads = CTX * CTY;
constexpr int kCOwned = CTX * CTY * CTZ;
constexpr uint16_t kOutside = 0xffff;           // unmasked vertex
static_assert(kCOwned < 65535, "tile-local roots are 16-bit");

struct CGeo {
  int64_t X, Y, Z, XY, N;
  int64_t ntx, nty, ntz;
};

__device__ __forceinline__ uint32_t cc_tile_of_block(uint32_t b, uint32_t nb) {
  const uint32_t per = nb / 8, rem = nb % 8, xcd = b % 8, idx = b / 8;
  return xcd < rem ? xcd * (per + 1) + idx
                   : rem * (per + 1) + (xcd - rem) * per + idx;
}

struct CTile {
  int64_t x0, y0, z0;
};

__device__ __forceinline__ CTile ctile_at(const CGeo &g, int64_t t) {
  int64_t tx = t % g.ntx, r = t / g.ntx;
  int64_t ty = r % g.nty, tz = r / g.nty;
  return CTile{tx * CTX, ty * CTY, tz * CTZ};
}

// The tile-local roots are stored tile-major: tile t's kCOwned entries,
// indexed by the tile-local index, are one contiguous run, so the passes
// read and write whole runs instead of a row of CTX entries per (y, z).
__device__ __forceinline__ int64_t loc_index(int64_t t, int l) {
  return t * kCOwned + l;
}

// Global id of the tile-local index l (lx + CTX*(ly + CTY*lz)).
__device__ __forceinline__ int64_t ctile_global(const CGeo &g, const CTile &t,
                                                int l) {
  const int lz = l / (CTX * CTY), r = l - lz * (CTX * CTY);
  const int ly = r / CTX, lx = r - ly * CTX;
  return (t.x0 + lx) + g.X * (t.y0 + ly) + g.XY * (t.z0 + lz);
}

// One mask of a launch: its buffers, shape and first tile.  A launch covers
// the tiles of up to B masks (B = 1 for a single mask), passed by value.
struct CGrid {
  const uint8_t *mask;
  int64_t *L;      // labels, also the union-find parent array
  uint16_t *loc;   // tile-local roots (workspace), tile-major (loc_index)
  int64_t off;     // added to every label (a slab inside a larger grid)
  int64_t X, Y, Z;
  uint32_t tile0;  // first tile of this mask in the launch
};

template <int B>
struct CBatch {
  int n;
  CGrid g[B];
};

// The mask and geometry of launch tile `tt`, and the tile's index within it.
template <int B>
__device__ __forceinline__ const CGrid &cgrid_of(const CBatch<B> &b,
                                                 uint32_t tt, CGeo *g,
                                                 int64_t *t) {
  int lo = 0;
  if (B > 1) {
    int hi = b.n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (b.g[mid].tile0 <= tt) lo = mid;
      else hi = mid - 1;
    }
  }
  const CGrid &d = b.g[lo];
  const int64_t X = d.X, Y = d.Y, Z = d.Z;
  *g = CGeo{X, Y, Z, X * Y, X * Y * Z, (X + CTX - 1) / CTX,
            (Y + CTY - 1) / CTY, (Z + CTZ - 1) / CTZ};
  *t = (int64_t)(tt - d.tile0);
  return d;
}

// First z of the run of consecutive set bits of `bits` that contains bit z.
__device__ __forceinline__ int run_start(uint32_t bits, int z) {
  const uint32_t zeros = ~bits & ((1u << z) - 1u);
  return zeros ? 32 - __clz(zeros) : 0;
}

template <int B>
__global__ void __launch_bounds__(kCThreads) k_cc_tile(CBatch<B> b) {
  __shared__ int32_t par[kCOwned];
  __shared__ uint32_t cols[kCThreads];  // mask bits of every column
  const int tid = threadIdx.x;
  CGeo g;
  int64_t ti;
  const CGrid &d = cgrid_of(b, cc_tile_of_block(blockIdx.x, gridDim.x), &g,
                            &ti);
  const uint8_t *__restrict__ mask = d.mask;
  uint16_t *__restrict__ loc = d.loc;
  int64_t *__restrict__ L = d.L;
  const CTile t = ctile_at(g, ti);
  const int cx = tid % CTX, cy = tid / CTX;
  const int64_t gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < g.X && gy < g.Y;
  int nz = (int)((g.Z - t.z0) < CTZ ? (g.Z - t.z0) : CTZ);
  if (!col_in) nz = 0;
  const int64_t v0 = gx + g.X * gy + g.XY * t.z0;
  auto local = [](int x, int y, int z) { return x + CTX * (y + CTY * z); };

  // This column's mask bits.  The loads are unconditional, at addresses
  // kept inside the mask (a plane past the column, or a column past the
  // grid, reads a vertex that exists), so that all of them are in flight
  // together; the planes past the column are then dropped.
  uint32_t m = 0;
  {
    const int64_t vb = col_in ? v0 : 0;
    uint8_t mv[CTZ];
#pragma unroll
    for (int lz = 0; lz < CTZ; ++lz) mv[lz] = mask[vb + g.XY * (lz < nz ? lz : 0)];
#pragma unroll
    for (int lz = 0; lz < CTZ; ++lz) m |= (uint32_t)(lz < nz && mv[lz] != 0) << lz;
  }
  // The column's runs of consecutive masked z: every vertex of a run points
  // at the run's first vertex, which settles every -z edge of the tile.
#pragma unroll
  for (int lz = 0; lz < CTZ; ++lz)
    par[local(cx, cy, lz)] =
        ((m >> lz) & 1u) ? local(cx, cy, run_start(m, lz)) : -1;
  cols[tid] = m;
  __syncthreads();

  // The other lower-id Freudenthal edges of each masked vertex, united run
  // head to run head.  The -x and -y edges are always taken; a diagonal one
  // is implied, and skipped, when an axis neighbour on its side is in the
  // mask: e.g. with v-x in the mask, v-x-y is v-x's own -y neighbour, so
  // v ~ v-x ~ v-x-y (by induction on id, as v-x < v settles its own lower
  // edges the same way; v ~ v-z through their run).  A lane skips a union of
  // the same two heads as its previous one in that direction, so runs that
  // lie side by side are united once.
  const uint32_t mx_ = cx > 0 ? cols[tid - 1] : 0u;
  const uint32_t my_ = cy > 0 ? cols[tid - CTX] : 0u;
  const uint32_t mxy = cx > 0 && cy > 0 ? cols[tid - CTX - 1] : 0u;
  uint32_t last[6] = {~0u, ~0u, ~0u, ~0u, ~0u, ~0u};
  auto unite = [&](int dir, int hl, int hu) {
    const uint32_t key = (uint32_t)hl | ((uint32_t)hu << 13);
    if (key == last[dir]) return;
    last[dir] = key;
    uf_unite<int32_t>(par, hl, hu);
  };
#pragma unroll
  for (int lz = 0; lz < CTZ; ++lz) {
    if (!((m >> lz) & 1u)) continue;
    const int hl = local(cx, cy, run_start(m, lz));
    const bool mx = (mx_ >> lz) & 1u, my = (my_ >> lz) & 1u;
    const bool mz = lz > 0 && ((m >> (lz - 1)) & 1u);
    if (mx) unite(0, hl, local(cx - 1, cy, run_start(mx_, lz)));
    if (my) unite(1, hl, local(cx, cy - 1, run_start(my_, lz)));
    if (!mx && !my && ((mxy >> lz) & 1u))
      unite(2, hl, local(cx - 1, cy - 1, run_start(mxy, lz)));
    if (lz > 0 && !mz) {
      if (!mx && ((mx_ >> (lz - 1)) & 1u))
        unite(3, hl, local(cx - 1, cy, run_start(mx_, lz - 1)));
      if (!my && ((my_ >> (lz - 1)) & 1u))
        unite(4, hl, local(cx, cy - 1, run_start(my_, lz - 1)));
      if (!mx && !my && ((mxy >> (lz - 1)) & 1u))
        unite(5, hl, local(cx - 1, cy - 1, run_start(mxy, lz - 1)));
    }
  }
  __syncthreads();

  // Tile-local roots, once per run.
  int run_head = -1, run_root = -1;
  for (int lz = 0; lz < nz; ++lz) {
    const int64_t v = v0 + g.XY * lz;
    const int l = local(cx, cy, lz);
    if (!((m >> lz) & 1u)) {
      loc[loc_index(ti, l)] = kOutside;
      continue;
    }
    const int h = local(cx, cy, run_start(m, lz));
    if (h != run_head) {
      run_head = h;
      run_root = uf_find<int32_t>(par, h);
    }
    loc[loc_index(ti, l)] = (uint16_t)run_root;
    if (run_root == l) L[v] = v;  // tile-local roots start as global roots
  }
}

// Unions across tile faces.  An edge between two tiles is handled by the tile
// that owns its lower endpoint, which sees it as one of the 7 higher-id
// neighbours leaving the tile through an upper face.  Both endpoints are
// replaced by their tile-local roots, and each distinct (local root,
// neighbour tile, its local root) triple is united once, after the block has
// collected them: a face of a smooth mask carries thousands of edges but
// only a few such triples.
constexpr int kCrossSlots = 2048;
constexpr int kCrossProbes = 16;

constexpr uint32_t kNoKey = 0xffffffffu;

// Inserts key into the block's set; false only when the set has no room
// for it (the caller then unites the pair itself).
__device__ __forceinline__ bool cross_insert(uint32_t *set, uint32_t key) {
  uint32_t h = (key * 0x9e3779b1u) >> (32 - 11);
#pragma unroll 1
  for (int probe = 0; probe < kCrossProbes; ++probe) {
    uint32_t cur = set[h];
    if (cur == key) return true;
    if (cur == kNoKey) {
      cur = atomicCAS(&set[h], kNoKey, key);
      if (cur == kNoKey || cur == key) return true;
    }
    h = (h + 1) & (kCrossSlots - 1);
  }
  return false;
}

// The two global ids a key stands for: the local root lv of tile t and the
// local root lu of the neighbour tile (bit k of nbr: one tile up along axis k).
__device__ __forceinline__ void cross_unite(const CGeo &g, const CTile &t,
                                            uint32_t key, int64_t *L) {
  const uint32_t lv = key & 0x1fffu, nbr = (key >> 13) & 7u, lu = key >> 16;
  const CTile tu{t.x0 + (nbr & 1u ? CTX : 0), t.y0 + (nbr & 2u ? CTY : 0),
                 t.z0 + (nbr & 4u ? CTZ : 0)};
  uf_unite_dev(L, ctile_global(g, t, (int)lv),
                    ctile_global(g, tu, (int)lu));
}

template <int B>
__global__ void __launch_bounds__(kCThreads) k_cc_cross(CBatch<B> b) {
  static_assert(kCOwned <= (1 << 13), "13-bit local roots in the keys");
  // The tile grown by one vertex on its upper sides; only the two upper
  // layers of each side are read: the tile's upper faces and the vertices
  // just beyond them.  Entries hold tile-local roots (kOutside: unmasked or
  // outside the domain), decoded with their own tile's origin later.
  constexpr int BX = CTX + 1, BY = CTY + 1, BZ = CTZ + 1, BXY = BX * BY;
  constexpr int BN = BXY * BZ;
  // The shell, in three disjoint slabs: bx >= CTX - 1 (all y, z); by >=
  // CTY - 1 (bx below that); bz >= CTZ - 1 (bx and by below).
  constexpr int S1 = 2 * BY * BZ, S2 = (CTX - 1) * 2 * BZ,
                S3 = (CTX - 1) * (CTY - 1) * 2, SN = S1 + S2 + S3;
  constexpr int K = (SN + kCThreads - 1) / kCThreads;
  __shared__ uint16_t box[BN];
  __shared__ uint32_t set[kCrossSlots];
  const int tid = threadIdx.x;
  for (int i = tid; i < kCrossSlots; i += kCThreads) set[i] = kNoKey;
  CGeo g;
  int64_t ti;
  const CGrid &d = cgrid_of(b, cc_tile_of_block(blockIdx.x, gridDim.x), &g,
                            &ti);
  const uint16_t *__restrict__ loc = d.loc;
  int64_t *L = d.L;
  const CTile t = ctile_at(g, ti);
  {
    uint16_t val[K];
    int at[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = tid + k * kCThreads;
      int bx, by, bz;
      if (i < S1) {
        bz = i / (2 * BY);
        const int r = i - bz * (2 * BY);
        by = r >> 1;
        bx = CTX - 1 + (r & 1);
      } else if (i < S1 + S2) {
        const int j = i - S1;
        bz = j / (2 * (CTX - 1));
        const int r = j - bz * (2 * (CTX - 1));
        by = CTY - 1 + r / (CTX - 1);
        bx = r % (CTX - 1);
      } else {
        const int j = i - S1 - S2;
        bz = CTZ - 1 + j / ((CTX - 1) * (CTY - 1));
        const int r = j % ((CTX - 1) * (CTY - 1));
        by = r / (CTX - 1);
        bx = r % (CTX - 1);
      }
      const int64_t x = t.x0 + bx, y = t.y0 + by, z = t.z0 + bz;
      const bool in = i < SN && x < g.X && y < g.Y && z < g.Z;
      at[k] = i < SN ? bx + BX * (by + BY * bz) : -1;
      const int64_t tn = x / CTX + g.ntx * (y / CTY + g.nty * (z / CTZ));
      const int ln = (int)(x % CTX) + CTX * ((int)(y % CTY) + CTY * (int)(z % CTZ));
      val[k] = in ? loc[loc_index(tn, ln)] : kOutside;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (at[k] >= 0) box[at[k]] = val[k];
  }
  __syncthreads();
  // Every masked vertex on an upper face, with each of its higher-id
  // Freudenthal neighbours that lies beyond the face (and in the mask).
  const int cx = tid % CTX, cy = tid / CTX;
  const bool xface = cx == CTX - 1, yface = cy == CTY - 1;
  uint32_t last = kNoKey;
  for (int lz = 0; lz < CTZ; ++lz) {
    const bool zface = lz == CTZ - 1;
    if (!(xface || yface || zface)) continue;
    const int bv = cx + BX * (cy + BY * lz);
    const uint32_t lv = box[bv];
    if (lv == kOutside) continue;
    const int dx[7] = {1, 0, 1, 0, 1, 0, 1};
    const int dy[7] = {0, 1, 1, 0, 0, 1, 1};
    const int dz[7] = {0, 0, 0, 1, 1, 1, 1};
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const bool leaves = (dx[k] && xface) || (dy[k] && yface) ||
                          (dz[k] && zface);
      if (!leaves) continue;
      const uint32_t lu = box[bv + dx[k] + BX * (dy[k] + BY * dz[k])];
      if (lu == kOutside) continue;
      // Which neighbour tile u lies in: one up along each axis it crossed.
      const uint32_t nbr = (uint32_t)(dx[k] && xface) |
                           ((uint32_t)(dy[k] && yface) << 1) |
                           ((uint32_t)(dz[k] && zface) << 2);
      const uint32_t key = lv | (nbr << 13) | (lu << 16);
      if (key == last) continue;  // a lane's edges mostly repeat their roots
      last = key;
      if (!cross_insert(set, key)) cross_unite(g, t, key, L);
    }
  }
  // Each distinct triple once, spread over the block.
  __syncthreads();
  for (int i = tid; i < kCrossSlots; i += kCThreads) {
    const uint32_t key = set[i];
    if (key != kNoKey) cross_unite(g, t, key, L);
  }
}

// Every vertex's final label, plus `off` (a slab labelled inside a larger
// grid writes global ids).  The tile-local roots keep the unshifted root
// here, since concurrent walks read their entries as indices; k_cc_root_shift
// adds the offset to them afterwards.
template <int B>
__global__ void __launch_bounds__(kCThreads) k_cc_final(CBatch<B> b) {
  const int tid = threadIdx.x;
  CGeo g;
  int64_t ti;
  const CGrid &d = cgrid_of(b, cc_tile_of_block(blockIdx.x, gridDim.x), &g,
                            &ti);
  const uint16_t *__restrict__ loc = d.loc;
  int64_t *L = d.L;
  const int64_t off = d.off;
  const CTile t = ctile_at(g, ti);
  const int cx = tid % CTX, cy = tid / CTX;
  const int64_t gx = t.x0 + cx, gy = t.y0 + cy;
  if (gx >= g.X || gy >= g.Y) return;
  const int nz = (int)((g.Z - t.z0) < CTZ ? (g.Z - t.z0) : CTZ);
  const int64_t v0 = gx + g.X * gy + g.XY * t.z0;
  // The column's tile-local roots, all loads in flight together (entries
  // past the domain's last plane exist in the tile's run and are not used).
  uint16_t sl[CTZ];
#pragma unroll
  for (int lz = 0; lz < CTZ; ++lz)
    sl[lz] = loc[loc_index(ti, tid + kCThreads * lz)];
  uint16_t last = kOutside;
  int64_t last_out = -1;
  for (int lz = 0; lz < nz; ++lz) {
    const uint16_t s = sl[lz];
    // Only tile-local roots are ever on a root path, and a root's entry is
    // overwritten (by its owner only) with its own final root, so concurrent
    // walks stay on ancestors and every entry ends as its final root.  A
    // column mostly repeats its local root: its final root is reused.
    if (s != last && s != kOutside) {
      last = s;
      last_out = uf_root<int64_t>(L, ctile_global(g, t, s));
    }
    const bool root = s == cx + CTX * (cy + CTY * lz);
    __atomic_store_n(&L[v0 + g.XY * lz],
                     s == kOutside ? -1 : last_out + (root ? 0 : off),
                     __ATOMIC_RELAXED);
  }
}

// The tile-local roots' labels take the offset once no walk is in flight.
template <int B>
__global__ void __launch_bounds__(kCThreads) k_cc_root_shift(CBatch<B> b) {
  const int tid = threadIdx.x;
  CGeo g;
  int64_t ti;
  const CGrid &d = cgrid_of(b, cc_tile_of_block(blockIdx.x, gridDim.x), &g,
                            &ti);
  const uint16_t *__restrict__ loc = d.loc;
  int64_t *L = d.L;
  const int64_t off = d.off;
  const CTile t = ctile_at(g, ti);
  const int cx = tid % CTX, cy = tid / CTX;
  const int64_t gx = t.x0 + cx, gy = t.y0 + cy;
  if (gx >= g.X || gy >= g.Y) return;
  int nz = (int)((g.Z - t.z0) < CTZ ? (g.Z - t.z0) : CTZ);
  for (int lz = 0; lz < nz; ++lz) {
    const int64_t v = gx + g.X * gy + g.XY * (t.z0 + lz);
    const int l = cx + CTX * (cy + CTY * lz);
    if (loc[loc_index(ti, l)] == l) L[v] += off;
  }
}

// ---------------------------------------------------------------------------
// CSR graphs
// ---------------------------------------------------------------------------

// Edges of a CSR row handled together, so that their gathers overlap.
constexpr int kEdgeChunk = 8;

// Unions of v with u[j] for every j with need[j]: the roots of v and of
// those u[j] are found first with all the walks side by side (each step's
// loads for every walk issued before any is used; walks that are done, or
// not needed, reload a root harmlessly), then each u[j]'s root is hooked to
// v's in turn, the smaller root winning.  A hook whose root has moved
// meanwhile walks that pair again and retries; the merged root is then v's.
__device__ __forceinline__ void uf_unite_row_dev(
    int64_t *par, int64_t v, const int64_t (&u)[kEdgeChunk],
    const bool (&need)[kEdgeChunk]) {
  constexpr int W = kEdgeChunk + 1;
  int64_t r[W];
  bool open[W];
  r[0] = v;
  open[0] = true;
#pragma unroll
  for (int j = 0; j < kEdgeChunk; ++j) {
    r[j + 1] = need[j] ? u[j] : v;
    open[j + 1] = need[j];
  }
  for (;;) {
    bool any = false;
#pragma unroll
    for (int i = 0; i < W; ++i) any |= open[i];
    if (!any) break;
    int64_t pr[W], gr[W];
#pragma unroll
    for (int i = 0; i < W; ++i) pr[i] = ld_dev(&par[r[i]]);
#pragma unroll
    for (int i = 0; i < W; ++i) gr[i] = ld_dev(&par[pr[i]]);
#pragma unroll
    for (int i = 0; i < W; ++i) {
      if (!open[i]) continue;
      if (pr[i] == r[i]) {
        open[i] = false;
      } else if (gr[i] == pr[i]) {
        r[i] = pr[i];
        open[i] = false;
      } else {
        __hip_atomic_store(&par[r[i]], gr[i], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        r[i] = gr[i];
      }
    }
  }
  int64_t rv = r[0];
#pragma unroll
  for (int j = 0; j < kEdgeChunk; ++j) {
    if (!need[j]) continue;
    int64_t a = rv, b = r[j + 1];
    for (;;) {
      if (a == b) {
        rv = a;
        break;
      }
      if (a > b) {
        const int64_t t = a;
        a = b;
        b = t;
      }
      int64_t expect = b;
      if (__hip_atomic_compare_exchange_strong(
              &par[b], &expect, a, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
              __HIP_MEMORY_SCOPE_AGENT)) {
        rv = a;
        break;
      }
      uf_find2_dev(par, a, b);  // b moved meanwhile; retry from the new trees
    }
  }
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
      // A row's edges in chunks whose loads are all in flight together.
      int64_t best = v;
      const int64_t end = rp[v + 1];
      for (int64_t e0 = rp[v]; e0 < end; e0 += kEdgeChunk) {
        int64_t u[kEdgeChunk];
        bool ok[kEdgeChunk];
        // Loads are unconditional, at indices kept in range (the chunk's
        // first entry; the vertex itself), so that a chunk's loads of each
        // kind are all issued before any is used.
#pragma unroll
        for (int j = 0; j < kEdgeChunk; ++j) {
          const int64_t c = (int64_t)ci[e0 + j < end ? e0 + j : e0];
          u[j] = e0 + j < end ? c : v;
          ok[j] = u[j] >= 0 && u[j] < n;
          bad |= !ok[j];
        }
        uint8_t mu[kEdgeChunk];
#pragma unroll
        for (int j = 0; j < kEdgeChunk; ++j)
          mu[j] = mask ? mask[ok[j] ? u[j] : v] : (uint8_t)1;
#pragma unroll
        for (int j = 0; j < kEdgeChunk; ++j)
          if (ok[j] && mu[j]) best = u[j] < best ? u[j] : best;
      }
      L[v] = best;
    }
  }
  flag_any(bad, ctr + kCtrBadIndex);
}

// Every vertex straight to its root (after the hooks of k_csr_init).
__global__ void __launch_bounds__(kBlock)
k_csr_compress(int64_t n, int64_t *L) {
  const int64_t v = gid();
  if (v >= n) return;
  if (__hip_atomic_load(&L[v], __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_WORKGROUP) < 0)
    return;
  __atomic_store_n(&L[v], uf_root<int64_t>(L, v), __ATOMIC_RELAXED);
}

// One union per listed edge between two masked vertices.  Most edges join
// vertices that already share a root after the hooks and the compression: a
// cached read of both entries shows it (an old value is still an ancestor,
// so equal values prove the two are connected), and only the rest take the
// lock-free union.
__global__ void __launch_bounds__(kBlock)
k_csr_union(int64_t n, const int64_t *__restrict__ rp,
            const int32_t *__restrict__ ci, const uint8_t *__restrict__ mask,
            int64_t *L) {
  const int64_t v = gid();
  if (v >= n || (mask && !mask[v])) return;
  const int64_t lv =
      __hip_atomic_load(&L[v], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  const int64_t end = rp[v + 1];
  for (int64_t e0 = rp[v]; e0 < end; e0 += kEdgeChunk) {
    int64_t u[kEdgeChunk], lu[kEdgeChunk];
    // Unconditional loads at in-range indices, each kind issued for the
    // whole chunk before any is used (the init pass has checked every index).
#pragma unroll
    for (int j = 0; j < kEdgeChunk; ++j) {
      const int64_t c = (int64_t)ci[e0 + j < end ? e0 + j : e0];
      u[j] = e0 + j < end ? c : v;
    }
    if (mask) {
      uint8_t mu[kEdgeChunk];
#pragma unroll
      for (int j = 0; j < kEdgeChunk; ++j) mu[j] = mask[u[j]];
#pragma unroll
      for (int j = 0; j < kEdgeChunk; ++j)
        if (!mu[j]) u[j] = v;
    }
#pragma unroll
    for (int j = 0; j < kEdgeChunk; ++j)
      lu[j] = __hip_atomic_load(&L[u[j]], __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
    bool need[kEdgeChunk];
#pragma unroll
    for (int j = 0; j < kEdgeChunk; ++j) need[j] = lu[j] != lv;
    uf_unite_row_dev(L, v, u, need);
  }
}

__global__ void __launch_bounds__(kBlock)
k_csr_final(int64_t n, int64_t *L) {
  int64_t v = gid();
  if (v >= n) return;
  if (__hip_atomic_load(&L[v], __ATOMIC_RELAXED,
                        __HIP_MEMORY_SCOPE_WORKGROUP) < 0)
    return;
  __atomic_store_n(&L[v], uf_root<int64_t>(L, v), __ATOMIC_RELAXED);
}

// ---------------------------------------------------------------------------
// Pointer forests
// ---------------------------------------------------------------------------

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

// Every pointer must be an id in [0, n) before any kernel follows it.
__global__ void __launch_bounds__(kBlock)
k_check_range(const int64_t *__restrict__ d, int64_t n,
              unsigned long long *ctr) {
  int64_t v = gid();
  flag_any(v < n && (d[v] < 0 || d[v] >= n), ctr + kCtrBadIndex);
}

int clear_changed(msc_ctx *ctx, hipStream_t s) {
  return zero_u64(ctx->dctr + kCtrChanged, 1, s);
}

// In-place doubling needs at most about log2(longest path) + 1 rounds; more
// than this many means the pointers hold a cycle (not a forest).
constexpr int kMaxRounds = 96;

}  // namespace

namespace {

// Masks per launch of a batched call: their descriptors travel as kernel
// arguments (64 bytes each).
constexpr int kCCBatch = 32;

// The grid-CC kernels over `nb` tiles of the masks in `b`.
template <int B>
int cc_launch(msc_ctx *ctx, const CBatch<B> &b, uint32_t nb, int64_t nverts,
              bool shift, hipStream_t s) {
  MSC_PHASE(ctx, s, "cc_tile", 3.0 * nverts,
            (k_cc_tile<B><<<nb, kCThreads, 0, s>>>(b)));
  MSC_PHASE(ctx, s, "cc_cross", 0.5 * nverts,
            (k_cc_cross<B><<<nb, kCThreads, 0, s>>>(b)));
  MSC_PHASE(ctx, s, "cc_final", 10.0 * nverts,
            (k_cc_final<B><<<nb, kCThreads, 0, s>>>(b)));
  if (shift)
    MSC_PHASE(ctx, s, "cc_root_shift", 2.0 * nverts,
              (k_cc_root_shift<B><<<nb, kCThreads, 0, s>>>(b)));
  return MSC_OK;
}

int64_t cc_tiles(int64_t X, int64_t Y, int64_t Z) {
  return ((X + CTX - 1) / CTX) * ((Y + CTY - 1) / CTY) * ((Z + CTZ - 1) / CTZ);
}

}  // namespace

size_t cc_grid_workspace(int n, const msc_mask *masks) {
  size_t need = 4096;
  for (int i = 0; i < n; ++i)
    need += align256((size_t)cc_tiles(masks[i].dims[0], masks[i].dims[1],
                                      masks[i].dims[2]) *
                     kCOwned * sizeof(uint16_t));
  return need;
}

int cc_grid_run(msc_ctx *ctx, const uint8_t *mask, int64_t X, int64_t Y,
                int64_t Z, int64_t *labels, hipStream_t s, bool sync,
                int64_t label_off) {
  const int64_t N = X * Y * Z;
  const int64_t ntiles = cc_tiles(X, Y, Z);
  if (ntiles > INT32_MAX) return MSC_ERANGE;
  MSC_TRY(reserve(ctx, ctx->ws,
                  align256(ntiles * kCOwned * sizeof(uint16_t)) + 4096));
  Carver cv(ctx->ws);
  uint16_t *loc = cv.take<uint16_t>(ntiles * kCOwned);
  CBatch<1> b{1, {CGrid{mask, labels, loc, label_off, X, Y, Z, 0u}}};
  MSC_TRY(cc_launch(ctx, b, (uint32_t)ntiles, N, label_off != 0, s));
  if (!sync) return MSC_OK;
  // Nothing to read back: the labels are the whole result.
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = N;
  ctx->stats.tile_x = CTX;
  ctx->stats.tile_y = CTY;
  ctx->stats.tile_z = CTZ;
  return MSC_OK;
}

int cc_grid_batch_run(msc_ctx *ctx, int n, const msc_mask *masks,
                      hipStream_t s) {
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t *d = masks[i].dims;
    if (cc_tiles(d[0], d[1], d[2]) > INT32_MAX) return MSC_ERANGE;
    total += d[0] * d[1] * d[2];
  }
  MSC_TRY(reserve(ctx, ctx->ws, cc_grid_workspace(n, masks)));
  Carver cv(ctx->ws);
  CBatch<kCCBatch> b{};
  uint64_t tiles = 0;
  int64_t verts = 0;
  for (int i = 0; i <= n; ++i) {
    const int64_t *d = i < n ? masks[i].dims : nullptr;
    const int64_t nt = d ? cc_tiles(d[0], d[1], d[2]) : 0;
    // Launch what is collected when the batch is full, would pass 2^31 - 1
    // tiles, or the masks are exhausted.
    if (b.n > 0 && (i == n || b.n == kCCBatch || tiles + nt > INT32_MAX)) {
      MSC_TRY(cc_launch(ctx, b, (uint32_t)tiles, verts, false, s));
      b.n = 0;
      tiles = 0;
      verts = 0;
    }
    if (i == n) break;
    const int64_t N = d[0] * d[1] * d[2];
    b.g[b.n++] = CGrid{masks[i].mask, masks[i].labels,
                       cv.take<uint16_t>(nt * kCOwned), 0, d[0], d[1], d[2],
                       (uint32_t)tiles};
    tiles += (uint64_t)nt;
    verts += N;
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = total;
  ctx->stats.tile_x = CTX;
  ctx->stats.tile_y = CTY;
  ctx->stats.tile_z = CTZ;
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
  MSC_PHASE(ctx, s, "csr_compress", 16.0 * n,
            (k_csr_compress<<<grid_for(n), kBlock, 0, s>>>(n, labels)));
  MSC_PHASE(ctx, s, "csr_union", 13.0 * n,
            (k_csr_union<<<grid_for(n), kBlock, 0, s>>>(n, row_ptr, col_idx,
                                                        mask, labels)));
  MSC_PHASE(ctx, s, "csr_final", 16.0 * n,
            (k_csr_final<<<grid_for(n), kBlock, 0, s>>>(n, labels)));
  MSC_TRY(read_counters(ctx, s));
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  return MSC_OK;
}

int jump_run(msc_ctx *ctx, int64_t *d, int64_t n, int rounds, int sync,
             hipStream_t s) {
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "check_range", 8.0 * n,
            (k_check_range<<<grid_for(n), kBlock, 0, s>>>(d, n, ctx->dctr)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrBadIndex]) return MSC_EINVAL;
  if (!sync) {
    for (int r = 0; rounds == 0 || r < rounds; ++r) {
      if (rounds == 0 && r == kMaxRounds) return MSC_EINVAL;
      MSC_TRY(clear_changed(ctx, s));
      MSC_PHASE(ctx, s, "jump64_round", 24.0 * n,
                (k_jump64<<<grid_for(n), kBlock, 0, s>>>(d, n, ctx->dctr)));
      if (rounds == 0) {
        MSC_TRY(read_counters(ctx, s));
        if (!ctx->hctr[kCtrChanged]) break;
      }
    }
    return MSC_OK;
  }
  MSC_TRY(reserve(ctx, ctx->ws, align256(n * sizeof(int64_t)) + 4096));
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

// ---------------------------------------------------------------------------
// Grid CC with no allocation (for callers that cannot allocate: code under
// graph capture, tight serving loops).  The tile-local roots live in one
// static device array per GPU, taken once per device by symbol address.
// ---------------------------------------------------------------------------

namespace {

// 16-bit tile-local root per vertex, stored by whole tiles: 2^27 entries
// (256 MiB per GPU the library runs on, held until the process ends) bound a
// call at 2^14 tiles of 32x16x16 (512^3 vertices).
constexpr int64_t kNoAllocEntries = INT64_C(1) << 27;
static __device__ __align__(256) uint16_t scratch[kNoAllocEntries];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint16_t *g_scratch_ptr[kMaxDevices] = {};

// The array's device address on `dev`, the current device (the host-side
// name `scratch` is only a stand-in, never a device address).
int scratch_of(int dev, uint16_t **out) {
  if (dev < 0 || dev >= kMaxDevices) return MSC_EINVAL;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return MSC_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<uint16_t *>(p);
  }
  *out = g_scratch_ptr[dev];
  return MSC_OK;
}

}  // namespace
}  // namespace msc

extern "C" int cc_label_grid_noalloc(const uint8_t *mask,
                                     const int64_t dims[3], int64_t *labels,
                                     void *stream) {
  using namespace msc;
  if (!mask || !labels || !dims) return MSC_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (dims[k] < 1) return MSC_EINVAL;
  // Each factor is bounded first, so that the tile count cannot overflow.
  if (dims[0] > kNoAllocEntries || dims[1] > kNoAllocEntries ||
      dims[2] > kNoAllocEntries ||
      cc_tiles(dims[0], dims[1], dims[2]) * kCOwned > kNoAllocEntries)
    return MSC_ERANGE;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MSC_EHIP;
  uint16_t *loc = nullptr;
  MSC_TRY(scratch_of(dev, &loc));
  const int64_t X = dims[0], Y = dims[1], Z = dims[2];
  const unsigned nb = (unsigned)cc_tiles(X, Y, Z);
  const CBatch<1> b{1, {CGrid{mask, labels, loc, 0, X, Y, Z, 0u}}};
  hipStream_t s = static_cast<hipStream_t>(stream);
  // Every entry of `loc` the kernels read is written first (k_cc_tile
  // writes each vertex's root or kOutside), so nothing is cleared.
  k_cc_tile<1><<<nb, kCThreads, 0, s>>>(b);
  k_cc_cross<1><<<nb, kCThreads, 0, s>>>(b);
  k_cc_final<1><<<nb, kCThreads, 0, s>>>(b);
  return hipGetLastError() == hipSuccess ? MSC_OK : MSC_EHIP;
}

namespace msc {

// ---------------------------------------------------------------------------
// Virtual ranks: slab-local labelling, then the exchange across slab
// boundaries (Alg. 3 with the distributed phase it shares with the MS
// segmentation).  Slab r holds planes [r*Z/R, (r+1)*Z/R).
// ---------------------------------------------------------------------------

namespace {

// A slab's labels name vertices by their id within the slab; adding the id
// of the slab's first vertex makes them global ids.
// The exchange at the boundary between plane zb (top of one slab) and
// zb + 1 (bottom of the next): every Freudenthal edge that crosses it,
// (x, y, zb) -- (x + dx, y + dy, zb + 1) for dx, dy in {0, 1}, joins the
// two endpoints' trees when both are in the mask.  L is the parent array:
// every label is a root of its slab's forest, and the smaller root wins.
// All R - 1 boundaries in one launch (grid y strides over them): unions are
// safe to run concurrently, and the boundaries' latency-bound root walks
// overlap.
__global__ void __launch_bounds__(kBlock)
k_rank_cc_stitch(const uint8_t *__restrict__ mask, int64_t X, int64_t Y,
                 int64_t Z, int64_t R, int64_t *L) {
  const int64_t XY = X * Y;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = i < XY;
  const int64_t x = in ? i % X : 0, y = in ? i / X : 0;
  for (int64_t r = 1 + blockIdx.y; r < R; r += gridDim.y) {
    const int64_t zb = r * Z / R - 1;
    const int64_t u = i + XY * zb;
    const bool mu = in && mask[u];
    // The slab labels of both ends, joined once per distinct pair in a run
    // of lanes: neighbouring vertices mostly carry the same two labels, and
    // letting every lane unite them would pile compare-and-swaps onto the
    // same root.
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int dx = e & 1, dy = e >> 1;
      int64_t a = -1, b = -1;
      if (mu && x + dx < X && y + dy < Y) {
        const int64_t w = u + XY + dx + X * dy;
        if (mask[w]) {
          a = L[u];
          b = L[w];
        }
      }
      const int64_t pa = __shfl_up(a, 1), pb = __shfl_up(b, 1);
      const bool first = (threadIdx.x & 63) == 0 || pa != a || pb != b;
      if (a >= 0 && a != b && first) uf_unite_dev(L, a, b);
    }
  }
}

// Every masked vertex takes the root of its label (the smallest id of its
// component); run once no union is in flight.
__global__ void __launch_bounds__(kBlock)
k_rank_cc_final(int64_t *L, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) {
    const int64_t v = L[i];
    if (v >= 0) L[i] = uf_root<int64_t>(L, v);
  }
}

unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int cc_grid_ranks_run(msc_ctx *ctx, const uint8_t *mask, int64_t X,
                      int64_t Y, int64_t Z, int ranks, int64_t *labels,
                      hipStream_t s) {
  const int64_t XY = X * Y, N = XY * Z;
  const int64_t thickest = (Z + ranks - 1) / ranks;
  MSC_TRY(reserve(ctx, ctx->ws, align256(XY * thickest * sizeof(uint16_t)) + 4096));
  for (int r = 0; r < ranks; ++r) {
    const int64_t z0 = r * Z / ranks, z1 = (r + 1) * Z / ranks;
    // No host round trip per slab: the slabs queue on the stream (the
    // tile-local workspace is sized for the largest slab up front).
    // Each slab is labelled in place with global ids (its first id as the
    // label offset).
    MSC_TRY(cc_grid_run(ctx, mask + XY * z0, X, Y, z1 - z0, labels + XY * z0,
                        s, false, XY * z0));
  }
  if (ranks > 1) {
    const unsigned by = ranks - 1 < 65535 ? (unsigned)(ranks - 1) : 65535u;
    MSC_PHASE(ctx, s, "rank_cc_stitch", 2.0 * XY * (ranks - 1),
              (k_rank_cc_stitch<<<dim3(blocks_for(XY), by), kBlock, 0, s>>>(
                  mask, X, Y, Z, ranks, labels)));
  }
  if (ranks > 1)
    MSC_PHASE(ctx, s, "rank_cc_final", 16.0 * N,
              (k_rank_cc_final<<<blocks_for(N), kBlock, 0, s>>>(labels, N)));
  MSC_TRY(read_counters(ctx, s));
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = N;
  return MSC_OK;
}

// ---------------------------------------------------------------------------
// CSR adjacency of a tetrahedral complex (the mesh of the explicit pipeline
// and of msc_segment_csr): every tetrahedron's vertices are neighbours of
// one another.  Per vertex: candidates gathered from its tetrahedra, then
// the distinct ones written in increasing order.  No global sort: vertex
// degrees are small, so each row is deduplicated and ranked by comparing
// its candidates with one another.
// ---------------------------------------------------------------------------

namespace {

constexpr int kScan = 1024;

// Exclusive prefix of x over the block (1024 threads) and the block total.
__device__ __forceinline__ uint64_t block_scan64(uint64_t x, uint64_t *tmp,
                                                 uint64_t *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t inc = x;
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) tmp[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t run = 0;
    for (int k = 0; k < kScan / 64; ++k) {
      const uint64_t t = tmp[k];
      tmp[k] = run;
      run += t;
    }
    tmp[kScan / 64] = run;
  }
  __syncthreads();
  const uint64_t ex = inc - x + tmp[w];
  *total = tmp[kScan / 64];
  __syncthreads();
  return ex;
}

__global__ void __launch_bounds__(kScan)
k_scan64_blocks(const uint32_t *__restrict__ cnt, int64_t n, int64_t *out,
                uint64_t *bsum) {
  __shared__ uint64_t tmp[kScan / 64 + 1];
  const int64_t i = (int64_t)blockIdx.x * kScan + threadIdx.x;
  uint64_t tot = 0;
  const uint64_t ex = block_scan64(i < n ? cnt[i] : 0u, tmp, &tot);
  if (i < n) out[i] = (int64_t)ex;
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// Block totals to block offsets in place (one block); the grand total goes
// to out[n].
__global__ void __launch_bounds__(kScan)
k_scan64_sums(uint64_t *bsum, int64_t nb, int64_t *out, int64_t n) {
  __shared__ uint64_t tmp[kScan / 64 + 1];
  uint64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kScan) {
    const int64_t i = b0 + threadIdx.x;
    uint64_t tot = 0;
    const uint64_t ex = block_scan64(i < nb ? bsum[i] : 0u, tmp, &tot);
    if (i < nb) bsum[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = (int64_t)carry;
}

__global__ void __launch_bounds__(kBlock)
k_scan64_add(int64_t *out, int64_t n, const uint64_t *__restrict__ bsum) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) out[i] += (int64_t)bsum[i / kScan];
}

__global__ void __launch_bounds__(kBlock)
k_zero32(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Every valid tetrahedron adds three candidates to each of its vertices; one
// with a vertex outside [0, n) is skipped and reported.
__global__ void __launch_bounds__(kBlock)
k_tet_count(int64_t ntets, const int32_t *__restrict__ tets, int64_t n,
            uint32_t *cnt, unsigned long long *ctr) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool bad = false;
  if (t < ntets) {
    int32_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = tets[4 * t + k];
      bad |= v[k] < 0 || (int64_t)v[k] >= n;
    }
    if (!bad)
#pragma unroll
      for (int k = 0; k < 4; ++k) atomicAdd(&cnt[v[k]], 3u);
  }
  flag_any(bad, ctr + kCtrBadIndex);
}

__global__ void __launch_bounds__(kBlock)
k_tet_scatter(int64_t ntets, const int32_t *__restrict__ tets, int64_t n,
              const int64_t *__restrict__ off, uint32_t *cursor,
              int32_t *__restrict__ cand) {
  const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (t >= ntets) return;
  int32_t v[4];
  bool bad = false;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = tets[4 * t + k];
    bad |= v[k] < 0 || (int64_t)v[k] >= n;
  }
  if (bad) return;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t at = off[v[k]] + atomicAdd(&cursor[v[k]], 3u);
    int j = 0;
#pragma unroll
    for (int m = 0; m < 4; ++m)
      if (m != k) cand[at + j++] = v[m];
  }
}

// A row's candidates are examined eight at a time.  The first pass moves
// the first occurrence of every neighbour (not the vertex itself) to the
// front of the row as it goes: a candidate is new when it matches neither
// that compacted prefix nor an earlier candidate of its batch, and the
// prefix never reaches past the batch being examined, so every candidate is
// read before it can be overwritten.  The second pass writes each of the
// prefix's values at its rank within the prefix.
constexpr int kRowBatch = 8;

__global__ void __launch_bounds__(kBlock)
k_row_distinct(int64_t n, const int64_t *__restrict__ off, int32_t *cand,
               uint32_t *ucnt) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  int32_t *seg = cand + off[v];
  const int64_t k = off[v + 1] - off[v];
  uint32_t count = 0;
  for (int64_t i0 = 0; i0 < k; i0 += kRowBatch) {
    int32_t c[kRowBatch];
    bool dup[kRowBatch];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t) {
      c[t] = i0 + t < k ? seg[i0 + t] : 0;
      dup[t] = i0 + t >= k || c[t] == (int32_t)v;
    }
    for (uint32_t j = 0; j < count; ++j) {
      const int32_t d = seg[j];
#pragma unroll
      for (int t = 0; t < kRowBatch; ++t) dup[t] |= d == c[t];
    }
#pragma unroll
    for (int t = 1; t < kRowBatch; ++t)
#pragma unroll
      for (int q = 0; q < t; ++q) dup[t] |= c[q] == c[t];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t)
      if (!dup[t]) seg[count++] = c[t];
  }
  ucnt[v] = count;
}

__global__ void __launch_bounds__(kBlock)
k_row_fill(int64_t n, const int64_t *__restrict__ off,
           const int32_t *__restrict__ cand,
           const int64_t *__restrict__ row_ptr, int32_t *__restrict__ col) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const int32_t *seg = cand + off[v];
  const int64_t base = row_ptr[v], u = row_ptr[v + 1] - base;
  for (int64_t i0 = 0; i0 < u; i0 += kRowBatch) {
    int32_t c[kRowBatch];
    uint32_t rank[kRowBatch];
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t) {
      c[t] = i0 + t < u ? seg[i0 + t] : 0;
      rank[t] = 0;
    }
    for (int64_t j = 0; j < u; ++j) {
      const int32_t d = seg[j];
#pragma unroll
      for (int t = 0; t < kRowBatch; ++t) rank[t] += d < c[t];
    }
#pragma unroll
    for (int t = 0; t < kRowBatch; ++t)
      if (i0 + t < u) col[base + rank[t]] = c[t];
  }
}

unsigned grid64(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int scan64(msc_ctx *ctx, const uint32_t *cnt, int64_t n, int64_t *out,
           uint64_t *bsum, hipStream_t s) {
  const int64_t nb = (n + kScan - 1) / kScan;
  if (n > 0)
    k_scan64_blocks<<<grid64(n, kScan), kScan, 0, s>>>(cnt, n, out, bsum);
  k_scan64_sums<<<1, kScan, 0, s>>>(bsum, nb, out, n);  // out[n]: the total
  if (n > 0) k_scan64_add<<<grid64(n, kBlock), kBlock, 0, s>>>(out, n, bsum);
  (void)ctx;
  return MSC_OK;
}

}  // namespace

int csr_from_tets_run(msc_ctx *ctx, int64_t n, int64_t ntets,
                      const int32_t *tets, int64_t *row_ptr, int32_t *col_idx,
                      int64_t capacity, int64_t *nnz, hipStream_t s) {
  const int64_t nb = (n + kScan - 1) / kScan;
  const int64_t ncand = 12 * ntets;
  MSC_TRY(reserve(ctx, ctx->ws, align256(n * 4) + align256((n + 1) * 8) +
                               align256(nb * 8 + 8) + align256(ncand * 4) +
                               4096));
  Carver cv(ctx->ws);
  uint32_t *cnt = cv.take<uint32_t>(n);
  int64_t *off = cv.take<int64_t>(n + 1);
  uint64_t *bsum = cv.take<uint64_t>(nb + 1);
  int32_t *cand = cv.take<int32_t>(ncand);
  MSC_TRY(clear_counters(ctx, s));
  if (n > 0) k_zero32<<<grid64(n, kBlock), kBlock, 0, s>>>(cnt, n);
  if (ntets > 0)
    MSC_PHASE(ctx, s, "tets_count", 16.0 * ntets,
              (k_tet_count<<<grid64(ntets, kBlock), kBlock, 0, s>>>(
                  ntets, tets, n, cnt, ctx->dctr)));
  MSC_PHASE(ctx, s, "tets_scan", 12.0 * n, (scan64(ctx, cnt, n, off, bsum, s)));
  if (n > 0) k_zero32<<<grid64(n, kBlock), kBlock, 0, s>>>(cnt, n);
  if (ntets > 0)
    MSC_PHASE(ctx, s, "tets_scatter", 16.0 * ntets + 4.0 * ncand,
              (k_tet_scatter<<<grid64(ntets, kBlock), kBlock, 0, s>>>(
                  ntets, tets, n, off, cnt, cand)));
  if (n > 0)
    MSC_PHASE(ctx, s, "rows_distinct", 4.0 * ncand + 12.0 * n,
              (k_row_distinct<<<grid64(n, kBlock), kBlock, 0, s>>>(n, off,
                                                                   cand,
                                                                   cnt)));
  MSC_PHASE(ctx, s, "rows_scan", 12.0 * n,
            (scan64(ctx, cnt, n, row_ptr, bsum, s)));
  int64_t total = 0;
  MSC_HIP_TRY(hipMemcpyAsync(&total, row_ptr + n, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrBadIndex]) return MSC_EINVAL;
  *nnz = total;
  if (col_idx && capacity >= total && total > 0)
    MSC_PHASE(ctx, s, "rows_fill", 4.0 * ncand + 4.0 * total,
              (k_row_fill<<<grid64(n, kBlock), kBlock, 0, s>>>(n, off, cand,
                                                               row_ptr,
                                                               col_idx)));
  MSC_TRY(read_counters(ctx, s));
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  return MSC_OK;
}

// ---------------------------------------------------------------------------
// Critical points and the extremum graph (background, "Critical Points";
// the extremum graph that the segmentations feed): the lower and upper link
// of every vertex and their connected components, from the 14 Freudenthal
// neighbours.  The triangulation is a flag complex, so two neighbours of v
// span a link edge exactly when they are neighbours of each other; a link
// vertex outside the domain is absent, which gives the link of boundary
// vertices and of 2-D and 1-D grids.
// ---------------------------------------------------------------------------

namespace {

struct NbVec {
  int dx, dy, dz;
};
// The neighbours in increasing (dz, dy, dx), i.e. in increasing vertex id.
constexpr NbVec kNb[14] = {
    {-1, -1, -1}, {0, -1, -1}, {-1, 0, -1}, {0, 0, -1}, {-1, -1, 0},
    {0, -1, 0},   {-1, 0, 0},  {1, 0, 0},   {0, 1, 0},  {1, 1, 0},
    {0, 0, 1},    {1, 0, 1},   {0, 1, 1},   {1, 1, 1}};

constexpr bool edge_vector(int a, int b, int c) {
  const bool nonneg = a >= 0 && b >= 0 && c >= 0 && a <= 1 && b <= 1 && c <= 1;
  const bool nonpos = a <= 0 && b <= 0 && c <= 0 && a >= -1 && b >= -1 &&
                      c >= -1;
  return (a | b | c) != 0 && (nonneg || nonpos);
}

constexpr uint32_t link_adj(int i) {
  uint32_t m = 0;
  for (int j = 0; j < 14; ++j)
    if (j != i && edge_vector(kNb[i].dx - kNb[j].dx, kNb[i].dy - kNb[j].dy,
                              kNb[i].dz - kNb[j].dz))
      m |= 1u << j;
  return m;
}

// Components of the link restricted to a set of neighbours depend on the set
// alone (the adjacency is fixed and absent neighbours are simply not in the
// set), so two tables over all 2^14 sets replace the per-vertex growth: the
// number of components, and the component that holds the set's lowest
// neighbour.  Removing that component leaves a set whose components are the
// remaining ones, so repeated lookups enumerate them.
constexpr int kLinkSets = 1 << 14;

__device__ __forceinline__ uint32_t grow_component(uint32_t seed,
                                                   uint32_t set) {
  uint32_t comp = seed, prev;
  do {
    prev = comp;
    uint32_t g = comp;
#pragma unroll
    for (int i = 0; i < 14; ++i)
      if ((prev >> i) & 1u) g |= link_adj(i);
    comp = g & set;
  } while (comp != prev);
  return comp;
}

__global__ void __launch_bounds__(kBlock)
k_link_tables(uint8_t *__restrict__ ncomp, uint16_t *__restrict__ first) {
  const uint32_t set = blockIdx.x * kBlock + threadIdx.x;
  if (set >= (uint32_t)kLinkSets) return;
  uint32_t rem = set, head = 0;
  int count = 0;
  while (rem) {
    const uint32_t comp = grow_component(rem & (0u - rem), rem);
    if (!count) head = comp;
    rem &= ~comp;
    ++count;
  }
  ncomp[set] = (uint8_t)count;
  first[set] = (uint16_t)head;
}

struct LinkSets {
  float fn[14];          // neighbour values (meaningless where absent)
  uint32_t lower, upper; // neighbours below / above v in the (f, id) order
  bool nan;
};

// Requires X·Y·Z <= INT32_MAX (checked by the entry points), so ids and id
// offsets fit 32 bits.
__device__ __forceinline__ LinkSets link_sets(const float *__restrict__ f,
                                              int64_t X, int64_t Y, int64_t Z,
                                              int64_t v) {
  const uint32_t vv = (uint32_t)v, X32 = (uint32_t)X, Y32 = (uint32_t)Y;
  const uint32_t row = vv / X32;
  const uint32_t x = vv - row * X32, y = row % Y32, z = row / Y32;
  const int32_t sx = 1, sy = (int32_t)X32, sz = (int32_t)(X32 * Y32);
  // Per axis, whether the step down / up stays in the grid; a step that
  // would leave it is taken as 0, so every load below stays in bounds and
  // the neighbour is marked absent.
  const bool lo[3] = {x > 0, y > 0, z > 0};
  const bool hi[3] = {x + 1 < X32, y + 1 < Y32, (int64_t)z + 1 < Z};
  const int32_t step[3] = {sx, sy, sz};
  const float *p = f + v;
  const float fv = p[0];
  LinkSets ls;
  uint32_t present = 0;
#pragma unroll
  for (int i = 0; i < 14; ++i) {
    const int d[3] = {kNb[i].dx, kNb[i].dy, kNb[i].dz};
    int32_t off = 0;
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (d[a] < 0) {
        in = in && lo[a];
        off -= lo[a] ? step[a] : 0;
      } else if (d[a] > 0) {
        in = in && hi[a];
        off += hi[a] ? step[a] : 0;
      }
    }
    ls.fn[i] = p[off];
    present |= (uint32_t)in << i;
  }
  ls.nan = fv != fv;
  uint32_t lower = 0;
#pragma unroll
  for (int i = 0; i < 14; ++i) {
    // the first 7 neighbours have smaller ids than v
    const bool below = ls.fn[i] < fv || (ls.fn[i] == fv && i < 7);
    lower |= (uint32_t)below << i;
  }
  ls.lower = lower & present;
  ls.upper = present & ~lower;
  return ls;
}

// The (f, id)-extreme neighbour of each component of `set` (the highest when
// `high`), as a neighbour mask.  Neighbour order is id order, so a tie in
// value goes to the larger index for the highest and the smaller for the
// lowest.
__device__ __forceinline__ uint32_t component_extremes(
    uint32_t set, const float *fn, bool high,
    const uint16_t *__restrict__ first) {
  uint32_t rem = set, ex = 0;
  while (rem) {
    const uint32_t comp = first[rem];
    int best = -1;
    float fb = 0.f;
#pragma unroll
    for (int i = 0; i < 14; ++i) {
      if (!((comp >> i) & 1u)) continue;
      const bool better = best < 0 || (high ? fn[i] >= fb : fn[i] < fb);
      if (better) {
        best = i;
        fb = fn[i];
      }
    }
    ex |= 1u << best;
    rem &= ~comp;
  }
  return ex;
}

__global__ void __launch_bounds__(kBlock)
k_critical(const float *__restrict__ f, int64_t X, int64_t Y, int64_t Z,
           const uint8_t *__restrict__ ncomp, uint8_t *__restrict__ code,
           unsigned long long *ctr) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool nan = false;
  if (v < X * Y * Z) {
    const LinkSets ls = link_sets(f, X, Y, Z, v);
    code[v] = (uint8_t)(ncomp[ls.lower] | (ncomp[ls.upper] << 4));
    nan = ls.nan;
  }
  flag_any(nan, ctr + kCtrNaN);
}

// Edges of a vertex: one per component of a side that has two or more.
__device__ __forceinline__ uint32_t edge_count(uint32_t lc, uint32_t uc) {
  return (uc >= 2 ? uc : 0u) + (lc >= 2 ? lc : 0u);
}

// Exclusive prefix over a block of kBlock threads and the block total, for
// per-thread counts below 16 (a vertex has at most 14 edges: its lower and
// upper link components together number at most its 14 link vertices).  One
// ballot per bit: a lane's prefix in its wave is the sum over bits k of 2^k
// times the number of lower lanes with bit k set.
__device__ __forceinline__ uint32_t block_scan16(uint32_t x, uint32_t *tmp,
                                                 uint32_t *total) {
  const int w = threadIdx.x >> 6;
  uint32_t pre = 0, sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const unsigned long long b = __ballot((x >> k) & 1u);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        (uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    pre += below << k;
    sum += (uint32_t)__popcll(b) << k;
  }
  if ((threadIdx.x & 63) == 0) tmp[w] = sum;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < kBlock / 64; ++k) {
    const uint32_t t = tmp[k];
    before += k < w ? t : 0u;
    all += t;
  }
  *total = all;
  return before + pre;
}

__global__ void __launch_bounds__(kBlock)
k_egraph_count(const float *__restrict__ f, int64_t X, int64_t Y, int64_t Z,
               const uint8_t *__restrict__ ncomp, uint32_t *bcount,
               unsigned long long *ctr) {
  __shared__ uint32_t tmp[kBlock / 64];
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t c = 0;
  bool nan = false;
  if (v < X * Y * Z) {
    const LinkSets ls = link_sets(f, X, Y, Z, v);
    c = edge_count(ncomp[ls.lower], ncomp[ls.upper]);
    nan = ls.nan;
  }
  flag_any(nan, ctr + kCtrNaN);
  uint32_t tot = 0;
  (void)block_scan16(c, tmp, &tot);
  if (threadIdx.x == 0) bcount[blockIdx.x] = tot;
}

// Edges of a vertex: ascending ones first, then descending; within a side,
// components by increasing id of their extreme vertex (= neighbour order).
__global__ void __launch_bounds__(kBlock)
k_egraph_write(const float *__restrict__ f, int64_t X, int64_t Y, int64_t Z,
               const uint8_t *__restrict__ ncomp,
               const uint16_t *__restrict__ first,
               const int32_t *__restrict__ asc,
               const int32_t *__restrict__ desc,
               const int64_t *__restrict__ boff, int32_t *__restrict__ out) {
  __shared__ uint32_t tmp[kBlock / 64];
  // A block without edges has nothing to write (the scan is block-local).
  if (boff[blockIdx.x + 1] == boff[blockIdx.x]) return;
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t XY = X * Y;
  LinkSets ls{};
  uint32_t lc = 0, uc = 0;
  if (v < X * Y * Z) {
    ls = link_sets(f, X, Y, Z, v);
    lc = ncomp[ls.lower];
    uc = ncomp[ls.upper];
  }
  const uint32_t c = edge_count(lc, uc);
  uint32_t tot = 0;
  const uint32_t ex = block_scan16(c, tmp, &tot);
  if (!c) return;
  int64_t at = boff[blockIdx.x] + ex;
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const bool high = side == 0;
    const uint32_t set = high ? (uc >= 2 ? ls.upper : 0u)
                              : (lc >= 2 ? ls.lower : 0u);
    const uint32_t m = component_extremes(set, ls.fn, high, first);
#pragma unroll
    for (int i = 0; i < 14; ++i) {
      if (!((m >> i) & 1u)) continue;
      const int64_t u = v + kNb[i].dx + (int64_t)X * kNb[i].dy +
                        XY * kNb[i].dz;
      out[3 * at] = (int32_t)v;
      out[3 * at + 1] = high ? asc[u] : desc[u];
      out[3 * at + 2] = high ? 1 : -1;
      ++at;
    }
  }
}

}  // namespace

int critical_points_run(msc_ctx *ctx, const float *field, const int64_t *dims,
                        uint8_t *code, hipStream_t s) {
  const int64_t X = dims[0], Y = dims[1], Z = dims[2], N = X * Y * Z;
  MSC_TRY(reserve(ctx, ctx->ws, align256(kLinkSets) + align256(2 * kLinkSets)));
  Carver cv(ctx->ws);
  uint8_t *ncomp = cv.take<uint8_t>(kLinkSets);
  uint16_t *first = cv.take<uint16_t>(kLinkSets);
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "link_tables", 3.0 * kLinkSets,
            (k_link_tables<<<kLinkSets / kBlock, kBlock, 0, s>>>(ncomp,
                                                                first)));
  MSC_PHASE(ctx, s, "critical", 5.0 * N,
            (k_critical<<<grid64(N, kBlock), kBlock, 0, s>>>(
                field, X, Y, Z, ncomp, code, ctx->dctr)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrNaN]) return MSC_ENAN;
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = N;
  return MSC_OK;
}

int extremum_graph_run(msc_ctx *ctx, const float *field, const int64_t *dims,
                       const int32_t *asc, const int32_t *desc, int32_t *edges,
                       int64_t capacity, int64_t *count, hipStream_t s) {
  const int64_t X = dims[0], Y = dims[1], Z = dims[2], N = X * Y * Z;
  const int64_t nb = (N + kBlock - 1) / kBlock;
  const int64_t nsb = (nb + kScan - 1) / kScan;
  MSC_TRY(reserve(ctx, ctx->ws, align256(nb * 4) + align256((nb + 1) * 8) +
                               align256(nsb * 8 + 8) + align256(kLinkSets) +
                               align256(2 * kLinkSets) + 4096));
  Carver cv(ctx->ws);
  uint32_t *bcount = cv.take<uint32_t>(nb);
  int64_t *boff = cv.take<int64_t>(nb + 1);
  uint64_t *bsum = cv.take<uint64_t>(nsb + 1);
  uint8_t *ncomp = cv.take<uint8_t>(kLinkSets);
  uint16_t *first = cv.take<uint16_t>(kLinkSets);
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "link_tables", 3.0 * kLinkSets,
            (k_link_tables<<<kLinkSets / kBlock, kBlock, 0, s>>>(ncomp,
                                                                first)));
  MSC_PHASE(ctx, s, "egraph_count", 4.0 * N,
            (k_egraph_count<<<(unsigned)nb, kBlock, 0, s>>>(
                 field, X, Y, Z, ncomp, bcount, ctx->dctr),
             scan64(ctx, bcount, nb, boff, bsum, s)));
  int64_t total = 0;
  MSC_HIP_TRY(hipMemcpyAsync(&total, boff + nb, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrNaN]) return MSC_ENAN;
  *count = total;
  if (edges && capacity >= total && total > 0)
    MSC_PHASE(ctx, s, "egraph_write", 4.0 * N + 12.0 * total,
              (k_egraph_write<<<(unsigned)nb, kBlock, 0, s>>>(
                  field, X, Y, Z, ncomp, first, asc, desc, boff, edges)));
  MSC_TRY(read_counters(ctx, s));
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = N;
  return MSC_OK;
}

}  // namespace msc
