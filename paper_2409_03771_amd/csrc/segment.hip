// Morse-Smale segmentation kernels (gfx950), for one field or a batch.
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
// onto the GPU's memory hierarchy, and every pass runs once over the tiles
// of all fields of a batch (one field is a batch of one):
//
//   tile_local    one workgroup per tile: the field plus a one-vertex halo is
//                 staged in LDS, both steepest pointers are computed from LDS
//                 (each thread walks a z-column with a three-plane register
//                 window), halo vertices point to themselves (the ghost
//                 rule), and pointer jumping runs in LDS until every owned
//                 vertex points to a tile-local extremum or to a halo vertex
//                 ("exit").  Writes a 16-bit code per vertex and direction
//                 (an owned extremum, or the tile-local number of an exit)
//                 and the tile's exit list at the tile's fixed slots
//                 (2 * halo size per tile, so node numbers need no scan).
//   exit_link     an exit lies on a neighbouring tile's shell; that tile's
//                 code for it gives the exit's successor: a final extremum or
//                 another tile's exit.  The exits form a dense graph.
//   tile_order    tiles sorted by mean value;
//   exit_resolve  one workgroup per tile and direction, in that order
//                 (ascent: high mean first; descent: low mean first), chases
//                 every exit's successors to a final value -- the paper's
//                 compression of the ghost graph after the exchange.
//   tile_pairs    per tile: decode every vertex's final (asc, desc) pair from
//                 its codes and the tile's resolved exits, dedupe in LDS, and
//                 insert into the field's hash table keeping the smallest id;
//   tile_write    the same decode, then asc, desc and the cell id per vertex
//                 (the paper's relabelling pass, Alg. 2).
#include <climits>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "msc_internal.hpp"

namespace msc {
namespace {

template <int TX_, int TY_, int TZ_>
struct Cfg {
  static constexpr int TX = TX_, TY = TY_, TZ = TZ_;
  static constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
  static constexpr int HXY = HX * HY;
  static constexpr int H = HXY * HZ;          // tile plus halo
  static constexpr int TXY = TX * TY;
  static constexpr int kThreads = TX * TY;    // one thread per z-column
  static constexpr int kHalo = H - TX * TY * TZ;
  // The in-LDS pointers are 16-bit byte addresses: 4 * (target index) for
  // ascent, 4 * (target index) + 2 for descent.
  static_assert(4 * (H - 1) + 2 <= 0xffff, "tile-local pointers are 16-bit");
  static_assert(kThreads % 64 == 0 && kThreads <= 1024, "block shape");
  static_assert((kHalo + kThreads - 1) / kThreads * (kThreads / 64) <= 64,
                "one wave scans the exit counts");
  static_assert(TX * TY * TZ <= 0x8000 && kHalo < 0x8000,
                "local pointer codes are 15-bit");
};

constexpr unsigned long long kEmptyKey = ~0ull;

// Per-field counters (kFieldCtrs per field).
enum FieldCtr : int { kFMaxima = 0, kFMinima = 1, kFCells = 2, kFNaN = 3,
                      kFExits = 4, kFieldCtrs = 5 };

struct Geo {
  uint32_t X, Y, Z, XY, N;
  uint32_t ntx, nty, ntz, ntiles;
};

// One field of a batch as the kernels see it.
struct FieldDev {
  const float *f;
  uint32_t *lp;                // packed codes, tile-major (code_word), one
                               // array for the whole batch
  int32_t *A, *D, *ms;         // outputs; NULL when not wanted
  unsigned long long *keys;    // the field's pair table
  int32_t *vals;
  uint32_t mask;               // table capacity - 1
  uint32_t tile0;              // first global tile of the field
  uint32_t ghost;              // bit 0 / bit 1: plane z = 0 / z = Z-1 holds
                               // ghost vertices (fixed points, Alg. 1)
  Geo g;
};

// A tile's exits in the list: `base`, then `na` ascent exits and `nd`
// descent exits, each group in increasing halo-index order.
struct Seg {
  uint32_t base;
  uint16_t na, nd;
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

// Field values read through a pointer known to be in global memory, so that
// the loads are global (not flat) ones.
typedef __attribute__((address_space(1))) float GlobalF;

// Plane z of a per-vertex array as a global-memory pointer: the base is
// uniform over a block and a column adds a 32-bit offset, so accesses need
// no per-lane 64-bit address arithmetic.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *plane_ptr(
    T *p, const Geo &g, int z) {
  return (__attribute__((address_space(1))) T *)p + (size_t)g.XY * (uint32_t)z;
}

// The packed codes are stored tile-major: a tile's TZ planes of TX*TY
// columns are one contiguous run, so every pass reads or writes whole runs
// instead of a row of TX words per (y, z).  Positions outside the domain
// have their word too (written and read, never used).
template <class C>
__device__ __forceinline__ size_t code_word(uint32_t gt, int lz, int tid) {
  return ((size_t)gt * C::TZ + (size_t)lz) * C::kThreads + (size_t)tid;
}

// A tile's codes of its first (side 0) and last (side 1) x column, side by
// side in one array: the x-face exits of its x-neighbours read them from
// there, consecutive exits from consecutive words, where a gather from the
// field-ordered codes would fetch a whole row for each.
template <class C>
__device__ __forceinline__ size_t shell_word(uint32_t gt, uint32_t side,
                                             uint32_t lz, uint32_t ly) {
  return (((size_t)gt * 2 + side) * C::TZ + lz) * C::TY + ly;
}

template <class C>
__device__ __forceinline__ Tile tile_at(const Geo &g, uint32_t t) {
  uint32_t tx = t % g.ntx, r = t / g.ntx;
  uint32_t ty = r % g.nty, tz = r / g.nty;
  return Tile{(int)tx * C::TX, (int)ty * C::TY, (int)tz * C::TZ};
}

// Global id of tile-local index p; p must lie inside the domain.
template <class C>
__device__ __forceinline__ uint32_t halo_global(const Geo &g, const Tile &t,
                                                int p) {
  int hz = p / C::HXY, r = p - hz * C::HXY, hy = r / C::HX, hx = r - hy * C::HX;
  return (uint32_t)(t.x0 - 1 + hx) + g.X * (uint32_t)(t.y0 - 1 + hy) +
         g.XY * (uint32_t)(t.z0 - 1 + hz);
}

// Tile-plus-halo index of halo entry i, 0 <= i < kHalo, enumerating the
// halo in increasing index: the bottom plane, then each middle plane's ring
// (its first row, the two ends of every inner row, its last row), then the
// top plane.
template <class C>
__device__ __forceinline__ int halo_index(int i) {
  constexpr uint32_t R = 2 * C::HX + 2 * (C::HY - 2);  // ring of a plane
  constexpr uint32_t B = C::HXY, M = B + (C::HZ - 2) * R;
  const uint32_t u = (uint32_t)i;
  if (u < B) return i;
  if (u >= M) return (int)((C::HZ - 1) * C::HXY + (u - M));
  const uint32_t r = u - B, pl = r / R, k = r - pl * R;
  uint32_t q;
  if (k < (uint32_t)C::HX) {
    q = k;
  } else if (k >= R - C::HX) {
    q = (C::HY - 1) * C::HX + (k - (R - C::HX));
  } else {
    const uint32_t k2 = k - C::HX;
    q = (1 + (k2 >> 1)) * C::HX + ((k2 & 1u) ? C::HX - 1 : 0);
  }
  return (int)((pl + 1) * C::HXY + q);
}

// Number of lanes below this one whose bit is set in a wave-wide mask.
__device__ __forceinline__ uint32_t lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Stored tile-local pointers are 16-bit codes: an owned target is
// lx + TX*(ly + TY*lz) (bit 15 clear); an exit target is its number among the
// tile's exits of that direction, with bit 15 set.
constexpr uint32_t kExitCode = 0x8000u;

// Global id of an owned code.
template <class C>
__device__ __forceinline__ uint32_t owned_global(const Geo &g, const Tile &t,
                                                 uint32_t code) {
  const uint32_t lx = code % C::TX, ly = (code / C::TX) % C::TY,
                 lz = code / (C::TX * C::TY);
  return ((uint32_t)t.x0 + lx) + g.X * ((uint32_t)t.y0 + ly) +
         g.XY * ((uint32_t)t.z0 + lz);
}

// A halo entry that some vertex's final pointer names.
constexpr uint32_t kMark = 0xffffu;

// 16-bit LDS entries addressed by byte offset from an array base.
__device__ __forceinline__ uint32_t ld16(const char *base, uint32_t off) {
  return *reinterpret_cast<const uint16_t *>(base + off);
}
__device__ __forceinline__ void st16(char *base, uint32_t off, uint32_t v) {
  *reinterpret_cast<uint16_t *>(base + off) = (uint16_t)v;
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

// Order-preserving map of a float to an unsigned key; only used to order
// work, never to decide a result.
__device__ __forceinline__ uint32_t float_key(float x) {
  uint32_t u = __float_as_uint(x);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Exclusive prefix sum over the block (at most 1024 threads = 16 waves).
// `tmp` holds 32 words of LDS.  Returns the prefix; *total gets the sum.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x,
                                                         uint32_t *tmp,
                                                         uint32_t *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nwaves = (blockDim.x + 63) >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(inc, o);
    if (lane >= o) inc += y;
  }
  if (lane == 63) tmp[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    uint32_t s = lane < nwaves ? tmp[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      uint32_t y = __shfl_up(s, o);
      if (lane >= o) s += y;
    }
    if (lane < 16) tmp[16 + lane] = s;  // inclusive wave totals
  }
  __syncthreads();
  const uint32_t before = wave ? tmp[16 + wave - 1] : 0;
  *total = tmp[16 + nwaves - 1];
  __syncthreads();
  return before + inc - x;
}

// The block's tile: global tile index, its field and the field's geometry.
struct BlockTile {
  uint32_t gt, fi, tile;
  FieldDev fd;
};

__device__ __forceinline__ BlockTile block_tile_at(const FieldDev *fds,
                                                   const uint32_t *tfield,
                                                   uint32_t blk, uint32_t nb) {
  BlockTile b;
  b.gt = tile_of_block(blk, nb);
  b.fi = tfield[b.gt];
  b.fd = fds[b.fi];
  b.tile = b.gt - b.fd.tile0;
  return b;
}

__device__ __forceinline__ BlockTile block_tile(const FieldDev *fds,
                                                const uint32_t *tfield) {
  BlockTile b;
  b.gt = tile_of_block(blockIdx.x, gridDim.x);
  b.fi = tfield[b.gt];
  b.fd = fds[b.fi];
  b.tile = b.gt - b.fd.tile0;
  return b;
}

// ---------------------------------------------------------------------------
// tile_local
// ---------------------------------------------------------------------------

// The 7 values of one plane a column needs: (dx,dy) = (-1,-1), (0,-1),
// (-1,0), (0,0), (1,0), (0,1), (1,1) -- the Freudenthal neighbours never use
// the (1,-1) and (-1,1) corners.
struct Plane {
  float v[7];
};

template <class C>
__device__ __forceinline__ Plane load_plane(const uint32_t *lds, int c) {
  Plane p;
  p.v[0] = __uint_as_float(lds[c - 1 - C::HX]);
  p.v[1] = __uint_as_float(lds[c - C::HX]);
  p.v[2] = __uint_as_float(lds[c - 1]);
  p.v[3] = __uint_as_float(lds[c]);
  p.v[4] = __uint_as_float(lds[c + 1]);
  p.v[5] = __uint_as_float(lds[c + C::HX]);
  p.v[6] = __uint_as_float(lds[c + C::HX + 1]);
  return p;
}

struct ExitOut {
  Seg *seg;            // per global tile: exit counts (base set later)
  uint32_t *tkey;      // per global tile: order key of its mean value
  uint32_t *tstat;     // per global tile: maxima, minima, cells, exits
  uint16_t *tlist;     // per global tile, 2*kHalo slots: halo index of each
                       // exit, ascent exits first (numbers are tile-local)
  uint32_t *xs;        // per global tile: the codes of its first and last
                       // x columns (shell_word)
};

// Counters are summed per block and written per tile, then folded by these
// small kernels: atomics on one device address are serialised across the
// chip and cost far more than the kernels' own work at one per wave.
// tstat[4 * tile + k] summed per field into fctr[field][which]; a wave whose
// tiles all belong to one field adds once.
// One tile counter per lane into its field's counter: summed over the wave
// when the wave's tiles share a field, else per lane.
__device__ __forceinline__ void fold_stat(bool in, uint32_t v, uint32_t fi,
                                          unsigned long long *fctr,
                                          int which) {
  const uint32_t f0 = __builtin_amdgcn_readlane(fi, 0);
  if (__ballot(in && fi != f0) == 0) {
    uint32_t sum = v;
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    if ((threadIdx.x & 63) == 0 && sum)
      atomicAdd(fctr + (size_t)f0 * kFieldCtrs + which,
                (unsigned long long)sum);
  } else if (in && v) {
    atomicAdd(fctr + (size_t)fi * kFieldCtrs + which, (unsigned long long)v);
  }
}

__global__ void __launch_bounds__(kBlock)
k_tile_stat_reduce(const uint32_t *__restrict__ tstat, int k, uint32_t nt,
                   const uint32_t *__restrict__ tfield,
                   unsigned long long *fctr, int which) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  const bool in = i < nt;
  const uint32_t v = in ? tstat[4 * (size_t)i + k] : 0u;
  const uint32_t fi = in ? tfield[i] : 0u;
  fold_stat(in, v, fi, fctr, which);
}

// Maxima, minima and exits of every tile in one pass (tile counters 0, 1
// and 3).
__global__ void __launch_bounds__(kBlock)
k_tile_stats3(const uint32_t *__restrict__ tstat, uint32_t nt,
              const uint32_t *__restrict__ tfield, unsigned long long *fctr) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  const bool in = i < nt;
  const uint4 c = in ? reinterpret_cast<const uint4 *>(tstat)[i]
                     : make_uint4(0u, 0u, 0u, 0u);
  const uint32_t fi = in ? tfield[i] : 0u;
  fold_stat(in, c.x, fi, fctr, kFMaxima);
  fold_stat(in, c.y, fi, fctr, kFMinima);
  fold_stat(in, c.w, fi, fctr, kFExits);
}

// Per-block (longest chain, links followed) of the exit resolution into the
// global counters: each thread folds a strided share, then the block, then
// one atomic pair per block.
constexpr int kStepsBlocks = 64;

__global__ void __launch_bounds__(1024)
k_steps_reduce(const unsigned long long *__restrict__ rstat, uint32_t nb,
               unsigned long long *ctr) {
  __shared__ unsigned long long smx[16], ssum[16];
  unsigned long long mx = 0, sum = 0;
  for (uint32_t i = blockIdx.x * 1024 + threadIdx.x; i < nb;
       i += kStepsBlocks * 1024) {
    const unsigned long long m = rstat[2 * (size_t)i];
    mx = m > mx ? m : mx;
    sum += rstat[2 * (size_t)i + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long a = __shfl_xor(mx, o);
    mx = a > mx ? a : mx;
    sum += __shfl_xor(sum, o);
  }
  if ((threadIdx.x & 63) == 0) {
    smx[threadIdx.x >> 6] = mx;
    ssum[threadIdx.x >> 6] = sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) {
      mx = smx[w] > mx ? smx[w] : mx;
      sum += ssum[w];
    }
    if (sum) {
      atomicMax(ctr + kCtrRounds, mx);
      atomicAdd(ctr + kCtrSteps, sum);
    }
  }
}

template <class C>
__global__ void __launch_bounds__(C::kThreads)
__attribute__((amdgpu_waves_per_eu(6, 6)))
k_tile_local(const FieldDev *__restrict__ fds,
             const uint32_t *__restrict__ tfield, ExitOut xo,
             unsigned long long *ctr, unsigned long long *fctr) {
  constexpr int HX = C::HX, HXY = C::HXY, H = C::H, T = C::kThreads;
  // The field while the steepest pointers are computed.  Then one word per
  // tile-plus-halo index p: the ascent pointer in its low half, the descent
  // pointer in its high half.  A pointer is the byte address of the half it
  // names (4 * target for ascent, 4 * target + 2 for descent), so following
  // it is a single 16-bit LDS read with no address arithmetic, and the value
  // read is the next pointer of the same direction.
  __shared__ uint32_t lds[H];
  char *const lb = reinterpret_cast<char *>(lds);
  // Marked halo entries per (round, wave) of the exit numbering, then
  // their exclusive prefixes and the total (ascent | descent << 16).
  __shared__ uint32_t s_cnt[(C::kHalo + C::kThreads - 1) / C::kThreads *
                                (C::kThreads / 64) + 1];
  __shared__ float s_wsum[16];
  __shared__ uint32_t s_wext[16];  // per wave: maxima | minima << 16

  const int tid = threadIdx.x;
  const BlockTile bt = block_tile(fds, tfield);
  const Geo &g = bt.fd.g;
  const float *__restrict__ f = bt.fd.f;
  unsigned long long *fc = fctr + (size_t)bt.fi * kFieldCtrs;
  const Tile t = tile_at<C>(g, bt.tile);
  // Stage the tile and its halo by z-columns: thread tid takes box columns
  // tid, tid + T, ... and issues a column's loads before storing any of
  // them.  Consecutive threads take consecutive columns (coalesced rows);
  // a column's offset within a plane is computed once, and each plane's
  // base is uniform over the block.  Positions outside the domain hold NaN,
  // which loses every comparison below and so is never chosen.
  // A NaN anywhere in the domain is reported (a halo value belongs to a
  // neighbouring tile, which reports it too).
  bool any_nan = false;
  {
    constexpr int KC = (HXY + T - 1) / T;
    const uint32_t kNaN = 0x7fc00000u;
#pragma unroll
    for (int sl = 0; sl < KC; ++sl) {
      const int col = tid + sl * T;
      if (col < HXY) {
        const int hy = col / HX, hx = col - hy * HX;
        const int gx = t.x0 - 1 + hx, gy = t.y0 - 1 + hy;
        const bool cin =
            gx >= 0 && gx < (int)g.X && gy >= 0 && gy < (int)g.Y;
        const uint32_t off = cin ? (uint32_t)gx + g.X * (uint32_t)gy : 0u;
        // Every load is issued before any is used (the addresses are
        // clamped into the field, so none needs a guard).
        uint32_t val[C::HZ];
#pragma unroll
        for (int hz = 0; hz < C::HZ; ++hz) {
          const int gz = t.z0 - 1 + hz;
          const bool zin = gz >= 0 && gz < (int)g.Z;
          const GlobalF *plane = (const GlobalF *)f +
                                 (size_t)g.XY * (uint32_t)(zin ? gz : 0);
          val[hz] = __float_as_uint(plane[off]);
        }
#pragma unroll
        for (int hz = 0; hz < C::HZ; ++hz) {
          const int gz = t.z0 - 1 + hz;
          const bool in = cin && gz >= 0 && gz < (int)g.Z;
          any_nan |= in && (val[hz] & 0x7fffffffu) > 0x7f800000u;
          lds[col + hz * HXY] = in ? val[hz] : kNaN;
        }
      }
    }
  }
  wave_count(any_nan, fc + kFNaN);
  __syncthreads();

  const int cx = tid % C::TX, cy = tid / C::TX;
  const int gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < (int)g.X && gy < (int)g.Y;
  int nz = (int)g.Z - t.z0;
  nz = col_in ? (nz < C::TZ ? nz : C::TZ) : 0;
  const int c0 = (cx + 1) + HX * (cy + 1);  // column index in plane 0

  // Steepest ascent / descent over the closed neighbourhood, ordered by
  // (value, id).  The 14 Freudenthal neighbours of a vertex at plane P are,
  // in plane P, the column's (-1,0), (0,-1), (-1,-1) and (+1,0), (0,+1),
  // (+1,+1) neighbours, and (0,0), (-1,0), (0,-1), (-1,-1) of plane P-1 and
  // (0,0), (+1,0), (0,+1), (+1,+1) of plane P+1.  So with, per plane,
  //   LF(P) = best of { c, (-1,0), (0,-1), (-1,-1) }   (c and lower ids)
  //   UF(P) = best of { c, (+1,0), (0,+1), (+1,+1) }   (c and higher ids)
  // the vertex at P takes the best of LF(P), UF(P), LF(P-1) and UF(P+1), and
  // each group is computed once and used by two vertices of the column.
  // Every id in plane P-1 is below every id in plane P, which is below every
  // id in plane P+1, so each merge knows which side has the larger id: a
  // challenger with larger ids wins the max when at least equal and the min
  // when strictly below; one with smaller ids wins the max when strictly
  // above and the min when at most equal.  Each chain starts from a vertex
  // of the domain and takes its challengers in one id order, so a position
  // outside the domain (NaN) never wins a comparison.
  // Ghost planes of a slab (the virtual-rank path): bit lz is set when
  // plane t.z0 + lz holds ghost vertices, which are fixed points
  // (block-uniform).
  uint32_t gmask = 0;
  if ((bt.fd.ghost & 1u) && t.z0 == 0) gmask |= 1u;
  if ((bt.fd.ghost & 2u) && (int)g.Z - 1 - t.z0 < C::TZ)
    gmask |= 1u << ((int)g.Z - 1 - t.z0);
  gmask = __builtin_amdgcn_readfirstlane(gmask);
  // Offsets are byte offsets of LDS words (four times the index
  // difference), relative to the plane's own column: the same seven
  // constants for every plane.  A vertex outside the domain holds NaN, so
  // it wins nothing and keeps pointing to itself.
  struct Best {
    float v;
    int o;
  };
  struct Groups {
    Best lmax, lmin, umax, umin;  // LF and UF of one plane, both directions
  };
  // The groups of box plane P (P = lz + 1 for the tile's planes); `want_l`
  // / `want_u` are compile-time after unrolling.
  auto groups = [&](int P, bool want_l, bool want_u) -> Groups {
    const int c = c0 + P * HXY;
    const float fc = __uint_as_float(lds[c]);
    Groups r;
    r.lmax = r.lmin = r.umax = r.umin = Best{fc, 0};
    if (want_l) {
      const float fxm = __uint_as_float(lds[c - 1]);
      const float fym = __uint_as_float(lds[c - HX]);
      const float fxym = __uint_as_float(lds[c - HX - 1]);
      // Challengers in decreasing id order: strict for the max, at most
      // equal for the min.
      if (fxm > r.lmax.v) r.lmax = Best{fxm, -4};
      if (fxm <= r.lmin.v) r.lmin = Best{fxm, -4};
      if (fym > r.lmax.v) r.lmax = Best{fym, -4 * HX};
      if (fym <= r.lmin.v) r.lmin = Best{fym, -4 * HX};
      if (fxym > r.lmax.v) r.lmax = Best{fxym, -4 * HX - 4};
      if (fxym <= r.lmin.v) r.lmin = Best{fxym, -4 * HX - 4};
    }
    if (want_u) {
      const float fxp = __uint_as_float(lds[c + 1]);
      const float fyp = __uint_as_float(lds[c + HX]);
      const float fxyp = __uint_as_float(lds[c + HX + 1]);
      // Challengers in increasing id order: at least equal for the max,
      // strict for the min.
      if (fxp >= r.umax.v) r.umax = Best{fxp, 4};
      if (fxp < r.umin.v) r.umin = Best{fxp, 4};
      if (fyp >= r.umax.v) r.umax = Best{fyp, 4 * HX};
      if (fyp < r.umin.v) r.umin = Best{fyp, 4 * HX};
      if (fxyp >= r.umax.v) r.umax = Best{fxyp, 4 * HX + 4};
      if (fxyp < r.umin.v) r.umin = Best{fxyp, 4 * HX + 4};
    }
    return r;
  };
  // The column's word at lz = 0; later planes are constant offsets.
  uint32_t *const own = lds + (c0 + HXY);
  // The tile's mean value orders the exit resolution (speed only, never a
  // result), so it is taken over one plane of the tile: the middle one, or
  // the last one inside the domain (block-uniform).  Read before the pointers
  // overwrite the field.
  float fsum = 0.f;
  {
    const int zs = min(C::TZ / 2, (int)g.Z - 1 - t.z0);
    if (nz > 0) fsum = __uint_as_float(own[HXY * zs]);
  }
  unsigned nmax = 0, nmin = 0;
  // Pointers wait in registers in groups of four planes: plane q's values
  // are last read in iteration q - 2, so once every thread has passed a
  // barrier after iteration lz, the words of planes up to lz + 2 are free
  // and the pointers computed so far replace their vertices' values.
  constexpr int kFlush = 4;
  static_assert(C::TZ % kFlush == 0, "tile depth");
  uint32_t ka[kFlush], kd[kFlush];
  Groups prev = groups(0, true, false);
  Groups cur = groups(1, true, true);
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz) {
    const int P = lz + 1;
    const Groups next = groups(P + 1, lz + 1 < C::TZ, true);
    // In plane P: LF then UF (ids at least as large; the two share only the
    // column's own vertex).  Then plane P-1 (smaller ids) and plane P+1
    // (larger), whose offsets move by one plane.
    Best mx = cur.lmax, mn = cur.lmin;
    if (cur.umax.v >= mx.v) mx = cur.umax;
    if (cur.umin.v < mn.v) mn = cur.umin;
    if (prev.lmax.v > mx.v) mx = Best{prev.lmax.v, prev.lmax.o - 4 * HXY};
    if (prev.lmin.v <= mn.v) mn = Best{prev.lmin.v, prev.lmin.o - 4 * HXY};
    if (next.umax.v >= mx.v) mx = Best{next.umax.v, next.umax.o + 4 * HXY};
    if (next.umin.v < mn.v) mn = Best{next.umin.v, next.umin.o + 4 * HXY};
    const uint32_t self = 4u * (uint32_t)(c0 + P * HXY);
    ka[lz % kFlush] = self + (uint32_t)mx.o;
    kd[lz % kFlush] = self + (uint32_t)mn.o + 2u;
    // Each test is one compare into a lane mask, restricted to the
    // columns that reach this plane.
    const unsigned long long inm = __builtin_amdgcn_ballot_w64(lz < nz);
    nmax += __popcll(__builtin_amdgcn_ballot_w64(mx.o == 0) & inm);
    nmin += __popcll(__builtin_amdgcn_ballot_w64(mn.o == 0) & inm);
    prev = cur;
    cur = next;
    if (lz % kFlush == kFlush - 1) {
      __syncthreads();
#pragma unroll
      for (int j = 0; j < kFlush; ++j)
        own[HXY * (lz - kFlush + 1 + j)] = ka[j] | (kd[j] << 16);
    }
    // Keep the scheduler from hoisting the next planes' work into this one
    // (register pressure).
    __builtin_amdgcn_sched_barrier(0);
  }
  if (gmask) {  // ghost vertices are fixed points (block-uniform branch)
    // The column's vertices inside the domain, as a mask of its own (the
    // steepest loop's per-plane tests would otherwise stay live until here).
    const uint32_t inmask = (1u << nz) - 1u;  // nz <= 16
    for (int lz = 0; lz < C::TZ; ++lz) {
      if ((gmask >> lz) & 1u) {
        const uint32_t self = 4u * (uint32_t)(c0 + (lz + 1) * HXY);
        const uint32_t w = own[HXY * lz];
        const bool in = (inmask >> lz) & 1u;
        nmax += __popcll(__ballot(in && (w & 0xffffu) != self));
        nmin += __popcll(__ballot(in && (w >> 16) != self + 2u));
        own[HXY * lz] = self | ((self + 2u) << 16);
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) fsum += __shfl_xor(fsum, o);
  if ((tid & 63) == 0) {
    s_wsum[tid >> 6] = fsum;
    s_wext[tid >> 6] = nmax | (nmin << 16);
  }
  __syncthreads();  // every thread is done reading the field
  if (tid < 2) {
    unsigned c = 0;
    for (int w = 0; w < T / 64; ++w) c += (s_wext[w] >> (16 * tid)) & 0xffffu;
    xo.tstat[4 * (size_t)bt.gt + tid] = c;
  } else if (tid == 64) {
    float sum = 0.f;
    for (int w = 0; w < T / 64; ++w) sum += s_wsum[w];
    const int cnt = min(C::TX, (int)g.X - t.x0) * min(C::TY, (int)g.Y - t.y0);
    xo.tkey[bt.gt] = float_key(sum / (float)cnt);
  }

  // Pointers replace the field: halo vertices point to themselves (whole
  // halo columns, and the bottom and top entries of the tile's columns).
  for (int col = tid; col < HXY; col += T) {
    const int hy = col / HX, hx = col - hy * HX;
    const bool edge = hx == 0 || hx == HX - 1 || hy == 0 || hy == C::HY - 1;
#pragma unroll
    for (int hz = 0; hz < C::HZ; ++hz) {
      if (edge || hz == 0 || hz == C::HZ - 1) {
        const uint32_t e = 4u * (uint32_t)(col + hz * HXY);
        lds[col + hz * HXY] = e | ((e + 2u) << 16);
      }
    }
  }
  __syncthreads();
  uint32_t pa[C::TZ], pd[C::TZ];
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz) {
    const uint32_t w = own[HXY * lz];
    pa[lz] = w & 0xffffu;
    pd[lz] = w >> 16;
  }

  // Pointer jumping inside the tile, in place.  Only the owner writes an
  // entry, so the owner's copy in registers is always current, and any value
  // read from another entry is an ancestor of it (a concurrent reader sees
  // the old or the new value, both on the vertex's own path).  Each round
  // gathers the successors of all the column's entries first (one wait for
  // the lot), then stores them.  Two rounds per iteration, alternating
  // between two register sets, so that no copies are needed.  A round
  // reports whether any of the wave's own entries changed.
  auto round = [&](const uint32_t (&sa)[C::TZ], const uint32_t (&sd)[C::TZ],
                   uint32_t (&da)[C::TZ], uint32_t (&dd)[C::TZ]) -> bool {
#pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz) {
      da[lz] = ld16(lb, sa[lz]);
      dd[lz] = ld16(lb, sd[lz]);
    }
    bool changed = false;
#pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz) {
      // The loaded entry as an opaque 32-bit value: keeps the compiler from
      // narrowing the pointers to 16 bits and widening them at every use.
      asm("" : "+v"(da[lz]));
      asm("" : "+v"(dd[lz]));
      changed |= (da[lz] != sa[lz]) | (dd[lz] != sd[lz]);
      own[HXY * lz] = da[lz] | (dd[lz] << 16);
    }
    return __ballot(changed) != 0ull;
  };
  {
    // Each wave jumps until its own entries are final, with no barrier
    // between rounds: a round that changes none of them leaves every one
    // naming a fixed point, which no later write changes, whatever the other
    // waves have stored so far.  A wave that is done leaves its SIMD to the
    // others until the block meets at the barrier.  Doubling settles within
    // about log2(H) + 1 rounds; the bound only turns a broken invariant into
    // an error (counter bit 2) instead of a hang.
    constexpr int kMaxPairs = 64;
    uint32_t qa[C::TZ], qd[C::TZ];
    bool open = true;
    for (int it = 0; it < kMaxPairs; ++it) {
      if (!round(pa, pd, qa, qd)) {
#pragma unroll
        for (int lz = 0; lz < C::TZ; ++lz) {
          pa[lz] = qa[lz];
          pd[lz] = qd[lz];
        }
        open = false;
        break;
      }
      if (!round(qa, qd, pa, pd)) {
        open = false;
        break;
      }
    }
    if (__syncthreads_or(open) && tid == 0) atomicOr(ctr + kCtrOverflow, 4ull);
  }

  // Every pointer is final: it names an extremum of the tile or a halo
  // vertex (an exit), both fixed points.  Each vertex marks its two targets'
  // halves; then every owner overwrites its own word with its stored code in
  // both halves, so that afterwards exactly the halo halves that are some
  // vertex's target hold the mark.  Entries that are nobody's target are
  // never read again.
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz) {
    st16(lb, pa[lz], kMark);
    st16(lb, pd[lz], kMark);
  }
  __syncthreads();
  {
    const uint32_t code0 = (uint32_t)(cx + C::TX * cy);
#pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz) {
      const uint32_t code = code0 + (uint32_t)(C::TXY * lz);
      own[HXY * lz] = code | (code << 16);
    }
  }
  __syncthreads();

  // Marked halves become exit codes.  Only halo entries can hold the mark,
  // so only the halo is walked: halo entry i (halo_index, increasing in p)
  // goes to thread i % T in round i / T.  Exits are numbered per direction
  // in increasing p; that is the order of (round, wave, lane), so a marked
  // entry's number is the count of marked entries of earlier (round, wave)
  // pairs, scanned once, plus the marked lanes below it in its wave.
  constexpr int KH = (C::kHalo + T - 1) / T, NW = T / 64;
  // Up to six rounds keep their halo indices and marks in registers for the
  // second loop; more would spill, so those are taken again (each entry
  // belongs to one thread, which reads it before rewriting it).
  constexpr bool kKeep = KH <= 6;
  const int lane = tid & 63, wv = tid >> 6;
  int hp[KH];
  bool am[KH], dm[KH];
  unsigned long long bma[KH], bmd[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) {
    const int i = tid + k * T;
    const bool ok = (k + 1) * T <= C::kHalo || i < C::kHalo;
    hp[k] = halo_index<C>(ok ? i : 0);
    const uint32_t e = lds[hp[k]];
    am[k] = ok && (e & 0xffffu) == kMark;
    dm[k] = ok && (e >> 16) == kMark;
    bma[k] = __ballot(am[k]);
    bmd[k] = __ballot(dm[k]);
    if (lane == 0)
      s_cnt[k * NW + wv] = (uint32_t)__popcll(bma[k]) |
                           ((uint32_t)__popcll(bmd[k]) << 16);
  }
  __syncthreads();
  if (tid < 64) {  // exclusive scan of the (round, wave) counts
    const uint32_t x = tid < KH * NW ? s_cnt[tid] : 0u;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    if (tid < KH * NW) s_cnt[tid] = inc - x;
    if (tid == 63) s_cnt[KH * NW] = inc;
  }
  __syncthreads();
  const uint32_t tot = s_cnt[KH * NW];
  const uint32_t na = tot & 0xffffu, nd = tot >> 16;
  {
    // Every halo entry's word gets both codes: a half that is nobody's
    // target is never read again.  The list gets each exit's index; the
    // stores of unmarked halves go to slot na + nd, which no exit uses (an
    // unmarked half means fewer than 2 * kHalo exits) and nothing reads.
    uint16_t *tl = xo.tlist + (size_t)bt.gt * (2 * C::kHalo);
    const uint32_t trash = na + nd;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int i = tid + k * T;
      const bool ok = (k + 1) * T <= C::kHalo || i < C::kHalo;
      const uint32_t base = s_cnt[k * NW + wv];
      const uint32_t ra = (base & 0xffffu) + lanes_below(bma[k]);
      const uint32_t rd = (base >> 16) + lanes_below(bmd[k]);
      if (ok) {
        int p = hp[k];
        bool ah = am[k], dh = dm[k];
        if (!kKeep) {
          p = halo_index<C>(i);
          const uint32_t e = lds[p];
          ah = (e & 0xffffu) == kMark;
          dh = (e >> 16) == kMark;
        }
        lds[p] = (kExitCode | ra) | ((kExitCode | rd) << 16);
        tl[ah ? ra : trash] = (uint16_t)p;
        tl[dh ? na + rd : trash] = (uint16_t)p;
      }
    }
  }
  __syncthreads();

  // The stored local pointer of every vertex is its target's code: an
  // owned target by its owned index, an exit by its number (bit 15 set), so
  // that later passes decode it with one lookup in the tile's resolved exits.
  // The first and last columns also go to the tile's shell copy (a
  // block-uniform base and a 32-bit offset per lane).
  const bool xedge = cx == 0 || cx == C::TX - 1;
  __attribute__((address_space(1))) uint32_t *const xsb =
      (__attribute__((address_space(1))) uint32_t *)xo.xs +
      shell_word<C>(bt.gt, 0u, 0u, 0u);
  const uint32_t xso = (cx == 0 ? 0u : (uint32_t)(C::TZ * C::TY)) + (uint32_t)cy;
  __attribute__((address_space(1))) uint32_t *const lpt =
      (__attribute__((address_space(1))) uint32_t *)bt.fd.lp +
      code_word<C>(bt.gt, 0, 0);
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz)
    lpt[(uint32_t)(lz * C::kThreads + tid)] =
        ld16(lb, pa[lz]) | (ld16(lb, pd[lz]) << 16);
  if (xedge) {
#pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz) {
      if (lz < nz)
        xsb[xso + (uint32_t)(lz * C::TY)] =
            ld16(lb, pa[lz]) | (ld16(lb, pd[lz]) << 16);
    }
  }
  if (tid == 0) {
    xo.seg[bt.gt] =
        Seg{bt.gt * (uint32_t)(2 * C::kHalo), (uint16_t)na, (uint16_t)nd};
    xo.tstat[4 * (size_t)bt.gt + 3] = na + nd;
  }
}

// ---------------------------------------------------------------------------
// exit graph
// ---------------------------------------------------------------------------

// Exit i (the k-th exit of its tile) lies on the shell of a neighbouring
// tile, whose stored code for it names either an extremum of that tile
// (final) or one of that tile's exits (the next node of the graph).  Nodes
// are numbered by list position, so the graph is a dense array: next[i] is a
// node index, or kRoot | vertex id once final.
constexpr uint32_t kRoot = 0x80000000u;

template <class C>
__device__ __forceinline__ Tile tile_of_vertex(const Geo &g, uint32_t v,
                                               uint32_t *tile) {
  uint32_t z = v / g.XY, r = v - z * g.XY, y = r / g.X, x = r - y * g.X;
  uint32_t tx = x / C::TX, ty = y / C::TY, tz = z / C::TZ;
  *tile = tx + g.ntx * (ty + g.nty * tz);
  return Tile{(int)(tx * C::TX), (int)(ty * C::TY), (int)(tz * C::TZ)};
}

// One block per tile links the tile's exits: exit k is the halo vertex v at
// tile-plus-halo index tlist[k]; its successor is the code that v's owner
// tile (a face, edge or corner neighbour, found from the index) stored for
// v -- an extremum of that tile (final) or one of that tile's exits (the
// next node of the graph).
template <class C>
__global__ void __launch_bounds__(kBlock)
k_exit_link(const FieldDev *__restrict__ fds,
            const uint32_t *__restrict__ tfield, const Seg *__restrict__ seg,
            const uint16_t *__restrict__ tlist,
            const uint32_t *__restrict__ xs, uint32_t *__restrict__ next) {
  const BlockTile bt = block_tile(fds, tfield);
  const Seg sg = seg[bt.gt];
  const uint32_t n = (uint32_t)sg.na + sg.nd;
  const uint16_t *tl = tlist + (size_t)bt.gt * (2 * C::kHalo);
  const Geo &g = bt.fd.g;
  const Tile t = tile_at<C>(g, bt.tile);
  const int ttx = t.x0 / C::TX, tty = t.y0 / C::TY, ttz = t.z0 / C::TZ;
  // Each thread links E exits per round, with each kind of load issued for
  // all of them before any is used (list entries, then the neighbours'
  // codes, then the slot records the descent exits need).
  constexpr int E = 4;
  for (uint32_t k0 = threadIdx.x; k0 < n; k0 += E * kBlock) {
    int p[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t k = k0 + e * kBlock;
      p[e] = k < n ? (int)tl[k] : -1;
    }
    uint32_t u[E], lw[E];
    const uint32_t *src[E];
    int dxs[E], dys[E], dzs[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = p[e] < 0 ? 0 : p[e];
      const int hz = q / C::HXY, r = q - hz * C::HXY, hy = r / C::HX,
                hx = r - hy * C::HX;
      dxs[e] = hx == 0 ? -1 : (hx == C::HX - 1 ? 1 : 0);
      dys[e] = hy == 0 ? -1 : (hy == C::HY - 1 ? 1 : 0);
      dzs[e] = hz == 0 ? -1 : (hz == C::HZ - 1 ? 1 : 0);
      u[e] = (uint32_t)(ttx + dxs[e]) +
             g.ntx * ((uint32_t)(tty + dys[e]) + g.nty * (uint32_t)(ttz + dzs[e]));
      // The exit's position in the owner tile; an exit on an x face lies in
      // the owner's last (dx = -1) or first (dx = +1) column and is read
      // from that tile's shell copy.
      const uint32_t ou = bt.fd.tile0 + u[e];
      const int lx = hx - 1 - dxs[e] * C::TX, ly = hy - 1 - dys[e] * C::TY,
                lzo = hz - 1 - dzs[e] * C::TZ;
      src[e] = dxs[e] != 0
                   ? xs + shell_word<C>(ou, dxs[e] < 0 ? 1u : 0u,
                                        (uint32_t)lzo, (uint32_t)ly)
                   : bt.fd.lp + code_word<C>(ou, lzo, lx + C::TX * ly);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) lw[e] = p[e] >= 0 ? *src[e] : 0u;
    uint32_t code[E], una[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const bool desc = k0 + e * kBlock >= sg.na;
      code[e] = desc ? (lw[e] >> 16) : (lw[e] & 0xffffu);
      // A tile's slots start at tile * 2 * kHalo; a descent exit's number
      // counts from after that tile's ascent exits.
      una[e] = p[e] >= 0 && desc && (code[e] & kExitCode)
                   ? (uint32_t)seg[bt.fd.tile0 + u[e]].na
                   : 0u;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (p[e] < 0) continue;
      const uint32_t k = k0 + e * kBlock;
      if (code[e] & kExitCode) {
        next[sg.base + k] = (bt.fd.tile0 + u[e]) * (uint32_t)(2 * C::kHalo) +
                            una[e] + (code[e] & (kExitCode - 1));
      } else {
        const Tile tu{t.x0 + dxs[e] * C::TX, t.y0 + dys[e] * C::TY,
                      t.z0 + dzs[e] * C::TZ};
        next[sg.base + k] = kRoot | owned_global<C>(g, tu, code[e]);
      }
    }
  }
}

// Tiles are resolved in order of their mean value: ascent chains climb, so
// a tile's ascent exits mostly lead into tiles of higher mean that were
// resolved just before (their graph segments are still in cache); descent
// runs the other way.  The order only affects speed: every chase follows
// its own path to a final value, whatever has been resolved already.
constexpr int kTileBuckets = 4096;

// The ordering kernels run 1024-thread blocks and fold per block in LDS
// first: tile means crowd into a few buckets, and global atomics on one
// address serialise across the chip.
constexpr int kOrderBlock = 1024;

inline unsigned order_grid(uint32_t n) {
  return (n + kOrderBlock - 1) / kOrderBlock;
}

__global__ void __launch_bounds__(kOrderBlock)
k_key_minmax(const uint32_t *__restrict__ key, uint32_t n, uint32_t *mm) {
  __shared__ uint32_t s_lo[kOrderBlock / 64], s_hi[kOrderBlock / 64];
  const uint32_t i = blockIdx.x * kOrderBlock + threadIdx.x;
  uint32_t lo = ~0u, hi = 0;
  if (i < n) lo = hi = key[i];
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t a = __shfl_xor(lo, o), b = __shfl_xor(hi, o);
    lo = a < lo ? a : lo;
    hi = b > hi ? b : hi;
  }
  if ((threadIdx.x & 63) == 0) {
    s_lo[threadIdx.x >> 6] = lo;
    s_hi[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kOrderBlock / 64; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    if (lo <= hi) {
      atomicMin(&mm[0], lo);
      atomicMax(&mm[1], hi);
    }
  }
}

__device__ __forceinline__ uint32_t key_bucket(uint32_t key,
                                               const uint32_t *mm) {
  const uint64_t span = (uint64_t)mm[1] - mm[0] + 1;
  const uint64_t b = ((uint64_t)(key - mm[0]) * kTileBuckets) / span;
  return b < kTileBuckets ? (uint32_t)b : kTileBuckets - 1;
}

__global__ void __launch_bounds__(kOrderBlock)
k_key_hist(const uint32_t *__restrict__ key, uint32_t n,
           const uint32_t *__restrict__ mm, uint32_t *hist) {
  __shared__ uint32_t cnt[kTileBuckets];
  for (int b = threadIdx.x; b < kTileBuckets; b += kOrderBlock) cnt[b] = 0;
  __syncthreads();
  const uint32_t i = blockIdx.x * kOrderBlock + threadIdx.x;
  if (i < n) atomicAdd(&cnt[key_bucket(key[i], mm)], 1u);
  __syncthreads();
  for (int b = threadIdx.x; b < kTileBuckets; b += kOrderBlock)
    if (cnt[b]) atomicAdd(&hist[b], cnt[b]);
}

// Exclusive scan of kTileBuckets counts in place (one block of 1024
// threads, four counts each).
__global__ void __launch_bounds__(1024) k_key_scan(uint32_t *hist) {
  __shared__ uint32_t tmp[32];
  const int b0 = threadIdx.x * 4;
  const uint32_t c0 = hist[b0], c1 = hist[b0 + 1], c2 = hist[b0 + 2],
                 c3 = hist[b0 + 3];
  uint32_t total;
  const uint32_t p = block_exclusive_scan(c0 + c1 + c2 + c3, tmp, &total);
  hist[b0] = p;
  hist[b0 + 1] = p + c0;
  hist[b0 + 2] = p + c0 + c1;
  hist[b0 + 3] = p + c0 + c1 + c2;
}

// The tiles' exit records in that order (the resolution reads its tile's
// record with one load).  A tile's place: its block's share of its bucket
// (one global atomic per bucket and block), then its rank in that share.
__global__ void __launch_bounds__(kOrderBlock)
k_key_scatter(const uint32_t *__restrict__ key, uint32_t n,
              const uint32_t *__restrict__ mm, uint32_t *cursor,
              const Seg *__restrict__ seg, Seg *__restrict__ oseg) {
  __shared__ uint32_t cnt[kTileBuckets];
  for (int b = threadIdx.x; b < kTileBuckets; b += kOrderBlock) cnt[b] = 0;
  __syncthreads();
  const uint32_t i = blockIdx.x * kOrderBlock + threadIdx.x;
  const bool in = i < n;
  const uint32_t b = in ? key_bucket(key[i], mm) : 0u;
  const uint32_t r = in ? atomicAdd(&cnt[b], 1u) : 0u;
  __syncthreads();
  for (int k = threadIdx.x; k < kTileBuckets; k += kOrderBlock)
    if (cnt[k]) cnt[k] = atomicAdd(&cursor[k], cnt[k]);
  __syncthreads();
  if (in) oseg[cnt[b] + r] = seg[i];
}

// Block b resolves one tile's exits of one direction: the first ntiles
// blocks take ascent exits in decreasing mean, the rest descent exits in
// increasing mean.  Each exit chases its successors until a final value.
// Values other blocks write are read and written at device scope, so that
// a chase can stop at an exit another tile has already resolved; whatever
// it reads (a link or a final value) lies on its own path.
constexpr int kResolveThreads = 256;
constexpr int kResolveE = 4;  // exits chased side by side per thread

__device__ __forceinline__ uint32_t load_dev(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kResolveThreads)
k_exit_resolve(const Seg *__restrict__ oseg, uint32_t ntiles, uint32_t count,
               uint32_t *next, unsigned long long *ctr,
               unsigned long long *rstat) {
  constexpr int T = kResolveThreads, E = kResolveE;
  __shared__ unsigned long long s_red[2][T / 64];
  const bool desc = blockIdx.x >= ntiles;
  const Seg sg =
      desc ? oseg[blockIdx.x - ntiles] : oseg[ntiles - 1 - blockIdx.x];
  const uint32_t first = sg.base + (desc ? sg.na : 0u);
  const uint32_t cnt = desc ? sg.nd : sg.na;
  unsigned steps_max = 0, steps_sum = 0;
  bool bad = false;
  for (uint32_t k0 = threadIdx.x; k0 < cnt; k0 += E * T) {
    // Every load of a round is issued before any is used: indices out of
    // range, or of chases already final, read the thread's first slot.
    uint32_t x[E];
    unsigned st[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t k = k0 + (uint32_t)(e * T);
      x[e] = next[first + (k < cnt ? k : k0)];
      st[e] = 0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (k0 + (uint32_t)(e * T) >= cnt) x[e] = kRoot;
    // Chains are acyclic and at most `count` long; the bound only turns a
    // broken invariant into an error instead of a hang.
    bool open = true;
    while (open) {
      uint32_t y[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const bool go = !(x[e] & kRoot) && x[e] < count;
        y[e] = load_dev(next + (go ? x[e] : first + k0));
      }
      open = false;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (!(x[e] & kRoot)) {
          if (x[e] >= count || ++st[e] > count) {
            bad = true;
            x[e] = kRoot;
          } else {
            x[e] = y[e];
          }
        }
        open |= !(x[e] & kRoot);
      }
    }
    unsigned sm = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t k = k0 + (uint32_t)(e * T);
      if (k < cnt)
        __hip_atomic_store(next + first + k, x[e], __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      sm = st[e] > sm ? st[e] : sm;
      steps_sum += st[e];
    }
    steps_max = sm > steps_max ? sm : steps_max;
  }
  if (bad) atomicOr(ctr + kCtrOverflow, 2ull);
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned other = __shfl_xor(steps_max, o);
    steps_max = other > steps_max ? other : steps_max;
    steps_sum += __shfl_xor(steps_sum, o);
  }
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = steps_max;
    s_red[1][threadIdx.x >> 6] = steps_sum;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long mx = 0, sum = 0;
    for (int w = 0; w < T / 64; ++w) {
      mx = s_red[0][w] > mx ? s_red[0][w] : mx;
      sum += s_red[1][w];
    }
    rstat[2 * (size_t)blockIdx.x] = mx;
    rstat[2 * (size_t)blockIdx.x + 1] = sum;
  }
}

// ---------------------------------------------------------------------------
// pairs and output
// ---------------------------------------------------------------------------

// A tile's decode table, staged in LDS: its resolved exits (ascent exits
// first, then descent) and, after them, the id offset X*ly + X*Y*lz of each
// row (ly, lz) of the tile, so that either reading of a stored code is one
// LDS read and an add (no 32-bit multiplies per vertex).
template <class C>
struct Decode {
  static constexpr int kRows = 2 * C::kHalo;
  int32_t tab[2 * C::kHalo + C::TY * C::TZ];
  uint32_t na;
  uint32_t base;  // id of the tile's first vertex
};

template <class C>
__device__ __forceinline__ void decode_setup(Decode<C> &s, uint32_t gt,
                                             const Seg *seg, const uint32_t *R,
                                             const Geo &g, const Tile &t) {
  const Seg sg = seg[gt];
  const uint32_t n = (uint32_t)sg.na + sg.nd;
  // Four resolved exits per thread and round, their loads in flight
  // together (indices past the tile's exits read its first slot, so that no
  // load sits in a branch of its own).  The first round, all that most
  // tiles need, stands outside the loop, so that its loads do not wait for
  // the caller's loads still in flight.
  constexpr uint32_t E = 4;
  auto round = [&](uint32_t k0) {
    uint32_t r[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t k = k0 + e * C::kThreads;
      r[e] = R[sg.base + (k < n ? k : 0u)];
    }
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t k = k0 + e * C::kThreads;
      if (k < n) s.tab[k] = (int32_t)(r[e] & ~kRoot);
    }
  };
  round(threadIdx.x);
  for (uint32_t k0 = threadIdx.x + E * C::kThreads; k0 < n;
       k0 += E * C::kThreads)
    round(k0);
  for (uint32_t r = threadIdx.x; r < (uint32_t)(C::TY * C::TZ);
       r += C::kThreads)
    s.tab[Decode<C>::kRows + r] =
        (int32_t)(g.X * (r % C::TY) + g.XY * (r / C::TY));
  if (threadIdx.x == 0) {
    s.na = sg.na;
    s.base = (uint32_t)t.x0 + g.X * (uint32_t)t.y0 + g.XY * (uint32_t)t.z0;
  }
  __syncthreads();
}

// Final extremum of a stored local pointer code, without branches (this is
// unrolled over a whole column): an exit reads its resolved extremum, an
// owned code its row offset, from the one table.
template <class C>
__device__ __forceinline__ int32_t decode_final(const Decode<C> &s,
                                                uint32_t code, bool desc) {
  static_assert((C::TX & (C::TX - 1)) == 0, "power-of-two tile width");
  const bool ex = (code & kExitCode) != 0u;
  const uint32_t low = code & (kExitCode - 1);
  const int32_t v = s.tab[ex ? (desc ? s.na : 0u) + low
                             : Decode<C>::kRows + low / C::TX];
  return ex ? v : (int32_t)(s.base + low % C::TX + (uint32_t)v);
}

__global__ void k_table_clear(unsigned long long *keys, int32_t *vals,
                              uint64_t cap) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < cap) {
    keys[i] = kEmptyKey;
    vals[i] = INT32_MAX;
  }
}

// Linear probing gives up after kTableProbes slots: an insert that finds no
// room reports an overflow (the host then grows the table and runs the pair
// pass again), and a lookup stops there too, since every key sits within
// that many slots of its hash.
constexpr uint32_t kTableProbes = 512;

// Insert (key, id) keeping the smallest id; reads before each atomic so that
// the common case (key present with a smaller id) stays a plain load.
// *at gets the key's slot when given.
__device__ __forceinline__ bool table_insert(unsigned long long *keys,
                                             int32_t *vals, uint32_t mask,
                                             unsigned long long key,
                                             int32_t id, unsigned *fresh,
                                             uint32_t *at = nullptr) {
  uint32_t h = (uint32_t)mix64(key) & mask;
#pragma unroll 1
  for (uint32_t probe = 0; probe <= mask && probe < kTableProbes; ++probe) {
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
      if (at) *at = h;
      return true;
    }
    h = (h + 1) & mask;
  }
  return false;
}

__device__ __forceinline__ unsigned long long pair_key(int32_t a, int32_t d) {
  return ((unsigned long long)(uint32_t)a << 32) | (uint32_t)d;
}

// Per-tile table of the distinct final (asc, desc) pairs: in smooth regions
// a tile holds few, so the global insert and the cell lookup run once per
// distinct pair.  Noise-dominated tiles hold thousands (a cell of pure noise
// has about three vertices); once half the slots are taken the table accepts
// no new pair, probes stay short, and the remaining vertices take the
// per-vertex path.  Linear probing without deletion: a pair that is in the
// table is found before any empty slot.  A lane consults the table only when
// its column's pair changes from one z to the next (a repeated pair has a
// larger id than the one already recorded), which in smooth regions is once
// or twice per column; concurrent inserts of one pair meet in one slot
// through the compare-and-swap.
constexpr int kPairSlots = 1024;
constexpr unsigned kPairLimit = kPairSlots / 2;
constexpr int kPairProbes = 16;

// A pair's first claim takes the next dense number (the fill count before
// it) into dense[slot], when given.
__device__ __forceinline__ int pair_slot(unsigned long long *skey,
                                         unsigned *fill,
                                         unsigned long long key,
                                         uint16_t *dense = nullptr) {
  // The slot is local to the tile, so a multiply-free hash of the two
  // labels serves (the global table keeps its 64-bit mix).
  const uint32_t a = (uint32_t)(key >> 32), d = (uint32_t)key;
  uint32_t h = (a ^ (a >> 10) ^ (d << 3) ^ (d >> 7)) & (kPairSlots - 1);
#pragma unroll 1
  for (int probe = 0; probe < kPairProbes; ++probe) {
    unsigned long long cur = skey[h];
    if (cur == kEmptyKey) {
      if (*fill >= kPairLimit) return -1;
      cur = atomicCAS(&skey[h], kEmptyKey, key);
      if (cur == kEmptyKey) {
        const unsigned k = atomicAdd(fill, 1u);
        if (dense) dense[h] = (uint16_t)k;
        return (int)h;
      }
    }
    if (cur == key) return (int)h;
    h = (h + 1) & (kPairSlots - 1);
  }
  return -1;
}

__device__ __forceinline__ int32_t table_lookup(
    const unsigned long long *__restrict__ keys,
    const int32_t *__restrict__ vals, uint32_t mask, unsigned long long key) {
  uint32_t h = (uint32_t)mix64(key) & mask;
#pragma unroll 1
  for (uint32_t probe = 0; probe <= mask && probe < kTableProbes; ++probe) {
    const unsigned long long cur = keys[h];
    if (cur == key) return vals[h];
    if (cur == kEmptyKey) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

// A tile whose vertices carry at most kCellIdx distinct pairs gets one byte
// per vertex, the pair's dense number within the tile (tile-major, four
// planes per word), and a record in its exit-list slots, which nothing reads
// once the exits are linked: the number of pairs, then the slot of each in
// the field's table.  The output pass then reads that byte instead of the
// codes and needs no decoding; a tile with one pair needs no bytes at all.
// Record 0 marks a tile that kept the per-vertex path.
constexpr unsigned kCellIdx = 255;

template <class C>
__device__ __forceinline__ uint32_t *cell_record(uint16_t *tlist,
                                                 uint32_t gt) {
  static_assert(kCellIdx + 1 <= (unsigned)C::kHalo, "record fits the slots");
  return reinterpret_cast<uint32_t *>(tlist + (size_t)gt * (2 * C::kHalo));
}

template <class C>
__device__ __forceinline__ size_t cell_word(uint32_t gt, int j, int tid) {
  return ((size_t)gt * (C::TZ / 4) + (size_t)j) * C::kThreads + (size_t)tid;
}

// Waves per SIMD that the pair pass's LDS (its decode and pair tables,
// about 14 KB besides the decode table) leaves room for, at most 8; the
// register budget is held to match (8 waves: 64 VGPRs).
template <class C>
constexpr int pair_waves() {
  constexpr int lds = 4 * (2 * C::kHalo + C::TY * C::TZ) + 14 * 1024 + 256;
  constexpr int w = (160 * 1024 / lds) * (C::kThreads / 64) / 4;
  return w < 8 ? w : 8;
}

template <class C>
__global__ void __launch_bounds__(C::kThreads)
__attribute__((amdgpu_waves_per_eu(pair_waves<C>(), pair_waves<C>())))
k_tile_pairs(const FieldDev *__restrict__ fds,
             const uint32_t *__restrict__ tfield, const Seg *__restrict__ seg,
             const uint32_t *__restrict__ R, unsigned long long *ctr,
             uint32_t *tstat, uint32_t ntiles, const uint32_t *run,
             uint16_t *tlist, uint32_t *cidx) {
  static_assert(C::TZ % 4 == 0, "four planes per index word");
  __shared__ Decode<C> s;
  __shared__ uint32_t s_fresh[C::kThreads / 64];
  __shared__ unsigned long long skey[kPairSlots];
  __shared__ int32_t sval[kPairSlots];
  __shared__ uint16_t sdense[kPairSlots];
  __shared__ unsigned sfill;
  const int tid = threadIdx.x;
  // The second pass (after an overflow) runs only when *run is set, over a
  // smaller grid that strides through the tiles.
  if (run && !*run) return;
  for (uint32_t blk = blockIdx.x; blk < ntiles; blk += gridDim.x) {
    const BlockTile bt = block_tile_at(fds, tfield, blk, ntiles);
    if (!bt.fd.ms) continue;  // uniform over the block
    const Geo &g = bt.fd.g;
    const Tile t = tile_at<C>(g, bt.tile);
    for (int i = tid; i < kPairSlots; i += C::kThreads) {
      skey[i] = kEmptyKey;
      sval[i] = INT32_MAX;
    }
    if (tid == 0) sfill = 0;
    const int cx = tid % C::TX, cy = tid / C::TX;
    const int gx = t.x0 + cx, gy = t.y0 + cy;
    const bool col_in = gx < (int)g.X && gy < (int)g.Y;
    int nz = (int)g.Z - t.z0;
    nz = col_in ? (nz < C::TZ ? nz : C::TZ) : 0;
    // Column offset within a plane; plane bases are uniform over the block.
    const uint32_t col = (uint32_t)gx + g.X * (uint32_t)gy;
    uint32_t code[C::TZ];
  #pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz)
      code[lz] = bt.fd.lp[code_word<C>(bt.gt, lz, tid)];
    decode_setup<C>(s, bt.gt, seg, R, g, t);

    unsigned fresh = 0;
    bool overflow = false, lost = false;
    // Every run of equal pairs down a column finds its slot in the tile's
    // table (two 16-bit slots per word).  Only the smallest id of each pair
    // matters: a vertex whose pair equals that of the vertex below it
    // (previous z of the column) or of the lane before it (a smaller id in
    // the same plane) is not that smallest id and inserts nothing; the
    // smallest one matches neither, so it is never skipped.
    const bool first_lane = (tid & 63) == 0;
    unsigned long long last = kEmptyKey;
    int last_slot = -1;
    uint32_t sp[C::TZ / 2];
  #pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz) {
      const bool in = lz < nz;
      unsigned long long key = kEmptyKey;
      if (in) {
        // The final labels are written here, where the pass is bound by its
        // arithmetic and the stores overlap it; the output pass then writes
        // only the cell ids.
        const int32_t a = decode_final<C>(s, code[lz] & 0xffffu, false);
        const int32_t d = decode_final<C>(s, code[lz] >> 16, true);
        // Only the labels the caller wants (block-uniform tests).
        if (bt.fd.A) plane_ptr(bt.fd.A, g, t.z0 + lz)[col] = a;
        if (bt.fd.D) plane_ptr(bt.fd.D, g, t.z0 + lz)[col] = d;
        key = pair_key(a, d);
      }
      if (in && key != last) {
        last_slot = pair_slot(skey, &sfill, key, sdense);
        lost |= last_slot < 0;
      }
      const unsigned long long left = __shfl_up(key, 1);
      const bool repeat = key == last || (!first_lane && key == left);
      last = key;
      const uint32_t s16 = (uint32_t)last_slot & 0xffffu;
      sp[lz / 2] = (lz & 1) ? (sp[lz / 2] | (s16 << 16)) : s16;
      if (!repeat && in) {
        const int32_t id = (int32_t)(col + g.XY * (uint32_t)(t.z0 + lz));
        if (last_slot >= 0)
          atomicMin(&sval[last_slot], id);
        else if (!table_insert(bt.fd.keys, bt.fd.vals, bt.fd.mask, key, id,
                               &fresh))
          overflow = true;
      }
    }
    // Block-uniform from here: the tile keeps the byte path when every
    // vertex found a slot and few enough pairs were claimed.
    const bool any_lost = __syncthreads_or(lost);
    const unsigned n = sfill;
    const bool indexed = !any_lost && n <= kCellIdx;
    uint32_t *rec = cell_record<C>(tlist, bt.gt);
    for (int i = tid; i < kPairSlots; i += C::kThreads) {
      if (skey[i] != kEmptyKey) {
        uint32_t at = 0;
        if (!table_insert(bt.fd.keys, bt.fd.vals, bt.fd.mask, skey[i], sval[i],
                          &fresh, &at))
          overflow = true;
        else if (indexed)
          rec[1 + sdense[i]] = at;
      }
    }
    if (tid == 0) rec[0] = indexed ? n : 0u;
    if (indexed && n > 1) {
  #pragma unroll
      for (int j = 0; j < C::TZ / 4; ++j) {
        uint32_t w = 0;
  #pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int lz = 4 * j + b;
          const uint32_t sl = (sp[lz / 2] >> (16 * (lz & 1))) & 0xffffu;
          if (lz < nz) w |= (uint32_t)sdense[sl] << (8 * b);
        }
        cidx[cell_word<C>(bt.gt, j, tid)] = w;
      }
    }
    // New pairs this tile inserted: summed per tile, folded per field later.
    for (int o = 32; o > 0; o >>= 1) fresh += __shfl_xor(fresh, o);
    if ((tid & 63) == 0) s_fresh[tid >> 6] = fresh;
    __syncthreads();
    if (tid == 0) {
      uint32_t c = 0;
      for (int w = 0; w < C::kThreads / 64; ++w) c += s_fresh[w];
      tstat[4 * (size_t)bt.gt + 2] = c;
    }
    if (overflow) atomicOr(ctr + kCtrOverflow, 1ull);
    __syncthreads();  // the LDS tables are cleared for the next tile
  }
}

template <class C>
__global__ void __launch_bounds__(C::kThreads)
k_tile_write(const FieldDev *__restrict__ fds,
             const uint32_t *__restrict__ tfield, const Seg *__restrict__ seg,
             const uint32_t *__restrict__ R, uint16_t *tlist,
             const uint32_t *__restrict__ cidx) {
  __shared__ Decode<C> s;
  __shared__ unsigned long long skey[kPairSlots];
  __shared__ int32_t scell[kPairSlots];
  __shared__ unsigned sfill;
  static_assert(kCellIdx <= (unsigned)C::kThreads, "a slot per thread");
  const int tid = threadIdx.x;
  // The tile's cell record needs only the tile index, so its count and
  // every slot it can hold (the record spans kHalo words) are loaded first,
  // together with the tile's descriptors; the cell ids and the bytes follow
  // in one more round trip.
  const uint32_t *rec =
      cell_record<C>(tlist, tile_of_block(blockIdx.x, gridDim.x));
  const uint32_t r0 = rec[0];
  const uint32_t rk = rec[1 + ((unsigned)tid < kCellIdx ? tid : 0)];
  const BlockTile bt = block_tile(fds, tfield);
  const Geo &g = bt.fd.g;
  int32_t *__restrict__ A = bt.fd.A;
  int32_t *__restrict__ D = bt.fd.D;
  int32_t *__restrict__ ms = bt.fd.ms;
  const Tile t = tile_at<C>(g, bt.tile);
  const int cx = tid % C::TX, cy = tid / C::TX;
  const int gx = t.x0 + cx, gy = t.y0 + cy;
  const bool col_in = gx < (int)g.X && gy < (int)g.Y;
  int nz = (int)g.Z - t.z0;
  nz = col_in ? (nz < C::TZ ? nz : C::TZ) : 0;
  const uint32_t col = (uint32_t)gx + g.X * (uint32_t)gy;
  // Block-uniform: the byte path when the field wants cells and the tile
  // kept one.
  const uint32_t n = __builtin_amdgcn_readfirstlane(ms ? r0 : 0u);
  const uint32_t cslot = (uint32_t)tid < n ? rk : 0u;
  if (n > 0) {  // each vertex's pair number in the tile
    uint32_t w[C::TZ / 4];
#pragma unroll
    for (int j = 0; j < C::TZ / 4; ++j)
      w[j] = n > 1 ? cidx[cell_word<C>(bt.gt, j, tid)] : 0u;
    const int32_t cell = bt.fd.vals[cslot];
    if ((uint32_t)tid < n) scell[tid] = cell;
    __syncthreads();
#pragma unroll
    for (int lz = 0; lz < C::TZ; ++lz)
      if (lz < nz)
        plane_ptr(ms, g, t.z0 + lz)[col] =
            scell[(w[lz / 4] >> (8 * (lz % 4))) & 0xffu];
    return;
  }
  if (ms) {  // uniform over the block: ms belongs to the field
    for (int i = tid; i < kPairSlots; i += C::kThreads) skey[i] = kEmptyKey;
  }
  if (tid == 0) sfill = 0;
  uint32_t code[C::TZ];
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz)
    code[lz] = bt.fd.lp[code_word<C>(bt.gt, lz, tid)];
  decode_setup<C>(s, bt.gt, seg, R, g, t);

  int16_t slot[C::TZ];
  // The slot (or, off the table, the cell) of the column's previous pair.
  unsigned long long last = kEmptyKey;
  int last_slot = -1;
  int32_t last_cell = -1;
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz) {
    const bool in = lz < nz;
    int32_t a = 0, d = 0;
    if (in) {
      a = decode_final<C>(s, code[lz] & 0xffffu, false);
      d = decode_final<C>(s, code[lz] >> 16, true);
      if (!ms) {  // with cells, the pair pass has written the labels
        if (A) plane_ptr(A, g, t.z0 + lz)[col] = a;
        if (D) plane_ptr(D, g, t.z0 + lz)[col] = d;
      }
    }
    slot[lz] = -1;
    if (ms) {  // uniform over the block: ms belongs to the field
      const unsigned long long key = pair_key(a, d);
      if (in && key != last) {
        last = key;
        last_slot = pair_slot(skey, &sfill, key);
        if (last_slot < 0)  // not in the tile's table: look this pair up alone
          last_cell = table_lookup(bt.fd.keys, bt.fd.vals, bt.fd.mask, key);
      }
      if (in) {
        slot[lz] = (int16_t)last_slot;
        if (last_slot < 0) plane_ptr(ms, g, t.z0 + lz)[col] = last_cell;
      }
    }
  }
  if (!ms) return;  // uniform over the block: ms belongs to the field
  __syncthreads();
  for (int i = tid; i < kPairSlots; i += C::kThreads)
    if (skey[i] != kEmptyKey)
      scell[i] = table_lookup(bt.fd.keys, bt.fd.vals, bt.fd.mask, skey[i]);
  __syncthreads();
#pragma unroll
  for (int lz = 0; lz < C::TZ; ++lz) {
    if (lz < nz && slot[lz] >= 0)
      plane_ptr(ms, g, t.z0 + lz)[col] = scell[slot[lz]];
  }
}

__global__ void k_fill_u32(uint32_t *p, uint32_t n, uint32_t value) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

__global__ void k_fill_u64(unsigned long long *p, uint32_t n,
                           unsigned long long value) {
  uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = value;
}

// Capacity of a pair table: a power of two at least twice the number of
// distinct pairs there can be (at most 2^32, so that the mask fits 32 bits).
__host__ __device__ inline uint64_t table_capacity(uint64_t n, uint64_t nmax,
                                                   uint64_t nmin) {
  uint64_t bound = nmax * nmin;
  if (nmax != 0 && bound / nmax != nmin) bound = n;  // product overflowed
  if (bound > n) bound = n;
  uint64_t cap = 1024;
  while (cap < 2 * bound && cap < (1ull << 32)) cap <<= 1;
  return cap;
}

// First capacity tried: the bound above, or twice an expected cell count of
// 8 per extremum (plus slack) when that is smaller, or the caller's choice.
// Cells are pairs of manifolds that meet, far fewer than all pairs of
// extrema: smooth, Perlin and pure-noise fields alike have 2 to 4 per
// extremum, so the table stays at most a quarter full and short to clear; a
// field with more makes the pair pass overflow and run again on the table of
// the full capacity.
__host__ __device__ inline uint64_t table_first_capacity(uint64_t n,
                                                         uint64_t nmax,
                                                         uint64_t nmin,
                                                         uint64_t requested) {
  const uint64_t full = table_capacity(n, nmax, nmin);
  uint64_t cap = 1024;
  const uint64_t want = requested ? (requested + 1) / 2
                                  : 8 * (nmax + nmin) + 4096;
  while (cap < 2 * want && cap < full) cap <<= 1;
  return cap;
}

// The tile -> field map, from the fields' first tiles (increasing).
__global__ void __launch_bounds__(kBlock)
k_fill_tfield(const FieldDev *__restrict__ fds, int nfields, uint32_t *tfield,
              uint32_t nt) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= nt) return;
  int lo = 0, hi = nfields - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (fds[mid].tile0 <= i) lo = mid;
    else hi = mid - 1;
  }
  tfield[i] = (uint32_t)lo;
}

// Everything a call clears or fills before its first pass, in one launch:
// the counter block, the tile -> field map, the per-field counters, the
// tile-order histogram with its min/max pair (min starts at ~0), and the
// per-tile counters.
__global__ void __launch_bounds__(kBlock)
k_call_setup(const FieldDev *__restrict__ fds, int nfields, uint32_t nt,
             unsigned long long *ctr, uint32_t *tfield,
             unsigned long long *fctr, uint32_t *hist, uint32_t *tstat) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i < (uint32_t)kNumCounters) ctr[i] = 0ull;
  if (i < (uint32_t)nfields * kFieldCtrs) fctr[i] = 0ull;
  if (i < (uint32_t)kTileBuckets + 2)
    hist[i] = i == (uint32_t)kTileBuckets ? ~0u : 0u;
  if (i < nt) {
    int lo = 0, hi = nfields - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (fds[mid].tile0 <= i) lo = mid;
      else hi = mid - 1;
    }
    tfield[i] = (uint32_t)lo;
    reinterpret_cast<uint4 *>(tstat)[i] = make_uint4(0u, 0u, 0u, 0u);
  }
}

// Table capacity of every field that wants cells, chosen on the device from
// its extremum counts: the first capacity (`regrow` == 0), or, when the pair
// pass overflowed (`regrow` != 0), the capacity that always suffices, with
// the field's cell counter cleared for the second pass.  *run tells the
// passes that follow whether they have work.  The host reserved each
// field's region for the largest capacity its vertex count allows.
__global__ void __launch_bounds__(kBlock)
k_table_plan(FieldDev *fds, int nfields, unsigned long long *fctr,
             unsigned long long *ctr, uint64_t requested, int regrow,
             uint32_t *run) {
  const bool again = regrow && (ctr[kCtrOverflow] & 1ull);
  for (int i = threadIdx.x; i < nfields; i += kBlock) {
    if (!fds[i].ms) continue;
    const uint64_t n = fds[i].g.N;
    const unsigned long long *fc = fctr + (size_t)i * kFieldCtrs;
    if (!regrow) {
      fds[i].mask = (uint32_t)(
          table_first_capacity(n, fc[kFMaxima], fc[kFMinima], requested) - 1);
    } else if (again) {
      fds[i].mask = (uint32_t)(table_capacity(n, fc[kFMaxima], fc[kFMinima]) - 1);
      fctr[(size_t)i * kFieldCtrs + kFCells] = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *run = regrow ? (again ? 1u : 0u) : 1u;
    if (again) ctr[kCtrOverflow] &= ~1ull;
  }
}

// Clear the tables of the fields that want cells (capacities from the
// plan), over a fixed grid; nothing to do when *run is 0.
constexpr unsigned kClearBlocks = 2048;

__global__ void __launch_bounds__(kBlock)
k_table_clear_all(const FieldDev *__restrict__ fds, int nfields,
                  const uint32_t *__restrict__ run) {
  if (!*run) return;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (int i = 0; i < nfields; ++i) {
    const FieldDev fd = fds[i];
    if (!fd.ms) continue;
    const uint64_t cap = (uint64_t)fd.mask + 1;
    for (uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < cap;
         k += stride) {
      fd.keys[k] = kEmptyKey;
      fd.vals[k] = INT32_MAX;
    }
  }
}

}  // namespace

// Fold the counters of the last segmentation call into the stats; waits for
// the call's work.
namespace {
// Outcome of a whole recorded call from its counter block.
int call_status(const CallRec &R) {
  const unsigned long long ovf = R.hctr[kCtrOverflow];
  if (ovf & 6) return MSC_EHIP;        // broken invariant (never expected)
  if (ovf & 1) return MSC_ENOMEM;      // table full at the full capacity
  return MSC_OK;
}
}  // namespace

int take_call(msc_ctx *ctx, int nfields, int *index) {
  const int k = ctx->next_call;
  CallRec &R = ctx->calls[k];
  if (R.pending) {
    MSC_TRY(host_wait(ctx, R.done));
    R.pending = false;
  }
  if (ctx->last_call == k) {
    // Its stats are replaced by the new call's.
    ctx->last_call = -1;
    ctx->last_folded = true;
  }
  if (!R.hctr &&
      host_malloc(reinterpret_cast<void **>(&R.hctr), kNumCounters * 8) !=
          hipSuccess) {
    R.hctr = nullptr;
    return MSC_ENOMEM;
  }
  const size_t want = (size_t)nfields * kFieldCtrs;
  if (want > R.hfctr_cap) {
    if (R.hfctr) (void)hipHostFree(R.hfctr);
    R.hfctr = nullptr;
    R.hfctr_cap = 0;
    const size_t cap = want * 2 + 64;
    if (host_malloc(reinterpret_cast<void **>(&R.hfctr), cap * 8) !=
        hipSuccess) {
      R.hfctr = nullptr;
      return MSC_ENOMEM;
    }
    R.hfctr_cap = cap;
  }
  ctx->next_call = (k + 1) % kCallRing;
  *index = k;
  return MSC_OK;
}

int call_field_status(const msc_ctx *ctx, int index, int i) {
  const CallRec &R = ctx->calls[index];
  const int all = call_status(R);
  if (all != MSC_OK) return all;
  return R.hfctr[(size_t)i * kFieldCtrs + kFNaN] ? MSC_ENAN : MSC_OK;
}

int call_field_stats(const msc_ctx *ctx, int index, int i, msc_stats *st) {
  const CallRec &R = ctx->calls[index];
  if (i < 0 || i >= R.nfields) return MSC_EINVAL;
  const unsigned long long *f = R.hfctr + (size_t)i * kFieldCtrs;
  *st = msc_stats{};
  st->n_vertices = R.n[i];
  st->n_maxima = (int64_t)f[kFMaxima];
  st->n_minima = (int64_t)f[kFMinima];
  st->n_cells = R.has_ms[i] ? (int64_t)f[kFCells] : -1;
  st->n_exits = (int64_t)f[kFExits];
  st->tile_x = R.tile[0];
  st->tile_y = R.tile[1];
  st->tile_z = R.tile[2];
  st->status = call_field_status(ctx, index, i);
  return MSC_OK;
}

int finish_last(msc_ctx *ctx) {
  if (ctx->last_call < 0 || ctx->last_folded) return MSC_OK;
  CallRec &R = ctx->calls[ctx->last_call];
  if (R.pending) {
    MSC_HIP_TRY(hipEventSynchronize(R.done));
    R.pending = false;
  }
  ctx->last_folded = true;
  const unsigned long long *fc = R.hfctr;
  const int status = call_status(R);
  int last = MSC_OK;
  ctx->stats = msc_stats{};
  ctx->field_stats.assign(R.nfields, msc_stats{});
  for (int i = 0; i < R.nfields; ++i) {
    msc_stats &st = ctx->field_stats[i];
    const unsigned long long *f = fc + (size_t)i * kFieldCtrs;
    st.n_vertices = R.n[i];
    st.n_maxima = (int64_t)f[kFMaxima];
    st.n_minima = (int64_t)f[kFMinima];
    st.n_cells = R.has_ms[i] ? (int64_t)f[kFCells] : -1;
    st.n_exits = (int64_t)f[kFExits];
    st.tile_x = R.tile[0];
    st.tile_y = R.tile[1];
    st.tile_z = R.tile[2];
    st.status = status != MSC_OK ? status : (f[kFNaN] ? MSC_ENAN : MSC_OK);
    if (st.status != MSC_OK && last == MSC_OK) last = st.status;
    ctx->stats.n_vertices += st.n_vertices;
    ctx->stats.n_maxima += st.n_maxima;
    ctx->stats.n_minima += st.n_minima;
    ctx->stats.n_cells += st.n_cells > 0 ? st.n_cells : 0;
    ctx->stats.n_exits += st.n_exits;
  }
  if (R.nfields == 1) ctx->stats.n_cells = ctx->field_stats[0].n_cells;
  ctx->stats.jump_rounds = (int32_t)R.hctr[kCtrRounds];
  ctx->stats.exit_steps = (int64_t)R.hctr[kCtrSteps];
  ctx->stats.tile_x = R.tile[0];
  ctx->stats.tile_y = R.tile[1];
  ctx->stats.tile_z = R.tile[2];
  ctx->stats.status = last;
  ctx->last_status = last;
  return MSC_OK;
}

namespace {

// Grow-only pinned host staging owned by the context (the synchronous
// virtual-rank path).
template <class T>
int stage(msc_ctx *ctx, size_t count, T **out) {
  const size_t bytes = count * sizeof(T);
  if (bytes > ctx->pinned_bytes) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    const size_t want = bytes + bytes / 4 + 4096;
    if (host_malloc(&ctx->pinned, want) != hipSuccess)
      return MSC_ENOMEM;
    ctx->pinned_bytes = want;
  }
  *out = static_cast<T *>(ctx->pinned);
  return MSC_OK;
}

// Geometry, tile ranges and workspace size of a batch.
struct BatchPlan {
  std::vector<FieldDev> fd;
  std::vector<uint64_t> tab_off;  // first slot of each field's pair table
  uint64_t total_n = 0, tab_slots = 0;
  uint32_t nt = 0, nslots = 0;
  bool any_ms = false;
  size_t need = 0;                // workspace bytes the call carves
};

template <class C>
int plan_batch(int nfields, const msc_field *fields, BatchPlan &p) {
  p.fd.assign(nfields, FieldDev{});
  p.tab_off.assign(nfields, 0);
  uint64_t total_tiles = 0;
  size_t need_lp = 0;
  for (int i = 0; i < nfields; ++i) {
    const int64_t X = fields[i].dims[0], Y = fields[i].dims[1],
                  Z = fields[i].dims[2];
    Geo &g = p.fd[i].g;
    g.X = (uint32_t)X;
    g.Y = (uint32_t)Y;
    g.Z = (uint32_t)Z;
    g.XY = (uint32_t)(X * Y);
    g.N = (uint32_t)(X * Y * Z);
    g.ntx = (uint32_t)((X + C::TX - 1) / C::TX);
    g.nty = (uint32_t)((Y + C::TY - 1) / C::TY);
    g.ntz = (uint32_t)((Z + C::TZ - 1) / C::TZ);
    const uint64_t nt = (uint64_t)g.ntx * g.nty * g.ntz;
    g.ntiles = (uint32_t)nt;
    p.fd[i].tile0 = (uint32_t)total_tiles;
    total_tiles += nt;
    p.total_n += g.N;
    if (total_tiles > INT32_MAX / 2) return MSC_ERANGE;
    if (fields[i].ms) {
      // Room for the largest table the field can need; the device uses
      // (and clears) only what its extremum counts call for.
      p.any_ms = true;
      p.tab_off[i] = p.tab_slots;
      p.tab_slots += table_capacity(g.N, g.N, g.N);
    }
  }
  // Exit-graph nodes: 2 * kHalo fixed slots per tile; node numbers and
  // final values share 32 bits (bit 31 tags a final value).
  if (total_tiles * 2 * (uint64_t)C::kHalo >= kRoot) return MSC_ERANGE;
  const uint32_t nt = (uint32_t)total_tiles;
  p.nt = nt;
  p.nslots = nt * (uint32_t)(2 * C::kHalo);
  need_lp = align256((size_t)nt * C::TX * C::TY * C::TZ * sizeof(uint32_t));
  p.need =
      need_lp + align256((size_t)p.nslots * sizeof(uint32_t)) +
      2 * align256(nt * sizeof(Seg)) + 2 * align256(nt * sizeof(uint32_t)) +
      align256((kTileBuckets + 2) * sizeof(uint32_t)) +
      align256(nfields * sizeof(FieldDev)) +
      align256(nfields * kFieldCtrs * sizeof(unsigned long long)) +
      align256(4ull * nt * sizeof(uint32_t)) +
      align256(4ull * nt * sizeof(unsigned long long)) +
      align256(2ull * C::kHalo * nt * sizeof(uint16_t)) +
      align256(2ull * C::TY * C::TZ * nt * sizeof(uint32_t)) + 8192 +
      (p.any_ms ? align256(p.tab_slots * 8) + align256(p.tab_slots * 4) +
                      align256((size_t)nt * C::TX * C::TY * C::TZ)
                : 0);
  return MSC_OK;
}

// One segmentation call over a batch of fields.  Everything is enqueued on
// `s`; the host never waits for the device (only a workspace growth or a
// record or pinned slot still in use by an earlier call can make it wait).
// Conditions the device detects (NaN, a broken invariant) are reported by
// the stats calls and msc_last_status once the work has run.
template <class C>
int segment_batch(msc_ctx *ctx, int nfields, const msc_field *fields,
                  const uint8_t *ghost, hipStream_t s, int *rec_out = nullptr) {
  BatchPlan plan;
  MSC_TRY(plan_batch<C>(nfields, fields, plan));
  std::vector<FieldDev> &fd = plan.fd;
  const std::vector<uint64_t> &tab_off = plan.tab_off;
  const uint64_t total_n = plan.total_n, tab_slots = plan.tab_slots;
  const uint32_t nt = plan.nt, nslots = plan.nslots;
  const bool any_ms = plan.any_ms;
  const size_t need = plan.need;
  unsigned long long *ctr = ctx->dctr;
  int rec = 0;
  MSC_TRY(take_call(ctx, nfields, &rec));
  MSC_TRY(begin_call(ctx, s));
  MSC_TRY(reserve(ctx, ctx->ws, need));
  Carver cv(ctx->ws);
  unsigned long long *keys = nullptr;
  int32_t *vals = nullptr;
  if (any_ms) {
    keys = cv.take<unsigned long long>(tab_slots);
    vals = cv.take<int32_t>(tab_slots);
  }
  uint32_t *lp = cv.take<uint32_t>((size_t)nt * C::TX * C::TY * C::TZ);
  for (int i = 0; i < nfields; ++i) {
    fd[i].f = fields[i].field;
    fd[i].lp = lp;
    fd[i].A = fields[i].asc;  // labels nobody wants are not written
    fd[i].D = fields[i].desc;
    fd[i].ms = fields[i].ms;
    fd[i].keys = fields[i].ms ? keys + tab_off[i] : nullptr;
    fd[i].vals = fields[i].ms ? vals + tab_off[i] : nullptr;
    fd[i].mask = 0;  // set on the device
    fd[i].ghost = ghost ? ghost[i] : 0u;
  }
  uint32_t *next = cv.take<uint32_t>(nslots);
  Seg *seg = cv.take<Seg>(nt);
  uint32_t *tkey = cv.take<uint32_t>(nt);
  Seg *oseg = cv.take<Seg>(nt);
  uint32_t *tfield = cv.take<uint32_t>(nt);
  uint32_t *hist = cv.take<uint32_t>(kTileBuckets + 2);
  uint32_t *mm = hist + kTileBuckets;
  FieldDev *fds = cv.take<FieldDev>(nfields);
  unsigned long long *fctr =
      cv.take<unsigned long long>((size_t)nfields * kFieldCtrs);
  uint32_t *tstat = cv.take<uint32_t>(4ull * nt);
  unsigned long long *rstat = cv.take<unsigned long long>(4ull * nt);
  uint16_t *tlist = cv.take<uint16_t>(2ull * C::kHalo * nt);
  uint32_t *xs = cv.take<uint32_t>(2ull * C::TY * C::TZ * nt);
  uint32_t *run = cv.take<uint32_t>(1);
  uint32_t *cidx = any_ms ? cv.take<uint32_t>((size_t)nt * C::kThreads *
                                               (C::TZ / 4))
                          : nullptr;

  // The descriptors go up through a pinned slot; the tile -> field map is
  // built on the device.
  {
    void *st = nullptr;
    int slot = 0;
    const size_t fbytes = nfields * sizeof(FieldDev);
    MSC_TRY(pinned_slot(ctx, fbytes, &st, &slot));
    std::memcpy(st, fd.data(), fbytes);
    MSC_HIP_TRY(hipMemcpyAsync(fds, st, fbytes, hipMemcpyHostToDevice, s));
    MSC_TRY(slot_copied(ctx, slot, s));
  }
  {
    const uint64_t span = std::max<uint64_t>(
        std::max<uint64_t>(nt, (uint64_t)nfields * kFieldCtrs),
        std::max<uint64_t>(kTileBuckets + 2, kNumCounters));
    k_call_setup<<<grid_for(span), kBlock, 0, s>>>(fds, nfields, nt, ctr,
                                                   tfield, fctr, hist, tstat);
  }
  MSC_HIP_TRY(hipGetLastError());
  ExitOut xo{seg, tkey, tstat, tlist, xs};
  MSC_PHASE(ctx, s, "tile_local", 12.0 * total_n,
            (k_tile_local<C><<<nt, C::kThreads, 0, s>>>(fds, tfield, xo, ctr,
                                                        fctr)));
  k_tile_stats3<<<grid_for(nt), kBlock, 0, s>>>(tstat, nt, tfield, fctr);
  // Exit slots are fixed per tile (2 * kHalo from the tile's own base), so
  // no count has to come back to the host before the graph is built.
  MSC_PHASE(ctx, s, "exit_link", 10.0 * nt * (double)C::kHalo * 0.5,
            (k_exit_link<C><<<nt, kBlock, 0, s>>>(fds, tfield, seg, tlist,
                                                  xs, next)));
  MSC_PHASE(ctx, s, "tile_order", 12.0 * nt,
            (k_key_minmax<<<order_grid(nt), kOrderBlock, 0, s>>>(tkey, nt,
                                                                 mm),
             k_key_hist<<<order_grid(nt), kOrderBlock, 0, s>>>(tkey, nt, mm,
                                                              hist),
             k_key_scan<<<1, 1024, 0, s>>>(hist),
             k_key_scatter<<<order_grid(nt), kOrderBlock, 0, s>>>(
                 tkey, nt, mm, hist, seg, oseg)));
  MSC_PHASE(ctx, s, "exit_resolve", 12.0 * nt * (double)C::kHalo * 0.5,
            (k_exit_resolve<<<2 * nt, kResolveThreads, 0, s>>>(
                oseg, nt, nslots, next, ctr, rstat)));
  k_steps_reduce<<<kStepsBlocks, 1024, 0, s>>>(rstat, 2 * nt, ctr);

  if (any_ms) {
    // Pair tables sized on the device; a pass that overflows its first
    // table runs once more on the capacity that always suffices (the second
    // pass and its clear return at once when nothing overflowed).
    const unsigned cb = (unsigned)std::min<uint64_t>(
        kClearBlocks, (tab_slots + kBlock - 1) / kBlock);
    k_table_plan<<<1, kBlock, 0, s>>>(fds, nfields, fctr, ctr,
                                      ctx->table_first, 0, run);
    MSC_PHASE(ctx, s, "table_clear", 12.0 * total_n,
              (k_table_clear_all<<<cb, kBlock, 0, s>>>(fds, nfields, run)));
    MSC_PHASE(ctx, s, "tile_pairs", 13.0 * total_n,
              (k_tile_pairs<C><<<nt, C::kThreads, 0, s>>>(
                  fds, tfield, seg, next, ctr, tstat, nt, nullptr, tlist,
                  cidx)));
    k_table_plan<<<1, kBlock, 0, s>>>(fds, nfields, fctr, ctr,
                                      ctx->table_first, 1, run);
    k_table_clear_all<<<cb, kBlock, 0, s>>>(fds, nfields, run);
    const unsigned rb = nt < 4096u ? nt : 4096u;
    k_tile_pairs<C><<<rb, C::kThreads, 0, s>>>(fds, tfield, seg, next, ctr,
                                               tstat, nt, run, tlist, cidx);
    MSC_HIP_TRY(hipGetLastError());
    k_tile_stat_reduce<<<grid_for(nt), kBlock, 0, s>>>(tstat, 2, nt, tfield,
                                                       fctr, kFCells);
  }
  MSC_PHASE(ctx, s, "tile_write", (any_ms ? 5.0 : 12.0) * total_n,
            (k_tile_write<C><<<nt, C::kThreads, 0, s>>>(fds, tfield, seg,
                                                        next, tlist, cidx)));
  // Counters back to the record's pinned memory, for the stats calls.
  CallRec &R = ctx->calls[rec];
  MSC_HIP_TRY(hipMemcpyAsync(R.hfctr, fctr, (size_t)nfields * kFieldCtrs * 8,
                             hipMemcpyDeviceToHost, s));
  MSC_HIP_TRY(hipMemcpyAsync(R.hctr, ctr, kNumCounters * 8,
                             hipMemcpyDeviceToHost, s));
  MSC_HIP_TRY(hipEventRecord(R.done, s));
  MSC_TRY(end_call(ctx, s));
  R.pending = true;
  R.nfields = nfields;
  R.n.resize(nfields);
  R.has_ms.resize(nfields);
  for (int i = 0; i < nfields; ++i) {
    R.n[i] = fd[i].g.N;
    R.has_ms[i] = fields[i].ms != nullptr;
  }
  R.tile[0] = C::TX;
  R.tile[1] = C::TY;
  R.tile[2] = C::TZ;
  ctx->last_call = rec;
  ctx->last_folded = false;
  if (rec_out) *rec_out = rec;
  return MSC_OK;
}

// Tile shapes compiled in, in the order of kTileShapes.
using Tile32x16x16 = Cfg<32, 16, 16>;
using Tile32x8x8 = Cfg<32, 8, 8>;
using Tile64x8x8 = Cfg<64, 8, 8>;
using Tile32x8x16 = Cfg<32, 8, 16>;
using Tile64x8x16 = Cfg<64, 8, 16>;

}  // namespace

int segment_workspace(const msc_ctx *ctx, int nfields, const msc_field *fields,
                      size_t *bytes) {
  BatchPlan p;
  int rc = MSC_OK;
  switch (ctx->tile_choice) {
    case 1: rc = plan_batch<Tile32x8x8>(nfields, fields, p); break;
    case 2: rc = plan_batch<Tile64x8x8>(nfields, fields, p); break;
    case 3: rc = plan_batch<Tile32x8x16>(nfields, fields, p); break;
    case 4: rc = plan_batch<Tile64x8x16>(nfields, fields, p); break;
    default: rc = plan_batch<Tile32x16x16>(nfields, fields, p); break;
  }
  *bytes = p.need;
  return rc;
}

int segment_batch_run(msc_ctx *ctx, int nfields, const msc_field *fields,
                      hipStream_t s, const uint8_t *ghost, int *rec) {
  switch (ctx->tile_choice) {
    case 1:
      return segment_batch<Tile32x8x8>(ctx, nfields, fields, ghost, s, rec);
    case 2:
      return segment_batch<Tile64x8x8>(ctx, nfields, fields, ghost, s, rec);
    case 3:
      return segment_batch<Tile32x8x16>(ctx, nfields, fields, ghost, s, rec);
    case 4:
      return segment_batch<Tile64x8x16>(ctx, nfields, fields, ghost, s, rec);
    default:
      return segment_batch<Tile32x16x16>(ctx, nfields, fields, ghost, s, rec);
  }
}


// ---------------------------------------------------------------------------
// Virtual ranks: the paper's distributed scheme on one device
// ---------------------------------------------------------------------------
//
// Alg. 1 and 2 with z-slabs as ranks.  Slab r owns planes [z0, z1) and is
// segmented as a field of its own that also holds the plane on each side
// owned by a neighbour; those ghost vertices are fixed points (every ghost
// is treated as an extremum).  An owned vertex then ends either at a true
// extremum of its slab or at a ghost vertex.  The exchange builds the ghost
// graph -- each ghost vertex gets its owner's result for it, which may be a
// ghost of the owner in turn -- compresses it, and relabels every vertex
// whose slab result is a ghost.  Cells are then paired over the final maps.

namespace {

struct SlabDev {
  uint32_t fs, z0, z1, fe;  // field planes [fs, fe), owned planes [z0, z1)
  uint64_t off;             // start of the slab's labels in the scratch
};

struct RankGeo {
  uint32_t X, XY, Z, R;
};

// Ghost node of slab r: side 0 = plane z0 - 1, side 1 = plane z1.
__device__ __forceinline__ uint32_t ghost_node(const RankGeo &g, uint32_t r,
                                               uint32_t side, uint32_t xy) {
  return (2u * r + side) * g.XY + xy;
}

// Node of the ghost vertex x of slab r, or ~0u when x is owned by r.
__device__ __forceinline__ uint32_t ghost_of(const RankGeo &g,
                                             const SlabDev &sl, uint32_t r,
                                             uint32_t x) {
  const uint32_t z = x / g.XY;
  if (r > 0 && z == sl.z0 - 1) return ghost_node(g, r, 0, x - z * g.XY);
  if (r + 1 < g.R && z == sl.z1) return ghost_node(g, r, 1, x - z * g.XY);
  return ~0u;
}

// Each ghost vertex takes its owner slab's result for it (as a global id).
__global__ void __launch_bounds__(kBlock)
k_rank_ghost_init(RankGeo g, const SlabDev *__restrict__ slabs,
                  const int32_t *__restrict__ A, const int32_t *__restrict__ D,
                  uint32_t *__restrict__ GA, uint32_t *__restrict__ GD) {
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= 2ull * g.R * g.XY) return;
  const uint32_t xy = (uint32_t)(i % g.XY), rs = (uint32_t)(i / g.XY);
  const uint32_t r = rs >> 1, side = rs & 1u;
  if ((side == 0 && r == 0) || (side == 1 && r + 1 == g.R)) return;
  const SlabDev me = slabs[r];
  const uint32_t zg = side ? me.z1 : me.z0 - 1;
  const SlabDev ow = slabs[side ? r + 1 : r - 1];
  const uint64_t local = (uint64_t)xy + (uint64_t)g.XY * (zg - ow.fs);
  const uint32_t base = ow.fs * g.XY;
  GA[i] = (uint32_t)A[ow.off + local] + base;
  GD[i] = (uint32_t)D[ow.off + local] + base;
}

// Ghost graph compression: each node follows its successors (a result that
// is a ghost of the slab that produced it leads to that ghost's node) to a
// final extremum.  A path may cross a slab boundary many times, but never
// visits a node twice (values rise strictly along an ascent, fall along a
// descent), so the walk ends within the number of nodes.
__global__ void __launch_bounds__(kBlock)
k_rank_ghost_resolve(RankGeo g, const SlabDev *__restrict__ slabs,
                     const uint32_t *__restrict__ G, uint32_t *__restrict__ F) {
  const uint64_t nodes = 2ull * g.R * g.XY;
  const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= nodes) return;
  const uint32_t rs = (uint32_t)(i / g.XY), r = rs >> 1, side = rs & 1u;
  if ((side == 0 && r == 0) || (side == 1 && r + 1 == g.R)) return;
  uint32_t s = side ? r + 1 : r - 1;  // the slab that produced G[i]
  uint32_t x = G[i];
  for (uint64_t step = 0; step < nodes; ++step) {
    const uint32_t nd = ghost_of(g, slabs[s], s, x);
    if (nd == ~0u) break;
    const uint32_t ns = (nd / g.XY) & 1u ? s + 1 : s - 1;
    x = G[nd];
    s = ns;
  }
  F[i] = x;
}

// Final labels: a slab result that is a ghost takes the ghost's resolved
// value.  Also counts the vertices that are their own labels (extrema).
// Grid: x over the plane's XY vertices, y over planes (strided by at most
// kRelabelPlanes, so that a block covers several planes and its fixed cost
// is shared), so a block's slab is uniform at each plane and a slab-local
// label is recognised as a ghost by its plane alone (first plane or last),
// without a division.
constexpr uint32_t kRelabelPlanes = 64;

__global__ void __launch_bounds__(kBlock)
k_rank_relabel(RankGeo g, const SlabDev *__restrict__ slabs,
               const int32_t *__restrict__ A, const int32_t *__restrict__ D,
               const uint32_t *__restrict__ FA, const uint32_t *__restrict__ FD,
               int32_t *__restrict__ asc, int32_t *__restrict__ desc,
               uint32_t *__restrict__ roots) {
  __shared__ uint32_t s_cnt[2];
  if (threadIdx.x < 2) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t xy = blockIdx.x * kBlock + threadIdx.x;
  uint32_t cmax = 0, cmin = 0;
  // The slab of the first plane, then advanced as z grows.
  uint32_t r = (uint32_t)(((uint64_t)blockIdx.y * g.R) / g.Z);
  while (r > 0 && slabs[r].z0 > blockIdx.y) --r;
  for (uint32_t z = blockIdx.y; z < g.Z; z += gridDim.y) {
    while (r + 1 < g.R && slabs[r + 1].z0 <= z) ++r;
    const SlabDev sl = slabs[r];
    if (xy >= g.XY) continue;
    const uint64_t v = (uint64_t)z * g.XY + xy;
    const uint64_t local = (uint64_t)(z - sl.fs) * g.XY + xy;
    const uint32_t base = sl.fs * g.XY;
    const uint32_t top = (sl.fe - sl.fs - 1) * g.XY;  // first of the last plane
    const bool lo = r > 0, hi = r + 1 < g.R;
    uint32_t a = (uint32_t)A[sl.off + local];
    uint32_t d = (uint32_t)D[sl.off + local];
    if (lo && a < g.XY) a = FA[ghost_node(g, r, 0, a)];
    else if (hi && a >= top) a = FA[ghost_node(g, r, 1, a - top)];
    else a += base;
    if (lo && d < g.XY) d = FD[ghost_node(g, r, 0, d)];
    else if (hi && d >= top) d = FD[ghost_node(g, r, 1, d - top)];
    else d += base;
    asc[v] = (int32_t)a;
    desc[v] = (int32_t)d;
    cmax += a == (uint32_t)v;
    cmin += d == (uint32_t)v;
  }
  for (int o = 32; o > 0; o >>= 1) {
    cmax += __shfl_xor(cmax, o);
    cmin += __shfl_xor(cmin, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (cmax) atomicAdd(&s_cnt[0], cmax);
    if (cmin) atomicAdd(&s_cnt[1], cmin);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t b = blockIdx.y * gridDim.x + blockIdx.x;
    roots[2 * b] = s_cnt[0];
    roots[2 * b + 1] = s_cnt[1];
  }
}

__global__ void __launch_bounds__(1024)
k_rank_roots_sum(const uint32_t *__restrict__ roots, uint32_t nb,
                 unsigned long long *ctr) {
  __shared__ unsigned long long sa[16], sd[16];
  unsigned long long a = 0, d = 0;
  for (uint32_t i = threadIdx.x; i < nb; i += 1024) {
    a += roots[2 * i];
    d += roots[2 * i + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    d += __shfl_xor(d, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sa[threadIdx.x >> 6] = a;
    sd[threadIdx.x >> 6] = d;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) {
      a += sa[w];
      d += sd[w];
    }
    ctr[kCtrRootsMax] = a;
    ctr[kCtrRootsMin] = d;
  }
}

// Cells over final labels: the smallest id of every (asc, desc) pair.  A
// lane whose pair equals the previous lane's (one id smaller) is not its
// pair's smallest id and inserts nothing; a run of equal pairs inserts once.
__global__ void __launch_bounds__(kBlock)
k_rank_pairs(uint64_t n, const int32_t *__restrict__ asc,
             const int32_t *__restrict__ desc, unsigned long long *keys,
             int32_t *vals, uint32_t mask, unsigned long long *ctr) {
  const uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool in = v < n;
  const unsigned long long key = in ? pair_key(asc[v], desc[v]) : kEmptyKey;
  const unsigned long long left = __shfl_up(key, 1);
  const bool start = (threadIdx.x & 63) == 0 || key != left;
  unsigned fresh = 0;
  bool ok = true;
  if (in && start) ok = table_insert(keys, vals, mask, key, (int32_t)v, &fresh);
  if (!ok) atomicOr(ctr + kCtrOverflow, 1ull);
}

// Cell ids, and per block the number of vertices that are their own cell
// id (one per cell).
__global__ void __launch_bounds__(kBlock)
k_rank_ms(uint64_t n, const int32_t *__restrict__ asc,
          const int32_t *__restrict__ desc,
          const unsigned long long *__restrict__ keys,
          const int32_t *__restrict__ vals, uint32_t mask, int32_t *ms,
          uint32_t *__restrict__ counts) {
  __shared__ uint32_t s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint64_t v = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  bool own = false;
  if (v < n) {
    const int32_t c = table_lookup(keys, vals, mask, pair_key(asc[v], desc[v]));
    ms[v] = c;
    own = (uint64_t)(uint32_t)c == v;
  }
  const uint32_t w = __popcll(__ballot(own));
  if ((threadIdx.x & 63) == 0 && w) atomicAdd(&s_cnt, w);
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[2 * blockIdx.x] = s_cnt;
    counts[2 * blockIdx.x + 1] = 0;
  }
}

// Cells over the final labels of a grid, per tile of kRankTX x kRankTY
// columns of kRankTZ vertices, with the tile passes' dedupe: a vertex whose
// pair equals that of the previous z of its column or of the lane before it
// (both smaller ids) is not its pair's smallest id and inserts nothing; the
// others go through a per-tile table of distinct pairs, so the global insert
// and the cell lookup run about once per pair and tile.  Requires
// X*Y*Z <= INT32_MAX.
constexpr uint32_t kRankTX = 32, kRankTY = kBlock / kRankTX, kRankTZ = 16;

__host__ __device__ inline uint32_t rank_tiles(uint32_t X, uint32_t Y,
                                               uint32_t Z) {
  return ((X + kRankTX - 1) / kRankTX) * ((Y + kRankTY - 1) / kRankTY) *
         ((Z + kRankTZ - 1) / kRankTZ);
}

struct RankCol {
  uint32_t col, z0, nz;  // column offset in its plane, first z, its height
};

__device__ __forceinline__ RankCol rank_col(uint32_t X, uint32_t Y,
                                            uint32_t Z) {
  const uint32_t ntx = (X + kRankTX - 1) / kRankTX;
  const uint32_t nty = (Y + kRankTY - 1) / kRankTY;
  const uint32_t tx = blockIdx.x % ntx, r = blockIdx.x / ntx;
  const uint32_t gx = tx * kRankTX + threadIdx.x % kRankTX;
  const uint32_t gy = (r % nty) * kRankTY + threadIdx.x / kRankTX;
  RankCol c;
  c.z0 = (r / nty) * kRankTZ;
  c.col = gx + X * gy;
  const uint32_t h = Z - c.z0;
  c.nz = gx < X && gy < Y ? (h < kRankTZ ? h : kRankTZ) : 0u;
  return c;
}

// A rank tile column's final labels, every load issued before any is used
// (unconditional: a plane past the column, or a column past the grid, reads
// vertex 0's labels, which are then ignored).
__device__ __forceinline__ void rank_col_labels(
    const RankCol &c, uint32_t XY, const int32_t *__restrict__ asc,
    const int32_t *__restrict__ desc, int32_t (&a)[kRankTZ],
    int32_t (&d)[kRankTZ]) {
#pragma unroll
  for (uint32_t lz = 0; lz < kRankTZ; ++lz) {
    const uint32_t v = lz < c.nz ? c.col + XY * (c.z0 + lz) : 0u;
    a[lz] = asc[v];
    d[lz] = desc[v];
  }
}

__global__ void __launch_bounds__(kBlock)
k_rank_tile_pairs(uint32_t X, uint32_t Y, uint32_t Z,
                  const int32_t *__restrict__ asc,
                  const int32_t *__restrict__ desc, unsigned long long *keys,
                  int32_t *vals, uint32_t mask, unsigned long long *ctr) {
  __shared__ unsigned long long skey[kPairSlots];
  __shared__ int32_t sval[kPairSlots];
  __shared__ unsigned sfill;
  const int tid = threadIdx.x;
  for (int i = tid; i < kPairSlots; i += kBlock) {
    skey[i] = kEmptyKey;
    sval[i] = INT32_MAX;
  }
  if (tid == 0) sfill = 0;
  __syncthreads();
  const RankCol c = rank_col(X, Y, Z);
  const uint32_t XY = X * Y;
  unsigned fresh = 0;
  bool overflow = false;
  const bool first_lane = (tid & 63) == 0;
  unsigned long long last = kEmptyKey;
  int32_t la[kRankTZ], ld[kRankTZ];
  rank_col_labels(c, XY, asc, desc, la, ld);
#pragma unroll
  for (uint32_t lz = 0; lz < kRankTZ; ++lz) {
    unsigned long long key = kEmptyKey;
    const uint32_t v = c.col + XY * (c.z0 + lz);
    if (lz < c.nz) key = pair_key(la[lz], ld[lz]);
    const unsigned long long left = __shfl_up(key, 1);
    const bool repeat = key == last || (!first_lane && key == left);
    last = key;
    if (!repeat && key != kEmptyKey) {
      const int slot = pair_slot(skey, &sfill, key);
      if (slot >= 0)
        atomicMin(&sval[slot], (int32_t)v);
      else if (!table_insert(keys, vals, mask, key, (int32_t)v, &fresh))
        overflow = true;
    }
  }
  __syncthreads();
  for (int i = tid; i < kPairSlots; i += kBlock)
    if (skey[i] != kEmptyKey &&
        !table_insert(keys, vals, mask, skey[i], sval[i], &fresh))
      overflow = true;
  if (overflow) atomicOr(ctr + kCtrOverflow, 1ull);
}

// Cell ids over the same tiles, and per tile the number of vertices that
// are their own cell id (one per cell).
__global__ void __launch_bounds__(kBlock)
k_rank_tile_ms(uint32_t X, uint32_t Y, uint32_t Z,
               const int32_t *__restrict__ asc,
               const int32_t *__restrict__ desc,
               const unsigned long long *__restrict__ keys,
               const int32_t *__restrict__ vals, uint32_t mask,
               int32_t *__restrict__ ms, uint32_t *__restrict__ counts) {
  __shared__ unsigned long long skey[kPairSlots];
  __shared__ int32_t scell[kPairSlots];
  __shared__ unsigned sfill;
  __shared__ uint32_t s_cnt;
  const int tid = threadIdx.x;
  for (int i = tid; i < kPairSlots; i += kBlock) skey[i] = kEmptyKey;
  if (tid == 0) {
    sfill = 0;
    s_cnt = 0;
  }
  __syncthreads();
  const RankCol c = rank_col(X, Y, Z);
  const uint32_t XY = X * Y;
  int16_t slot[kRankTZ];
  unsigned long long last = kEmptyKey;
  int last_slot = -1;
  int32_t last_cell = -1;
  uint32_t own = 0;
  int32_t la[kRankTZ], ld[kRankTZ];
  rank_col_labels(c, XY, asc, desc, la, ld);
#pragma unroll
  for (uint32_t lz = 0; lz < kRankTZ; ++lz) {
    slot[lz] = -1;
    if (lz < c.nz) {
      const uint32_t v = c.col + XY * (c.z0 + lz);
      const unsigned long long key = pair_key(la[lz], ld[lz]);
      if (key != last) {
        last = key;
        last_slot = pair_slot(skey, &sfill, key);
        if (last_slot < 0)  // not in the tile's table: look this pair up alone
          last_cell = table_lookup(keys, vals, mask, key);
      }
      slot[lz] = (int16_t)last_slot;
      if (last_slot < 0) {
        ms[v] = last_cell;
        own += (uint32_t)last_cell == v;
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < kPairSlots; i += kBlock)
    if (skey[i] != kEmptyKey) scell[i] = table_lookup(keys, vals, mask, skey[i]);
  __syncthreads();
#pragma unroll
  for (uint32_t lz = 0; lz < kRankTZ; ++lz) {
    if (lz < c.nz && slot[lz] >= 0) {
      const uint32_t v = c.col + XY * (c.z0 + lz);
      const int32_t cell = scell[slot[lz]];
      ms[v] = cell;
      own += (uint32_t)cell == v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) own += __shfl_xor(own, o);
  if ((tid & 63) == 0 && own) atomicAdd(&s_cnt, own);
  __syncthreads();
  if (tid == 0) {
    counts[2 * blockIdx.x] = s_cnt;
    counts[2 * blockIdx.x + 1] = 0;
  }
}

template <class C>
int segment_ranks(msc_ctx *ctx, const float *field, const int64_t dims[3],
                  int ranks, int32_t *asc, int32_t *desc, int32_t *ms,
                  hipStream_t s) {
  const uint32_t X = (uint32_t)dims[0], Y = (uint32_t)dims[1],
                 Z = (uint32_t)dims[2], R = (uint32_t)ranks;
  const uint64_t XY = (uint64_t)X * Y, N = XY * Z;
  std::vector<SlabDev> sl(R);
  std::vector<msc_field> fields(R);
  std::vector<uint8_t> ghost(R);
  uint64_t total = 0;
  for (uint32_t r = 0; r < R; ++r) {
    SlabDev &q = sl[r];
    q.z0 = (uint32_t)((uint64_t)r * Z / R);
    q.z1 = (uint32_t)((uint64_t)(r + 1) * Z / R);
    q.fs = r > 0 ? q.z0 - 1 : 0;
    q.fe = r + 1 < R ? q.z1 + 1 : Z;
    q.off = total;
    total += XY * (q.fe - q.fs);
    ghost[r] = (uint8_t)((r > 0 ? 1 : 0) | (r + 1 < R ? 2 : 0));
  }
  const uint64_t nodes = 2ull * R * XY;
  const dim3 rgrid((unsigned)((XY + kBlock - 1) / kBlock),
                   Z < kRelabelPlanes ? Z : kRelabelPlanes);
  const uint32_t ntile = rank_tiles(X, Y, Z);
  // per-block root counts: for the cell tiles and for the relabel grid
  const uint64_t nroot = std::max<uint64_t>(ntile, (uint64_t)rgrid.x * rgrid.y);
  MSC_TRY(reserve(ctx, ctx->rk, 2 * align256(total * 4) + 4 * align256(nodes * 4) +
                               align256(R * sizeof(SlabDev)) +
                               2 * align256(N * 4) + align256(nroot * 8ull) +
                               4096));
  Carver cv(ctx->rk);
  int32_t *A = cv.take<int32_t>(total), *D = cv.take<int32_t>(total);
  uint32_t *GA = cv.take<uint32_t>(nodes), *GD = cv.take<uint32_t>(nodes);
  uint32_t *FA = cv.take<uint32_t>(nodes), *FD = cv.take<uint32_t>(nodes);
  SlabDev *dsl = cv.take<SlabDev>(R);
  uint32_t *roots = cv.take<uint32_t>(2ull * nroot);
  int32_t *fa = asc ? asc : cv.take<int32_t>(N);
  int32_t *fd = desc ? desc : cv.take<int32_t>(N);
  for (uint32_t r = 0; r < R; ++r) {
    fields[r].field = field + XY * sl[r].fs;
    fields[r].dims[0] = X;
    fields[r].dims[1] = Y;
    fields[r].dims[2] = sl[r].fe - sl[r].fs;
    fields[r].asc = A + sl[r].off;
    fields[r].desc = D + sl[r].off;
    fields[r].ms = nullptr;
  }
  // Alg. 1 on every rank, all ranks in one batched call.
  MSC_TRY(segment_batch<C>(ctx, (int)R, fields.data(), ghost.data(), s));
  // This path reads counts back anyway: take the slabs' outcome now.
  MSC_TRY(finish_last(ctx));
  if (ctx->last_status != MSC_OK) return ctx->last_status;

  char *st = nullptr;
  MSC_TRY(stage(ctx, R * sizeof(SlabDev), &st));
  std::memcpy(st, sl.data(), R * sizeof(SlabDev));
  MSC_HIP_TRY(hipMemcpyAsync(dsl, st, R * sizeof(SlabDev),
                             hipMemcpyHostToDevice, s));
  MSC_TRY(clear_counters(ctx, s));
  const RankGeo rg{X, (uint32_t)XY, Z, R};
  // Alg. 2: ghost graph, compression, relabelling.
  MSC_PHASE(ctx, s, "rank_exchange", 24.0 * nodes,
            (k_rank_ghost_init<<<grid_for(nodes), kBlock, 0, s>>>(
                 rg, dsl, A, D, GA, GD),
             k_rank_ghost_resolve<<<grid_for(nodes), kBlock, 0, s>>>(
                 rg, dsl, GA, FA),
             k_rank_ghost_resolve<<<grid_for(nodes), kBlock, 0, s>>>(
                 rg, dsl, GD, FD)));
  MSC_PHASE(ctx, s, "rank_relabel", 16.0 * N,
            (k_rank_relabel<<<rgrid, kBlock, 0, s>>>(rg, dsl, A, D, FA, FD, fa,
                                                    fd, roots),
             k_rank_roots_sum<<<1, 1024, 0, s>>>(roots, rgrid.x * rgrid.y,
                                                 ctx->dctr)));
  MSC_TRY(read_counters(ctx, s));
  const uint64_t nmax = ctx->hctr[kCtrRootsMax], nmin = ctx->hctr[kCtrRootsMin];
  int64_t cells = -1;
  if (ms) {
    const uint64_t cap = table_capacity(N, nmax, nmin);
    MSC_TRY(reserve(ctx, ctx->tab, align256(cap * 8) + align256(cap * 4) + 4096));
    Carver tc(ctx->tab);
    unsigned long long *keys = tc.take<unsigned long long>(cap);
    int32_t *vals = tc.take<int32_t>(cap);
    MSC_PHASE(ctx, s, "rank_pairs", 12.0 * N,
              (k_table_clear<<<(unsigned)((cap + kBlock - 1) / kBlock), kBlock,
                               0, s>>>(keys, vals, cap),
               k_rank_tile_pairs<<<ntile, kBlock, 0, s>>>(
                   X, Y, Z, fa, fd, keys, vals, (uint32_t)(cap - 1),
                   ctx->dctr)));
    MSC_PHASE(ctx, s, "rank_ms", 12.0 * N,
              (k_rank_tile_ms<<<ntile, kBlock, 0, s>>>(
                   X, Y, Z, fa, fd, keys, vals, (uint32_t)(cap - 1), ms,
                   roots),
               k_rank_roots_sum<<<1, 1024, 0, s>>>(roots, ntile, ctx->dctr)));
    MSC_TRY(read_counters(ctx, s));
    if (ctx->hctr[kCtrOverflow]) return MSC_ENOMEM;
    cells = (int64_t)ctx->hctr[kCtrRootsMax];
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = (int64_t)N;
  ctx->stats.n_maxima = (int64_t)nmax;
  ctx->stats.n_minima = (int64_t)nmin;
  ctx->stats.n_cells = cells;
  ctx->stats.tile_x = C::TX;
  ctx->stats.tile_y = C::TY;
  ctx->stats.tile_z = C::TZ;
  return MSC_OK;
}

}  // namespace

int segment_ranks_run(msc_ctx *ctx, const float *field, const int64_t dims[3],
                      int ranks, int32_t *asc, int32_t *desc, int32_t *ms,
                      hipStream_t s) {
  return segment_ranks<Tile32x16x16>(ctx, field, dims, ranks, asc, desc, ms,
                                     s);
}

// ---------------------------------------------------------------------------
// Segmentation on a complex given as CSR adjacency (the problem statement's
// general K): steepest neighbours over the closed row neighbourhoods, path
// compression in place, cells over the final labels.
// ---------------------------------------------------------------------------

namespace {

constexpr int kRowChunk = 8;  // column entries gathered per round trip

// sp[v] / sm[v]: the (f, id)-largest / -smallest of v and its row.  Column
// indices are checked before use (an out-of-range one is skipped and
// reported); NaN values lose every comparison and are reported.  Each block
// counts its extrema (vertices that are their own successor).
__global__ void __launch_bounds__(kBlock)
k_csr_steepest(int64_t n, int64_t nnz, const int64_t *__restrict__ rp,
               const int32_t *__restrict__ col, const float *__restrict__ f,
               int32_t *__restrict__ sp, int32_t *__restrict__ sm,
               uint32_t *__restrict__ counts, unsigned long long *ctr) {
  __shared__ uint32_t s_max, s_min;
  if (threadIdx.x == 0) s_max = s_min = 0;
  __syncthreads();
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool bad = false, nan = false, is_max = false, is_min = false;
  if (v < n) {
    const float fv = f[v];
    nan = fv != fv;
    float bmax = fv, bmin = fv;
    int32_t imax = (int32_t)v, imin = (int32_t)v;
    // A row is read only inside [0, nnz); a row pointer outside it is
    // reported like a bad column index.
    int64_t e1 = rp[v + 1], e0 = rp[v];
    bad |= e0 < 0 || e1 > nnz;
    e0 = e0 < 0 ? 0 : e0;
    e1 = e1 > nnz ? nnz : e1;
    for (; e0 < e1; e0 += kRowChunk) {
      int32_t u[kRowChunk];
      float fu[kRowChunk];
      // Unconditional loads at in-range indices (the chunk's first entry;
      // the vertex itself), each kind issued for the whole chunk first.
#pragma unroll
      for (int k = 0; k < kRowChunk; ++k) {
        const int32_t c = col[e0 + k < e1 ? e0 + k : e0];
        u[k] = e0 + k < e1 ? c : -1;
        const bool ok = u[k] >= 0 && (int64_t)u[k] < n;
        bad |= e0 + k < e1 && !ok;
        if (!ok) u[k] = -1;
      }
#pragma unroll
      for (int k = 0; k < kRowChunk; ++k) fu[k] = f[u[k] >= 0 ? u[k] : v];
#pragma unroll
      for (int k = 0; k < kRowChunk; ++k) {
        if (u[k] < 0) continue;
        if (fu[k] > bmax || (fu[k] == bmax && u[k] > imax)) {
          bmax = fu[k];
          imax = u[k];
        }
        if (fu[k] < bmin || (fu[k] == bmin && u[k] < imin)) {
          bmin = fu[k];
          imin = u[k];
        }
      }
    }
    sp[v] = imax;
    sm[v] = imin;
    is_max = imax == (int32_t)v;
    is_min = imin == (int32_t)v;
  }
  const uint32_t wmax = __popcll(__ballot(is_max));
  const uint32_t wmin = __popcll(__ballot(is_min));
  if ((threadIdx.x & 63) == 0) {
    if (wmax) atomicAdd(&s_max, wmax);
    if (wmin) atomicAdd(&s_min, wmin);
  }
  if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(ctr + kCtrBadIndex, 1ull);
  if (__ballot(nan) && (threadIdx.x & 63) == 0) atomicOr(ctr + kCtrNaN, 1ull);
  __syncthreads();
  if (threadIdx.x == 0) {
    counts[2 * blockIdx.x] = s_max;
    counts[2 * blockIdx.x + 1] = s_min;
  }
}

// Root of v in a successor forest, compressing as it goes (path halving:
// an entry only ever moves to an ancestor, so concurrent chases agree).
// Successors climb the (f, id) order strictly, so every chase ends.
__device__ __forceinline__ int32_t chase_halving(int32_t *S, int32_t x) {
  for (;;) {
    const int32_t p = __atomic_load_n(&S[x], __ATOMIC_RELAXED);
    if (p == x) return x;
    const int32_t g = __atomic_load_n(&S[p], __ATOMIC_RELAXED);
    if (g == p) return p;
    __atomic_store_n(&S[x], g, __ATOMIC_RELAXED);
    x = g;
  }
}

// First pass: every vertex chases its root with path halving, which
// shortens every path but writes no final value -- a halving store may land
// after another thread's, so a root written here could be overwritten by an
// older ancestor.
__global__ void __launch_bounds__(kBlock)
k_csr_compress(int64_t n, int32_t *A, int32_t *D) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  (void)chase_halving(A, (int32_t)v);
  (void)chase_halving(D, (int32_t)v);
}

// Root of x without writing (every value read is an ancestor of x).
__device__ __forceinline__ int32_t walk_root(const int32_t *S, int32_t x) {
  for (;;) {
    const int32_t p = __hip_atomic_load(&S[x], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    x = p;
  }
}

// Second pass: only the owner writes an entry, and it writes the root, so a
// concurrent reader sees the old pointer or the root, both ancestors.
__global__ void __launch_bounds__(kBlock)
k_csr_roots(int64_t n, int32_t *A, int32_t *D) {
  const int64_t v = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (v >= n) return;
  const int32_t a = walk_root(A, (int32_t)v);
  const int32_t d = walk_root(D, (int32_t)v);
  __hip_atomic_store(&A[v], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&D[v], d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

int segment_csr_run(msc_ctx *ctx, int64_t n, const int64_t *row_ptr,
                    const int32_t *col_idx, const float *field, int32_t *asc,
                    int32_t *desc, int32_t *ms, hipStream_t s) {
  if (n == 0) {
    ctx->stats = msc_stats{};
    ctx->stats.n_cells = ms ? 0 : -1;
    return MSC_OK;
  }
  const uint32_t nblk = (uint32_t)((n + kBlock - 1) / kBlock);
  // Edge count, for the pass's algorithmic bytes (row pointer, column index
  // and the neighbour's value per entry).
  int64_t nnz = 0;
  MSC_HIP_TRY(hipMemcpyAsync(&nnz, row_ptr + n, sizeof(int64_t),
                             hipMemcpyDeviceToHost, s));
  MSC_HIP_TRY(hipStreamSynchronize(s));
  if (nnz < 0 || (nnz > 0 && !col_idx)) return MSC_EINVAL;
  MSC_TRY(reserve(ctx, ctx->rk, 2 * align256((uint64_t)n * 4) +
                               align256(nblk * 8ull) + 4096));
  Carver cv(ctx->rk);
  uint32_t *roots = cv.take<uint32_t>(2ull * nblk);
  int32_t *A = asc ? asc : cv.take<int32_t>(n);
  int32_t *D = desc ? desc : cv.take<int32_t>(n);
  MSC_TRY(clear_counters(ctx, s));
  MSC_PHASE(ctx, s, "csr_steepest", 20.0 * n + 8.0 * (double)nnz,
            (k_csr_steepest<<<nblk, kBlock, 0, s>>>(n, nnz, row_ptr, col_idx,
                                                    field,
                                                    A, D, roots, ctx->dctr),
             k_rank_roots_sum<<<1, 1024, 0, s>>>(roots, nblk, ctx->dctr)));
  MSC_PHASE(ctx, s, "csr_compress", 16.0 * n,
            (k_csr_compress<<<nblk, kBlock, 0, s>>>(n, A, D),
             k_csr_roots<<<nblk, kBlock, 0, s>>>(n, A, D)));
  MSC_TRY(read_counters(ctx, s));
  if (ctx->hctr[kCtrBadIndex]) return MSC_EINVAL;
  if (ctx->hctr[kCtrNaN]) return MSC_ENAN;
  const uint64_t nmax = ctx->hctr[kCtrRootsMax], nmin = ctx->hctr[kCtrRootsMin];
  int64_t cells = -1;
  if (ms) {
    // Pair table: first capacity from the extremum counts, grown fourfold
    // while the pair pass overflows.
    uint64_t cap = table_first_capacity((uint64_t)n, nmax, nmin,
                                        ctx->table_first);
    const uint64_t full = table_capacity((uint64_t)n, nmax, nmin);
    for (;;) {
      MSC_TRY(reserve(ctx, ctx->tab, align256(cap * 8) + align256(cap * 4) + 4096));
      Carver tc(ctx->tab);
      unsigned long long *keys = tc.take<unsigned long long>(cap);
      int32_t *vals = tc.take<int32_t>(cap);
      MSC_PHASE(ctx, s, "csr_pairs", 12.0 * n,
                (k_table_clear<<<(unsigned)((cap + kBlock - 1) / kBlock),
                                 kBlock, 0, s>>>(keys, vals, cap),
                 k_rank_pairs<<<nblk, kBlock, 0, s>>>((uint64_t)n, A, D, keys,
                                                      vals, (uint32_t)(cap - 1),
                                                      ctx->dctr)));
      MSC_TRY(read_counters(ctx, s));
      if (!ctx->hctr[kCtrOverflow]) {
        MSC_PHASE(ctx, s, "csr_ms", 12.0 * n,
                  (k_rank_ms<<<nblk, kBlock, 0, s>>>(
                       (uint64_t)n, A, D, keys, vals, (uint32_t)(cap - 1), ms,
                       roots),
                   k_rank_roots_sum<<<1, 1024, 0, s>>>(roots, nblk,
                                                       ctx->dctr)));
        MSC_TRY(read_counters(ctx, s));
        cells = (int64_t)ctx->hctr[kCtrRootsMax];
        break;
      }
      if (cap >= full) return MSC_ENOMEM;
      cap = cap * 4 < full ? cap * 4 : full;
      k_fill_u64<<<1, kBlock, 0, s>>>(ctx->dctr + kCtrOverflow, 1, 0ull);
    }
  }
  ctx->stats = msc_stats{};
  ctx->stats.n_vertices = n;
  ctx->stats.n_maxima = (int64_t)nmax;
  ctx->stats.n_minima = (int64_t)nmin;
  ctx->stats.n_cells = cells;
  return MSC_OK;
}

}  // namespace msc
