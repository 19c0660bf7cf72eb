// Stage kernels of the repeat-finding path (everything except the segmented
// sort engine): token ranking, LCP construction, candidate generation,
// greedy selection and output compaction.
#include "apo_internal.h"
#include "device_util.h"
#include "stages.h"
#include <algorithm>

namespace apo {

static inline dim3 grid_for(uint64_t n, int threads, int cap_blocks) {
  uint64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap_blocks) b = cap_blocks;
  return dim3((unsigned)b);
}

#define GRID_STRIDE(i, n) \
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (uint64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) { GRID_STRIDE(i, n) p[i] = v; }
__global__ void k_fill_u8(uint8_t *p, uint64_t n, uint8_t v) { GRID_STRIDE(i, n) p[i] = v; }

void fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u32, grid_for(n, 256, 8192), dim3(256), 0, s, p, n, v);
}
void fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill_u8, grid_for(n, 256, 8192), dim3(256), 0, s, p, n, v);
}

// ------------------------------------------------------ device-wide scan
// Exclusive prefix sum of u32 values (sums fit in u32).  Three phases:
// per-tile sums, one-workgroup scan of the tile sums, per-tile rescan.
constexpr int kScanNT = 256, kScanPer = 16, kScanTile = kScanNT * kScanPer;

__global__ __launch_bounds__(kScanNT) void k_scan_tiles(const uint32_t *in, const uint32_t *n_dev, uint32_t *tile_sum) {
  __shared__ uint32_t sh[kScanNT / 64];
  const uint64_t n = *n_dev;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  if (base >= n && blockIdx.x > 0) return;
  uint32_t loc = 0;
  for (int q = 0; q < kScanPer; q++) {
    const uint64_t i = base + (uint64_t)q * kScanNT + threadIdx.x;
    loc += i < n ? in[i] : 0u;
  }
  uint32_t tot;
  (void)block_excl_sum<kScanNT>(loc, sh, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *tile_sum, const uint32_t *n_dev, uint32_t *total) {
  __shared__ uint32_t sh[1024 / 64];
  __shared__ uint32_t carry;
  const uint32_t ntiles = (uint32_t)(((uint64_t)*n_dev + kScanTile - 1) / kScanTile);
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (uint32_t b0 = 0; b0 < ntiles; b0 += 1024) {
    const uint32_t i = b0 + threadIdx.x;
    const uint32_t v = i < ntiles ? tile_sum[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_sum<1024>(v, sh, &tot);
    if (i < ntiles) tile_sum[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

__global__ __launch_bounds__(kScanNT) void k_scan_apply(const uint32_t *in, const uint32_t *n_dev,
                                                        const uint32_t *tile_sum, uint32_t *out) {
  __shared__ uint32_t sh[kScanNT / 64];
  const uint64_t n = *n_dev;
  if ((uint64_t)blockIdx.x * kScanTile >= n) return;
  // thread owns kScanPer consecutive elements
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint32_t loc = 0;
  for (int q = 0; q < kScanPer; q++) {
    const uint64_t i = base + q;
    v[q] = i < n ? in[i] : 0u;
    loc += v[q];
  }
  uint32_t tot;
  uint32_t ex = block_excl_sum<kScanNT>(loc, sh, &tot) + tile_sum[blockIdx.x];
  for (int q = 0; q < kScanPer; q++) {
    const uint64_t i = base + q;
    if (i < n) out[i] = ex;
    ex += v[q];
  }
}

// n_dev: element count in device memory; bound: host upper bound (grid size).
void scan_excl(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t bound, uint32_t *tile_tmp,
               uint32_t *total, hipStream_t s) {
  const uint32_t tiles = (uint32_t)std::max<uint64_t>((bound + kScanTile - 1) / kScanTile, 1);
  hipLaunchKernelGGL(k_scan_tiles, dim3(tiles), dim3(kScanNT), 0, s, in, n_dev, tile_tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tile_tmp, n_dev, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(tiles), dim3(kScanNT), 0, s, in, n_dev, tile_tmp, out);
}

// ---------------------------------------------------- byte-flag compaction
// Stream compaction over a byte array with a predicate: per-tile counts, a
// scan of the tile counts, then each thread takes kScanPer consecutive flags
// (one 16-byte load) and scans its count across the workgroup; the output
// positions go through LDS so that the gather act.get(k) / act.put(o, rec)
// runs with consecutive threads on consecutive entries.  No flag or position
// array is written to global memory.
struct FlagNonZero {
  __device__ bool operator()(uint8_t x) const { return x != 0; }
};
struct FlagIsOne {
  __device__ bool operator()(uint8_t x) const { return x == 1; }
};

template <class P>
__device__ __forceinline__ uint32_t flag_mask16(const uint8_t *f, uint64_t base, uint64_t n, P pred) {
  static_assert(kScanPer == 16, "one 16-byte load per thread");
  uint32_t mask = 0;
  if (base + 16 <= n) {
    const uint4 v = *reinterpret_cast<const uint4 *>(f + base);
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int b = 0; b < 16; b++)
      if (pred((uint8_t)(w[b >> 2] >> (8 * (b & 3))))) mask |= 1u << b;
  } else {
    for (int b = 0; b < 16; b++)
      if (base + b < n && pred(f[base + b])) mask |= 1u << b;
  }
  return mask;
}

template <class P>
__global__ __launch_bounds__(kScanNT) void k_flag_tiles(const uint8_t *f, P pred, const uint32_t *n_dev,
                                                        uint32_t *tile_sum) {
  __shared__ uint32_t sh[kScanNT / 64];
  const uint64_t n = *n_dev;
  if ((uint64_t)blockIdx.x * kScanTile >= n && blockIdx.x > 0) return;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
  const uint32_t loc = base < n ? (uint32_t)__popc(flag_mask16(f, base, n, pred)) : 0u;
  uint32_t tot;
  (void)block_excl_sum<kScanNT>(loc, sh, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

template <class P, class A>
__global__ __launch_bounds__(kScanNT) void k_flag_compact(const uint8_t *f, P pred, const uint32_t *n_dev,
                                                          const uint32_t *tile_sum, A act) {
  __shared__ uint32_t sh[kScanNT / 64];
  __shared__ uint32_t opos[pad16(kScanTile)];  // output position of each flagged entry of the tile, else ~0
  const uint64_t n = *n_dev;
  const uint64_t tile0 = (uint64_t)blockIdx.x * kScanTile;
  if (tile0 >= n) return;
  const int first = threadIdx.x * kScanPer;
  const uint64_t base = tile0 + first;
  const uint32_t mask = base < n ? flag_mask16(f, base, n, pred) : 0u;
  uint32_t tot;
  uint32_t o = block_excl_sum<kScanNT>((uint32_t)__popc(mask), sh, &tot) + tile_sum[blockIdx.x];
#pragma unroll
  for (int b = 0; b < kScanPer; b++) opos[pad16(first + b)] = ((mask >> b) & 1u) ? o++ : ~0u;
  __syncthreads();
  // gather with consecutive threads on consecutive entries, every load of
  // the thread's entries issued before any store
  typename A::Rec rec[kScanPer];
  uint32_t dst[kScanPer];
#pragma unroll
  for (int q = 0; q < kScanPer; q++) {
    const int e = q * kScanNT + threadIdx.x;
    dst[q] = tile0 + e < n ? opos[pad16(e)] : ~0u;
    if (dst[q] != ~0u) rec[q] = act.get(tile0 + e);
  }
#pragma unroll
  for (int q = 0; q < kScanPer; q++)
    if (dst[q] != ~0u) act.put(dst[q], rec[q]);
}

// *total receives the number of flagged entries.
template <class P, class A>
static void flag_compact(const uint8_t *f, P pred, const uint32_t *n_dev, uint64_t bound, uint32_t *tile_tmp,
                         uint32_t *total, A act, hipStream_t s) {
  const uint32_t tiles = (uint32_t)std::max<uint64_t>((bound + kScanTile - 1) / kScanTile, 1);
  hipLaunchKernelGGL((k_flag_tiles<P>), dim3(tiles), dim3(kScanNT), 0, s, f, pred, n_dev, tile_tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(1024), 0, s, tile_tmp, n_dev, total);
  hipLaunchKernelGGL((k_flag_compact<P, A>), dim3(tiles), dim3(kScanNT), 0, s, f, pred, n_dev, tile_tmp, act);
}

__global__ void k_fill_u8_dev(uint8_t *p, const uint32_t *n_dev, uint8_t v) {
  const uint64_t n = *n_dev;
  GRID_STRIDE(i, n) p[i] = v;
}
void fill_u8_dev(uint8_t *p, const uint32_t *n_dev, uint64_t bound, uint8_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u8_dev, grid_for(bound, 256, 8192), dim3(256), 0, s, p, n_dev, v);
}
__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src) {
  if (threadIdx.x == 0) *dst = *src;
}
__global__ void k_copy_n_u32(uint32_t *dst, const uint32_t *src, uint64_t n) { GRID_STRIDE(i, n) dst[i] = src[i]; }

void copy_n_u32(uint32_t *dst, const uint32_t *src, uint64_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_copy_n_u32, grid_for(n, 256, 8192), dim3(256), 0, s, dst, src, n);
}

void copy_u32(uint32_t *dst, const uint32_t *src, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_u32, dim3(1), dim3(64), 0, s, dst, src);
}

// ------------------------------------------------------ token ranking (u64)
// Open-addressing table of the distinct 64-bit token values themselves
// (kEmpty marks a free slot; the token value equal to kEmpty has the extra
// slot mask+1 of its own).  Each workgroup first removes duplicates within
// its tile of tokens with a table in LDS, so only one thread per distinct
// value and tile probes the global table (loop streams repeat a few hundred
// hashes thousands of times); a probe compares the stored key, with no
// dependent read of the token array.  The threads whose CAS claims a slot
// collect their new distinct values in LDS, and the tile reserves their list
// entries with one atomic.
constexpr int kHashTile = 2048, kHashLds = 4096;
constexpr uint64_t kEmpty = ~0ull;

// Returns whether the key was new; *slot receives its slot either way.
__device__ __forceinline__ bool global_insert(uint64_t key, unsigned long long *tab, uint64_t mask,
                                              uint64_t *slot) {
  if (key == kEmpty) {
    *slot = mask + 1;
    return atomicCAS(&tab[mask + 1], 0ull, 1ull) == 0ull;
  }
  uint64_t h = mix64(key) & mask;
  while (true) {
    unsigned long long cur = tab[h];
    if (cur == kEmpty) {
      cur = atomicCAS(&tab[h], (unsigned long long)kEmpty, (unsigned long long)key);
      if (cur == kEmpty) {
        *slot = h;
        return true;
      }
    }
    if (cur == key) {
      *slot = h;
      return false;
    }
    h = (h + 1) & mask;
  }
}

// Also writes every token's global slot to tok_slot (the tile's first
// occurrence of a value finds it; the local table hands it to the others), so
// the ranks come later from one gather per token instead of a second probe.
// With `wflag` set only the tokens of flagged windows are inserted and get a
// slot (window of token i: wid[i]), and nothing runs unless *gate > 0.
__global__ __launch_bounds__(256) void k_hash_insert(const uint64_t *tok, uint64_t n, unsigned long long *tab,
                                                     uint64_t mask, uint32_t *dist_idx, uint32_t *dist_slot,
                                                     uint32_t *nd, uint32_t *tok_slot, const uint32_t *wid,
                                                     const uint8_t *wflag, const uint32_t *gate) {
  constexpr int NT = 256;
  if (gate && *gate == 0) return;
  constexpr int PER = kHashTile / NT;
  __shared__ uint64_t lt[kHashTile];   // the tile's tokens
  __shared__ uint32_t ls[kHashLds];    // local table: tile index + 1 (0 = empty); then global slots
  __shared__ uint32_t new_i[kHashTile], new_h[kHashTile];
  __shared__ uint32_t nnew, nbase;
  for (uint64_t t0 = (uint64_t)blockIdx.x * kHashTile; t0 < n; t0 += (uint64_t)gridDim.x * kHashTile) {
    const uint32_t m = (uint32_t)min((uint64_t)kHashTile, n - t0);
    for (uint32_t k = threadIdx.x; k < kHashLds; k += NT) ls[k] = 0;
    for (uint32_t k = threadIdx.x; k < m; k += NT) lt[k] = tok[t0 + k];
    if (threadIdx.x == 0) nnew = 0;
    __syncthreads();
    uint32_t hl[PER], gs[PER];  // local table entry of each token; global slot (first occurrences)
    uint32_t first = 0;
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const uint32_t k = threadIdx.x + (uint32_t)u * NT;
      hl[u] = 0;
      gs[u] = 0;
      if (k >= m) continue;
      if (wflag && !wflag[wid[t0 + k]]) {
        hl[u] = kHashLds;  // not this table's token
        continue;
      }
      const uint64_t key = lt[k];
      uint32_t h = (uint32_t)(mix64(key) >> 40) & (kHashLds - 1);
      while (true) {
        uint32_t prev = ls[h];
        if (prev == 0u) prev = atomicCAS(&ls[h], 0u, k + 1);
        if (prev == 0u) {  // first in this tile
          uint64_t slot;
          if (global_insert(key, tab, mask, &slot)) {
            const uint32_t q = atomicAdd(&nnew, 1u);
            new_i[q] = (uint32_t)(t0 + k);
            new_h[q] = (uint32_t)slot;
          }
          gs[u] = (uint32_t)slot;
          first |= 1u << u;
          break;
        }
        if (lt[prev - 1] == key) break;
        h = (h + 1) & (kHashLds - 1);
      }
      hl[u] = h;
    }
    __syncthreads();  // every probe of the local table is done
#pragma unroll
    for (int u = 0; u < PER; u++)
      if (first & (1u << u)) ls[hl[u]] = gs[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; u++) {
      const uint32_t k = threadIdx.x + (uint32_t)u * NT;
      if (k < m && hl[u] < kHashLds) tok_slot[t0 + k] = ls[hl[u]];
    }
    if (threadIdx.x == 0) nbase = nnew ? atomicAdd(nd, nnew) : 0u;
    __syncthreads();
    for (uint32_t k = threadIdx.x; k < nnew; k += blockDim.x) {
      dist_idx[nbase + k] = new_i[k];
      dist_slot[nbase + k] = new_h[k];
    }
    __syncthreads();
  }
}

__global__ void k_hash_fields(const uint64_t *tok, const uint32_t *dist_idx, const uint32_t *nd,
                              uint32_t *hi, uint32_t *lo) {
  const uint32_t m = *nd;
  GRID_STRIDE(d, m) {
    const uint64_t t = tok[dist_idx[d]];
    hi[d] = (uint32_t)(t >> 32);
    lo[d] = (uint32_t)t;
  }
}

__global__ void k_hash_assign(const uint32_t *sorted_d, const uint32_t *nd, const uint32_t *dist_slot,
                              uint32_t *slot_rank) {
  const uint32_t m = *nd;
  GRID_STRIDE(q, m) slot_rank[dist_slot[sorted_d[q]]] = (uint32_t)q + 1u;
}

// rank of every token from its slot (in place: out may be tok_slot); four
// tokens per thread with the loads issued together.
__global__ void k_hash_rank(const uint32_t *tok_slot, uint64_t n, const uint32_t *slot_rank, uint32_t *out,
                            const uint32_t *wid, const uint8_t *wflag, const uint32_t *gate) {
  if (gate && *gate == 0) return;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x * 4;
  for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x * 4; b0 < n; b0 += step) {
    uint32_t sl[4], r[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t i = b0 + (uint64_t)u * blockDim.x + threadIdx.x;
      const bool mine = i < n && (!wflag || wflag[wid[i]]);
      sl[u] = mine ? tok_slot[i] : ~0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      r[u] = sl[u] != ~0u ? slot_rank[sl[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t i = b0 + (uint64_t)u * blockDim.x + threadIdx.x;
      if (sl[u] != ~0u) out[i] = r[u];
    }
  }
}

__global__ void k_fill_u64(unsigned long long *p, uint64_t n, unsigned long long v, const uint32_t *gate) {
  if (gate && *gate == 0) return;
  GRID_STRIDE(i, n) p[i] = v;
}

void hash_clear(uint64_t *tab, uint64_t mask, hipStream_t s, const uint32_t *gate) {
  auto *t = reinterpret_cast<unsigned long long *>(tab);
  hipLaunchKernelGGL(k_fill_u64, grid_for(mask + 1, 256, 8192), dim3(256), 0, s, t, mask + 1,
                     (unsigned long long)kEmpty, gate);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, t + mask + 1, (uint64_t)1, 0ull, gate);
}

void hash_insert(const uint64_t *tok, uint64_t n, uint64_t *tab, uint64_t mask, uint32_t *dist_idx,
                 uint32_t *dist_slot, uint32_t *nd, uint32_t *tok_slot, hipStream_t s, const uint32_t *wid,
                 const uint8_t *wflag, const uint32_t *gate) {
  const uint64_t tiles = (n + kHashTile - 1) / kHashTile;
  hipLaunchKernelGGL(k_hash_insert, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>(tiles, 1), 4096)), dim3(256),
                     0, s, tok, n, reinterpret_cast<unsigned long long *>(tab), mask, dist_idx, dist_slot, nd,
                     tok_slot, wid, wflag, gate);
}
void hash_fields(const uint64_t *tok, const uint32_t *dist_idx, const uint32_t *nd, uint32_t *hi,
                 uint32_t *lo, uint64_t hint, hipStream_t s) {
  hipLaunchKernelGGL(k_hash_fields, grid_for(hint, 256, 8192), dim3(256), 0, s, tok, dist_idx, nd, hi, lo);
}
void hash_assign(const uint32_t *sorted_d, const uint32_t *nd, const uint32_t *dist_slot, uint32_t *slot_rank,
                 uint64_t hint, hipStream_t s) {
  hipLaunchKernelGGL(k_hash_assign, grid_for(hint, 256, 8192), dim3(256), 0, s, sorted_d, nd, dist_slot,
                     slot_rank);
}
void hash_rank(const uint32_t *tok_slot, uint64_t n, const uint32_t *slot_rank, uint32_t *out, hipStream_t s,
               const uint32_t *wid, const uint8_t *wflag, const uint32_t *gate) {
  hipLaunchKernelGGL(k_hash_rank, grid_for((n + 3) / 4, 256, 8192), dim3(256), 0, s, tok_slot, n, slot_rank, out,
                     wid, wflag, gate);
}

// Appends a large unit to a list of the sort engine: packed (units << 32 |
// chunks) counter, chunk base from the old value (the engine's list format).
__device__ __forceinline__ void append_big_unit(BigUnit *list, unsigned long long *pk, uint32_t cap, uint32_t start,
                                                uint32_t len, uint32_t meta, uint32_t *err, uint32_t chunk_log) {
  const unsigned long long old = atomicAdd(pk, (1ull << 32) | ((len + (1u << chunk_log) - 1) >> chunk_log));
  const uint32_t k = (uint32_t)(old >> 32);
  if (k < cap) list[k] = BigUnit{start, len, (uint32_t)old, meta};
  else atomicOr(err, 2u);
}

// ------------------------------------------------ per-window token ranks
// Only the order of tokens within a window matters (the first doubling round
// sorts each window's suffixes by first token, and the LCP walk compares
// tokens of one window), so a batch ranks each window on its own, one
// workgroup per window at a time (workgroups take windows from a counter, so
// a long window never holds up the dispatch of the others):
//  1. the window's distinct values go into an LDS hash table (and a list);
//  2. each value's slot receives its 1-based rank among them: the list is
//     sorted in runs of 64 by a bitonic network over lane shuffles within
//     each wavefront, then runs are merged pairwise up to the whole list,
//     each element finding its place by a binary search in the other run
//     (one barrier per merge level: 6 for 4096 values);
//  3. every token's rank is read from its slot (one probe, usually one LDS
//     read).
// The token value kEmpty (the largest) marks free slots, so it is counted
// aside and ranks last.  A window with more than kWinRankCap distinct values
// is flagged instead and ranked through the shared global table.
// cnt[0] += distinct values of a ranked window, cnt[1] = their maximum,
// cnt[2] += 1 per flagged window, cnt[3]: window counter (zeroed by the caller).
constexpr int kWinRankThreads = 1024;
constexpr int kWinRankSlots = 8192;
constexpr uint32_t kWinRankCap = 4096;
constexpr int kWinRankRegs = kWinRankCap / kWinRankThreads;  // sorted values per thread
constexpr int kWinRankBatch = 16;

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange of element i with its partner value p in the bitonic
// merge of size k at distance j: the element that ends up lower keeps the
// minimum when the block of size k is ascending.
__device__ __forceinline__ uint64_t bitonic_keep(uint64_t v, uint64_t p, uint32_t i, uint32_t j, uint32_t k) {
  const bool lower = (i & j) == 0, asc = (i & k) == 0;
  return (lower == asc) ? (v < p ? v : p) : (v < p ? p : v);
}

__device__ __forceinline__ uint32_t win_probe(const unsigned long long *tab, uint64_t key) {
  uint32_t h = (uint32_t)(mix64(key) >> 40) & (kWinRankSlots - 1);
  while (tab[h] != (unsigned long long)key) h = (h + 1) & (kWinRankSlots - 1);
  return h;
}

__global__ __launch_bounds__(kWinRankThreads) void k_win_rank(const uint64_t *tok, const uint64_t *off,
                                                             const uint32_t *order, uint32_t nw, uint32_t *rank,
                                                             uint8_t *wflag, uint32_t *cnt) {
  constexpr int NT = kWinRankThreads;
  __shared__ unsigned long long tab[kWinRankSlots];
  __shared__ uint64_t dist[kWinRankCap];   // distinct values; then merge buffers with mrg
  __shared__ uint64_t mrg[kWinRankCap];
  __shared__ uint16_t srank[kWinRankSlots];    // rank of the value in each slot
  __shared__ uint32_t nd, ovf, hasmax, cur_w;
  const int tid = threadIdx.x;
  for (;;) {
    __syncthreads();  // the previous window's reads of the shared state are done
    if (tid == 0) {
      cur_w = atomicAdd(&cnt[3], 1u);
      nd = 0;
      ovf = 0;
      hasmax = 0;
    }
    for (int k = tid; k < kWinRankSlots; k += NT) tab[k] = (unsigned long long)kEmpty;
    __syncthreads();
    if (cur_w >= nw) return;  // uniform
    const uint32_t w = order ? order[cur_w] : cur_w;
    const uint64_t b = off[w] - off[0], e = off[w + 1] - off[0];
    // 1. distinct values, kWinRankBatch tokens per thread per pass (loads first)
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint64_t kv[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        kv[u] = i < e ? tok[i] : 0ull;
      }
      if (*(volatile uint32_t *)&ovf) break;  // the window goes to the shared table anyway
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        if (i0 + (uint64_t)u * NT + tid >= e) break;
        const uint64_t key = kv[u];
        if (key == kEmpty) {
          hasmax = 1;
          continue;
        }
        uint32_t h = (uint32_t)(mix64(key) >> 40) & (kWinRankSlots - 1);
        for (int probe = 0;; probe++) {
          if (probe == kWinRankSlots) {  // full table (only after the cap is passed)
            ovf = 1;
            break;
          }
          unsigned long long c = tab[h];
          if (c == (unsigned long long)kEmpty) {
            c = atomicCAS(&tab[h], (unsigned long long)kEmpty, (unsigned long long)key);
            if (c == (unsigned long long)kEmpty) {
              const uint32_t q = atomicAdd(&nd, 1u);
              if (q < kWinRankCap) dist[q] = key;
              else ovf = 1;
              break;
            }
          }
          if (c == key) break;
          h = (h + 1) & (kWinRankSlots - 1);
        }
      }
    }
    __syncthreads();
    const bool flagged = ovf != 0;
    if (tid == 0) {
      wflag[w] = flagged ? 1 : 0;
      if (flagged) atomicAdd(&cnt[2], 1u);
    }
    if (flagged) continue;  // uniform
    const uint32_t D = nd;
    uint32_t P = 64;
    while (P < D) P <<= 1;
    const int R = (int)((P + NT - 1) / NT);
    const bool holds = (uint32_t)tid < P;  // P < NT: whole wavefronts hold one value or none
    // 2a. element i = r * NT + tid in v[r] (pads: kEmpty); each wavefront's
    // 64 elements of one register sorted ascending by a bitonic network over
    // lane shuffles (constant distances after unrolling)
    uint64_t v[kWinRankRegs];
#pragma unroll
    for (int r = 0; r < kWinRankRegs; r++) {
      const uint32_t i = (uint32_t)r * NT + tid;
      v[r] = (r < R && holds && i < D) ? dist[i] : kEmpty;
    }
    const uint32_t ln = (uint32_t)tid & 63;
#pragma unroll
    for (uint32_t k = 2; k <= 64; k <<= 1)
#pragma unroll
      for (uint32_t j = k >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int r = 0; r < kWinRankRegs; r++)
          if (r < R) v[r] = bitonic_keep(v[r], shfl_xor_u64(v[r], (int)j), ln, j, k == 64 ? 128 : k);
    __syncthreads();  // every list read is done before the buffers are reused
    // 2b. runs of 64 merged pairwise, 64 -> P: an element's place in the
    // merged run is its index in its own run plus the number of elements of
    // the other run before it (lower bound from the left run, upper bound
    // from the right one, so equal pads keep distinct places)
    int cb = 0;  // merge source: dist (0) or mrg (1)
#pragma unroll
    for (int r = 0; r < kWinRankRegs; r++)
      if (r < R && holds) dist[(uint32_t)r * NT + tid] = v[r];
    __syncthreads();
    uint32_t pos[kWinRankRegs];
#pragma unroll
    for (int r = 0; r < kWinRankRegs; r++) pos[r] = (uint32_t)r * NT + tid;
    for (uint32_t L = 64; L < P; L <<= 1) {
      const uint64_t *src = cb ? mrg : dist;
      uint64_t *dst = cb ? dist : mrg;
#pragma unroll
      for (int r = 0; r < kWinRankRegs; r++) {
        if (!(r < R && holds)) continue;
        const uint32_t i = pos[r];
        const uint64_t x = v[r];
        const uint32_t base = i & ~(2 * L - 1), right = i & L;
        const bool rt = right != 0;
        const uint64_t *o = src + (right ? base : base + L);  // the other run
        uint32_t c = 0;  // elements of the other run before x
        // branch-free steps (the comparison depends on the lane's run; as
        // a branch it compiled to divergent control flow per step)
        for (uint32_t step = L >> 1; step > 0; step >>= 1) {
          const uint64_t y = o[c + step - 1];
          c += ((y < x) | ((y == x) & rt)) ? step : 0u;
        }
        c += ((o[c] < x) | ((o[c] == x) & rt)) ? 1u : 0u;  // c <= L - 1 before this step
        pos[r] = base + (i - base - right) + c;
        dst[pos[r]] = x;
      }
      __syncthreads();
      cb ^= 1;
    }
    // 3. ranks into the slots
#pragma unroll
    for (int r = 0; r < kWinRankRegs; r++)
      if (r < R && holds && v[r] != kEmpty) srank[win_probe(tab, v[r])] = (uint16_t)(pos[r] + 1);
    __syncthreads();
    // every token's rank from its slot
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint64_t kv[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        kv[u] = i < e ? tok[i] : kEmpty;
      }
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        if (i < e) rank[i] = kv[u] == kEmpty ? D + 1 : (uint32_t)srank[win_probe(tab, kv[u])];
      }
    }
    if (tid == 0) {
      const uint32_t sig = D + hasmax;
      atomicAdd(&cnt[0], sig);
      atomicMax(&cnt[1], sig);
    }
  }
}

static unsigned cu_count() {
  static const unsigned cus = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || n <= 0) {
      (void)hipGetLastError();
      n = 256;
    }
    return (unsigned)n;
  }();
  return cus;
}

void win_rank(const uint64_t *tok, const uint64_t *off, const uint32_t *order, uint32_t nw, uint32_t *rank,
              uint8_t *wflag, uint32_t *cnt, hipStream_t s) {
  // one workgroup per compute unit (the LDS footprint allows one), each
  // taking windows until none is left
  if (nw) hipLaunchKernelGGL(k_win_rank, dim3(std::min<unsigned>(cu_count(), nw)), dim3(kWinRankThreads), 0, s, tok, off,
                             order, nw, rank, wflag, cnt);
}

// ------------------------------------------- per-window ranks of token pairs
// The doubling rounds refine groups of equal 2^r-token prefixes.  A batch
// whose windows all have few distinct adjacent pairs gets the state after
// the second round (groups of equal two-token prefix) directly from the
// window's token ranks, and the engine starts at offset 2.  Per window, one
// workgroup at a time (windows taken from a counter):
//  1. the window's distinct pair keys (rank of token i, rank of token i+1 or
//     0 past the window's end) go into an LDS hash table and a list, and the
//     occurrences of each first token are counted (the suffixes that the
//     first round leaves grouped: that round's active count, added to *act1);
//  2. the list is sorted (bitonic runs of 64 over lane shuffles, then merges
//     by binary search) and each slot receives its key's 1-based rank;
//  3. every suffix's pair rank is read from its slot.
// Token ranks are at most kWinRankCap + 1 (13 bits), so a pair key fits in
// 26 bits and 0xFFFFFFFF marks free slots.  A window with more than
// kPairCap distinct pairs, or without ranks of its own (wflag set), is
// counted in cnt[1] and left alone: the caller then takes the first two
// rounds the usual way for the whole batch.  cnt[0]: window counter.  When
// *wcount (windows without ranks of their own) is not zero the kernel only
// sets cnt[1].
constexpr int kPairSlots = 16384;
constexpr uint32_t kPairCap = 8192;
constexpr int kPairRegs = kPairCap / kWinRankThreads;  // sorted keys per thread
constexpr uint32_t kPairEmpty = 0xFFFFFFFFu;
constexpr uint32_t kTokRanks = kWinRankCap + 2;  // token ranks 1..kWinRankCap + 1

__device__ __forceinline__ uint32_t pair_probe(const uint32_t *tab, uint32_t key) {
  uint32_t h = (uint32_t)(mix64(key) >> 40) & (kPairSlots - 1);
  while (tab[h] != key) h = (h + 1) & (kPairSlots - 1);
  return h;
}

__device__ __forceinline__ uint32_t bitonic_keep32(uint32_t v, uint32_t p, uint32_t i, uint32_t j, uint32_t k) {
  const bool lower = (i & j) == 0, asc = (i & k) == 0;
  return (lower == asc) ? (v < p ? v : p) : (v < p ? p : v);
}

__global__ __launch_bounds__(kWinRankThreads) void k_win_pair(const uint64_t *off, const uint32_t *order, uint32_t nw,
                                                             const uint8_t *wflag,
                                                             const uint32_t *tokrank, uint32_t *prank, uint32_t *cnt,
                                                             uint32_t *act1, const uint32_t *wcount) {
  constexpr int NT = kWinRankThreads;
  if (*wcount) {  // uniform: the batch takes the usual first rounds anyway
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&cnt[1], 1u);
    return;
  }
  __shared__ uint32_t tab[kPairSlots];
  __shared__ uint32_t dist[kPairCap];
  // first-token counts (kTokRanks words), then the merge buffer, then the
  // slots' ranks (kPairSlots u16): never two of them at once
  __shared__ uint32_t aux[kPairCap];
  __shared__ uint32_t nd, ovf, cur_w, a1;
  static_assert(kTokRanks <= kPairCap && kPairSlots * 2 <= kPairCap * 4, "aux too small");
  uint32_t *const hc = aux;
  uint16_t *const srank = reinterpret_cast<uint16_t *>(aux);
  const int tid = threadIdx.x;
  for (;;) {
    __syncthreads();  // the previous window's reads of the shared state are done
    if (tid == 0) {
      cur_w = atomicAdd(&cnt[0], 1u);
      nd = 0;
      ovf = 0;
      a1 = 0;
    }
    for (int k = tid; k < kPairSlots; k += NT) tab[k] = kPairEmpty;
    for (uint32_t k = tid; k < kTokRanks; k += NT) hc[k] = 0;
    __syncthreads();
    if (cur_w >= nw) return;  // uniform
    const uint32_t w = order ? order[cur_w] : cur_w;
    if (wflag[w]) {       // the same word for every thread
      if (tid == 0) atomicAdd(&cnt[1], 1u);
      continue;
    }
    const uint64_t b = off[w] - off[0], e = off[w + 1] - off[0];
    // 1. distinct pairs and first-token counts (loads of a pass first)
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint32_t r1[kWinRankBatch], r2[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        r1[u] = i < e ? tokrank[i] : 0u;
        r2[u] = i + 1 < e ? tokrank[i + 1] : 0u;
      }
      if (*(volatile uint32_t *)&ovf) break;  // the batch takes the usual path anyway
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        if (i0 + (uint64_t)u * NT + tid >= e) break;
        atomicAdd(&hc[r1[u]], 1u);
        const uint32_t key = (r1[u] << 13) | r2[u];
        uint32_t h = (uint32_t)(mix64(key) >> 40) & (kPairSlots - 1);
        for (int probe = 0;; probe++) {
          if (probe == kPairSlots) {  // full table (only after the cap is passed)
            ovf = 1;
            break;
          }
          uint32_t c = tab[h];
          if (c == kPairEmpty) {
            c = atomicCAS(&tab[h], kPairEmpty, key);
            if (c == kPairEmpty) {
              const uint32_t q = atomicAdd(&nd, 1u);
              if (q < kPairCap) dist[q] = key;
              else ovf = 1;
              break;
            }
          }
          if (c == key) break;
          h = (h + 1) & (kPairSlots - 1);
        }
      }
    }
    __syncthreads();
    const bool flagged = ovf != 0;
    if (flagged) {  // uniform
      if (tid == 0) atomicAdd(&cnt[1], 1u);
      continue;
    }
    {
      uint32_t part = 0;
      for (uint32_t k = tid; k < kTokRanks; k += NT) {
        const uint32_t c = hc[k];
        part += c >= 2 ? c : 0u;
      }
      part = wave_incl_sum(part);
      if ((tid & 63) == 63 && part) atomicAdd(&a1, part);
    }
    const uint32_t D = nd;
    uint32_t P = 64;
    while (P < D) P <<= 1;
    const int R = (int)((P + NT - 1) / NT);
    const bool holds = (uint32_t)tid < P;  // P < NT: whole wavefronts hold one key or none
    // 2a. element i = r * NT + tid in v[r] (pads: kPairEmpty), each
    // wavefront's 64 elements of one register sorted ascending
    uint32_t v[kPairRegs];
#pragma unroll
    for (int r = 0; r < kPairRegs; r++) {
      const uint32_t i = (uint32_t)r * NT + tid;
      v[r] = (r < R && holds && i < D) ? dist[i] : kPairEmpty;
    }
    const uint32_t ln = (uint32_t)tid & 63;
#pragma unroll
    for (uint32_t k = 2; k <= 64; k <<= 1)
#pragma unroll
      for (uint32_t j = k >> 1; j > 0; j >>= 1)
#pragma unroll
        for (int r = 0; r < kPairRegs; r++)
          if (r < R)
            v[r] = bitonic_keep32(v[r], (uint32_t)__shfl_xor((int)v[r], (int)j, 64), ln, j, k == 64 ? 128 : k);
    __syncthreads();  // list and counts read, a1 complete
    if (tid == 0 && a1) atomicAdd(act1, a1);
#pragma unroll
    for (int r = 0; r < kPairRegs; r++)
      if (r < R && holds) dist[(uint32_t)r * NT + tid] = v[r];
    __syncthreads();
    // 2b. runs merged pairwise, 64 -> P: an element's place is its index in
    // its own run plus the elements of the other run before it (strictly
    // smaller ones from the left run, smaller or equal ones from the right
    // one; keys are distinct, pads all equal)
    uint32_t pos[kPairRegs];
#pragma unroll
    for (int r = 0; r < kPairRegs; r++) pos[r] = (uint32_t)r * NT + tid;
    int cb = 0;  // merge source: dist (0) or aux (1)
    for (uint32_t L = 64; L < P; L <<= 1) {
      const uint32_t *src = cb ? aux : dist;
      uint32_t *dst = cb ? dist : aux;
#pragma unroll
      for (int r = 0; r < kPairRegs; r++) {
        if (!(r < R && holds)) continue;
        const uint32_t i = pos[r], x = v[r];
        const uint32_t base = i & ~(2 * L - 1), right = i & L;
        const bool rt = right != 0;
        const uint32_t *o = src + (right ? base : base + L);
        uint32_t c = 0;
        for (uint32_t step = L >> 1; step > 0; step >>= 1) {  // branch-free steps
          const uint32_t y = o[c + step - 1];
          c += ((y < x) | ((y == x) & rt)) ? step : 0u;
        }
        c += ((o[c] < x) | ((o[c] == x) & rt)) ? 1u : 0u;  // c <= L - 1 before this step
        pos[r] = base + (i - base - right) + c;
        dst[pos[r]] = x;
      }
      __syncthreads();
      cb ^= 1;
    }
    // 3. ranks into the slots (aux is free now), then every suffix's rank
#pragma unroll
    for (int r = 0; r < kPairRegs; r++)
      if (r < R && holds && v[r] != kPairEmpty) srank[pair_probe(tab, v[r])] = (uint16_t)(pos[r] + 1);
    __syncthreads();
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint32_t r1[kWinRankBatch], r2[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        r1[u] = i < e ? tokrank[i] : 0u;
        r2[u] = i + 1 < e ? tokrank[i + 1] : 0u;
      }
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        if (i < e) prank[i] = srank[pair_probe(tab, (r1[u] << 13) | r2[u])];
      }
    }
  }
}

void win_pair(const uint64_t *off, const uint32_t *order, uint32_t nw, const uint8_t *wflag, const uint32_t *tokrank,
              uint32_t *prank, uint32_t *cnt, uint32_t *act1, const uint32_t *wcount, hipStream_t s) {
  // one workgroup per compute unit (the LDS footprint allows one)
  if (nw) hipLaunchKernelGGL(k_win_pair, dim3(std::min<unsigned>(cu_count(), nw)), dim3(kWinRankThreads), 0, s, off,
                             order, nw, wflag, tokrank, prank, cnt, act1, wcount);
}

// ------------------------------------ first doubling round, per window
// The first round of the suffix sort for the windows ranked on their own:
// each window's suffixes grouped by their rank (first token, or first two
// tokens after k_win_pair), by a counting sort on the window's ranks (at most
// RANKS - 1 of them) in LDS, written in the form the later doubling rounds
// take over from a round of the sort engine: the suffix arrangement in
// val[0], rank[i] = 1 + slot of the first suffix of i's group, the
// grouped-slot flags, and every group of two or more as a unit of list LIST
// (kHeadBit set: its suffixes' ranks are its start + 1) in its size class,
// or in the large-unit list when it exceeds the LDS tile (next_bits key
// bits), with the active-slot count.  Flagged windows are left to the
// engine.  Workgroups take windows from the counter *wnext.  With pflag set
// the kernel runs only when *pflag == 0 (pair ranks for every window) for
// the pair form, only when *pflag != 0 for the first-token form.  The pair
// form also records the first round's active count *a1 in *hist0.
constexpr uint32_t kR0SingleWords = 4096;  // singleton-slot bitmap: windows up to 2^17 slots

template <uint32_t RANKS, int LIST>
__global__ __launch_bounds__(kWinRankThreads) void k_win_round0(SortBufs B, const uint64_t *off,
                                                               const uint32_t *order, uint32_t nw,
                                                               const uint8_t *wflag, const uint32_t *keyrank,
                                                               uint32_t *rank, uint8_t *aflag, uint32_t next_bits,
                                                               uint32_t *wnext, const uint32_t *pflag,
                                                               const uint32_t *a1, uint32_t *hist0) {
  constexpr int NT = kWinRankThreads;
  constexpr int PER = (RANKS + NT - 1) / NT;
  constexpr uint32_t TOP = 1u << (31 - __builtin_clz(RANKS - 1));  // largest power of two below RANKS
  // cnt: counts, then each group's next free slot; gst: group starts
  // (window-relative), gst[RANKS] = window length, so a count is a difference
  __shared__ uint32_t cnt[RANKS], gst[RANKS + 1];
  __shared__ uint32_t single[kR0SingleWords];  // bit s: slot s holds a group of one
  __shared__ uint32_t sh[NT / 64];
  __shared__ uint32_t cls_loc[kClasses], cls_base[kClasses];
  __shared__ uint32_t cur_w;
  const int tid = threadIdx.x;
  const uint32_t tile = 1u << B.tile_log;
  if (pflag && ((*pflag == 0) != (LIST == 0))) return;  // uniform: the other form runs
  if (a1 && blockIdx.x == 0 && tid == 0) *hist0 = *a1;
  for (;;) {
    __syncthreads();  // the previous window's reads of the shared state are done
    if (tid == 0) cur_w = atomicAdd(wnext, 1u);
    for (uint32_t r = tid; r < RANKS; r += NT) cnt[r] = 0;
    if (tid < kClasses) cls_loc[tid] = 0;
    __syncthreads();
    if (cur_w >= nw) return;  // uniform
    const uint32_t w = order ? order[cur_w] : cur_w;
    if (wflag[w]) continue;  // the same word for every thread
    const uint64_t b = off[w] - off[0], e = off[w + 1] - off[0];
    const bool bits = e - b <= 32ull * kR0SingleWords;  // uniform
    if (bits)
      for (uint32_t k = tid; k < (uint32_t)((e - b + 31) / 32); k += NT) single[k] = 0;
    // counts of the ranks
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint32_t rq[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        rq[u] = i < e ? keyrank[i] : 0u;
      }
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++)
        if (i0 + (uint64_t)u * NT + tid < e) atomicAdd(&cnt[rq[u]], 1u);
    }
    __syncthreads();
    // group starts: exclusive scan, PER consecutive ranks a thread
    {
      const uint32_t r0 = (uint32_t)tid * PER;
      uint32_t c[PER], loc = 0;
#pragma unroll
      for (int q = 0; q < PER; q++) {
        c[q] = r0 + q < RANKS ? cnt[r0 + q] : 0u;
        loc += c[q];
      }
      uint32_t tot;
      uint32_t ex = block_excl_sum<NT>(loc, sh, &tot);  // its barriers order the reads above before the writes
#pragma unroll
      for (int q = 0; q < PER; q++)
        if (r0 + q < RANKS) {
          gst[r0 + q] = ex;
          cnt[r0 + q] = ex;
          ex += c[q];
        }
      if (tid == 0) gst[RANKS] = tot;
    }
    __syncthreads();
    // groups of two or more: units of the next list, reserved once per class
    uint32_t ur[PER], ui[PER];
    uint32_t act = 0;
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const uint32_t r = (uint32_t)tid * PER + q;
      ur[q] = 0;
      ui[q] = 0;
      const uint32_t c = r < RANKS ? gst[r + 1] - gst[r] : 0u;
      if (c == 1 && bits) atomicOr(&single[gst[r] >> 5], 1u << (gst[r] & 31));
      if (c < 2) continue;
      act += c;
      ur[q] = r;
      if (c <= tile) ui[q] = atomicAdd(&cls_loc[class_of(c)], 1u);
      else append_big_unit(B.big[LIST][0], &B.ctr->big_pk[LIST][0], B.big_cap, (uint32_t)b + gst[r], c, next_bits,
                           &B.ctr->err, B.chunk_log);
    }
    {
      uint32_t tot;
      (void)block_excl_sum<NT>(act, sh, &tot);
      if (tid == 0 && tot) atomicAdd(&B.ctr->act_cnt[LIST], tot);
    }
    if (tid < kClasses) cls_base[tid] = cls_loc[tid] ? atomicAdd(&B.ctr->cls_cnt[LIST][tid], cls_loc[tid]) : 0u;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PER; q++) {
      const uint32_t r = ur[q];
      if (!r) continue;
      const uint32_t c = gst[r + 1] - gst[r];
      if (c > tile) continue;
      const int ci = class_of(c);
      const uint32_t k = cls_base[ci] + ui[q];
      if (k < B.cls_off[ci + 1] - B.cls_off[ci]) B.cls[LIST][B.cls_off[ci] + k] = Unit{(uint32_t)b + gst[r], c | kHeadBit};
      else atomicOr(&B.ctr->err, 8u);
    }
    // suffixes into their groups' slots; ranks and flags
    for (uint64_t i0 = b; i0 < e; i0 += (uint64_t)NT * kWinRankBatch) {
      uint32_t rq[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        rq[u] = i < e ? keyrank[i] : 0u;
      }
      // every slot reservation of the batch first, then the stores
      uint32_t sq[kWinRankBatch];
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++)
        sq[u] = i0 + (uint64_t)u * NT + tid < e ? atomicAdd(&cnt[rq[u]], 1u) : 0u;
#pragma unroll
      for (int u = 0; u < kWinRankBatch; u++) {
        const uint64_t i = i0 + (uint64_t)u * NT + tid;
        if (i >= e) continue;
        const uint32_t r = rq[u], slot = (uint32_t)b + sq[u];
        B.val[0][slot] = (uint32_t)i;
        rank[i] = (uint32_t)b + gst[r] + 1;
      }
    }
    // grouped-slot flags in slot order (coalesced, where scattering them with
    // the suffixes cost as much as the suffixes): a slot is grouped unless it
    // holds a group of one, marked in the bitmap by the units pass; windows
    // too long for the bitmap search the group starts (the last rank whose
    // start is <= s; gst[RANKS], the window length, stops the search)
    for (uint64_t s0 = 0; s0 < e - b; s0 += NT) {
      const uint32_t sl = (uint32_t)s0 + tid;
      if (sl >= e - b) break;
      if (bits) {
        aflag[b + sl] = ((single[sl >> 5] >> (sl & 31)) & 1u) ? 0 : 1;
      } else {
        uint32_t lo = 0;  // gst[0] = 0
        for (uint32_t step = TOP; step > 0; step >>= 1) {
          const uint32_t t = min(lo + step, RANKS);
          lo = gst[t] <= sl ? t : lo;
        }
        aflag[b + sl] = gst[lo + 1] - gst[lo] >= 2 ? 1 : 0;
      }
    }
  }
}

void win_round0(const SortBufs &B, const uint64_t *off, const uint32_t *order, uint32_t nw, const uint8_t *wflag,
                const uint32_t *keyrank, uint32_t *rank, uint8_t *aflag, uint32_t next_bits, uint32_t *wnext, bool pairs,
                const uint32_t *pflag, const uint32_t *a1, uint32_t *hist0, hipStream_t s) {
  if (!nw) return;
  const dim3 grid(std::min<unsigned>(2 * cu_count(), nw)), block(kWinRankThreads);
  if (pairs)
    hipLaunchKernelGGL((k_win_round0<kPairCap + 2, 0>), grid, block, 0, s, B, off, order, nw, wflag, keyrank, rank, aflag,
                       next_bits, wnext, pflag, a1, hist0);
  else
    hipLaunchKernelGGL((k_win_round0<kTokRanks, 1>), grid, block, 0, s, B, off, order, nw, wflag, keyrank, rank, aflag,
                       next_bits, wnext, pflag, nullptr, nullptr);
}

// -------------------------------------------------------------- windows
// Per-slot window bounds for batched input (offsets are global, ascending).
__global__ void k_window_bounds(const uint64_t *off, uint32_t nw, uint32_t *wbeg, uint32_t *wend,
                                uint32_t *wid) {
  const uint32_t w = blockIdx.x;
  if (w >= nw) return;
  const uint32_t b = (uint32_t)(off[w] - off[0]), e = (uint32_t)(off[w + 1] - off[0]);
  for (uint32_t p = b + threadIdx.x; p < e; p += blockDim.x) {
    wbeg[p] = b;
    wend[p] = e;
    wid[p] = w;
  }
}

void window_bounds(const uint64_t *off, uint32_t nw, uint32_t *wbeg, uint32_t *wend, uint32_t *wid,
                   hipStream_t s) {
  if (nw) hipLaunchKernelGGL(k_window_bounds, dim3(nw), dim3(256), 0, s, off, nw, wbeg, wend, wid);
}

// ------------------------------------------------------------------- LCP
// Snapshot level j is the whole rank array after doubling round j: two
// suffixes of one window carry equal ranks there iff their 2^j-prefixes are
// equal (a suffix alone in its group has a rank no other suffix has).  It is
// a coalesced copy taken once per round instead of a scattered write of every
// grouped suffix's rank by the sort kernels.
__global__ void k_snapshot(const uint32_t *rank, uint32_t *snap_r, uint64_t n, const uint32_t *act_dev,
                           uint32_t *snaps, int r) {
  if (*act_dev == 0) return;  // nothing was sorted: no later level is read
  if (blockIdx.x == 0 && threadIdx.x == 0) *snaps = (uint32_t)r + 1;
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x * 4;
  for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x * 4; b0 < n; b0 += step) {
    uint32_t v[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t i = b0 + (uint64_t)u * blockDim.x + threadIdx.x;  // coalesced for each u
      v[u] = i < n ? rank[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t i = b0 + (uint64_t)u * blockDim.x + threadIdx.x;
      if (i < n) snap_r[i] = v[u];
    }
  }
}

void snapshot_ranks(const uint32_t *rank, uint32_t *snap_r, uint64_t n, const uint32_t *act_dev, uint32_t *snaps,
                    int r, hipStream_t s) {
  hipLaunchKernelGGL(k_snapshot, grid_for((n + 3) / 4, 256, 8192), dim3(256), 0, s, rank, snap_r, n, act_dev, snaps,
                     r);
}

// lcp(x, y) >= acc known; extend by binary lifting over the per-round rank
// snapshots: 2^j-prefixes at x+acc and y+acc are equal iff their ranks after
// round j are equal.  Snapshots exist for rounds >= kSnapFrom only; the last
// < 2^kSnapFrom tokens are compared directly (key0: order-preserving token
// keys).
__device__ __forceinline__ uint32_t lcp_lift(uint32_t x, uint32_t y, uint32_t acc, uint32_t we, int top,
                                             const uint32_t *snap, uint64_t n, const uint32_t *key0) {
  for (int j = top; j >= kSnapFrom; j--) {
    const uint32_t a = x + acc, b = y + acc;
    if (a >= we || b >= we) break;
    if (snap[(uint64_t)j * n + a] == snap[(uint64_t)j * n + b]) acc += 1u << j;
  }
  // the remaining < 2^kSnapFrom tokens: issue all loads at once, then find
  // the first mismatch (or the window end)
  constexpr int kTail = 1 << kSnapFrom;
  const uint32_t a = x + acc, b = y + acc;
  const uint32_t room = (a < we && b < we) ? we - max(a, b) : 0u;
  uint32_t ka[kTail], kb[kTail];
#pragma unroll
  for (int k = 0; k < kTail; k++) {
    const bool in = (uint32_t)k < room;
    ka[k] = in ? key0[a + k] : 0u;
    kb[k] = in ? key0[b + k] : 1u;
  }
  uint32_t t = kTail;
#pragma unroll
  for (int k = kTail - 1; k >= 0; k--)
    if (ka[k] != kb[k]) t = (uint32_t)k;
  return acc + t;
}

// lcp(x, y) knowing that the first acc tokens match, for a remainder that
// is usually short: blocks of 2^kSnapFrom, 2^(kSnapFrom+1), ... tokens are
// compared while they match (an exponential search over the snapshot
// levels), then the lifting goes down from below the first level that
// differed, so a remainder r reads about 2 log2(r / 2^kSnapFrom) levels
// instead of every level up to the last snapshot.
__device__ __forceinline__ uint32_t lcp_gallop(uint32_t x, uint32_t y, uint32_t acc, uint32_t we, int top,
                                               const uint32_t *snap, uint64_t n, const uint32_t *key0) {
  int j = kSnapFrom;
  for (; j <= top; j++) {
    const uint32_t a = x + acc, b = y + acc;
    if (a >= we || b >= we || snap[(uint64_t)j * n + a] != snap[(uint64_t)j * n + b]) break;
    acc += 1u << j;
  }
  return lcp_lift(x, y, acc, we, j - 1, snap, n, key0);
}

// Kasai extension tokens read before switching to lifting: the walk of a
// workgroup lasts as long as its slowest thread, and a long extension is a
// chain of dependent reads, where lifting is a bounded one (on the batched
// loop streams: 64 tokens 1.93 ms per launch, 16: 1.79, 4: 1.58, 0 (one
// batch of 4 tokens, then lifting): 1.50)
constexpr int kKasaiCap = 0;
constexpr int kSeedGroup = 8;
constexpr int kPlcpChunk = 8;                        // positions per thread
constexpr int kPlcpSpan = 256 * kPlcpChunk;          // positions per workgroup pass
constexpr int kPlcpMargin = 256;                     // staged tokens past the span

// lcp(x, y) from scratch for y = Phi[x], the suffix just before x in the
// suffix array (rank: final ranks, rank[x] = x's slot + 1).  Groups are refined in
// place, so x's final slot lies in its group's slot range after every round,
// and y shares that group iff the group starts before x's slot: iff x's
// snapshot rank (group start + 1) is below rank[x].  Only x's snapshots are read
// (neighbouring positions for neighbouring threads), kSeedGroup levels at a
// time with independent loads; equal 2^j-prefixes imply equal 2^i-prefixes
// for i < j, so the highest shared level j* gives lcp in [2^j*, 2^(j*+1)),
// and lifting goes on below it.
__device__ __forceinline__ uint32_t lcp_seed(uint32_t x, uint32_t y, const uint32_t *rank, uint32_t we, int top,
                                             const uint32_t *snap, uint64_t n, const uint32_t *key0) {
  const uint32_t rx = rank[x];  // issued with the probe loads (their addresses do not depend on it)
  const int J = top;
  int best = kSnapFrom - 1;
  for (int lo = kSnapFrom; lo <= J; lo += kSeedGroup) {
#pragma unroll
    for (int k = 0; k < kSeedGroup; k++) {
      const int j = lo + k;
      if (j <= J && snap[(uint64_t)j * n + x] < rx) best = j;
    }
    if (best < lo + kSeedGroup - 1) break;  // a level of this group differed (or J ended it)
  }
  if (best < kSnapFrom) return lcp_lift(x, y, 0u, we, kSnapFrom - 1, snap, n, key0);  // tail only
  return lcp_lift(x, y, 1u << best, we, best - 1, snap, n, key0);
}

// Kasai's recurrence PLCP[j] >= PLCP[j-1] - 1 within chunks of kPlcpChunk
// consecutive positions; each chunk (and each window start) is seeded exactly
// by lifting, and an extension past its first kExt tokens switches to
// lifting.  Where Phi[j] = Phi[j-1] + 1 (a reducible position: most of a
// repetitive stream) the value is PLCP[j-1] - 1 exactly, with no token read.
// Phi[j] = SA[ISA[j] - 1] comes from the final ranks (rank =
// 1 + slot once every suffix is alone in its group).  A workgroup stages its
// span's Phi values and tokens in LDS with coalesced loads, so each thread's
// sequential walk reads LDS; only the Phi side of the comparisons reads
// tokens from global memory.  Each PLCP value goes straight to the LCP array
// at the slot before its suffix's (LCP[ISA[j] - 1] = PLCP[j]), so no PLCP
// array is written and no second pass permutes it.
__global__ __launch_bounds__(256) void k_plcp(const uint32_t *sa, const uint32_t *rank, uint64_t n,
                                              const uint32_t *wbeg, const uint32_t *wend, const uint32_t *snap,
                                              const uint32_t *snaps, const uint32_t *key0, int top_bound,
                                              uint32_t *lcp) {
  static_assert(kPlcpSpan == 256 * kPlcpChunk, "one staged position per thread and chunk slot");
  __shared__ uint32_t ps[pad16(kPlcpSpan)];
  __shared__ uint32_t ks[pad16(kPlcpSpan + kPlcpMargin)];
  const int top = min(top_bound, (int)*snaps - 1);  // last snapshot level (< kSnapFrom: none)
  const uint64_t nspan = (n + kPlcpSpan - 1) / kPlcpSpan;
  // spans are handed out XCD by XCD: the Phi-side reads of neighbouring spans
  // fall in the same windows, so one L2 holds them
  for (uint64_t base = 0; base < nspan; base += gridDim.x) {
    const uint64_t sp = xcd_item(base, nspan, blockIdx.x, gridDim.x);
    if (sp >= nspan) break;
    const uint64_t j0 = sp * kPlcpSpan;
    const int len = (int)min((uint64_t)kPlcpSpan, n - j0);
    const int klen = (int)min((uint64_t)(kPlcpSpan + kPlcpMargin), n - j0);
    uint32_t islot[kPlcpChunk];  // slot of each of this thread's staged positions
    uint32_t first = 0;          // bit q: that position's suffix is first of its window in the suffix array
#pragma unroll
    for (int q = 0; q < kPlcpChunk; q++) {
      const int p = threadIdx.x + q * 256;
      islot[q] = 0;
      if (p < len) {
        const uint32_t i = rank[j0 + p] - 1u;  // slot of suffix j0 + p
        const uint32_t b = wbeg ? wbeg[j0 + p] : 0u;
        ps[pad16(p)] = i > b ? sa[i - 1] : kNone;
        islot[q] = i;
        if (i <= b) first |= 1u << q;
      }
    }
    for (int p = threadIdx.x; p < klen; p += blockDim.x) ks[pad16(p)] = key0[j0 + p];
    __syncthreads();
    const int c0 = threadIdx.x * kPlcpChunk;
    if (c0 < len) {
      const int c1 = min(c0 + kPlcpChunk, len);
      uint64_t j = j0 + c0;
      uint32_t wb = wbeg ? wbeg[j] : 0u, we = wend ? wend[j] : (uint32_t)n;
      uint32_t h = 0, py = kNone;  // py: Phi of the previous position
      bool fresh = true;
      for (int c = c0; c < c1; c++, j++) {
        if (j == we) {  // the next window starts here (only with window bounds: otherwise we == n > j)
          wb = (uint32_t)j;
          we = wend[j];
        }
        if (j == wb) fresh = true;
        const uint32_t y = ps[pad16(c)];
        if (y == kNone) {
          h = 0;
          fresh = true;
        } else if (fresh) {
          h = lcp_seed((uint32_t)j, y, rank, we, top, snap, n, key0);
          fresh = false;
        } else if (y == py + 1 && h > 0) {
          // Phi[j] = Phi[j-1] + 1: suffix j-1 and its predecessor shared h
          // tokens and then differed (or met the window end), so j and its
          // predecessor share exactly h - 1: no token is read
          h--;
        } else {
          // extend from h - 1, kExt tokens per step with independent loads
          constexpr int kExt = 4;
          h = h > 0 ? h - 1 : 0;
          int steps = 0;
          for (;;) {
            const uint32_t a = (uint32_t)j + h, b = y + h;
            if (a >= we || b >= we) break;
            const uint32_t room = we - max(a, b);
            const uint32_t q = a - (uint32_t)j0;
            uint32_t ka[kExt], kb[kExt];
#pragma unroll
            for (int k = 0; k < kExt; k++) {
              const bool in = (uint32_t)k < room;
              kb[k] = in ? key0[b + k] : 0u;
              ka[k] = in ? (q + k < (uint32_t)klen ? ks[pad16((int)(q + k))] : key0[a + k]) : 1u;
            }
            uint32_t m = kExt;
#pragma unroll
            for (int k = kExt - 1; k >= 0; k--)
              if (ka[k] != kb[k]) m = (uint32_t)k;
            h += m;
            if (m < (uint32_t)kExt) break;
            steps += kExt;
            if (steps > kKasaiCap) { h = lcp_gallop((uint32_t)j, y, h, we, top, snap, n, key0); break; }
          }
        }
        ps[pad16(c)] = h;  // this thread's own slot, already read
        py = y;
      }
    }
    __syncthreads();
    // LCP[i - 1] = lcp(SA[i - 1], SA[i]) = PLCP[SA[i]]: each value goes to the
    // slot before its suffix's (0 across a window boundary)
#pragma unroll
    for (int q = 0; q < kPlcpChunk; q++) {
      const int p = threadIdx.x + q * 256;
      if (p < len && islot[q] > 0) lcp[islot[q] - 1] = ((first >> q) & 1u) ? 0u : ps[pad16(p)];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && n > 0) lcp[n - 1] = 0;  // the last slot has no successor
}

void build_lcp(const uint32_t *sa, const uint32_t *rank, uint64_t n, const uint32_t *wbeg, const uint32_t *wend,
               const uint32_t *snap, const uint32_t *snaps, const uint32_t *key0, int top, uint32_t *lcp,
               hipStream_t s) {
  const uint64_t nspan = (n + kPlcpSpan - 1) / kPlcpSpan;
  hipLaunchKernelGGL(k_plcp, dim3((unsigned)std::min<uint64_t>(std::max<uint64_t>(nspan, 1), 8192)), dim3(256), 0, s,
                     sa, rank, n, wbeg, wend, snap, snaps, key0, top, lcp);
}

// ------------------------------------------------------------ candidates
// Block minima of LCP (kMinFan-ary levels) for previous-smaller-value queries.
// Full blocks are read with four 16-byte loads (levels are 16-entry aligned).
__global__ void k_blockmin(const uint32_t *src, uint64_t nsrc, uint32_t *dst, uint64_t ndst) {
  static_assert(kMinFan == 16, "four uint4 loads per block");
  GRID_STRIDE(k, ndst) {
    uint32_t m = 0xFFFFFFFFu;
    const uint64_t b = k * kMinFan, e = min(b + kMinFan, nsrc);
    if (e - b == kMinFan) {
      const uint4 *q = reinterpret_cast<const uint4 *>(src + b);
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint4 v = q[u];
        m = min(min(m, min(v.x, v.y)), min(v.z, v.w));
      }
    } else {
      for (uint64_t i = b; i < e; i++) m = min(m, src[i]);
    }
    dst[k] = m;
  }
}

struct MinLevels {
  const uint32_t *lv[kMinLevels];
  uint64_t sz[kMinLevels];
  int nlev;
};

// Largest e in [lo, hi) with L[e] < l, or -1; lo is a multiple of kMinFan
// and the aligned block [lo, lo + kMinFan) lies inside L's allocation.  The
// block is read with four independent 16-byte loads.
__device__ __forceinline__ int64_t last_below(const uint32_t *L, uint64_t lo, uint64_t hi, uint32_t l) {
  static_assert(kMinFan == 16, "one block is four uint4 loads");
  const uint4 *q = reinterpret_cast<const uint4 *>(L + lo);
  const uint4 a = q[0], b = q[1], c = q[2], d = q[3];
  const uint32_t v[16] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w, d.x, d.y, d.z, d.w};
  int f = -1;
#pragma unroll
  for (int k = 0; k < 16; k++)
    if (lo + k < hi && v[k] < l) f = k;
  return f >= 0 ? (int64_t)(lo + f) : -1;
}

// Largest j < i with lcp[j] < l, or -1: scans the aligned block of kMinFan
// entries left of the bound at each level, climbing while nothing below l is
// found, then descends to the rightmost qualifying leaf.  Each step is one
// block read; near answers (the common case) take one or two.
__device__ int64_t psv_query(const uint32_t *const *lv, const uint64_t *sz, int nlev, uint64_t i, uint32_t l) {
  uint64_t pos = i;  // exclusive bound at level `lev`: its entries below pos cover [0, i)
  int lev = 0;
  int64_t found;
  for (;;) {
    if (pos == 0) return -1;
    const uint64_t lo = (pos - 1) / kMinFan * kMinFan;
    found = last_below(lv[lev], lo, pos, l);
    if (found >= 0) break;
    if (lev + 1 < nlev) {
      pos = lo / kMinFan;
      lev++;
    } else {
      pos = lo;  // top level: go on down the same level
    }
  }
  while (lev > 0) {
    lev--;
    const uint64_t lo = (uint64_t)found * kMinFan;
    found = last_below(lv[lev], lo, min(lo + kMinFan, sz[lev]), l);  // found: the parent minimum is < l
    if (found < 0) return -1;
  }
  return found;
}

// Loop body of the paper's candidate pass for every adjacent pair i (both
// suffixes in one window): disjoint branch -> (p, s1), (p, s2); overlap branch
// -> l = floor((p+d)/2) - remainder mod d, at base and base+l.  Candidates
// with l >= min_len are appended with their substring ID.  When pairs i-1 and
// i are both in the disjoint branch with LCP[i-1] == LCP[i], pair i's first
// candidate (LCP[i], SA[i]) equals pair i-1's second one, ID included (no
// LCP value between them is below the length), so it is counted but not
// written: on loop streams this removes nearly all exact duplicates before
// the sort.  A workgroup takes kCandItems consecutive pairs per thread per
// pass (a tile of 256 * kCandItems pairs).  Two passes keep the output in
// suffix-array order: the first counts each tile's records (and the longest
// length and the skipped repeats), a scan turns the counts into tile offsets,
// and the second computes the IDs and writes every record at its place.
constexpr int kCandItems = 8;

// tile_val: count pass: records per tile (then scanned to offsets); the
// tile's skipped repeats and longest length go to tile_val[ntiles + tile]
// and tile_val[2 ntiles + tile] (summed by k_tile_totals, not by atomics on
// one word from every workgroup).
// The write pass stages the tile's records in LDS, kCandStage at a time, so
// they leave in consecutive words (a thread's own records are consecutive,
// but neighbouring threads' are not).
constexpr uint32_t kCandStage = 1024;

// Occupancy of 6 wavefronts per SIMD: the ID queries are latency-bound, and
// the write pass would otherwise take ~127 registers (4 wavefronts); on the
// batched workload analysed on one stream the write pass went from 825 to
// 754 us per launch, a few spilled registers included (a gain within the
// noise of the whole step).
template <bool WRITE>
__global__ __launch_bounds__(256, 6) void k_candidates(const uint32_t *sa, const uint32_t *lcp, uint64_t n,
                                                    const uint32_t *wend, uint32_t min_len, MinLevels M,
                                                    uint32_t *tile_val, uint32_t *crec) {
  __shared__ uint32_t sh[4];
  __shared__ uint32_t stage[WRITE ? kCandStage * kCandWords : 1];
  __shared__ uint32_t bmax;
  // level pointers in LDS: per-lane indexing of the kernel argument would
  // cost a dependent global load per level step
  __shared__ const uint32_t *slv[kMinLevels];
  __shared__ uint64_t ssz[kMinLevels];
  if (threadIdx.x == 0) bmax = 0;
  if (threadIdx.x < kMinLevels) {
    slv[threadIdx.x] = M.lv[threadIdx.x];
    ssz[threadIdx.x] = M.sz[threadIdx.x];
  }
  __syncthreads();
  const uint64_t span = (uint64_t)blockDim.x * kCandItems;
  const uint64_t ntiles = (n + span - 1) / span;
  for (uint64_t i0 = (uint64_t)blockIdx.x * span; i0 < n; i0 += (uint64_t)gridDim.x * span) {
    const uint64_t tile = i0 / span;
    uint32_t mymax = 0, myskip = 0;
    const uint64_t ib = i0 + (uint64_t)threadIdx.x * kCandItems;  // a thread's pairs are consecutive
    // every input of the thread's pairs (and of the pair before them) is
    // loaded before any is used; index 0 is pair ib - 1
    uint32_t S[kCandItems + 2], P[kCandItems + 1], WE[kCandItems + 1];
    static_assert(kCandItems == 8, "two 16-byte loads per array");
    if (ib + kCandItems + 1 <= n) {  // ib is a multiple of 8: aligned 16-byte loads
      const uint4 s0 = reinterpret_cast<const uint4 *>(sa + ib)[0], s1 = reinterpret_cast<const uint4 *>(sa + ib)[1];
      const uint4 p0 = reinterpret_cast<const uint4 *>(lcp + ib)[0], p1 = reinterpret_cast<const uint4 *>(lcp + ib)[1];
      S[0] = ib ? sa[ib - 1] : 0u;
      S[1] = s0.x; S[2] = s0.y; S[3] = s0.z; S[4] = s0.w; S[5] = s1.x; S[6] = s1.y; S[7] = s1.z; S[8] = s1.w;
      S[9] = sa[ib + kCandItems];
      P[0] = ib ? lcp[ib - 1] : 0u;
      P[1] = p0.x; P[2] = p0.y; P[3] = p0.z; P[4] = p0.w; P[5] = p1.x; P[6] = p1.y; P[7] = p1.z; P[8] = p1.w;
      if (wend) {
        const uint4 e0 = reinterpret_cast<const uint4 *>(wend + ib)[0], e1 = reinterpret_cast<const uint4 *>(wend + ib)[1];
        WE[0] = ib ? wend[ib - 1] : (uint32_t)n;
        WE[1] = e0.x; WE[2] = e0.y; WE[3] = e0.z; WE[4] = e0.w; WE[5] = e1.x; WE[6] = e1.y; WE[7] = e1.z; WE[8] = e1.w;
      } else {
#pragma unroll
        for (int k = 0; k < kCandItems + 1; k++) WE[k] = (uint32_t)n;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kCandItems + 2; k++) {
        const uint64_t i = ib + k - 1;
        S[k] = (ib + k >= 1 && i < n) ? sa[i] : 0u;
      }
#pragma unroll
      for (int k = 0; k < kCandItems + 1; k++) {
        const uint64_t i = ib + k - 1;
        const bool in = ib + k >= 1 && i < n;
        P[k] = in ? lcp[i] : 0u;
        WE[k] = (wend && in) ? wend[i] : (uint32_t)n;
      }
    }
    uint32_t L[kCandItems + 1], A[kCandItems + 1], B[kCandItems + 1];
    bool D[kCandItems + 1];  // pair in the disjoint branch with l >= min_len
#pragma unroll
    for (int k = 0; k < kCandItems + 1; k++) {
      const uint64_t i = ib + k - 1;
      L[k] = 0;
      A[k] = B[k] = 0;
      D[k] = false;
      if (ib + k < 1 || i + 1 >= n || i + 1 >= WE[k]) continue;
      const uint32_t s1 = S[k], s2 = S[k + 1], p = P[k];
      const uint32_t lo = min(s1, s2), hi = max(s1, s2);
      uint32_t l, a, b;
      bool disj = false;
      if (lo + p <= hi) {
        l = p; a = s1; b = s2;
        disj = true;
      } else {
        const uint32_t d = hi - lo;
        l = (p + d) / 2;
        l -= l % d;
        a = lo; b = lo + l;
      }
      if (l >= min_len) {  // min_len >= 1, so L[k] != 0 marks an emitted pair
        L[k] = l; A[k] = a; B[k] = b;
        D[k] = disj;
      }
    }
    uint32_t mine = 0;
#pragma unroll
    for (int k = 1; k < kCandItems + 1; k++) {
      if (!L[k]) continue;
      const bool rep = D[k] && D[k - 1] && L[k - 1] == L[k];
      mine += rep ? 1u : 2u;
      if (!WRITE) {
        myskip += rep ? 1u : 0u;
        mymax = max(mymax, L[k]);
      }
    }
    uint32_t tot;
    const uint32_t off = block_excl_sum<256>(mine, sh, &tot);
    if (!WRITE) {
      uint32_t tskip;
      (void)block_excl_sum<256>(myskip, sh, &tskip);
      const uint32_t wm = wave_incl_max(mymax);
      if ((threadIdx.x & 63) == 63 && wm) atomicMax(&bmax, wm);
      __syncthreads();
      if (threadIdx.x == 0) {
        tile_val[tile] = tot;
        tile_val[ntiles + tile] = tskip;
        tile_val[2 * ntiles + tile] = bmax;
        bmax = 0;  // the next tile's first LDS max follows two more barriers
      }
      continue;
    }
    uint32_t id[kCandItems + 1];
#pragma unroll
    for (int k = 1; k < kCandItems + 1; k++)
      id[k] = L[k] ? (uint32_t)(psv_query(slv, ssz, M.nlev, ib + k - 1, L[k]) + 1) : 0u;
    uint32_t *dst = crec + kCandWords * (uint64_t)tile_val[tile];
    for (uint32_t w0 = 0; w0 < tot; w0 += kCandStage) {  // workgroup-uniform
      uint32_t q = off;  // the thread's next record index within the tile
#pragma unroll
      for (int k = 1; k < kCandItems + 1; k++) {
        if (!L[k]) continue;
        if (!(D[k] && D[k - 1] && L[k - 1] == L[k])) {
          if (q >= w0 && q - w0 < kCandStage) {
            uint32_t *r = stage + kCandWords * (q - w0);
            r[0] = L[k]; r[1] = A[k]; r[2] = id[k];
          }
          q++;
        }
        if (q >= w0 && q - w0 < kCandStage) {
          uint32_t *r = stage + kCandWords * (q - w0);
          r[0] = L[k]; r[1] = B[k]; r[2] = id[k];
        }
        q++;
      }
      __syncthreads();
      const uint32_t words = kCandWords * min(kCandStage, tot - w0);
      for (uint32_t j = threadIdx.x; j < words; j += blockDim.x) dst[(uint64_t)kCandWords * w0 + j] = stage[j];
      __syncthreads();
    }
  }
}

// Sum of the tiles' skipped repeats and maximum of their longest lengths.
__global__ __launch_bounds__(1024) void k_tile_totals(const uint32_t *skip, const uint32_t *mx, uint32_t ntiles,
                                                      uint32_t *skipped, uint32_t *maxl) {
  __shared__ uint32_t ssum, smax;
  if (threadIdx.x == 0) ssum = smax = 0;
  __syncthreads();
  uint32_t a = 0, b = 0;
  for (uint32_t t = threadIdx.x; t < ntiles; t += blockDim.x) {
    a += skip[t];
    b = max(b, mx[t]);
  }
  const uint32_t wa = wave_incl_sum(a), wb = wave_incl_max(b);
  if ((threadIdx.x & 63) == 63) {
    atomicAdd(&ssum, wa);
    atomicMax(&smax, wb);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *skipped = ssum;
    *maxl = smax;
  }
}

void gen_candidates(const uint32_t *sa, const uint32_t *lcp, uint64_t n, const uint32_t *wend, uint32_t min_len,
                    uint32_t *const *levels, int nlev, uint32_t *crec, uint32_t *cnt, uint32_t *skipped,
                    uint32_t *maxl, uint32_t *tile_val, uint32_t *ntiles_dev, uint32_t *tile_tmp, hipStream_t s) {
  MinLevels M{};
  uint64_t sz = n;
  M.lv[0] = lcp;
  M.sz[0] = n;
  M.nlev = 1;
  for (int k = 1; k < nlev && k < kMinLevels && sz > (uint64_t)kMinFan; k++) {
    const uint64_t nd = (sz + kMinFan - 1) / kMinFan;
    hipLaunchKernelGGL(k_blockmin, grid_for(nd, 256, 8192), dim3(256), 0, s, M.lv[k - 1], sz, levels[k], nd);
    M.lv[k] = levels[k];
    M.sz[k] = nd;
    M.nlev = k + 1;
    sz = nd;
  }
  const uint64_t span = 256 * kCandItems;
  const uint64_t ntiles = std::max<uint64_t>((n + span - 1) / span, 1);
  const dim3 grid((unsigned)std::min<uint64_t>(ntiles, 8192));
  hipLaunchKernelGGL((k_candidates<false>), grid, dim3(256), 0, s, sa, lcp, n, wend, min_len, M, tile_val, crec);
  hipLaunchKernelGGL(k_tile_totals, dim3(1), dim3(1024), 0, s, tile_val + ntiles, tile_val + 2 * ntiles,
                     (uint32_t)((n + span - 1) / span), skipped, maxl);
  fill_u32(ntiles_dev, 1, (uint32_t)ntiles, s);
  scan_excl(tile_val, tile_val, ntiles_dev, ntiles, tile_tmp, cnt, s);  // tile offsets; *cnt = records
  hipLaunchKernelGGL((k_candidates<true>), grid, dim3(256), 0, s, sa, lcp, n, wend, min_len, M, tile_val, crec);
}

// Keep the first of each run of identical candidates, in sorted order.
struct GatherSorted {
  using Rec = uint3;
  const uint32_t *order, *crec;
  uint32_t *s_len, *s_start, *s_id;
  __device__ Rec get(uint64_t k) const {
    const uint32_t *r = crec + kCandWords * (uint64_t)order[k];
    return make_uint3(r[0], r[1], r[2]);
  }
  __device__ void put(uint32_t o, Rec r) const { s_len[o] = r.x; s_start[o] = r.y; s_id[o] = r.z; }
};

void compact_sorted(const uint32_t *order, const uint8_t *keep, const uint32_t *m_dev, uint64_t bound,
                    const uint32_t *crec, uint32_t *s_len, uint32_t *s_start, uint32_t *s_id, uint32_t *tile_tmp,
                    uint32_t *total, hipStream_t s) {
  flag_compact(keep, FlagNonZero{}, m_dev, bound, tile_tmp, total, GatherSorted{order, crec, s_len, s_start, s_id}, s);
}

// ------------------------------------------------- stable LSD digit passes
// Stable sort of (key, p1, p2) triples by kLsdBits-bit digits of the key,
// least significant first (8-bit digits measured faster than 10-bit ones,
// even where they need one pass more).  A tile of kLsdTile entries is 4 wavefronts x 16 slots x
// 64 lanes with entry index tile0 + 1024 w + 64 e + lane, so each slot's
// loads are coalesced and index order is (wavefront, slot, lane) order.  Per
// tile: a digit histogram (lanes with equal digits found by ballots, one LDS
// add per digit group); the histograms of all tiles, bin-major, are scanned
// once; the scatter ranks every entry among the tile's equal digits in index
// order (running per-wavefront digit counts in LDS) and writes it to the
// bin's global offset.  The first pass reads the candidate records
// (key = maxl - length, p1 = start, p2 = ID).
constexpr int kLsdNT = 256, kLsdSlots = 16, kLsdTile = kLsdNT * kLsdSlots, kLsdBits = 8,
              kLsdBins = 1 << kLsdBits;

struct LsdSrc {
  const uint32_t *rec;           // candidate records, or null
  const uint32_t *maxl;          // with records: key = *maxl - length
  const uint32_t *key, *p1, *p2; // without records
  const uint32_t *wid;           // with records (nullable): key |= window << wshift
  int wshift;
};

__device__ __forceinline__ void lsd_load(const LsdSrc &in, uint64_t i, uint32_t maxl, uint32_t &k, uint32_t &a,
                                         uint32_t &b) {
  if (in.rec) {
    const uint32_t *r = in.rec + kCandWords * i;
    k = maxl - r[0]; a = r[1]; b = r[2];
    // the window of a candidate is the window of its ID (a slot of the same
    // window: pairs across windows have LCP 0, so the ID never reaches back
    // past the window's first slot); records come in suffix-array order, so
    // the IDs of neighbouring records are close and these reads share lines
    if (in.wid) k |= in.wid[b] << in.wshift;
  } else {
    k = in.key[i]; a = in.p1[i]; b = in.p2[i];
  }
}

// Lanes of the wavefront whose digit equals this lane's (valid lanes only).
__device__ __forceinline__ uint64_t digit_peers(uint32_t d, bool valid) {
  uint64_t peers = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kLsdBits; b++) {
    const bool bit = (d >> b) & 1u;
    const uint64_t m = __ballot(bit);
    peers &= bit ? m : ~m;
  }
  return valid ? peers : 0ull;
}

// Tiles never straddle a segment (a window, when records come window by
// window): segment g holds records [off[g], off[g+1]) and tiles [tb[g],
// tb[g+1]); tseg[t] is the segment of tile t.  The histograms are laid out
// segment by segment, each segment's block digit-major over its own tiles,
// so one exclusive scan gives every (tile, digit) run its output offset, and
// every pass keeps each segment's records together, stable inside it.
struct LsdTiles {
  const uint32_t *off, *tb, *tseg;
  uint32_t nseg;
};

struct LsdTile {
  uint64_t lo;      // first record
  uint32_t cnt;     // records (<= kLsdTile)
  uint64_t hbase;   // first histogram word of the tile's segment
  uint32_t nt, j;   // tiles of the segment, index of this tile in it
};

__device__ __forceinline__ LsdTile lsd_tile(const LsdTiles &T, uint32_t t) {
  LsdTile r;
  const uint32_t g = T.tseg[t];
  const uint32_t tb0 = T.tb[g];
  r.nt = T.tb[g + 1] - tb0;
  r.j = t - tb0;
  r.lo = (uint64_t)T.off[g] + (uint64_t)r.j * kLsdTile;
  r.cnt = (uint32_t)min((uint64_t)kLsdTile, (uint64_t)T.off[g + 1] - r.lo);
  r.hbase = (uint64_t)tb0 * kLsdBins;
  return r;
}

// First record k in [0, n) whose window (wid of its ID) is >= target: a
// 64-ary search by the whole wavefront (each step probes 64 evenly spaced
// records; the window never decreases along the records).
__device__ uint32_t rec_window_bound(const uint32_t *rec, const uint32_t *wid, uint32_t n, uint32_t target) {
  const int lane = threadIdx.x & 63;
  uint32_t lo = 0, hi = n;
  while (hi - lo > 64) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t k = lo + (uint32_t)lane * step;
    const int nb = __popcll(__ballot(k < hi && wid[rec[kCandWords * (uint64_t)k + 2]] < target));
    if (nb == 0) return lo;
    const uint32_t nlo = lo + (uint32_t)(nb - 1) * step + 1, nhi = min(hi, lo + (uint32_t)nb * step);
    lo = nlo;
    hi = nhi;
  }
  const uint32_t k = lo + (uint32_t)lane;
  return lo + (uint32_t)__popcll(__ballot(k < hi && wid[rec[kCandWords * (uint64_t)k + 2]] < target));
}

// Segment g's records (one wavefront per segment) and its tile count.
__global__ __launch_bounds__(64) void k_lsd_segments(const uint32_t *rec, const uint32_t *n_dev, const uint32_t *wid,
                                                     uint32_t nseg, uint32_t *off, uint32_t *nt) {
  const uint32_t g = blockIdx.x;
  const uint32_t n = *n_dev;
  uint32_t lo = 0, hi = n;
  if (wid) {
    lo = rec_window_bound(rec, wid, n, g);
    hi = rec_window_bound(rec, wid, n, g + 1);
  }
  if (threadIdx.x == 0) {
    off[g] = lo;
    nt[g] = (hi - lo + kLsdTile - 1) / kLsdTile;
    if (g == 0) {
      off[nseg] = n;
      nt[nseg] = 0;
    }
  }
}

// tseg of every tile; *hist_words = tiles * kLsdBins.
__global__ __launch_bounds__(64) void k_lsd_seg_fill(const uint32_t *tb, uint32_t nseg, uint32_t *tseg,
                                                     uint32_t *hist_words) {
  const uint32_t g = blockIdx.x;
  for (uint32_t t = tb[g] + threadIdx.x; t < tb[g + 1]; t += 64) tseg[t] = g;
  if (g == 0 && threadIdx.x == 0) *hist_words = tb[nseg] * kLsdBins;
}

__global__ __launch_bounds__(kLsdNT) void k_lsd_hist(LsdSrc in, int shift, uint32_t *hist, LsdTiles T) {
  __shared__ uint32_t h[kLsdBins];
  const uint32_t maxl = in.maxl ? *in.maxl : 0u;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t ntiles = T.tb[T.nseg];
  for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const LsdTile tl = lsd_tile(T, t);
    for (int d = threadIdx.x; d < kLsdBins; d += kLsdNT) h[d] = 0;
    __syncthreads();
    // every slot's key is loaded before the first ballot, so the loads (and
    // a record pass's window lookups) overlap instead of queueing
    uint32_t K[kLsdSlots];
#pragma unroll
    for (int e = 0; e < kLsdSlots; e++) {
      const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
      uint32_t a, b;
      K[e] = 0;
      if (q < tl.cnt) lsd_load(in, tl.lo + q, maxl, K[e], a, b);
    }
#pragma unroll
    for (int e = 0; e < kLsdSlots; e++) {
      const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
      const bool valid = q < tl.cnt;
      const uint32_t d = (K[e] >> shift) & (kLsdBins - 1);
      const uint64_t peers = digit_peers(d, valid);
      if (valid && lane == __ffsll((unsigned long long)peers) - 1) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kLsdBins; d += kLsdNT) hist[tl.hbase + (uint64_t)d * tl.nt + tl.j] = h[d];
    __syncthreads();
  }
}

// oa2 (nullable): a second output of p1.
__global__ __launch_bounds__(kLsdNT) void k_lsd_scatter(LsdSrc in, int shift, const uint32_t *offs, LsdTiles T,
                                                        uint32_t *ok, uint32_t *oa, uint32_t *ob, uint32_t *oa2) {
  static_assert(kLsdBins == kLsdNT, "one digit per thread in the run offsets");
  __shared__ uint32_t wcnt[4][kLsdBins];   // per-wavefront digit counts; then tile-local run starts
  __shared__ uint32_t wstart[4][kLsdBins];  // global run starts
  __shared__ uint32_t lg[kLsdTile];         // global position of each tile-local sorted slot
  __shared__ uint32_t lv[kLsdTile];         // one output array's values in tile-local sorted order
  __shared__ uint32_t sh[kLsdNT / 64];
  const uint32_t maxl = in.maxl ? *in.maxl : 0u;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t ntiles = T.tb[T.nseg];
  for (uint32_t tb = 0; tb < ntiles; tb += gridDim.x) {  // tiles handed out XCD by XCD
    const uint32_t t = (uint32_t)xcd_item(tb, ntiles, blockIdx.x, gridDim.x);
    if (t >= ntiles) break;
    const LsdTile tl = lsd_tile(T, t);
    for (int d = threadIdx.x; d < kLsdBins; d += kLsdNT)
      for (int q = 0; q < 4; q++) wcnt[q][d] = 0;
    __syncthreads();
    uint32_t K[kLsdSlots], A[kLsdSlots], Bv[kLsdSlots], rank[kLsdSlots];
#pragma unroll
    for (int e = 0; e < kLsdSlots; e++) {
      const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
      K[e] = 0;
      if (q < tl.cnt) lsd_load(in, tl.lo + q, maxl, K[e], A[e], Bv[e]);
    }
#pragma unroll
    for (int e = 0; e < kLsdSlots; e++) {
      const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
      const bool valid = q < tl.cnt;
      const uint32_t d = (K[e] >> shift) & (kLsdBins - 1);
      const uint64_t peers = digit_peers(d, valid);
      const int leader = valid ? __ffsll((unsigned long long)peers) - 1 : lane;
      uint32_t base = 0;
      if (valid && lane == leader) {
        base = wcnt[w][d];
        wcnt[w][d] = base + (uint32_t)__popcll(peers);
      }
      base = (uint32_t)__shfl((int)base, leader, 64);
      rank[e] = base + (uint32_t)__popcll(peers & lt);
    }
    __syncthreads();
    {
      // run starts of (wavefront, digit): global from the scanned
      // histograms, tile-local from a scan of the tile's digit totals
      const int d = threadIdx.x;
      uint32_t c[4], tot = 0;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        c[q] = wcnt[q][d];
        tot += c[q];
      }
      uint32_t ttot;
      uint32_t lrun = block_excl_sum<kLsdNT>(tot, sh, &ttot);  // (has barriers)
      uint32_t run = offs[tl.hbase + (uint64_t)d * tl.nt + tl.j];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        wstart[q][d] = run;
        wcnt[q][d] = lrun;
        run += c[q];
        lrun += c[q];
      }
    }
    __syncthreads();
    // every entry's tile-local sorted slot (kept in rank[]) and global position
#pragma unroll
    for (int e = 0; e < kLsdSlots; e++) {
      const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
      if (q >= tl.cnt) continue;
      const uint32_t d = (K[e] >> shift) & (kLsdBins - 1);
      const uint32_t loc = wcnt[w][d] + rank[e];
      lg[loc] = wstart[w][d] + rank[e];
      rank[e] = loc;
    }
    // each output array goes through LDS in sorted order, so consecutive
    // threads write consecutive words of a digit's run
    const uint32_t cnt = tl.cnt;
#pragma unroll
    for (int a = 0; a < 4; a++) {
      uint32_t *out = a == 0 ? ok : a == 1 ? oa : a == 2 ? ob : oa2;
      if (!out) continue;  // uniform
#pragma unroll
      for (int e = 0; e < kLsdSlots; e++) {
        const uint32_t q = (uint32_t)w * (kLsdTile / 4) + (uint32_t)e * 64 + lane;
        if (q < tl.cnt) lv[rank[e]] = a == 0 ? K[e] : a == 2 ? Bv[e] : A[e];
      }
      __syncthreads();
      for (uint32_t j = threadIdx.x; j < cnt; j += kLsdNT) out[lg[j]] = lv[j];
      __syncthreads();
    }
  }
}

void lsd_sort_candidates(const uint32_t *crec, const uint32_t *maxl_dev, const uint32_t *n_dev, uint64_t bound,
                         int key_bits, uint32_t *const *xs, uint32_t *const *ys, uint32_t *start_copy,
                         uint32_t *hist, uint32_t *hist_n, uint32_t *tile_tmp, hipStream_t s, const uint32_t *wid,
                         int wshift, const uint32_t *seg_wid, uint32_t nseg, uint32_t *seg) {
  if (!seg_wid) nseg = 1;
  const int passes = std::max(1, (key_bits + kLsdBits - 1) / kLsdBits);
  const uint64_t tiles_bound = (bound + kLsdTile - 1) / kLsdTile + nseg;
  const unsigned grid = (unsigned)std::min<uint64_t>(std::max<uint64_t>(tiles_bound, 1), 8192);
  uint32_t *off = seg, *nt = seg + (nseg + 1), *tb = seg + 2 * (nseg + 1), *tseg = seg + 3 * (nseg + 1);
  hipLaunchKernelGGL(k_lsd_segments, dim3(nseg), dim3(64), 0, s, crec, n_dev, seg_wid, nseg, off, nt);
  fill_u32(hist_n, 1, nseg + 1, s);
  scan_excl(nt, tb, hist_n, nseg + 1, tile_tmp, nullptr, s);
  hipLaunchKernelGGL(k_lsd_seg_fill, dim3(nseg), dim3(64), 0, s, tb, nseg, tseg, hist_n);
  const LsdTiles T{off, tb, tseg, nseg};
  LsdSrc in{crec, maxl_dev, nullptr, nullptr, nullptr, wid, wshift};
  for (int ps = 0; ps < passes; ps++) {
    uint32_t *const *out = ((passes - 1 - ps) % 2 == 0) ? xs : ys;  // the last pass writes xs
    hipLaunchKernelGGL(k_lsd_hist, dim3(grid), dim3(kLsdNT), 0, s, in, kLsdBits * ps, hist, T);
    scan_excl(hist, hist, hist_n, (uint64_t)kLsdBins * tiles_bound, tile_tmp, nullptr, s);
    hipLaunchKernelGGL(k_lsd_scatter, dim3(grid), dim3(kLsdNT), 0, s, in, kLsdBits * ps, hist, T, out[0], out[1],
                       out[2], ps == passes - 1 ? start_copy : nullptr);
    in = LsdSrc{nullptr, nullptr, out[0], out[1], out[2], nullptr, 0};
  }
}

// Run starts of equal (key, p2) in the sorted order, as byte flags.
__global__ void k_run_flags(const uint32_t *key, const uint32_t *p2, const uint32_t *n_dev, uint8_t *flag) {
  const uint64_t n = *n_dev;
  GRID_STRIDE(i, n) flag[i] = (i == 0 || key[i] != key[i - 1] || p2[i] != p2[i - 1]) ? 1 : 0;
}
void run_flags(const uint32_t *key, const uint32_t *p2, const uint32_t *n_dev, uint64_t bound, uint8_t *flag,
               hipStream_t s) {
  hipLaunchKernelGGL(k_run_flags, grid_for(bound, 256, 8192), dim3(256), 0, s, key, p2, n_dev, flag);
}

struct StoreIndex {
  using Rec = uint32_t;
  uint32_t *out;
  __device__ Rec get(uint64_t k) const { return (uint32_t)k; }
  __device__ void put(uint32_t o, Rec r) const { out[o] = r; }
};
void flag_positions(const uint8_t *flag, const uint32_t *n_dev, uint64_t bound, uint32_t *out, uint32_t *count,
                    uint32_t *tile_tmp, hipStream_t s) {
  flag_compact(flag, FlagNonZero{}, n_dev, bound, tile_tmp, count, StoreIndex{out}, s);
}

// Keep the first of each run of identical candidates, in sorted order: slot k
// holds position order[k] of the length-sorted arrays.
struct GatherSortedRuns {
  using Rec = uint3;
  const uint32_t *order, *lkey, *start, *id, *maxl;
  uint32_t *s_len, *s_start, *s_id;
  uint32_t lmask;  // bits of the key that hold maxl - length (a window may sit above them)
  __device__ Rec get(uint64_t k) const {
    const uint32_t q = order[k];
    return make_uint3(*maxl - (lkey[q] & lmask), start[q], id[q]);
  }
  __device__ void put(uint32_t o, Rec r) const { s_len[o] = r.x; s_start[o] = r.y; s_id[o] = r.z; }
};
void compact_sorted_runs(const uint32_t *order, const uint8_t *keep, const uint32_t *m_dev, uint64_t bound,
                         const uint32_t *lkey, const uint32_t *start, const uint32_t *id, const uint32_t *maxl,
                         uint32_t *s_len, uint32_t *s_start, uint32_t *s_id, uint32_t *tile_tmp, uint32_t *total,
                         hipStream_t s, uint32_t lmask) {
  flag_compact(keep, FlagNonZero{}, m_dev, bound, tile_tmp, total,
               GatherSortedRuns{order, lkey, start, id, maxl, s_len, s_start, s_id, lmask}, s);
}

// ------------------------------------------------------------- selection
// Round-based exact evaluation of the greedy.  Accepted candidates are final
// and pairwise disjoint; each one paints its interval into `mark` when it is
// accepted.  Round r >= 1 first rejects every undecided candidate with a
// painted endpoint (an accepted candidate overlapping it always has higher
// priority) and keeps the rest as the round's working list.  Then a working
// candidate is accepted when no working candidate of higher priority covers
// its first or last position (sufficient because higher priority means not
// shorter).  Coverage minima of the working list come from one of two
// structures, chosen on the device from the list's size:
//  * dense: a sparse table over all positions -- every working interval
//    writes its priority into the two power-of-two blocks that tile it, then
//    minima are pushed down level by level (levels above kSelSmall one pass
//    each, the rest inside one tiled LDS kernel); two tables alternate, and
//    a dense round after the first empties its table before inserting;
//  * sparse (at most n / kSparseDiv working candidates): canonical
//    power-of-two blocks of each interval (at most two per level, as in a
//    segment tree); a point's minimum is the minimum over its enclosing
//    blocks, and the round resets the blocks it wrote.
// Round r runs only if round r-1 left candidates undecided, so rounds can be
// launched ahead of the host.
constexpr int kSelSmall = 8;
constexpr int kPushTile = 1024;
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr uint32_t kSparseDiv = 32;

struct SelArgs {
  const uint32_t *len, *start;
  uint32_t *Tc, *To;        // dense: this round's table and the other one; level j at + j*n
  uint64_t n;
  int top;
  uint8_t *state;           // 0 undecided, 1 accepted, 2 rejected
  uint32_t *pend;           // undecided candidates entering round r (r >= 1)
  uint32_t *work;           // round r's working list (round 0: every candidate)
  uint32_t *nlive;          // nlive[r]: entries of pend at round r (nlive[0]: all candidates)
  uint32_t *nwork;          // nwork[r]: entries of work at round r (r >= 1)
  uint32_t *undec;          // undec[r]: undecided after round r (equal to nlive[r + 1]; not written on the device)
  int r;
  const uint32_t *maxl;     // longest candidate: table levels above log2 of it stay empty
  uint32_t *ctree;          // sparse: canonical-block tree (all kInf between rounds)
  uint64_t npad;            // power of two >= n: level j of ctree has npad >> j nodes
  uint8_t *mark;            // positions covered by accepted candidates
};

// round r runs when round r - 1 left candidates undecided: nlive[r] of them
__device__ __forceinline__ bool sel_active(const SelArgs &a) { return a.r == 0 || a.nlive[a.r] > 0; }
__device__ __forceinline__ uint32_t sel_nwork(const SelArgs &a) { return a.r == 0 ? a.nlive[0] : a.nwork[a.r]; }
__device__ __forceinline__ bool sel_dense(const SelArgs &a) {
  return a.r == 0 || (uint64_t)a.nwork[a.r] * kSparseDiv > a.n;
}
__device__ __forceinline__ bool sel_run_dense(const SelArgs &a) { return sel_active(a) && sel_dense(a); }
__device__ __forceinline__ bool sel_run_sparse(const SelArgs &a) { return sel_active(a) && !sel_dense(a); }

// Paints [s, s + l) for every lane with `on` set; called by the whole
// wavefront.  Short intervals are painted by their own lane; long ones (up to
// half a window on runs) by all 64 lanes together with 16-byte stores.
constexpr uint32_t kPaintShort = 64;

__device__ __forceinline__ void paint_wave(uint8_t *mark, bool on, uint32_t s, uint32_t l) {
  const int lane = threadIdx.x & 63;
  const bool lng = on && l > kPaintShort;
  if (on && !lng)
    for (uint32_t x = s; x < s + l; x++) mark[x] = 1;
  uint64_t lm = __ballot(lng);
  while (lm) {
    const int src = __ffsll((unsigned long long)lm) - 1;
    lm &= lm - 1;
    const uint32_t S = (uint32_t)__shfl((int)s, src, 64), E = S + (uint32_t)__shfl((int)l, src, 64);
    const uint32_t A = min((S + 15u) & ~15u, E), B = max(A, E & ~15u);  // [A, B) 16-byte aligned
    if (S + (uint32_t)lane < A) mark[S + lane] = 1;
    if (B + (uint32_t)lane < E) mark[B + lane] = 1;
    uint4 *body = reinterpret_cast<uint4 *>(mark + A);
    const uint4 ones = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
    for (uint32_t q = lane; q < (B - A) / 16; q += 64) body[q] = ones;
  }
}

// Lists built by a pass (working list, next round's undecided list) reserve
// their space once per workgroup pass of 256 * kSelItems entries.
constexpr int kSelItems = 8;

// Round r >= 1: reject undecided candidates with a painted endpoint; the
// others form the working list.
__global__ void k_sel_filter(SelArgs a) {
  if (!sel_active(a)) return;
  __shared__ uint32_t sh[4];
  __shared__ uint32_t base;
  const uint32_t m = a.nlive[a.r];
  const uint64_t span = (uint64_t)blockDim.x * kSelItems;
  for (uint64_t q0 = (uint64_t)blockIdx.x * span; q0 < m; q0 += (uint64_t)gridDim.x * span) {
    // loads of all items first (entries, then intervals, then marks)
    uint32_t K[kSelItems], S[kSelItems], E[kSelItems];
    uint8_t M1[kSelItems], M2[kSelItems];
#pragma unroll
    for (int t = 0; t < kSelItems; t++) {
      const uint64_t q = q0 + threadIdx.x + (uint64_t)t * blockDim.x;
      K[t] = q < m ? a.pend[q] : kInf;
    }
#pragma unroll
    for (int t = 0; t < kSelItems; t++) {
      S[t] = K[t] != kInf ? a.start[K[t]] : 0u;
      E[t] = K[t] != kInf ? S[t] + a.len[K[t]] - 1 : 0u;
    }
#pragma unroll
    for (int t = 0; t < kSelItems; t++) {
      M1[t] = K[t] != kInf ? a.mark[S[t]] : 0;
      M2[t] = K[t] != kInf ? a.mark[E[t]] : 0;
    }
    uint32_t mine = 0, kept = 0;
#pragma unroll
    for (int t = 0; t < kSelItems; t++) {
      if (K[t] == kInf) continue;
      if (M1[t] || M2[t]) {
        a.state[K[t]] = 2;
      } else {
        kept |= 1u << t;
        mine++;
      }
    }
    uint32_t tot;
    const uint32_t off = block_excl_sum<256>(mine, sh, &tot);
    if (threadIdx.x == 0) base = tot ? atomicAdd(&a.nwork[a.r], tot) : 0u;
    __syncthreads();
    uint32_t w = base + off;
#pragma unroll
    for (int t = 0; t < kSelItems; t++)
      if (kept & (1u << t)) a.work[w++] = K[t];
    __syncthreads();
  }
}

// Min-writes k into T[addr] for every lane with `pending` set (valid, and the
// table held more than k when read).  Lanes that share the address of the
// first remaining lane are combined into one atomic with their minimum, twice;
// the others write alone.  Long periodic runs send many candidates of a
// wavefront to one word (the right blocks of a run's candidates all end at
// its end, every other candidate in priority order).
__device__ __forceinline__ void min_write_grouped(uint32_t *T, uint64_t addr, uint32_t k, bool pending) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int it = 0; it < 2; it++) {
    const uint64_t todo = __ballot(pending);
    if (!todo) return;  // wavefront-uniform
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const uint64_t la = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(addr >> 32), leader, 64) << 32) |
                        (uint32_t)__shfl((int)(uint32_t)addr, leader, 64);
    const bool mine = pending && addr == la;
    uint32_t v = mine ? k : kInf;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o, 64));
    if (lane == leader) atomicMin(&T[la], v);
    if (mine) pending = false;
  }
  if (pending) atomicMin(&T[addr], k);
}

// Round-0 style insert: each working candidate min-writes its priority into
// the two blocks of level floor(log2 l) that tile it.  Four candidates per
// thread (consecutive in the working list across the workgroup), all loads
// issued before any atomic; a write is skipped when the table already holds
// a smaller priority.
__global__ __launch_bounds__(256) void k_sel_insert(SelArgs a) {
  if (!sel_run_dense(a)) return;
  constexpr int NT = 256;
  const uint32_t m = sel_nwork(a);
  const uint64_t step = (uint64_t)gridDim.x * NT * 4;
  for (uint64_t b0 = (uint64_t)blockIdx.x * NT * 4; b0 < m; b0 += step) {  // wavefront-uniform trip count
    uint32_t k[4], l[4], st[4], t1[4], t2[4];
    uint64_t a1[4], a2[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t q = b0 + (uint64_t)u * NT + threadIdx.x;
      k[u] = q < m ? a.work[q] : kInf;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      l[u] = k[u] != kInf ? a.len[k[u]] : 1u;
      st[u] = k[u] != kInf ? a.start[k[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int j = 31 - __clz((int)l[u]);
      a1[u] = (uint64_t)j * a.n + st[u];  // word index in the table
      a2[u] = (uint64_t)j * a.n + st[u] + l[u] - (1u << j);
      t1[u] = k[u] != kInf ? a.Tc[a1[u]] : 0u;
      t2[u] = k[u] != kInf ? a.Tc[a2[u]] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) {
      min_write_grouped(a.Tc, a1[u], k[u], t1[u] > k[u]);
      min_write_grouped(a.Tc, a2[u], k[u], t2[u] > k[u]);
    }
  }
}

// A dense round r >= 1 starts by emptying the levels of its table that a
// run can use (round 0's table is emptied before the rounds); sparse rounds
// leave the tables alone, so a run whose later rounds are all sparse never
// pays for it.
__global__ void k_sel_clear(SelArgs a) {
  if (a.r == 0 || !sel_run_dense(a)) return;
  const uint32_t ml = *a.maxl;
  const int lv = ml ? 32 - __clz((int)ml) : 1;
  const uint64_t lim = (uint64_t)min(lv, a.top + 1) * a.n;
  GRID_STRIDE(i, lim) a.Tc[i] = kInf;
}

// Level j -> j-1 for the large levels.
__global__ void k_sel_push(SelArgs a, int j) {
  if (!sel_run_dense(a) || (1u << j) > *a.maxl) return;  // level j empty
  const uint32_t *Tj = a.Tc + (uint64_t)j * a.n;
  uint32_t *Td = a.Tc + (uint64_t)(j - 1) * a.n;
  const uint64_t half = 1ull << (j - 1);
  GRID_STRIDE(x, a.n) {
    uint32_t v = Td[x];
    v = min(v, Tj[x]);
    if (x >= half) v = min(v, Tj[x - half]);
    Td[x] = v;
  }
}

// Levels min(top, kSelSmall)..0 for one tile of positions, halos included;
// writes level 0.
__global__ __launch_bounds__(256) void k_sel_push_tile(SelArgs a) {
  if (!sel_run_dense(a)) return;
  constexpr int HMAX = 1 << kSelSmall;
  __shared__ uint32_t buf[2][kPushTile + HMAX];
  const uint32_t ml = *a.maxl;
  const int J = min(min(a.top, kSelSmall), ml ? 31 - __clz((int)ml) : 0);  // levels above log2(maxl) are empty
  const uint64_t ntiles = (a.n + kPushTile - 1) / kPushTile;
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t x0 = (int64_t)t * kPushTile;
    const int64_t x1 = min((int64_t)a.n, x0 + kPushTile);
    // level J over [x0 - 2^J + 1, x1)
    int64_t lo = x0 - (1ll << J) + 1;
    const uint32_t *TJ = a.Tc + (uint64_t)J * a.n;
    for (int64_t x = lo + threadIdx.x; x < x1; x += blockDim.x) buf[0][x - lo] = x >= 0 ? TJ[x] : kInf;
    __syncthreads();
    int c = 0;
    for (int j = J; j >= 1; j--) {
      const int64_t half = 1ll << (j - 1);
      const int64_t nlo = x0 - half + 1;  // level j-1 range [nlo, x1)
      const uint32_t *Td = a.Tc + (uint64_t)(j - 1) * a.n;
      for (int64_t x = nlo + threadIdx.x; x < x1; x += blockDim.x) {
        uint32_t v = x >= 0 ? Td[x] : kInf;
        v = min(v, buf[c][x - lo]);
        if (x - half >= lo) v = min(v, buf[c][x - half - lo]);
        buf[c ^ 1][x - nlo] = v;
      }
      __syncthreads();
      c ^= 1;
      lo = nlo;
    }
    uint32_t *T0 = a.Tc;
    for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) T0[x] = buf[c][x - lo];
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t *ctree_level(const SelArgs &a, int j) {
  return a.ctree + (j == 0 ? 0 : 2 * a.npad - (a.npad >> (j - 1)));
}

__device__ __forceinline__ uint32_t ctree_point(const SelArgs &a, uint32_t x, int levels) {
  uint32_t v = kInf;
  for (int j = 0; j < levels; j++) v = min(v, ctree_level(a, j)[x >> j]);
  return v;
}

// Accept the working candidates with no higher-priority working candidate on
// an endpoint (and paint them); the others stay undecided for round r + 1.
template <bool DENSE>
__global__ void k_sel_decide(SelArgs a) {
  if (DENSE ? !sel_run_dense(a) : !sel_run_sparse(a)) return;
  __shared__ uint32_t sh[4];
  __shared__ uint32_t base;
  __syncthreads();
  const uint32_t m = sel_nwork(a);
  const uint32_t ml = *a.maxl;
  const int levels = ml ? 32 - __clz((int)ml) : 1;  // sparse: blocks of size <= maxl
  const uint64_t span = (uint64_t)blockDim.x * kSelItems;
  for (uint64_t q0 = (uint64_t)blockIdx.x * span; q0 < m; q0 += (uint64_t)gridDim.x * span) {
    uint32_t K[kSelItems];
    uint32_t mine = 0, kept = 0;
#pragma unroll
    for (int t = 0; t < kSelItems; t++) {
      const uint64_t q = q0 + threadIdx.x + (uint64_t)t * blockDim.x;
      bool acc = false;
      uint32_t k = 0, l = 0, s = 0;
      if (q < m) {
        k = a.work[q];
        l = a.len[k];
        s = a.start[k];
        const uint32_t e = s + l - 1;
        const uint32_t t1 = DENSE ? a.Tc[s] : ctree_point(a, s, levels);
        const uint32_t t2 = DENSE ? a.Tc[e] : ctree_point(a, e, levels);
        if (t1 >= k && t2 >= k) {
          a.state[k] = 1;
          acc = true;
        } else {
          kept |= 1u << t;
          mine++;
        }
      }
      K[t] = k;
      paint_wave(a.mark, acc, s, l);
    }
    uint32_t tot;
    const uint32_t off = block_excl_sum<256>(mine, sh, &tot);
    if (threadIdx.x == 0) {
      base = tot ? atomicAdd(&a.nlive[a.r + 1], tot) : 0u;
    }
    __syncthreads();
    uint32_t w = base + off;
#pragma unroll
    for (int t = 0; t < kSelItems; t++)
      if (kept & (1u << t)) a.pend[w++] = K[t];
    __syncthreads();
  }
}

template <bool CLEAR>
__device__ __forceinline__ void ctree_cover(const SelArgs &a, uint32_t s, uint32_t l, uint32_t k) {
  uint64_t lo = s, hi = (uint64_t)s + l;
  for (int j = 0; lo < hi; j++) {
    uint32_t *Tj = ctree_level(a, j);
    if (lo & 1) {
      if (CLEAR) Tj[lo] = kInf;
      else if (Tj[lo] > k) atomicMin(&Tj[lo], k);
      lo++;
    }
    if (hi & 1) {
      hi--;
      if (CLEAR) Tj[hi] = kInf;
      else if (Tj[hi] > k) atomicMin(&Tj[hi], k);
    }
    lo >>= 1;
    hi >>= 1;
  }
}

template <bool CLEAR>
__global__ void k_sel_sparse_cover(SelArgs a) {
  if (!sel_run_sparse(a)) return;
  const uint32_t m = sel_nwork(a);
  GRID_STRIDE(q, m) {
    const uint32_t k = a.work[q];
    ctree_cover<CLEAR>(a, a.start[k], a.len[k], k);
  }
}

__global__ void k_iota(uint32_t *p, const uint32_t *n) {
  const uint32_t m = *n;
  GRID_STRIDE(i, m) p[i] = (uint32_t)i;
}

// Fills levels 0..min(top, log2 maxl) of a sparse table (the only ones a
// run touches).
__global__ void k_fill_levels(uint32_t *p, uint64_t n, const uint32_t *maxl, int top, uint32_t v) {
  const uint32_t ml = *maxl;
  const int lv = ml ? 32 - __clz((int)ml) : 1;
  const uint64_t lim = (uint64_t)min(lv, top + 1) * n;
  GRID_STRIDE(i, lim) p[i] = v;
}

void sel_table_init(uint32_t *T, uint64_t n, const uint32_t *maxl, int top, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_levels, grid_for((uint64_t)(top + 1) * n, 256, 8192), dim3(256), 0, s, T, n, maxl, top,
                     kInf);
}

void sel_init(uint32_t *work, const uint32_t *nlive_dev, uint8_t *state, uint64_t bound, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, grid_for(bound, 256, 8192), dim3(256), 0, s, work, nlive_dev);
  fill_u8_dev(state, nlive_dev, bound, 0, s);
}

void sel_round(const uint32_t *len, const uint32_t *start, uint32_t *Tc, uint32_t *To, int top, uint64_t n,
               uint8_t *state, uint32_t *pend, uint32_t *work, uint32_t *nlive, uint32_t *nwork, uint32_t *undec,
               int r, uint64_t live_hint, const uint32_t *maxl, uint32_t *ctree, uint64_t npad, uint8_t *mark,
               hipStream_t s) {
  SelArgs a{len, start, Tc, To, n, top, state, pend, work, nlive, nwork, undec, r, maxl, ctree, npad, mark};
  const dim3 g = grid_for((live_hint + kSelItems - 1) / kSelItems, 256, 8192);
  if (r > 0) hipLaunchKernelGGL(k_sel_filter, g, dim3(256), 0, s, a);
  // dense round (each kernel returns at once when the round is sparse or not needed)
  if (r > 0) hipLaunchKernelGGL(k_sel_clear, grid_for((uint64_t)(top + 1) * n, 256, 8192), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sel_insert, g, dim3(256), 0, s, a);
  for (int j = top; j > kSelSmall; j--)
    hipLaunchKernelGGL(k_sel_push, grid_for(n, 256, 8192), dim3(256), 0, s, a, j);
  const uint64_t ntiles = (n + kPushTile - 1) / kPushTile;
  hipLaunchKernelGGL(k_sel_push_tile, dim3((unsigned)std::min<uint64_t>(ntiles, 4096)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sel_decide<true>, g, dim3(256), 0, s, a);
  // sparse round (returns at once unless the working list is short)
  if (r > 0) {
    hipLaunchKernelGGL(k_sel_sparse_cover<false>, g, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sel_decide<false>, g, dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sel_sparse_cover<true>, g, dim3(256), 0, s, a);
  }
}

// Exact sequential completion for whatever is still undecided after the
// round cap: one thread walks the sorted list with a mark array.
__global__ void k_sel_paint(const uint8_t *state, const uint32_t *len, const uint32_t *start, const uint32_t *m_dev,
                            uint8_t *mark) {
  const uint64_t m = *m_dev;
  GRID_STRIDE(k, m) {
    if (state[k] == 1) {
      const uint32_t s = start[k], l = len[k];
      for (uint32_t x = s; x < s + l; x++) mark[x] = 1;
    }
  }
}

__global__ void k_sel_sequential(uint8_t *state, const uint32_t *len, const uint32_t *start, const uint32_t *m_dev,
                                 uint8_t *mark) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  const uint64_t m = *m_dev;
  for (uint64_t k = 0; k < m; k++) {
    if (state[k] != 0) continue;
    const uint32_t s = start[k], l = len[k];
    if (mark[s] || mark[s + l - 1]) { state[k] = 2; continue; }
    state[k] = 1;
    for (uint32_t x = s; x < s + l; x++) mark[x] = 1;
  }
}

void sel_sequential(uint8_t *state, const uint32_t *len, const uint32_t *start, const uint32_t *m_dev, uint64_t bound,
                    uint8_t *mark, uint64_t n, hipStream_t s) {
  fill_u8(mark, n, 0, s);
  hipLaunchKernelGGL(k_sel_paint, grid_for(bound, 256, 8192), dim3(256), 0, s, state, len, start, m_dev, mark);
  hipLaunchKernelGGL(k_sel_sequential, dim3(1), dim3(64), 0, s, state, len, start, m_dev, mark);
}

// Exact greedy over a prefix of the priority order (the first k
// candidates), by one workgroup: the first wavefront takes 64 candidates at a
// time, rejects those with a marked end (exact: every candidate accepted
// before is at least as long, so an overlap covers an end), settles the rest
// of the batch among itself in priority order with ballots, and the whole
// workgroup paints the batch's accepted intervals before the next batch
// reads the marks.  The longest candidates come first, so when they are long
// a short prefix paints most of the window; the rounds then go on from round
// 1 over the candidates after the prefix, and its filter rejects every one
// with a marked end.
constexpr int kPrefixThreads = 1024;

__global__ __launch_bounds__(kPrefixThreads) void k_sel_prefix(const uint32_t *len, const uint32_t *start, uint32_t k,
                                                                uint8_t *state, uint8_t *mark) {
  __shared__ uint32_t as[64], ae[64];
  __shared__ uint32_t nacc;
  const int tid = threadIdx.x, lane = tid & 63;
  const uint4 ones = make_uint4(0x01010101u, 0x01010101u, 0x01010101u, 0x01010101u);
  for (uint32_t b0 = 0; b0 < k; b0 += 64) {
    if (tid < 64) {
      const uint32_t q = b0 + (uint32_t)lane;
      const bool valid = q < k;
      const uint32_t l = valid ? len[q] : 1u, st = valid ? start[q] : 0u, e = st + l - 1;
      const bool pass = valid && !mark[st] && !mark[e];
      uint64_t cand = __ballot(pass);
      uint64_t acc = 0;
      while (cand) {  // wavefront-uniform
        const int i = __ffsll((unsigned long long)cand) - 1;
        acc |= 1ull << i;
        const uint32_t si = (uint32_t)__shfl((int)st, i, 64), ei = (uint32_t)__shfl((int)e, i, 64);
        const bool hit = lane > i && st <= ei && si <= e;
        cand &= ~__ballot(hit);
        cand &= cand - 1;  // lane i itself
      }
      const bool a = (acc >> lane) & 1ull;
      if (valid) state[q] = a ? 1 : 2;
      if (a) {
        const int pos = __popcll(acc & ((1ull << lane) - 1ull));
        as[pos] = st;
        ae[pos] = e + 1;
      }
      if (lane == 0) nacc = (uint32_t)__popcll(acc);
    }
    __syncthreads();
    const uint32_t na = nacc;
    for (uint32_t i = 0; i < na; i++) {
      const uint32_t S = as[i], E = ae[i];
      const uint32_t A = min((S + 15u) & ~15u, E), B = max(A, E & ~15u);  // [A, B) 16-byte aligned
      if (S + (uint32_t)tid < A) mark[S + tid] = 1;
      if (B + (uint32_t)tid < E) mark[B + tid] = 1;
      uint4 *body = reinterpret_cast<uint4 *>(mark + A);
      for (uint32_t x = tid; x < (B - A) / 16; x += kPrefixThreads) body[x] = ones;
    }
    __threadfence();  // the next batch's mark reads see every wavefront's paint
    __syncthreads();
  }
}

// Round 1's undecided list after a prefix of k: candidates k..m-1 in order.
__global__ void k_sel_prefix_rest(uint32_t *pend, uint32_t k, const uint32_t *m_dev, uint32_t *nlive1) {
  const uint32_t m = *m_dev;
  const uint32_t rest = m > k ? m - k : 0u;
  if (blockIdx.x == 0 && threadIdx.x == 0) *nlive1 = rest;
  GRID_STRIDE(i, rest) pend[i] = k + (uint32_t)i;
}

void sel_prefix(const uint32_t *len, const uint32_t *start, uint32_t k, uint8_t *state, uint8_t *mark,
                uint32_t *pend, const uint32_t *m_dev, uint32_t *nlive1, uint64_t bound, hipStream_t s) {
  hipLaunchKernelGGL(k_sel_prefix, dim3(1), dim3(kPrefixThreads), 0, s, len, start, k, state, mark);
  hipLaunchKernelGGL(k_sel_prefix_rest, grid_for(bound, 256, 8192), dim3(256), 0, s, pend, k, m_dev, nlive1);
}

// ----------------------------------------- per-window sequential greedy
// For candidate lists ordered window by window (each window's candidates in
// priority order): one wavefront per window walks its list in batches of 64
// over an LDS bitmap of the window's accepted positions, which reproduces
// the sequential greedy exactly.  A lane passes when neither end of its
// interval is marked (exact, because every interval accepted before it is at
// least as long); the lowest passing lane is accepted and knocks out every
// later passing lane whose interval intersects it, until no passing lane is
// left; the accepted intervals are then painted, one at a time by the whole
// wavefront.  The walk is sequential, so its time is the latency of one
// batch times the batches of the longest window: candidate loads run
// kWinSelDepth batches ahead in a register ring so that they never wait.
// state[k] = 1 (accepted) or 2 (rejected) for every candidate.
constexpr int kWinSelDepth = 16;
constexpr uint32_t kOwnPaint = 4;  // intervals of up to this many bitmap words are painted by their own lane

// First index k in [lo, hi) whose window is >= w (hi if none), for a
// window-major list: a 64-ary search by the whole wavefront (each step
// probes 64 evenly spaced entries), window of entry k = wid[start[k]].
__device__ uint32_t window_lower_bound(const uint32_t *start, const uint32_t *wid, uint32_t lo, uint32_t hi,
                                       uint32_t w) {
  const int lane = threadIdx.x & 63;
  while (hi - lo > 64) {
    const uint32_t step = (hi - lo + 63) / 64;
    const uint32_t k = lo + (uint32_t)lane * step;
    const bool below = k < hi && wid[start[k]] < w;
    const uint64_t m = __ballot(below);
    // probes below w form a prefix of the lanes
    const int nb = __popcll(m);
    if (nb == 0) return lo;  // probe 0 is lo itself: nothing below
    const uint32_t nlo = lo + (uint32_t)(nb - 1) * step + 1;
    const uint32_t nhi = min(hi, lo + (uint32_t)nb * step);
    lo = nlo;
    hi = nhi;
  }
  const uint32_t k = lo + (uint32_t)lane;
  const bool below = k < hi && wid[start[k]] < w;
  return lo + (uint32_t)__popcll(__ballot(below));
}

__global__ __launch_bounds__(64) void k_sel_window(const uint32_t *len, const uint32_t *start, const uint32_t *m_dev,
                                                   const uint32_t *wid, const uint64_t *woff, uint32_t nwin,
                                                   uint8_t *state) {
  extern __shared__ uint32_t bm[];
  const uint32_t w = blockIdx.x;
  if (w >= nwin) return;
  const int lane = threadIdx.x;
  const uint32_t m = *m_dev;
  uint32_t c0 = 0, c1 = m;
  if (wid) {
    c0 = window_lower_bound(start, wid, 0, m, w);
    c1 = window_lower_bound(start, wid, c0, m, w + 1);
  }
  if (c0 >= c1) return;
  const uint32_t ws = (uint32_t)woff[w];
  const uint32_t L = (uint32_t)(woff[w + 1] - woff[w]);
  for (uint32_t x = lane; x < (L + 31) / 32; x += 64) bm[x] = 0;
  // Chunks of kWinSelDepth batches, double-buffered in registers: the next
  // chunk's loads are issued (unconditionally, indices clamped, so the
  // compiler can count them) before the current chunk is walked, and the
  // chunk's states are stored after the walk, so no memory wait sits inside
  // the walk.
  const uint32_t last = c1 - 1;
  uint32_t cs[kWinSelDepth], cl[kWinSelDepth], ns[kWinSelDepth], nl[kWinSelDepth];
#pragma unroll
  for (int d = 0; d < kWinSelDepth; d++) {
    const uint32_t k = min(c0 + (uint32_t)(d * 64 + lane), last);
    cs[d] = start[k];
    cl[d] = len[k];
  }
  __syncthreads();
  for (uint32_t base = c0; base < c1; base += 64 * kWinSelDepth) {
#pragma unroll
    for (int d = 0; d < kWinSelDepth; d++) {
      const uint32_t k = min(base + (uint32_t)(64 * kWinSelDepth + d * 64 + lane), last);
      ns[d] = start[k];
      nl[d] = len[k];
    }
    uint64_t acc[kWinSelDepth];
#pragma unroll
    for (int d = 0; d < kWinSelDepth; d++) {
      const uint32_t k = base + d * 64 + lane;
      const bool valid = k < c1;
      const uint32_t s = cs[d] - ws, e = s + cl[d] - 1u;
      // both end words read together (one LDS round trip, not two)
      const uint32_t ws0 = valid ? bm[s >> 5] : 0u, we0 = valid ? bm[e >> 5] : 0u;
      const bool ok = valid && !((ws0 >> (s & 31)) & 1u) && !((we0 >> (e & 31)) & 1u);
      uint64_t pass = __ballot(ok);
      uint64_t a = 0;
      while (pass) {
        const int j = __ffsll((unsigned long long)pass) - 1;
        const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)s, j),
                       ej = (uint32_t)__builtin_amdgcn_readlane((int)e, j);  // j is uniform
        a |= 1ull << j;
        pass &= ~__ballot(valid && s <= ej && e >= sj);  // j itself and the later lanes it overlaps
      }
      // accepted lanes whose interval spans at most kOwnPaint words paint it
      // themselves; longer ones are painted by the whole wavefront, one by one
      const bool mine = (a >> lane) & 1ull;
      const bool own = mine && ((e >> 5) - (s >> 5)) < kOwnPaint;
      if (own) {
        for (uint32_t x = s >> 5; x <= (e >> 5); x++) {
          uint32_t msk = 0xFFFFFFFFu;
          if (x == (s >> 5)) msk &= 0xFFFFFFFFu << (s & 31);
          if (x == (e >> 5)) msk &= 0xFFFFFFFFu >> (31 - (e & 31));
          atomicOr(&bm[x], msk);
        }
      }
      uint64_t todo = a & ~__ballot(own);
      while (todo) {
        const int j = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const uint32_t sj = (uint32_t)__builtin_amdgcn_readlane((int)s, j),
                       ej = (uint32_t)__builtin_amdgcn_readlane((int)e, j);  // j is uniform
        const uint32_t w0 = sj >> 5, w1 = ej >> 5;
        for (uint32_t x = w0 + lane; x <= w1; x += 64) {
          uint32_t msk = 0xFFFFFFFFu;
          if (x == w0) msk &= 0xFFFFFFFFu << (sj & 31);
          if (x == w1) msk &= 0xFFFFFFFFu >> (31 - (ej & 31));
          atomicOr(&bm[x], msk);  // accepted intervals may share their end words
        }
      }
      acc[d] = a;
    }
#pragma unroll
    for (int d = 0; d < kWinSelDepth; d++) {
      const uint32_t k = base + d * 64 + lane;
      if (k < c1) state[k] = ((acc[d] >> lane) & 1ull) ? 1 : 2;
    }
#pragma unroll
    for (int d = 0; d < kWinSelDepth; d++) {
      cs[d] = ns[d];
      cl[d] = nl[d];
    }
  }
}

void sel_windows(const uint32_t *len, const uint32_t *start, const uint32_t *m_dev, uint64_t bound,
                 const uint32_t *wid, const uint64_t *woff, uint32_t nwin, uint64_t maxwin, uint8_t *state,
                 hipStream_t s) {
  (void)bound;
  const size_t lds = ((maxwin + 31) / 32) * 4;
  hipLaunchKernelGGL(k_sel_window, dim3(nwin), dim3(64), lds, s, len, start, m_dev, wid, woff, nwin, state);
}

// ------------------------------------------------- per-interval greedy counts
// Candidates sorted by (length desc, ID asc, start asc): a group of equal
// (length, ID) is one substring, its occurrences in increasing start order.
// next[k] = first member k' of k's group with start[k'] >= start[k] + len[k]
// (the next occurrence the equal-length greedy of Algorithm 2 would keep
// after k, ignoring other substrings), found by binary search in priority
// order; count[k] = length of the chain k, next[k], next[next[k]], ...  by
// pointer jumping.  count at a group's first member is the substring's
// isolated non-overlapping occurrence count.

__global__ void k_group_next(const uint32_t *len, const uint32_t *start, const uint32_t *id, uint32_t m,
                             uint32_t *next, uint32_t *cnt, uint32_t *ptr) {
  GRID_STRIDE(k, m) {
    const uint32_t l = len[k], g = id[k];
    const uint64_t e = (uint64_t)start[k] + l;
    // first index in (k, m) whose key is not below (l, g, e) in priority order
    uint32_t lo = (uint32_t)k + 1, hi = m;
    while (lo < hi) {
      const uint32_t mid = lo + (hi - lo) / 2;
      const uint32_t lm = len[mid];
      const bool below = lm > l || (lm == l && (id[mid] < g || (id[mid] == g && (uint64_t)start[mid] < e)));
      if (below) lo = mid + 1;
      else hi = mid;
    }
    const uint32_t nx = (lo < m && len[lo] == l && id[lo] == g) ? lo : kNone;
    next[k] = nx;
    ptr[k] = nx;
    cnt[k] = 1;
  }
}

__global__ void k_chain_jump(uint32_t m, const uint32_t *cnt, const uint32_t *ptr, uint32_t *cnt2, uint32_t *ptr2) {
  GRID_STRIDE(k, m) {
    const uint32_t p = ptr[k];
    if (p == kNone) {
      cnt2[k] = cnt[k];
      ptr2[k] = kNone;
    } else {
      cnt2[k] = cnt[k] + cnt[p];
      ptr2[k] = ptr[p];
    }
  }
}

void interval_counts(const uint32_t *len, const uint32_t *start, const uint32_t *id, uint32_t m, uint32_t *next,
                     uint32_t *count, uint32_t *tmp, hipStream_t s) {
  if (m == 0) return;
  uint32_t *c[2] = {count, tmp}, *p[2] = {tmp + m, tmp + 2 * (uint64_t)m};
  hipLaunchKernelGGL(k_group_next, grid_for(m, 256, 8192), dim3(256), 0, s, len, start, id, m, next, c[0], p[0]);
  // a chain is at most m long: ceil(log2 m) doublings reach every end
  int cur = 0;
  for (uint64_t span = 1; span < m; span <<= 1) {
    hipLaunchKernelGGL(k_chain_jump, grid_for(m, 256, 8192), dim3(256), 0, s, m, c[cur], p[cur], c[cur ^ 1],
                       p[cur ^ 1]);
    cur ^= 1;
  }
  if (cur) copy_n_u32(count, c[1], m, s);
}

// ---------------------------------------------------------------- output
struct GatherAccepted {
  using Rec = uint3;
  const uint32_t *len, *start, *id;
  uint32_t *o_len, *o_start, *o_id;
  __device__ Rec get(uint64_t k) const { return make_uint3(len[k], start[k], id[k]); }
  __device__ void put(uint32_t o, Rec r) const { o_len[o] = r.x; o_start[o] = r.y; o_id[o] = r.z; }
};

void gather_accepted(const uint8_t *state, const uint32_t *m_dev, uint64_t bound, const uint32_t *len,
                     const uint32_t *start, const uint32_t *id, uint32_t *o_len, uint32_t *o_start, uint32_t *o_id,
                     uint32_t *tile_tmp, uint32_t *total, hipStream_t s) {
  flag_compact(state, FlagIsOne{}, m_dev, bound, tile_tmp, total, GatherAccepted{len, start, id, o_len, o_start, o_id},
               s);
}

// Occurrence o (in final order: window, then priority) opens a row when its
// window, length or substring ID differs from occurrence o-1.
__global__ void k_row_flags(const uint32_t *order, const uint32_t *a_dev, const uint32_t *o_len,
                            const uint32_t *o_start, const uint32_t *o_id, const uint32_t *wid, uint32_t *f) {
  const uint64_t a = *a_dev;
  GRID_STRIDE(o, a) {
    const uint32_t c = order ? order[o] : (uint32_t)o;
    bool nr = (o == 0);
    if (!nr) {
      const uint32_t p = order ? order[o - 1] : (uint32_t)(o - 1);
      nr = o_len[c] != o_len[p] || o_id[c] != o_id[p] ||
           (wid && wid[o_start[c]] != wid[o_start[p]]);
    }
    f[o] = nr ? 1u : 0u;
  }
}

struct OutRow { uint32_t start, length, count; };
struct OutOcc { uint32_t start, length, cand; };

// woff: window offsets (window w starts at position woff[w]; null for one
// window).  Rows come in window order, so a wavefront's new rows fall into one
// or two windows and their per-window counts are added once per window.
__global__ void k_emit(const uint32_t *order, const uint32_t *a_dev, const uint32_t *o_len, const uint32_t *o_start,
                       const uint32_t *wid, const uint64_t *woff, const uint32_t *f, const uint32_t *rowidx,
                       uint32_t *row_first, OutRow *rows, OutOcc *occ, uint32_t *win_rows) {
  const uint64_t a = *a_dev;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t o0 = (uint64_t)blockIdx.x * blockDim.x; o0 < a; o0 += stride) {  // wavefront-uniform trip count
    const uint64_t o = o0 + threadIdx.x;
    if (o >= a) continue;
    const uint32_t c = order ? order[o] : (uint32_t)o;
    const uint32_t r = rowidx[o] + f[o] - 1u;  // row of this occurrence (inclusive count - 1)
    const uint32_t st = o_start[c];
    const uint32_t w = wid ? wid[st] : 0u;
    const uint32_t rel = st - (woff ? (uint32_t)woff[w] : 0u);
    if (f[o]) {
      row_first[r] = (uint32_t)o;
      rows[r].start = rel;
      rows[r].length = o_len[c];
      if (win_rows) agg_add_any(&win_rows[w], 1u);
    }
    if (occ) { occ[o].start = rel; occ[o].length = o_len[c]; occ[o].cand = r; }
  }
}

__global__ void k_row_counts(const uint32_t *row_first, const uint32_t *nrows_dev, const uint32_t *a_dev,
                             OutRow *rows) {
  const uint32_t nrows = *nrows_dev, a = *a_dev;
  GRID_STRIDE(r, nrows) {
    const uint32_t e = (r + 1 < nrows) ? row_first[r + 1] : a;
    rows[r].count = e - row_first[r];
  }
}

void emit_rows(const uint32_t *order, const uint32_t *a_dev, uint64_t bound, const uint32_t *o_len,
               const uint32_t *o_start, const uint32_t *o_id, const uint32_t *wid, const uint64_t *woff, uint32_t *f,
               uint32_t *rowidx, uint32_t *row_first, void *rows, void *occ, uint32_t *win_rows, uint32_t *tile_tmp,
               uint32_t *nrows, hipStream_t s) {
  hipLaunchKernelGGL(k_row_flags, grid_for(bound, 256, 8192), dim3(256), 0, s, order, a_dev, o_len, o_start, o_id, wid,
                     f);
  scan_excl(f, rowidx, a_dev, bound, tile_tmp, nrows, s);
  hipLaunchKernelGGL(k_emit, grid_for(bound, 256, 8192), dim3(256), 0, s, order, a_dev, o_len, o_start, wid, woff, f,
                     rowidx, row_first, (OutRow *)rows, (OutOcc *)occ, win_rows);
  hipLaunchKernelGGL(k_row_counts, grid_for(bound, 256, 8192), dim3(256), 0, s, row_first, nrows, a_dev,
                     (OutRow *)rows);
}

}  // namespace apo

namespace apo {

__global__ void k_window_of_occ(const uint32_t *o_start, const uint32_t *wid, const uint32_t *a_dev, uint32_t *out) {
  const uint64_t a = *a_dev;
  GRID_STRIDE(o, a) out[o] = wid[o_start[o]];
}
__global__ void k_iota_n(uint32_t *p, const uint32_t *n_dev) {
  const uint64_t n = *n_dev;
  GRID_STRIDE(i, n) p[i] = (uint32_t)i;
}

void window_of_occ(const uint32_t *o_start, const uint32_t *wid, const uint32_t *a_dev, uint64_t bound, uint32_t *out,
                   hipStream_t s) {
  hipLaunchKernelGGL(k_window_of_occ, grid_for(bound, 256, 8192), dim3(256), 0, s, o_start, wid, a_dev, out);
}
void iota_u32(uint32_t *p, const uint32_t *n_dev, uint64_t bound, hipStream_t s) {
  hipLaunchKernelGGL(k_iota_n, grid_for(bound, 256, 8192), dim3(256), 0, s, p, n_dev);
}

}  // namespace apo
