// Small device helpers (wave64 scans, hashing) shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apo {

// LDS index with one skew word per 16: threads that each walk 16
// consecutive words then hit different banks.
__host__ __device__ constexpr int pad16(int p) { return p + (p >> 4); }

// The command processor hands workgroups to the eight XCDs in turn (block b
// to XCD b mod 8), and each XCD has its own L2.  Renumbering the blocks so
// that every XCD runs one contiguous share of the logical block range keeps
// the lines that neighbouring blocks share (one window's ranks, suffixes and
// tokens) in a single L2 instead of fetching them into all eight.  A
// bijection on [0, G): XCD x's blocks x, x + 8, ... become x*q + min(x, G mod 8)
// + 0, 1, ... with q = G / 8.
__host__ __device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
  const uint32_t q = G >> 3, rem = G & 7u, x = b & 7u;
  return x * q + (x < rem ? x : rem) + (b >> 3);
}

// Grid-stride form: the item of physical block b in the pass that starts at
// item `base` (G blocks, `total` items).  The blocks are renumbered over the
// g = min(G, total - base) of them that have an item in this pass, so a short
// pass still spreads over every XCD; a block without an item gets `total`.
__host__ __device__ __forceinline__ uint64_t xcd_item(uint64_t base, uint64_t total, uint32_t b, uint32_t G) {
  const uint64_t left = total - base;
  const uint32_t g = left < (uint64_t)G ? (uint32_t)left : G;
  return b < g ? base + xcd_block(b, g) : total;
}

__device__ __forceinline__ uint32_t wave_incl_sum(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ uint32_t wave_incl_max(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x = x > y ? x : y;
  }
  return x;
}

// Block-wide exclusive sum over NT threads.  `sh` needs NT/64 words.  Returns
// the exclusive prefix of the calling thread; *total receives the block sum.
template <int NT>
__device__ __forceinline__ uint32_t block_excl_sum(uint32_t x, uint32_t *sh, uint32_t *total) {
  const uint32_t inc = wave_incl_sum(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; i++) {
    const uint32_t v = sh[i];
    before += (i < w) ? v : 0u;
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return before + inc - x;
}

// Block-wide inclusive max over NT threads.
template <int NT>
__device__ __forceinline__ uint32_t block_incl_max(uint32_t x, uint32_t *sh) {
  const uint32_t inc = wave_incl_max(x);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 63) sh[w] = inc;
  __syncthreads();
  uint32_t before = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; i++) {
    const uint32_t v = sh[i];
    if (i < w) before = before > v ? before : v;
  }
  __syncthreads();
  return before > inc ? before : inc;
}

// SplitMix64 finaliser (Steele/Lea/Flood; constants by Vigna), used as a hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ int class_of(uint32_t len) {
  // 1-based class c with len in (2^(c-1), 2^c], len==1 -> c=1; returns c-1
  int c = 32 - __clz((int)(len - 1u));  // ceil(log2(len)) for len>=2, 0 for len==1
  if (len <= 1u) c = 0;
  c = c < 1 ? 1 : c;
  return c - 1;
}

}  // namespace apo

namespace apo {

// Wave-aggregated increment of an LDS/global counter: when every active lane
// of the wavefront targets the same counter (the common case for the heavily
// repeated keys of loop-structured token streams), one lane adds the number
// of active lanes and the others derive their slot from their rank; otherwise
// each lane increments on its own.  Returns the counter value before this
// lane's increment (a unique slot among all callers).
__device__ __forceinline__ uint32_t agg_inc(uint32_t *ctr) {
  const uint64_t active = __ballot(1);
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)active) - 1;
  const uintptr_t mine = reinterpret_cast<uintptr_t>(ctr);
  const uint32_t lo = (uint32_t)mine, hi = (uint32_t)(mine >> 32);
  const bool same = __all(lo == (uint32_t)__shfl((int)lo, leader, 64) && hi == (uint32_t)__shfl((int)hi, leader, 64));
  if (same) {
    const uint32_t rank = (uint32_t)__popcll(active & ((1ull << lane) - 1ull));
    uint32_t old = 0;
    if (lane == leader) old = atomicAdd(ctr, (uint32_t)__popcll(active));
    old = (uint32_t)__shfl((int)old, leader, 64);
    return old + rank;
  }
  return atomicAdd(ctr, 1u);
}

// Same, when only the total matters.
// atomicAdd(ctr, v) for every active lane, one atomic per distinct address
// among the wavefront's active lanes (v must agree among lanes that share an
// address).  For counters that a few addresses share per wavefront.
__device__ __forceinline__ void agg_add_any(uint32_t *ctr, uint32_t v) {
  uint64_t todo = __ballot(1);
  const int lane = __lane_id();
  const uint64_t mine = reinterpret_cast<uintptr_t>(ctr);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const uint64_t la = ((uint64_t)(uint32_t)__shfl((int)(mine >> 32), leader, 64) << 32) |
                        (uint32_t)__shfl((int)(uint32_t)mine, leader, 64);
    const uint64_t grp = __ballot(mine == la) & todo;
    if (lane == leader) atomicAdd(ctr, v * (uint32_t)__popcll(grp));
    todo &= ~grp;
  }
}

__device__ __forceinline__ void agg_add(uint32_t *ctr, uint32_t v) {
  const uint64_t active = __ballot(1);
  const int lane = __lane_id();
  const int leader = __ffsll((unsigned long long)active) - 1;
  const uintptr_t mine = reinterpret_cast<uintptr_t>(ctr);
  const uint32_t lo = (uint32_t)mine, hi = (uint32_t)(mine >> 32);
  const bool same = __all(lo == (uint32_t)__shfl((int)lo, leader, 64) && hi == (uint32_t)__shfl((int)hi, leader, 64));
  if (same) {
    // every lane adds the same v in all call sites
    if (lane == leader) atomicAdd(ctr, v * (uint32_t)__popcll(active));
    return;
  }
  atomicAdd(ctr, v);
}

}  // namespace apo
