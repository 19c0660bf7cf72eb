// Segmented refine-sort engine.
//
// State: slots [0, cap) hold (key, val) pairs; a set of "units" (contiguous
// slot ranges) must each be sorted by key, after which every run of equal keys
// becomes a group.  Groups of size >= 2 become the units of the next level
// (next doubling round, or the next key of a multi-key sort).  Order among
// equal keys is left unspecified: every consumer only depends on group
// membership, and the final order is fully determined once all groups are
// singletons or exact duplicates.
//
// Units of up to 64 entries are sorted one per wavefront row in registers;
// units of 65..2^tile_log entries are grouped in LDS (a hash table counts the
// distinct keys of a tile's units, only those are sorted, and every entry is
// placed at its group's offset), with an LDS bitonic sort for class 13 when
// the tile is 8192 entries.  Longer units are split by MSD bucketing passes on
// digit_bits-bit digits (histogram, scan, scatter into the alternate buffer)
// until the pieces fit the LDS path or all key bits are consumed (the piece
// then is one group).
#include "apo_internal.h"
#include "device_util.h"
#include "segsort.h"
#include <algorithm>

namespace apo {

enum { MODE_SA = 0, MODE_PLAIN = 1 };

// Buffer b of the key/value pairs.  A per-lane index into the kernel
// argument's pointer array would be a dependent global load; selecting
// between the two pointers (scalar kernel-argument loads) avoids it.
__device__ __forceinline__ uint32_t *key_buf(const SortBufs &B, int b) { return b ? B.key[1] : B.key[0]; }
__device__ __forceinline__ uint32_t *val_buf(const SortBufs &B, int b) { return b ? B.val[1] : B.val[0]; }

// ------------------------------------------------------------------ resets
__global__ void k_round_begin(SortCounters *c, int cur) {
  const int nxt = cur ^ 1;
  const int t = threadIdx.x;
  if (t < kClasses) c->cls_cnt[nxt][t] = 0;
  if (t >= 1 && t < kMsdLists) c->big_pk[cur][t] = 0;
  if (t == 0) {
    c->big_pk[nxt][0] = 0;
    c->bulk_pk = 0;
    c->act_cnt[nxt] = 0;
    c->lds_elems = 0;
  }
}

// Records the outcome of round `r` (active slots and large units handed to
// the next round, entries sorted in LDS) so the host can read several rounds
// at once.
__global__ void k_round_end(const SortCounters *c, int cur, int r, uint32_t *hist) {
  if (threadIdx.x == 0) {
    hist[4 * r] = c->act_cnt[cur ^ 1];
    hist[4 * r + 1] = (uint32_t)(c->big_pk[cur ^ 1][0] >> 32);
    hist[4 * r + 2] = c->lds_elems;
  }
}

__device__ __forceinline__ uint32_t chunks_of(uint32_t len, uint32_t chunk_log) {
  return (len + (1u << chunk_log) - 1) >> chunk_log;
}

// Appends one large unit to a list with its chunk base.
__device__ __forceinline__ void append_big(BigUnit *list, unsigned long long *pk, uint32_t cap, uint32_t start,
                                           uint32_t len, uint32_t meta, uint32_t *err, uint32_t chunk_log) {
  const unsigned long long old = atomicAdd(pk, (1ull << 32) | chunks_of(len, chunk_log));
  const uint32_t k = (uint32_t)(old >> 32);
  if (k < cap) list[k] = BigUnit{start, len, (uint32_t)old, meta};
  else atomicOr(err, 2u);
}

// Number of units of a list (clamped to its capacity) and of their chunks.
__device__ __forceinline__ void list_size(unsigned long long pk, uint32_t cap, uint32_t &units, uint32_t &chunks) {
  units = min((uint32_t)(pk >> 32), cap);
  chunks = (uint32_t)pk;
}

// Largest u < units with U[u].cbase <= ch.
__device__ __forceinline__ uint32_t find_unit(const BigUnit *U, uint32_t units, uint32_t ch) {
  uint32_t lo = 0, hi = units;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (U[mid].cbase <= ch) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_counters_reset(SortCounters *c) {
  uint32_t *w = reinterpret_cast<uint32_t *>(c);
  const int nw = sizeof(SortCounters) / 4;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) w[i] = 0;
}

// -------------------------------------------------------------- unit setup
// Routes the ranges [off[w], off[w+1]) to the class lists or the level-0 big
// list of list `cur`.  Empty ranges are skipped, and with `only` set the
// ranges w with only[w] == 0.
__global__ void k_init_units(SortBufs B, int cur, const uint64_t *off, uint32_t nranges,
                             uint32_t base, uint32_t key_bits, const uint8_t *only) {
  const uint32_t w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nranges || (only && !only[w])) return;
  const uint32_t s = (uint32_t)(off[w] - off[0]) + base;
  const uint32_t len = (uint32_t)(off[w + 1] - off[w]);
  if (len == 0) return;
  if (len <= (1u << B.tile_log)) {
    const int ci = class_of(len);
    const uint32_t k = atomicAdd(&B.ctr->cls_cnt[cur][ci], 1u);
    const uint32_t capc = B.cls_off[ci + 1] - B.cls_off[ci];
    if (k >= capc) { atomicOr(&B.ctr->err, 1u); return; }
    B.cls[cur][B.cls_off[ci] + k] = Unit{s, len};
  } else {
    append_big(B.big[cur][0], &B.ctr->big_pk[cur][0], B.big_cap, s, len, key_bits, &B.ctr->err, B.chunk_log);
  }
}

// Routes runs [rs[r], rs[r+1]) (the last one ends at *total_dev) of length
// >= 2 to the class lists or the level-0 big list of list `cur`; *nruns_dev
// runs.  A thread takes kRunItems consecutive runs, and class-list slots are
// reserved once per workgroup pass and class (most runs are singletons).
constexpr int kRunItems = 8;

__global__ __launch_bounds__(256) void k_init_runs(SortBufs B, int cur, const uint32_t *rs,
                                                   const uint32_t *nruns_dev, const uint32_t *total_dev,
                                                   uint32_t key_bits) {
  __shared__ uint32_t cnt[kClasses], cbase[kClasses];
  const uint32_t R = *nruns_dev, total = *total_dev;
  const int lane = threadIdx.x & 63;
  const uint64_t span = (uint64_t)blockDim.x * kRunItems;
  for (uint64_t r0 = (uint64_t)blockIdx.x * span; r0 < R; r0 += (uint64_t)gridDim.x * span) {
    if (threadIdx.x < kClasses) cnt[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t rb = r0 + (uint64_t)threadIdx.x * kRunItems;
    uint32_t bound[kRunItems + 1];
#pragma unroll
    for (int k = 0; k <= kRunItems; k++) bound[k] = rb + k < R ? rs[rb + k] : total;
    uint32_t loc[kRunItems];
    int ci[kRunItems];
#pragma unroll
    for (int k = 0; k < kRunItems; k++) {
      const uint32_t len = rb + k < R ? bound[k + 1] - bound[k] : 0u;
      ci[k] = -1;
      loc[k] = 0;
      if (len >= 2 && len <= (1u << B.tile_log)) ci[k] = class_of(len);
      else if (len > (1u << B.tile_log))
        append_big(B.big[cur][0], &B.ctr->big_pk[cur][0], B.big_cap, bound[k], len, key_bits, &B.ctr->err,
                   B.chunk_log);
      // slot within the workgroup's share of the class: one LDS add per
      // class present in the wavefront
      uint64_t todo = __ballot(ci[k] >= 0);
      while (todo) {
        const int leader = __ffsll((unsigned long long)todo) - 1;
        const int lc = __shfl(ci[k], leader, 64);
        const uint64_t grp = __ballot(ci[k] == lc) & todo;
        uint32_t b = 0;
        if (lane == leader) b = atomicAdd(&cnt[lc], (uint32_t)__popcll(grp));
        b = (uint32_t)__shfl((int)b, leader, 64);
        if ((grp >> lane) & 1ull) loc[k] = b + (uint32_t)__popcll(grp & ((1ull << lane) - 1ull));
        todo &= ~grp;
      }
    }
    __syncthreads();
    if (threadIdx.x < kClasses) {
      const uint32_t c = cnt[threadIdx.x];
      cbase[threadIdx.x] = c ? atomicAdd(&B.ctr->cls_cnt[cur][threadIdx.x], c) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRunItems; k++) {
      if (ci[k] < 0) continue;
      const uint32_t slot = cbase[ci[k]] + loc[k];
      const uint32_t capc = B.cls_off[ci[k] + 1] - B.cls_off[ci[k]];
      if (slot < capc) B.cls[cur][B.cls_off[ci[k]] + slot] = Unit{bound[k], bound[k + 1] - bound[k]};
      else atomicOr(&B.ctr->err, 1u);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ gathers
// Round 0 of suffix sorting: slot p holds suffix p, keyed by its first token
// (its dense rank or, for 32-bit input, the token itself).  With `only` set,
// just the slots p whose window wid[p] has only[wid[p]] != 0, and nothing
// unless *gate > 0.
__global__ void k_gather_identity(SortBufs B, const uint32_t *src, uint32_t n, const uint32_t *wid,
                                  const uint8_t *only, const uint32_t *gate) {
  if (gate && *gate == 0) return;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    if (only && !only[wid[p]]) continue;
    B.key[0][p] = src[p];
    B.val[0][p] = p;
  }
}

// Doubling round with offset h: key = rank of the suffix h positions later,
// 0 when that lies past the end of the suffix's window.
// Block 0 also closes the previous round (records its outcome in hist[r-1])
// and clears the counters of this round (what k_round_end / k_round_begin do).
// Opens round r (records round r-1's outcome, resets the list counters) and
// gathers the sort key of every still-grouped slot: the rank of the suffix
// 2^(r-1) positions later (0 past the window end).  A dense pass over the
// slots (the grouped-slot flags are sequential) instead of an active list.
__global__ void k_gather_sa(SortBufs B, int cur, const uint32_t *rank, const uint8_t *aflag,
                            const uint32_t *slot_wend, uint32_t n, uint32_t h, uint32_t *hist, int r) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SortCounters *c = B.ctr;
    const int nxt = cur ^ 1;
    hist[4 * (r - 1)] = c->act_cnt[cur];
    hist[4 * (r - 1) + 1] = (uint32_t)(c->big_pk[cur][0] >> 32);
    hist[4 * (r - 1) + 2] = c->lds_elems;
    for (int t = 0; t < kClasses; t++) c->cls_cnt[nxt][t] = 0;
    for (int t = 1; t < kMsdLists; t++) c->big_pk[cur][t] = 0;
    c->big_pk[nxt][0] = 0;
    c->bulk_pk = 0;
    c->act_cnt[nxt] = 0;
    c->lds_elems = 0;
  }
  if (B.ctr->act_cnt[cur] == 0) return;  // nothing grouped: a round launched past the last one
  // four consecutive slots per thread: flags, suffixes and window ends are
  // single 4- and 16-byte loads and the four partner-rank reads are issued
  // together.  Keys of slots no longer grouped are never read (only units
  // are sorted), so all four keys go out as one 16-byte store.  Blocks of
  // slots are handed out XCD by XCD: partner ranks lie in the same window, so
  // one XCD's L2 holds the lines its neighbouring blocks gather.
  const uint32_t *val = B.val[0];
  uint32_t *key = B.key[0];
  const uint64_t n4 = n / 4, nblk = (n4 + blockDim.x - 1) / blockDim.x;
  for (uint64_t base = 0; base < nblk; base += gridDim.x) {
    const uint64_t bk = xcd_item(base, nblk, blockIdx.x, gridDim.x);
    if (bk >= nblk) break;
    const uint64_t q = bk * blockDim.x + threadIdx.x;
    if (q >= n4) continue;
    const uint32_t fl = reinterpret_cast<const uint32_t *>(aflag)[q];
    if (!fl) continue;
    const uint4 v = reinterpret_cast<const uint4 *>(val)[q];
    const uint4 we = slot_wend ? reinterpret_cast<const uint4 *>(slot_wend)[q] : make_uint4(n, n, n, n);
    const uint32_t x[4] = {v.x + h, v.y + h, v.z + h, v.w + h}, e[4] = {we.x, we.y, we.z, we.w};
    uint32_t k[4];
#pragma unroll
    for (int u = 0; u < 4; u++) k[u] = (((fl >> (8 * u)) & 0xFFu) && x[u] < e[u]) ? rank[x[u]] : 0u;
    reinterpret_cast<uint4 *>(key)[q] = make_uint4(k[0], k[1], k[2], k[3]);
  }
  const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t p = 4 * n4 + gid;  // the last n mod 4 slots
  if (p < n && aflag[p]) {
    const uint32_t x = val[p] + h;
    const uint32_t we = slot_wend ? slot_wend[p] : n;
    key[p] = x < we ? rank[x] : 0u;
  }
}

__global__ void k_gather_field(SortBufs B, int cur, const uint32_t *field, int stride, const uint32_t *all_dev,
                               int sub, const uint32_t *c_dev, uint32_t c) {
  const uint32_t cnt = all_dev ? *all_dev : B.ctr->act_cnt[cur];
  if (c_dev) c = *c_dev;
  // four entries per thread, each step's loads issued together
  const uint32_t *act = B.act[cur], *val = B.val[0];
  uint32_t *key = B.key[0];
  const uint64_t step = (uint64_t)gridDim.x * blockDim.x * 4;
  for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x * 4; b0 < cnt; b0 += step) {
    uint32_t p[4], v[4], f[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint64_t q = b0 + (uint64_t)u * blockDim.x + threadIdx.x;  // coalesced for each u
      p[u] = q < cnt ? (all_dev ? (uint32_t)q : act[q]) : ~0u;
    }
#pragma unroll
    for (int u = 0; u < 4; u++) v[u] = p[u] != ~0u ? val[p[u]] : 0u;
#pragma unroll
    for (int u = 0; u < 4; u++) f[u] = p[u] != ~0u ? field[(uint64_t)v[u] * stride] : 0u;
#pragma unroll
    for (int u = 0; u < 4; u++)
      if (p[u] != ~0u) key[p[u]] = sub ? c - f[u] : f[u];
  }
}

__global__ void k_iota_val(SortBufs B, const uint32_t *n_dev) {
  const uint32_t n = *n_dev;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    B.val[0][p] = p;
}

// -------------------------------------------------------------- LDS sorting
template <int MODE, int TL>
__global__ __launch_bounds__(kLdsThreads) void k_lds_sort(SortBufs B, int cur, RankOut R,
                                                          uint32_t next_bits, int last_level,
                                                          uint8_t *keep, int ci_lo, int ci_hi) {
  constexpr int NT = kLdsThreads;
  constexpr int kLdsTile = 1 << TL;
  constexpr int kTileClasses = TL;
  constexpr int PER = kLdsTile / NT;  // consecutive slots per thread
  __shared__ uint64_t d[kLdsTile];
  __shared__ uint32_t hd[kLdsTile];
  __shared__ Unit ud[kLdsTile / 2];
  __shared__ uint32_t sh[NT / 64];
  __shared__ uint32_t cls_loc[kClasses], cls_base[kClasses];
  __shared__ uint32_t act_base;
  __shared__ uint32_t item_c, item_b, items_total;
  __shared__ uint32_t cnt_c[kClasses];

  const int nxt = cur ^ 1;
  const int tid = threadIdx.x;
  if (tid < kClasses) cnt_c[tid] = B.ctr->cls_cnt[cur][tid];
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0;
    for (int ci = ci_lo; ci < ci_hi && ci < kTileClasses; ci++) {
      const uint32_t per = (uint32_t)kLdsTile >> (ci + 1);
      tot += (cnt_c[ci] + per - 1) / per;
    }
    items_total = tot;
  }
  __syncthreads();
  const uint32_t total = items_total;

  uint32_t act_deferred = 0;
  for (uint32_t item = blockIdx.x; item < total; item += gridDim.x) {
    if (tid == 0) {
      uint32_t it = item;
      int ci = ci_lo;
      for (; ci < ci_hi && ci < kTileClasses; ci++) {
        const uint32_t per = (uint32_t)kLdsTile >> (ci + 1);
        const uint32_t ni = (cnt_c[ci] + per - 1) / per;
        if (it < ni) break;
        it -= ni;
      }
      item_c = (uint32_t)ci;
      item_b = it;
    }
    if (tid < kClasses) cls_loc[tid] = 0;
    __syncthreads();
    const int ci = (int)item_c;
    const int c = ci + 1;
    const uint32_t sub = 1u << c;
    const uint32_t per = (uint32_t)kLdsTile >> c;
    const uint32_t first = item_b * per;
    const uint32_t nb = min(per, cnt_c[ci] - first);
    const Unit *src = B.cls[cur] + B.cls_off[ci] + first;
    for (uint32_t j = tid; j < nb; j += NT) ud[j] = src[j];
    __syncthreads();
    if (tid == 0) {
      uint32_t tot = 0;
      for (uint32_t j = 0; j < nb; j++) tot += ud[j].len & kLenMask;
      atomicAdd(&B.ctr->lds_elems, tot);
    }

    // load (key, val) pairs; pad with all-ones
    for (int s = tid; s < kLdsTile; s += NT) {
      const uint32_t j = (uint32_t)s >> c, idx = (uint32_t)s & (sub - 1);
      uint64_t v = ~0ull;
      if (j < nb) {
        const Unit u = ud[j];
        const uint32_t len = u.len & kLenMask;
        if (idx < len) {
          const int b = (u.len & kBufBit) ? 1 : 0;
          const uint32_t p = u.start + idx;
          v = ((uint64_t)key_buf(B, b)[p] << 32) | val_buf(B, b)[p];
        }
      }
      d[s] = v;
    }
    __syncthreads();

    // bitonic sort of every sub-block of size `sub`, ascending
    for (uint32_t k = 2; k <= sub; k <<= 1) {
      for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
        for (uint32_t t = tid; t < (uint32_t)kLdsTile / 2; t += NT) {
          const uint32_t i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
          const uint32_t l = i | jj;
          const bool asc = (k == sub) || ((i & k) == 0);
          const uint64_t a = d[i], b = d[l];
          if ((a > b) == asc) { d[i] = b; d[l] = a; }
        }
        __syncthreads();
      }
    }

    // group heads: hd[s] = last boundary slot <= s.  Every sub-block starts
    // with a boundary, so the running maximum never leaves the sub-block.
    const int s0 = tid * PER;
    uint32_t run = 0;  // last boundary + 1 seen in this thread's chunk (0: none)
    for (int q = 0; q < PER; q++) {
      const int s = s0 + q;
      const uint32_t idx = (uint32_t)s & (sub - 1);
      const bool bnd = (idx == 0) || ((uint32_t)(d[s] >> 32) != (uint32_t)(d[s - 1] >> 32));
      if (bnd) run = (uint32_t)s + 1;
      hd[s] = run;
    }
    __shared__ uint32_t tmax[NT];
    tmax[tid] = block_incl_max<NT>(run, sh);
    __syncthreads();
    const uint32_t carry = tid > 0 ? tmax[tid - 1] : 0u;
    for (int q = 0; q < PER; q++) {
      const int s = s0 + q;
      const uint32_t h = hd[s];
      hd[s] = (h ? h : carry) - 1u;
    }
    __syncthreads();

    // regroup
    uint32_t my_act = 0;
    for (int q = 0; q < PER; q++) {
      const int s = s0 + q;
      const uint32_t j = (uint32_t)s >> c, idx = (uint32_t)s & (sub - 1);
      if (j >= nb) continue;
      const Unit u = ud[j];
      const uint32_t len = u.len & kLenMask;
      if (idx >= len) continue;
      const uint32_t hs = hd[s];
      const bool bnd = hs == (uint32_t)s;
      const bool last = (idx + 1 == len) || ((uint32_t)(d[s + 1] >> 32) != (uint32_t)(d[s] >> 32));
      const bool single = bnd && last;
      const uint32_t v = (uint32_t)d[s];
      const uint32_t gpos = u.start + (hs - (j << c));
      const uint32_t p = u.start + idx;
      B.val[0][p] = v;
      if (MODE == MODE_SA) {
        if (!((u.len & kHeadBit) && gpos == u.start)) R.rank[v] = gpos + 1;  // else unchanged
      }
      if (last_level) {
        keep[p] = bnd ? 1 : 0;
      } else {
        if (!single) my_act++;
        if (last && !bnd) {
          const uint32_t size = (uint32_t)s - hs + 1;
          atomicAdd(&cls_loc[class_of(size)], 1u);
        }
      }
    }
    if (!last_level) {
      uint32_t tot;
      const uint32_t off = block_excl_sum<NT>(my_act, sh, &tot);
      if (tid == 0) {
        if (R.aflag) act_deferred += tot;  // SA rounds keep flags: the count only, once per workgroup
        else act_base = tot ? atomicAdd(&B.ctr->act_cnt[nxt], tot) : 0u;
      }
      if (tid < kClasses) {
        const uint32_t m = cls_loc[tid];
        cls_base[tid] = m ? atomicAdd(&B.ctr->cls_cnt[nxt][tid], m) : 0u;
        cls_loc[tid] = 0;
      }
      __syncthreads();
      uint32_t w = act_base + off;
      for (int q = 0; q < PER; q++) {
        const int s = s0 + q;
        const uint32_t j = (uint32_t)s >> c, idx = (uint32_t)s & (sub - 1);
        if (j >= nb) continue;
        const Unit u = ud[j];
        const uint32_t len = u.len & kLenMask;
        if (idx >= len) continue;
        const uint32_t hs = hd[s];
        const bool bnd = hs == (uint32_t)s;
        const bool last = (idx + 1 == len) || ((uint32_t)(d[s + 1] >> 32) != (uint32_t)(d[s] >> 32));
        if (R.aflag) {
          R.aflag[u.start + idx] = (bnd && last) ? 0 : 1;
        } else if (!(bnd && last)) {
          if (w < B.cap) B.act[nxt][w] = u.start + idx;
          else atomicOr(&B.ctr->err, 4u);
          w++;
        }
        if (last && !bnd) {
          const uint32_t size = (uint32_t)s - hs + 1;
          const int cc = class_of(size);
          const uint32_t k = cls_base[cc] + atomicAdd(&cls_loc[cc], 1u);
          const uint32_t capc = B.cls_off[cc + 1] - B.cls_off[cc];
          if (k < capc)
            B.cls[nxt][B.cls_off[cc] + k] = Unit{u.start + (hs - (j << c)), size | (MODE == MODE_SA ? kHeadBit : 0u)};
          else atomicOr(&B.ctr->err, 8u);
        }
      }
    }
    (void)next_bits;
    __syncthreads();
  }
  if (threadIdx.x == 0 && act_deferred) atomicAdd(&B.ctr->act_cnt[nxt], act_deferred);
}

// ---------------------------------------------- wavefront sort (tiny units)
// Units of at most 64 entries (classes 1..6) are sorted inside one wavefront:
// a 64-lane row holds 64/2^c units of class c, bitonic stages are cross-lane
// exchanges, group heads come from a wave-wide max-scan, and appends are
// aggregated per wavefront with ballots.  No LDS, no barriers.
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, m, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}

constexpr int kWaveMaxCi = 6;  // classes 1..6 (0-based 0..5)
constexpr int kWaveItems = 8;  // items per wavefront per block batch
constexpr int kWaveCtrs = kWaveMaxCi + 2;  // new units per class, active entries, sorted entries

// Units of <= 64 entries, several per wavefront (2^(6-c) units of class c
// side by side), sorted by a bitonic network over lane shuffles.  A block
// takes a batch of 4 x kWaveItems items; the slots its new active entries
// and units need are reserved with one atomic per counter per batch (the
// per-item counts are wave ballots), so the hot list counters see few
// atomics.  The batch loop is uniform across the block.
template <int MODE>
__global__ __launch_bounds__(256, 5) void k_wave_sort(SortBufs B, int cur, RankOut R, int last_level, uint8_t *keep) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nxt = cur ^ 1;
  __shared__ uint32_t wtot[4][kWaveCtrs];
  __shared__ uint32_t wbase[4][kWaveCtrs];
  uint32_t cnt[kWaveMaxCi], first_item[kWaveMaxCi + 1];
  first_item[0] = 0;
#pragma unroll
  for (int ci = 0; ci < kWaveMaxCi; ci++) {
    cnt[ci] = B.ctr->cls_cnt[cur][ci];
    const uint32_t per = 64u >> (ci + 1);
    first_item[ci + 1] = first_item[ci] + (cnt[ci] + per - 1) / per;
  }
  const uint32_t total = first_item[kWaveMaxCi];
  const uint64_t lanes_lt = (1ull << lane) - 1ull;
  constexpr uint32_t kBatch = 4 * kWaveItems;
  uint32_t deferred = 0;  // threads kWaveMaxCi (SA active count) and kWaveMaxCi + 1 (sorted entries)
  for (uint64_t b0 = (uint64_t)blockIdx.x * kBatch; b0 < total; b0 += (uint64_t)gridDim.x * kBatch) {
    // per item and lane: slot of an entry that stays active, and a new unit
    uint32_t act_p[kWaveItems], unit_pos[kWaveItems], unit_code[kWaveItems];
    uint32_t tot[kWaveCtrs];
#pragma unroll
    for (int q = 0; q < kWaveCtrs; q++) tot[q] = 0;
    // the batch's global loads first (unit descriptors, then entries), so
    // that their latencies overlap instead of adding up item by item
    int ck[kWaveItems];
    uint32_t nbk[kWaveItems];
    Unit uk[kWaveItems];
    uint64_t vk[kWaveItems];
#pragma unroll
    for (int k = 0; k < kWaveItems; k++) {
      ck[k] = 0;
      nbk[k] = 0;
      uk[k] = Unit{0, 0};
      const uint64_t item = b0 + (uint64_t)wid * kWaveItems + k;
      if (item >= total) continue;  // wave-uniform
      int ci = 0;
#pragma unroll
      for (int q = 1; q < kWaveMaxCi; q++) ci += item >= first_item[q] ? 1 : 0;
      uint32_t cnt_ci = 0, off_ci = 0;
#pragma unroll
      for (int q = 0; q < kWaveMaxCi; q++)
        if (q == ci) { cnt_ci = cnt[q]; off_ci = first_item[q]; }
      const uint32_t per = 64u >> (ci + 1);
      const uint32_t first = (uint32_t)(item - off_ci) * per;
      const uint32_t nb = min(per, cnt_ci - first);
      const uint32_t j = (uint32_t)lane >> (ci + 1);
      ck[k] = ci;
      nbk[k] = nb;
      if (j < nb) uk[k] = B.cls[cur][B.cls_off[ci] + first + j];
    }
#pragma unroll
    for (int k = 0; k < kWaveItems; k++) {
      vk[k] = ~0ull;
      const int c = ck[k] + 1;
      const uint32_t j = (uint32_t)lane >> c, idx = (uint32_t)lane & ((1u << c) - 1);
      const Unit u = uk[k];
      if (j < nbk[k] && idx < (u.len & kLenMask)) {
        const int bb = (u.len & kBufBit) ? 1 : 0;
        const uint32_t p = u.start + idx;
        vk[k] = ((uint64_t)key_buf(B, bb)[p] << 32) | val_buf(B, bb)[p];
      }
    }
#pragma unroll
    for (int k = 0; k < kWaveItems; k++) {
      act_p[k] = kNone;
      unit_code[k] = 0;
      unit_pos[k] = 0;
      const uint64_t item = b0 + (uint64_t)wid * kWaveItems + k;
      if (item >= total) continue;  // wave-uniform
      const int c = ck[k] + 1;
      const uint32_t sub = 1u << c;
      const uint32_t nb = nbk[k];
      const uint32_t j = (uint32_t)lane >> c, idx = (uint32_t)lane & (sub - 1);
      const Unit u = uk[k];
      const uint32_t len = u.len & kLenMask;
      const bool valid = j < nb && idx < len;
      uint64_t v = vk[k];
      for (uint32_t kk = 2; kk <= sub; kk <<= 1) {
        for (uint32_t jj = kk >> 1; jj > 0; jj >>= 1) {
          const uint64_t o = shfl_xor64(v, (int)jj);
          const bool asc = (kk == sub) || (((uint32_t)lane & kk) == 0);
          const bool lower = ((uint32_t)lane & jj) == 0;
          v = (lower == asc) ? (v < o ? v : o) : (v > o ? v : o);
        }
      }
      const uint32_t key = (uint32_t)(v >> 32);
      const uint32_t prevkey = (uint32_t)__shfl_up((int)key, 1, 64);
      const uint32_t nextkey = (uint32_t)__shfl_down((int)key, 1, 64);
      const bool bnd = valid && (idx == 0 || key != prevkey);
      const bool last = valid && (idx + 1 == len || nextkey != key);
      const uint32_t hs = wave_incl_max(bnd ? (uint32_t)lane : 0u);  // head lane of this lane's group
      const bool single = bnd && last;
      const uint32_t p = u.start + idx;
      const uint32_t gpos = u.start + (hs - (j << c));
      if (valid) {
        const uint32_t val = (uint32_t)v;
        B.val[0][p] = val;
        if (MODE == MODE_SA) {
          if (!((u.len & kHeadBit) && gpos == u.start)) R.rank[val] = gpos + 1;  // else unchanged
        }
        if (last_level) keep[p] = bnd ? 1 : 0;
      }
      tot[kWaveMaxCi + 1] += (uint32_t)__popcll(__ballot(valid));
      if (!last_level) {
        const bool stay = valid && !single;
        tot[kWaveMaxCi] += (uint32_t)__popcll(__ballot(stay));
        if (R.aflag) {
          if (valid) R.aflag[p] = stay ? 1 : 0;
        } else if (stay) {
          act_p[k] = p;
        }
        // new units: groups of size >= 2, emitted by their last lane
        const bool emit = last && !bnd;
        const uint32_t size = (uint32_t)lane - hs + 1;
        const int mycc = emit ? class_of(size) : -1;
#pragma unroll
        for (int cc = 0; cc < kWaveMaxCi; cc++) tot[cc] += (uint32_t)__popcll(__ballot(mycc == cc));
        if (emit) {
          unit_pos[k] = gpos;
          unit_code[k] = (size << 8) | (uint32_t)(mycc + 1);
        }
      }
    }
    // reserve list slots: one atomic per counter per block batch
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < kWaveCtrs; q++) wtot[wid][q] = tot[q];
    }
    __syncthreads();
    if (threadIdx.x < kWaveCtrs) {
      const int q = threadIdx.x;
      uint32_t sum = 0;
      for (int w = 0; w < 4; w++) sum += wtot[w][q];
      uint32_t base = 0;
      if (sum) {
        // counts whose positions nobody needs (the active count of SA rounds,
        // which keep flags instead of a list, and the statistics) are added
        // once per workgroup at the end
        if (q < kWaveMaxCi) base = atomicAdd(&B.ctr->cls_cnt[nxt][q], sum);
        else if (q == kWaveMaxCi && !R.aflag) base = atomicAdd(&B.ctr->act_cnt[nxt], sum);
        else deferred += sum;
      }
      for (int w = 0; w < 4; w++) {
        wbase[w][q] = base;
        base += wtot[w][q];
      }
    }
    __syncthreads();
    if (!last_level) {
      uint32_t abase = wbase[wid][kWaveMaxCi];
      uint32_t cbase[kWaveMaxCi];
#pragma unroll
      for (int cc = 0; cc < kWaveMaxCi; cc++) cbase[cc] = wbase[wid][cc];
#pragma unroll
      for (int k = 0; k < kWaveItems; k++) {
        const bool stay = act_p[k] != kNone;
        const uint64_t am = __ballot(stay);
        if (stay) {
          const uint32_t w = abase + (uint32_t)__popcll(am & lanes_lt);
          if (w < B.cap) B.act[nxt][w] = act_p[k];
          else atomicOr(&B.ctr->err, 4u);
        }
        abase += (uint32_t)__popcll(am);
        const int mycc = (int)(unit_code[k] & 0xFF) - 1;
#pragma unroll
        for (int cc = 0; cc < kWaveMaxCi; cc++) {
          const uint64_t m = __ballot(mycc == cc);
          if (mycc == cc) {
            const uint32_t kk = cbase[cc] + (uint32_t)__popcll(m & lanes_lt);
            const uint32_t capc = B.cls_off[cc + 1] - B.cls_off[cc];
            if (kk < capc)
              B.cls[nxt][B.cls_off[cc] + kk] = Unit{unit_pos[k], (unit_code[k] >> 8) | (MODE == MODE_SA ? kHeadBit : 0u)};
            else atomicOr(&B.ctr->err, 8u);
          }
          cbase[cc] += (uint32_t)__popcll(m);
        }
      }
    }
    __syncthreads();  // wtot/wbase are reused by the next batch
  }
  if (threadIdx.x == kWaveMaxCi && deferred) atomicAdd(&B.ctr->act_cnt[nxt], deferred);
  if (threadIdx.x == kWaveMaxCi + 1 && deferred) atomicAdd(&B.ctr->lds_elems, deferred);
}

// ------------------------------------------------- LDS grouping (large units)
// For units of 65..2^TLG entries: count the entries of every distinct
// (unit, key) pair in an LDS hash table, sort only the distinct pairs, turn
// their counts into offsets and drop every entry into its group's range.  Work
// per entry is a few LDS operations plus a share of the distinct-pair sort,
// instead of a full bitonic network; loop-structured streams have few
// distinct keys per group.
constexpr int kGroupMinCi = 6;  // 0-based class 6 = lengths 65..128
constexpr int kGroupThreads = 512;

template <int MODE, int TLG>
__global__ __launch_bounds__(kGroupThreads, TLG == 11 ? 6 : 2) void k_lds_group(SortBufs B, int cur, RankOut R, int last_level,
                                                            uint8_t *keep) {
  constexpr int NT = kGroupThreads;
  constexpr int T = 1 << TLG;
  constexpr int HT = 2 * T;            // hash slots (load <= 1/2)
  constexpr int PER = T / NT;
  constexpr int MAXU = T >> (kGroupMinCi + 1);  // units per tile of the smallest handled class
  __shared__ uint32_t K[T], V[T];
  __shared__ uint16_t EJ[T];           // unit of each entry
  __shared__ uint32_t tab[HT];         // insert: (count << 16) | (entry + 1); after scan: (count << 16) | base
  __shared__ uint64_t D[T];            // distinct (unit, key, slot); after scan: fill cursors (u32[HT])
  __shared__ Unit ud[MAXU];
  __shared__ uint32_t uoff[MAXU + 1];
  __shared__ uint32_t sh[NT / 64];
  __shared__ uint32_t nd, act_base, items_total, item_c, item_b;
  __shared__ uint32_t cls_loc[kClasses], cls_base[kClasses], cnt_c[kClasses];
  uint32_t *cursor = reinterpret_cast<uint32_t *>(D);
  const int nxt = cur ^ 1;
  const int tid = threadIdx.x;
  const int ci_hi = min((int)B.tile_log, TLG);
  if (tid < kClasses) cnt_c[tid] = B.ctr->cls_cnt[cur][tid];
  __syncthreads();
  if (tid == 0) {
    uint32_t tot = 0;
    for (int ci = kGroupMinCi; ci < ci_hi; ci++) {
      const uint32_t per = (uint32_t)T >> (ci + 1);
      tot += (cnt_c[ci] + per - 1) / per;
    }
    items_total = tot;
  }
  __syncthreads();
  const uint32_t total_items = items_total;
  uint32_t elems = 0, act_deferred = 0;
  // items are handed out XCD by XCD: neighbouring tiles hold units of
  // neighbouring windows, whose scattered rank writes then merge in one L2
  for (uint32_t base = 0; base < total_items; base += gridDim.x) {
    const uint32_t item = (uint32_t)xcd_item(base, total_items, blockIdx.x, gridDim.x);
    if (item >= total_items) break;
    if (tid == 0) {
      uint32_t it = item;
      int ci = kGroupMinCi;
      for (; ci < ci_hi; ci++) {
        const uint32_t per = (uint32_t)T >> (ci + 1);
        const uint32_t ni = (cnt_c[ci] + per - 1) / per;
        if (it < ni) break;
        it -= ni;
      }
      item_c = (uint32_t)ci;
      item_b = it;
      nd = 0;
    }
    if (tid < kClasses) cls_loc[tid] = 0;
    for (int h = tid; h < HT; h += NT) tab[h] = 0;
    __syncthreads();
    const int ci = (int)item_c;
    const uint32_t per = (uint32_t)T >> (ci + 1);
    const uint32_t first = item_b * per;
    const uint32_t nb = min(per, cnt_c[ci] - first);
    const Unit *src = B.cls[cur] + B.cls_off[ci] + first;
    // unit descriptors and compact offsets (nb <= MAXU <= NT)
    {
      uint32_t len = 0;
      if (tid < (int)nb) {
        ud[tid] = src[tid];
        len = src[tid].len & kLenMask;
      }
      uint32_t tot;
      const uint32_t ex = block_excl_sum<NT>(len, sh, &tot);
      if (tid < (int)nb) uoff[tid] = ex;
      if (tid == 0) uoff[nb] = tot;
      elems += tot;  // statistics: one atomic per workgroup at the end
    }
    __syncthreads();
    const uint32_t total = uoff[nb];
    // load entries: all of a thread's global loads are issued before the
    // first is waited for
    {
      uint32_t kq[PER], vq[PER], jq[PER];
#pragma unroll
      for (int q = 0; q < PER; q++) {
        const uint32_t p = tid + q * NT;
        jq[q] = 0;
        if (p < total) {
          uint32_t lo = 0, hi = nb;  // unit j: uoff[j] <= p < uoff[j+1]
          while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (uoff[mid] <= p) lo = mid; else hi = mid;
          }
          const Unit u = ud[lo];
          const int b = (u.len & kBufBit) ? 1 : 0;
          const uint32_t g = u.start + (p - uoff[lo]);
          kq[q] = key_buf(B, b)[g];
          vq[q] = val_buf(B, b)[g];
          jq[q] = lo;
        }
      }
#pragma unroll
      for (int q = 0; q < PER; q++) {
        const uint32_t p = tid + q * NT;
        if (p < total) {
          K[p] = kq[q];
          V[p] = vq[q];
          EJ[p] = (uint16_t)jq[q];
        }
      }
    }
    __syncthreads();
    // insert into the hash table
    uint32_t eslot[PER];
    for (int q = 0; q < PER; q++) {
      const uint32_t p = tid + q * NT;
      eslot[q] = 0;
      if (p < total) {
        const uint32_t key = K[p], j = EJ[p];
        uint32_t h = (uint32_t)(mix64(((uint64_t)j << 32) | key) >> 20) & (HT - 1);
        while (true) {
          uint32_t prev = tab[h];
          if (prev == 0u) prev = atomicCAS(&tab[h], 0u, (1u << 16) | (p + 1));
          if (prev == 0u) {
            const uint32_t d = atomicAdd(&nd, 1u);
            D[d] = ((uint64_t)j << 46) | ((uint64_t)key << 14) | h;
            break;
          }
          const uint32_t e = (prev & 0xFFFFu) - 1;
          if (K[e] == key && EJ[e] == j) {
            agg_add(&tab[h], 1u << 16);
            break;
          }
          h = (h + 1) & (HT - 1);
        }
        eslot[q] = h;
      }
    }
    __syncthreads();
    // sort the distinct pairs (bitonic over the next power of two)
    const uint32_t m = nd;
    uint32_t m2 = 1;
    while (m2 < m) m2 <<= 1;
    for (uint32_t i = m + tid; i < m2; i += NT) D[i] = ~0ull;
    __syncthreads();
    for (uint32_t k = 2; k <= m2; k <<= 1) {
      for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
        for (uint32_t t = tid; t < m2 / 2; t += NT) {
          const uint32_t i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
          const uint32_t l = i | jj;
          const bool asc = (i & k) == 0;
          const uint64_t a = D[i], b = D[l];
          if ((a > b) == asc) { D[i] = b; D[l] = a; }
        }
        __syncthreads();
      }
    }
    // offsets: exclusive scan of counts in (unit, key) order
    {
      const uint32_t chunk = (m + NT - 1) / NT;
      const uint32_t d0 = tid * chunk, d1 = min(d0 + chunk, m);
      uint32_t loc = 0;
      for (uint32_t d = d0; d < d1; d++) loc += tab[(uint32_t)D[d] & (HT - 1)] >> 16;
      uint32_t tot;
      uint32_t ex = block_excl_sum<NT>(loc, sh, &tot);
      uint32_t slots[8];
      uint32_t bases[8];
      int nsl = 0;
      for (uint32_t d = d0; d < d1; d++) {
        const uint32_t h = (uint32_t)D[d] & (HT - 1);
        const uint32_t c = tab[h] >> 16;
        if (nsl < 8) { slots[nsl] = h; bases[nsl] = ex; nsl++; }
        else { tab[h] = (c << 16) | ex; }  // only when chunk > 8 (m > 8 * NT): never for T <= 4096
        ex += c;
      }
      __syncthreads();  // every D read done before D is reused as cursors
      for (int z = 0; z < nsl; z++) {
        const uint32_t c = tab[slots[z]] >> 16;
        tab[slots[z]] = (c << 16) | bases[z];
        cursor[slots[z]] = bases[z];
      }
    }
    __syncthreads();
    // place entries and regroup
    uint32_t my_act = 0;
    uint32_t pos_q[PER];
    for (int q = 0; q < PER; q++) {
      const uint32_t p = tid + q * NT;
      pos_q[q] = 0;
      if (p < total) {
        const uint32_t h = eslot[q];
        const uint32_t info = tab[h];
        const uint32_t gbase = info & 0xFFFFu, gcnt = info >> 16;
        const uint32_t pos = agg_inc(&cursor[h]);
        pos_q[q] = pos;
        const uint32_t j = EJ[p];
        const Unit u = ud[j];
        const uint32_t slot = u.start + (pos - uoff[j]);
        const uint32_t head = u.start + (gbase - uoff[j]);
        const uint32_t v = V[p];
        B.val[0][slot] = v;
        if (MODE == MODE_SA) {
          if (!((u.len & kHeadBit) && head == u.start)) R.rank[v] = head + 1;  // else unchanged
          if (R.aflag) R.aflag[slot] = gcnt >= 2 ? 1 : 0;
        }
        if (last_level) {
          keep[slot] = (pos == gbase) ? 1 : 0;
        } else if (gcnt >= 2) {
          my_act++;
          if (pos == gbase) atomicAdd(&cls_loc[class_of(gcnt)], 1u);
        }
      }
    }
    if (!last_level) {
      uint32_t tot;
      const uint32_t off = block_excl_sum<NT>(my_act, sh, &tot);
      if (tid == 0) {
        if (R.aflag) act_deferred += tot;  // SA rounds keep flags: the count only, once per workgroup
        else act_base = tot ? atomicAdd(&B.ctr->act_cnt[nxt], tot) : 0u;
      }
      if (tid < kClasses) {
        const uint32_t mm = cls_loc[tid];
        cls_base[tid] = mm ? atomicAdd(&B.ctr->cls_cnt[nxt][tid], mm) : 0u;
        cls_loc[tid] = 0;
      }
      __syncthreads();
      uint32_t w = act_base + off;
      for (int q = 0; q < PER; q++) {
        const uint32_t p = tid + q * NT;
        if (p >= total) continue;
        const uint32_t info = tab[eslot[q]];
        const uint32_t gbase = info & 0xFFFFu, gcnt = info >> 16;
        if (gcnt < 2) continue;
        const uint32_t j = EJ[p];
        const Unit u = ud[j];
        const uint32_t slot = u.start + (pos_q[q] - uoff[j]);
        if (!R.aflag) {
          if (w < B.cap) B.act[nxt][w] = slot;
          else atomicOr(&B.ctr->err, 4u);
          w++;
        }
        if (pos_q[q] == gbase) {
          const int cc = class_of(gcnt);
          const uint32_t k = cls_base[cc] + atomicAdd(&cls_loc[cc], 1u);
          const uint32_t capc = B.cls_off[cc + 1] - B.cls_off[cc];
          if (k < capc)
            B.cls[nxt][B.cls_off[cc] + k] = Unit{u.start + (gbase - uoff[j]), gcnt | (MODE == MODE_SA ? kHeadBit : 0u)};
          else atomicOr(&B.ctr->err, 8u);
        }
      }
    }
    __syncthreads();
  }
  if (tid == 0 && elems) atomicAdd(&B.ctr->lds_elems, elems);
  if (tid == 0 && act_deferred) atomicAdd(&B.ctr->act_cnt[nxt], act_deferred);
}

// ----------------------------------------------------------- MSD bucketing
__device__ __forceinline__ void digit_params(uint32_t bits, uint32_t dbits, uint32_t &shift, uint32_t &mask) {
  const uint32_t d = bits < dbits ? bits : dbits;
  shift = bits - d;
  mask = (d >= 32) ? 0xFFFFFFFFu : ((1u << d) - 1u);
}

// Digit of a key relative to its unit's base (0 stays 0: past the window end).
__device__ __forceinline__ uint32_t rel_key(uint32_t k, uint32_t base) { return k ? k - base : 0u; }

__global__ __launch_bounds__(256) void k_msd_hist(SortBufs B, int cur, int level, const uint32_t *slot_base) {
  __shared__ uint32_t h[kBins];
  uint32_t units, total;
  list_size(B.ctr->big_pk[cur][level], B.big_cap, units, total);
  const BigUnit *U = B.big[cur][level];
  for (uint32_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
    for (int b = threadIdx.x; b < (1 << B.digit_bits); b += blockDim.x) h[b] = 0;
    __syncthreads();
    const uint32_t u = find_unit(U, units, ch);
    const BigUnit bu = U[u];
    uint32_t shift, mask;
    digit_params(bu.meta & 0xFFu, B.digit_bits, shift, mask);
    const uint32_t lo = bu.start + ((ch - bu.cbase) << B.chunk_log);
    const uint32_t hi = min(lo + (1u << B.chunk_log), bu.start + bu.len);
    const uint32_t *key = key_buf(B, (bu.meta & kMetaAlt) ? 1 : 0);
    const uint32_t base = slot_base ? slot_base[bu.start] : 0u;
    for (uint32_t p = lo + threadIdx.x; p < hi; p += blockDim.x)
      agg_add(&h[(rel_key(key[p], base) >> shift) & mask], 1u);
    __syncthreads();
    uint32_t *gh = B.hist + (size_t)u * kBins;
    for (int b = threadIdx.x; b <= (int)mask; b += blockDim.x)
      if (h[b]) atomicAdd(&gh[b], h[b]);
    __syncthreads();
  }
}

// Destinations of a bucket: LDS class lists (0..kClasses-1), the bulk list,
// the next MSD level.
enum { kDestBulk = kClasses, kDestNext = kClasses + 1, kDests = kClasses + 2 };

__device__ __forceinline__ int dest_of(const SortBufs &B, uint32_t len, uint32_t bits_left, int level) {
  if (len <= (1u << B.tile_log)) return class_of(len);
  if (bits_left == 0 || level + 1 >= kMaxMsdLevels) return kDestBulk;
  return kDestNext;
}

// One workgroup per large unit: exclusive scan of its digit histogram into
// scatter cursors, then every non-empty bucket becomes a piece routed to a
// class list, the bulk list or the next level.  Appends are aggregated per
// workgroup (one global atomic per destination).  A unit whose digit puts
// everything into one bucket is not scattered: it continues in place.
__global__ __launch_bounds__(256) void k_msd_scan(SortBufs B, int cur, int level) {
  constexpr int NT = 256;
  constexpr int PER = kBins / NT;
  __shared__ uint32_t sh[NT / 64];
  __shared__ unsigned long long dl[kDests];  // per destination: (units << 32) | chunks, local
  __shared__ unsigned long long dg[kDests];  // global base of this workgroup's range
  __shared__ int one;
  uint32_t units, total;
  list_size(B.ctr->big_pk[cur][level], B.big_cap, units, total);
  BigUnit *U = B.big[cur][level];
  for (uint32_t u = blockIdx.x; u < units; u += gridDim.x) {
    const BigUnit bu = U[u];
    const uint32_t buf = (bu.meta & kMetaAlt) ? 1u : 0u;
    uint32_t shift, mask;
    digit_params(bu.meta & 0xFFu, B.digit_bits, shift, mask);
    uint32_t *gh = B.hist + (size_t)u * kBins;
    uint32_t *cu = B.cursor + (size_t)u * kBins;
    if (threadIdx.x < kDests) dl[threadIdx.x] = 0;
    if (threadIdx.x == 0) one = 0;
    uint32_t v[PER];
    uint32_t loc = 0;
    for (int q = 0; q < PER; q++) {
      const uint32_t b = threadIdx.x * PER + q;
      v[q] = b <= mask ? gh[b] : 0u;
      loc += v[q];
    }
    uint32_t tot;
    const uint32_t ex0 = block_excl_sum<NT>(loc, sh, &tot);  // (has barriers)
    for (int q = 0; q < PER; q++)
      if (v[q] == bu.len) one = 1;
    __syncthreads();
    const bool single = one != 0;
    // pass 1: local offsets per destination
    unsigned long long lo[PER];
    uint32_t ex = ex0;
    for (int q = 0; q < PER; q++) {
      const uint32_t b = threadIdx.x * PER + q;
      lo[q] = 0;
      if (b <= mask) {
        cu[b] = bu.start + ex;
        gh[b] = 0;
        if (v[q]) {
          const int d = dest_of(B, v[q], shift, level);
          const unsigned long long inc = (d >= kDestBulk) ? ((1ull << 32) | chunks_of(v[q], B.chunk_log)) : (1ull << 32);
          lo[q] = atomicAdd(&dl[d], inc);
        }
      }
      ex += v[q];
    }
    __syncthreads();
    if (threadIdx.x < kDests) {
      const int d = threadIdx.x;
      const unsigned long long m = dl[d];
      unsigned long long g = 0;
      if (m) {
        if (d < kClasses) g = (unsigned long long)atomicAdd(&B.ctr->cls_cnt[cur][d], (uint32_t)(m >> 32)) << 32;
        else if (d == kDestBulk) g = atomicAdd(&B.ctr->bulk_pk, m);
        else g = atomicAdd(&B.ctr->big_pk[cur][level + 1], m);
      }
      dg[d] = g;
    }
    __syncthreads();
    // pass 2: write the pieces
    ex = ex0;
    for (int q = 0; q < PER; q++) {
      const uint32_t b = threadIdx.x * PER + q;
      if (b <= mask && v[q]) {
        const uint32_t pstart = single ? bu.start : bu.start + ex;
        const uint32_t pbuf = single ? buf : buf ^ 1u;
        const int d = dest_of(B, v[q], shift, level);
        const uint32_t k = (uint32_t)(dg[d] >> 32) + (uint32_t)(lo[q] >> 32);
        const uint32_t cb = (uint32_t)dg[d] + (uint32_t)lo[q];
        if (d < kClasses) {
          const uint32_t capc = B.cls_off[d + 1] - B.cls_off[d];
          if (k < capc) B.cls[cur][B.cls_off[d] + k] = Unit{pstart, v[q] | (pbuf ? kBufBit : 0u)};
          else atomicOr(&B.ctr->err, 16u);
        } else if (k < B.big_cap) {
          BigUnit *L = (d == kDestBulk) ? B.bulk : B.big[cur][level + 1];
          L[k] = BigUnit{pstart, v[q], cb, shift | (pbuf ? kMetaAlt : 0u)};
        } else {
          atomicOr(&B.ctr->err, 32u);
        }
      }
      ex += v[q];
    }
    if (threadIdx.x == 0 && single) U[u].meta = bu.meta | kMetaSkip;
    __syncthreads();
  }
}

template <int CL>
__global__ __launch_bounds__(256) void k_msd_scatter(SortBufs B, int cur, int level, const uint32_t *slot_base) {
  constexpr int NT = 256;
  constexpr int PER = (1 << CL) / NT;
  __shared__ uint32_t cnt[kBins];
  uint32_t units, total;
  list_size(B.ctr->big_pk[cur][level], B.big_cap, units, total);
  const BigUnit *U = B.big[cur][level];
  for (uint32_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
    const uint32_t u = find_unit(U, units, ch);
    const BigUnit bu = U[u];
    if (bu.meta & kMetaSkip) continue;  // uniform across the block
    for (int b = threadIdx.x; b < (1 << B.digit_bits); b += NT) cnt[b] = 0;
    __syncthreads();
    uint32_t shift, mask;
    digit_params(bu.meta & 0xFFu, B.digit_bits, shift, mask);
    const uint32_t lo = bu.start + ((ch - bu.cbase) << CL);
    const uint32_t hi = min(lo + (1u << CL), bu.start + bu.len);
    const int sb = (bu.meta & kMetaAlt) ? 1 : 0, db = sb ^ 1;
    const uint32_t base = slot_base ? slot_base[bu.start] : 0u;
    uint32_t kk[PER], vv[PER], oo[PER];
    for (int q = 0; q < PER; q++) {
      const uint32_t p = lo + threadIdx.x + q * NT;
      if (p < hi) {
        kk[q] = key_buf(B, sb)[p];
        vv[q] = val_buf(B, sb)[p];
        oo[q] = agg_inc(&cnt[(rel_key(kk[q], base) >> shift) & mask]);
      }
    }
    __syncthreads();
    uint32_t *cu = B.cursor + (size_t)u * kBins;
    for (int b = threadIdx.x; b <= (int)mask; b += NT) {
      const uint32_t m = cnt[b];
      cnt[b] = m ? atomicAdd(&cu[b], m) : 0u;
    }
    __syncthreads();
    for (int q = 0; q < PER; q++) {
      const uint32_t p = lo + threadIdx.x + q * NT;
      if (p < hi) {
        const uint32_t dst = cnt[(rel_key(kk[q], base) >> shift) & mask] + oo[q];
        key_buf(B, db)[dst] = kk[q];
        val_buf(B, db)[dst] = vv[q];
      }
    }
    __syncthreads();
  }
}

// --------------------------------------------------- bulk (one-group) units
// Pieces whose key bits are used up are one group each.  Processed chunk by
// chunk: SA-mode ranks and grouped-slot flags, copy-back from the
// alternate buffer, the next level's active slots (plain mode), and (by the
// unit's first chunk) the unit itself as a large unit of the next level.
template <int MODE, int CL>
__global__ __launch_bounds__(256) void k_bulk(SortBufs B, int cur, RankOut R, uint32_t next_bits,
                                              int last_level, uint8_t *keep) {
  constexpr int NT = 256;
  constexpr int PER = (1 << CL) / NT;
  __shared__ uint32_t sh[NT / 64];
  __shared__ uint32_t base;
  const int nxt = cur ^ 1;
  uint32_t units, total;
  list_size(B.ctr->bulk_pk, B.big_cap, units, total);
  for (uint32_t ch = blockIdx.x; ch < total; ch += gridDim.x) {
    const uint32_t u = find_unit(B.bulk, units, ch);
    const BigUnit bu = B.bulk[u];
    const bool alt = (bu.meta & kMetaAlt) != 0;
    const uint32_t lo = bu.start + ((ch - bu.cbase) << CL);
    const uint32_t hi = min(lo + (1u << CL), bu.start + bu.len);
    if (threadIdx.x == 0 && !last_level && ch == bu.cbase)
      append_big(B.big[nxt][0], &B.ctr->big_pk[nxt][0], B.big_cap, bu.start, bu.len, next_bits, &B.ctr->err,
                 CL);
    for (int q = 0; q < PER; q++) {
      const uint32_t p = lo + threadIdx.x + q * NT;
      if (p < hi) {
        const uint32_t v = val_buf(B, alt ? 1 : 0)[p];
        if (alt) B.val[0][p] = v;
        if (MODE == MODE_SA) {
          R.rank[v] = bu.start + 1;
          if (R.aflag) R.aflag[p] = 1;
        }
        if (last_level) keep[p] = (p == bu.start) ? 1 : 0;
      }
    }
    if (!last_level) {
      const uint32_t cnt = hi - lo;
      if (threadIdx.x == 0) base = atomicAdd(&B.ctr->act_cnt[nxt], cnt);
      __syncthreads();
      for (uint32_t e = threadIdx.x; e < cnt && !R.aflag; e += NT) {
        const uint32_t w = base + e;
        if (w < B.cap) B.act[nxt][w] = lo + e;
        else atomicOr(&B.ctr->err, 256u);
      }
      __syncthreads();
    }
  }
  (void)sh;
}

// =================================================================== host
static inline dim3 grid_for(uint64_t n, int threads, int cap_blocks) {
  uint64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > (uint64_t)cap_blocks) b = cap_blocks;
  return dim3((unsigned)b);
}

size_t SortEngine::bytes_for(uint64_t capacity) {
  SortEngine probe;
  size_t b = 0;
  probe.alloc(capacity, &b);
  return b;
}

int SortEngine::alloc(uint64_t capacity, size_t *dry_bytes, void *ext) {
  cap_ = capacity;
  SortBufs &B = b_;
  B.cap = capacity;
  // class regions: class c (1-based) holds at most cap >> (c-1) units (+1 slack)
  uint32_t off = 0;
  for (int ci = 0; ci < kClasses; ci++) {
    B.cls_off[ci] = off;
    off += (uint32_t)((capacity >> ci) + 1);
  }
  B.cls_off[kClasses] = off;
  B.big_cap = (uint32_t)(capacity / (1u << kMinTileLog) + 64);
  B.tile_log = kDefaultTileLog;
  B.digit_bits = kDefaultDigitBits;
  B.chunk_log = kChunkLogLarge;
  size_t bytes = 0;
  auto take = [&](size_t n) { size_t o = bytes; bytes += (n + 255) & ~(size_t)255; return o; };
  size_t o_key0 = take(capacity * 4), o_key1 = take(capacity * 4);
  size_t o_val0 = take(capacity * 4), o_val1 = take(capacity * 4);
  size_t o_cls0 = take((size_t)off * sizeof(Unit)), o_cls1 = take((size_t)off * sizeof(Unit));
  size_t o_big[2][kMsdLists];
  for (int l = 0; l < 2; l++)
    for (int v = 0; v < kMsdLists; v++) o_big[l][v] = take((size_t)B.big_cap * sizeof(BigUnit));
  size_t o_bulk = take((size_t)B.big_cap * sizeof(BigUnit));
  size_t o_hist = take((size_t)B.big_cap * kBins * 4);
  size_t o_cur = take((size_t)B.big_cap * kBins * 4);
  size_t o_act0 = take(capacity * 4), o_act1 = take(capacity * 4);
  size_t o_ctr = take(sizeof(SortCounters));
  if (dry_bytes) {  // size only
    *dry_bytes = bytes;
    return 0;
  }
  if (ext) {
    mem_ = ext;
    external_ = true;
  } else {
    APO_HIP_TRY(hipMalloc(&mem_, bytes));
    external_ = false;
  }
  bytes_ = bytes;
  char *m = static_cast<char *>(mem_);
  B.key[0] = (uint32_t *)(m + o_key0); B.key[1] = (uint32_t *)(m + o_key1);
  B.val[0] = (uint32_t *)(m + o_val0); B.val[1] = (uint32_t *)(m + o_val1);
  B.cls[0] = (Unit *)(m + o_cls0); B.cls[1] = (Unit *)(m + o_cls1);
  for (int l = 0; l < 2; l++)
    for (int v = 0; v < kMsdLists; v++) B.big[l][v] = (BigUnit *)(m + o_big[l][v]);
  B.bulk = (BigUnit *)(m + o_bulk);
  B.hist = (uint32_t *)(m + o_hist);
  B.cursor = (uint32_t *)(m + o_cur);
  B.act[0] = (uint32_t *)(m + o_act0); B.act[1] = (uint32_t *)(m + o_act1);
  B.ctr = (SortCounters *)(m + o_ctr);
  APO_HIP_TRY(hipMemset(B.hist, 0, (size_t)B.big_cap * kBins * 4));
  APO_HIP_TRY(hipMemset(B.ctr, 0, sizeof(SortCounters)));
  return 0;
}

void SortEngine::release() {
  if (mem_ && !external_) (void)hipFree(mem_);
  mem_ = nullptr;
  external_ = false;
}

void SortEngine::reset_counters(hipStream_t s) {
  hipLaunchKernelGGL(k_counters_reset, dim3(1), dim3(64), 0, s, b_.ctr);
}

void SortEngine::round_begin(int cur, hipStream_t s) {
  hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(64), 0, s, b_.ctr, cur);
}

void SortEngine::round_end(int cur, int r, uint32_t *hist, hipStream_t s) {
  hipLaunchKernelGGL(k_round_end, dim3(1), dim3(64), 0, s, b_.ctr, cur, r, hist);
}

void SortEngine::init_units(int cur, const uint64_t *d_off, uint32_t nranges, uint32_t base,
                            uint32_t key_bits, hipStream_t s, const uint8_t *only) {
  hipLaunchKernelGGL(k_init_units, grid_for(nranges, 256, 1 << 16), dim3(256), 0, s, b_, cur, d_off,
                     nranges, base, key_bits, only);
}

void SortEngine::init_runs(int cur, const uint32_t *run_start, const uint32_t *nruns_dev, const uint32_t *total_dev,
                           uint64_t bound, uint32_t key_bits, hipStream_t s) {
  hipLaunchKernelGGL(k_init_runs, grid_for((bound + kRunItems - 1) / kRunItems, 256, 8192), dim3(256), 0, s, b_, cur,
                     run_start, nruns_dev, total_dev, key_bits);
}

void SortEngine::gather_identity(const uint32_t *src, uint32_t n, hipStream_t s, const uint32_t *wid,
                                 const uint8_t *only, const uint32_t *gate) {
  hipLaunchKernelGGL(k_gather_identity, grid_for(n, 256, 4096), dim3(256), 0, s, b_, src, n, wid, only, gate);
}

void SortEngine::gather_sa(int cur, const uint32_t *rank, const uint8_t *aflag, const uint32_t *slot_wend,
                           uint32_t n, uint32_t h, uint32_t *hist, int r, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_sa, dim3(4096), dim3(256), 0, s, b_, cur, rank, aflag, slot_wend, n, h, hist, r);
}

void SortEngine::gather_field(int cur, const uint32_t *field, int stride, const uint32_t *all_dev, int sub,
                              const uint32_t *c_dev, uint32_t c, uint64_t bound, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_field, grid_for((bound + 3) / 4, 256, 4096), dim3(256), 0, s, b_, cur, field, stride,
                     all_dev, sub, c_dev, c);
}

void SortEngine::iota_val(const uint32_t *n_dev, uint64_t bound, hipStream_t s) {
  hipLaunchKernelGGL(k_iota_val, grid_for(bound, 256, 4096), dim3(256), 0, s, b_, n_dev);
}

void SortEngine::msd(int cur, uint64_t work_hint, int max_bits, hipStream_t s, const uint32_t *slot_base) {
  const unsigned g = (unsigned)std::min<uint64_t>(4096, std::max<uint64_t>(256, (work_hint >> b_.chunk_log) + 1));
  const int levels = std::min(kMaxMsdLevels, (max_bits + (int)b_.digit_bits - 1) / (int)b_.digit_bits);
  for (int level = 0; level < levels; level++) {
    hipLaunchKernelGGL(k_msd_hist, dim3(g), dim3(256), 0, s, b_, cur, level, slot_base);
    hipLaunchKernelGGL(k_msd_scan, dim3(256), dim3(256), 0, s, b_, cur, level);
    if (b_.chunk_log == kChunkLogSmall)
      hipLaunchKernelGGL(k_msd_scatter<kChunkLogSmall>, dim3(g), dim3(256), 0, s, b_, cur, level, slot_base);
    else
      hipLaunchKernelGGL(k_msd_scatter<kChunkLogLarge>, dim3(g), dim3(256), 0, s, b_, cur, level, slot_base);
  }
}

template <int MODE>
static void launch_lds(const SortBufs &b, int cur, RankOut R, uint32_t next_bits, int last_level, uint8_t *keep,
                       uint64_t work_hint, hipStream_t s) {
  const uint64_t tile = 1ull << b.tile_log;
  const unsigned g = (unsigned)std::min<uint64_t>(2048, std::max<uint64_t>(64, 2 * work_hint / tile + 16));
  const int tl = (int)b.tile_log;
  // classes below kGroupMinCi: wavefront sort; kGroupMinCi..min(tl,12)-1:
  // hash grouping; class 13 (tile 2^13 only): LDS bitonic
  const int grp_hi = std::min(tl, 12);
  // units of <= 64 entries: one wavefront each row
  const unsigned gw = (unsigned)std::min<uint64_t>(4096, std::max<uint64_t>(64, work_hint / 256 + 1));
  hipLaunchKernelGGL(k_wave_sort<MODE>, dim3(gw), dim3(256), 0, s, b, cur, R, last_level, keep);
  if (tl == 13)
    hipLaunchKernelGGL((k_lds_sort<MODE, 13>), dim3(g), dim3(kLdsThreads), 0, s, b, cur, R, next_bits, last_level,
                       keep, 12, 13);
  if (grp_hi > kGroupMinCi) {
    if (tl == 11)
      hipLaunchKernelGGL((k_lds_group<MODE, 11>), dim3(g), dim3(kGroupThreads), 0, s, b, cur, R, last_level, keep);
    else
      hipLaunchKernelGGL((k_lds_group<MODE, 12>), dim3(g), dim3(kGroupThreads), 0, s, b, cur, R, last_level, keep);
  }
}

void SortEngine::set_params(int tile_log, int digit_bits) {
  b_.tile_log = (uint32_t)std::min(std::max(tile_log, kMinTileLog), kMaxTileLog);
  b_.digit_bits = (uint32_t)std::min(std::max(digit_bits, kMinDigitBits), kMaxDigitBits);
}

// On small analyses the large units hold few chunks, and 2^13-entry chunks
// left most CUs idle in the MSD passes (n = 2^20: 3.0 -> 2.7 ms per window
// with 2^12); on large ones the bigger chunks save per-chunk histogram work.
void SortEngine::set_chunk_for(uint64_t n) {
  b_.chunk_log = n <= kSmallChunkMaxN ? (uint32_t)kChunkLogSmall : (uint32_t)kChunkLogLarge;
}

void SortEngine::lds_sa(int cur, RankOut R, uint32_t next_bits, uint64_t work_hint, hipStream_t s) {
  launch_lds<MODE_SA>(b_, cur, R, next_bits, 0, nullptr, work_hint, s);
}

void SortEngine::lds_plain(int cur, uint32_t next_bits, int last_level, uint8_t *keep,
                           uint64_t work_hint, hipStream_t s) {
  RankOut R{};
  launch_lds<MODE_PLAIN>(b_, cur, R, next_bits, last_level, keep, work_hint, s);
}

void SortEngine::bulk_sa(int cur, RankOut R, uint32_t next_bits, uint64_t work_hint, hipStream_t s) {
  const unsigned g = (unsigned)std::min<uint64_t>(2048, std::max<uint64_t>(64, (work_hint >> b_.chunk_log) + 1));
  if (b_.chunk_log == kChunkLogSmall)
    hipLaunchKernelGGL((k_bulk<MODE_SA, kChunkLogSmall>), dim3(g), dim3(256), 0, s, b_, cur, R, next_bits, 0,
                       (uint8_t *)nullptr);
  else
    hipLaunchKernelGGL((k_bulk<MODE_SA, kChunkLogLarge>), dim3(g), dim3(256), 0, s, b_, cur, R, next_bits, 0,
                       (uint8_t *)nullptr);
}

void SortEngine::bulk_plain(int cur, uint32_t next_bits, int last_level, uint8_t *keep,
                            uint64_t work_hint, hipStream_t s) {
  RankOut R{};
  const unsigned g = (unsigned)std::min<uint64_t>(2048, std::max<uint64_t>(64, (work_hint >> b_.chunk_log) + 1));
  if (b_.chunk_log == kChunkLogSmall)
    hipLaunchKernelGGL((k_bulk<MODE_PLAIN, kChunkLogSmall>), dim3(g), dim3(256), 0, s, b_, cur, R, next_bits,
                       last_level, keep);
  else
    hipLaunchKernelGGL((k_bulk<MODE_PLAIN, kChunkLogLarge>), dim3(g), dim3(256), 0, s, b_, cur, R, next_bits,
                       last_level, keep);
}

}  // namespace apo
