// Internal declarations shared by the HIP translation units of libapo.
// Not part of the public C ABI (see include/apo.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace apo {

// ---------------------------------------------------------------- tuning
constexpr int kLdsTileLog = 12;             // LDS sort tile: 4096 64-bit entries (32 KB)
constexpr int kLdsTile = 1 << kLdsTileLog;
constexpr int kClasses = kLdsTileLog;       // size class c holds units of length (2^(c-1), 2^c]
constexpr int kLdsThreads = 256;
constexpr int kDigitBits = 11;              // MSD bucket pass digit width
constexpr int kBins = 1 << kDigitBits;
constexpr int kChunk = 8192;                // elements per workgroup in MSD passes
constexpr int kMaxRounds = 32;              // doubling rounds (n <= 2^26 needs <= 28)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kBufBit = 0x80000000u;   // unit data lives in the alternate buffer

// Unit descriptor for the LDS sort: a contiguous slot range sorted by key.
struct Unit {
  uint32_t start;
  uint32_t len;     // low 31 bits length, top bit = alternate buffer
};

// Large unit for MSD bucketing passes.
struct BigUnit {
  uint32_t start;
  uint32_t len;
  uint32_t bits;    // key bits still unsorted (from the top)
  uint32_t flags;   // bit0: data in alternate buffer, bit1: skip scatter (single bucket)
};

// Device-side counters of one segmented-sort level/round.  Lives in device
// memory; the host reads it back between rounds.
struct SortCounters {
  uint32_t cls_cnt[2][kClasses];  // per class unit counts, [list][class]
  uint32_t big_cnt[2][4];         // large units: [list][level]  (level 0 = from previous round)
  uint32_t bulk_cnt;              // units with all key bits consumed (single group)
  uint32_t act_cnt[2];            // active slot list lengths
  uint32_t chunk_total[4];        // chunks per MSD level
  uint32_t err;                   // nonzero: capacity overflow detected on device
  uint32_t lds_elems;             // entries sorted by the LDS path this round
  uint32_t pad[2];
};

// Pointers of one segmented-sort "engine" (arrays of capacity cap elements).
struct SortBufs {
  uint32_t *key[2];     // [0] main, [1] alternate
  uint32_t *val[2];
  Unit *cls[2];         // class lists, [list] each with per-class regions
  uint32_t cls_off[kClasses + 1];   // region offsets (in units) within one list
  BigUnit *big[2][4];   // [list][level]
  uint32_t big_cap;
  BigUnit *bulk;
  uint32_t *hist;       // big_cap * kBins
  uint32_t *cursor;     // big_cap * kBins
  uint32_t *chunk_base; // big_cap + 1
  uint32_t *act[2];
  SortCounters *ctr;
  uint64_t cap;
};

// Regroup side effects for suffix-array rounds.
struct RankOut {
  uint32_t *rank;       // rank[pos] = 1 + SA slot of the first suffix of its group
  uint32_t *snap;       // snapshot of this round: snap[pos]
  uint8_t *fin;         // round in which the suffix became a singleton
  uint32_t round;
};

inline int ceil_log2_u64(uint64_t x) {
  int b = 0;
  while ((1ull << b) < x) b++;
  return b;
}

inline int bit_length_u64(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b)) b++;
  return b;
}

}  // namespace apo

#define APO_HIP_TRY(expr)                                      \
  do {                                                         \
    hipError_t _e = (expr);                                    \
    if (_e != hipSuccess) return ::apo::hip_fail(_e, #expr, __FILE__, __LINE__); \
  } while (0)

namespace apo {
int hip_fail(hipError_t e, const char *what, const char *file, int line);
}
