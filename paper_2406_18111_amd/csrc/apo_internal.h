// Internal declarations shared by the HIP translation units of libapo.
// Not part of the public C ABI (see include/apo.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace apo {

// ---------------------------------------------------------------- tuning
// The LDS sort tile (2^tile_log 64-bit entries) and the MSD digit width are
// chosen per run (defaults below, or the autotuner's table).
constexpr int kMinTileLog = 11, kMaxTileLog = 13, kDefaultTileLog = 11;
constexpr int kClasses = kMaxTileLog;       // size class c holds units of length (2^(c-1), 2^c]
constexpr int kLdsThreads = 256;
// Doubling rounds from this one on keep a rank snapshot for the LCP stage;
// shorter prefixes are compared token by token there.
constexpr int kSnapFrom = 4;
constexpr int kMinDigitBits = 8, kMaxDigitBits = 12, kDefaultDigitBits = 11;
constexpr int kBins = 1 << kMaxDigitBits;   // histogram stride per large unit
constexpr int kMaxMsdLevels = 4;            // 32-bit keys / 8-bit digits
constexpr int kMsdLists = kMaxMsdLevels + 1;
// Entries per workgroup in the MSD and bulk passes: 2^12 for analyses of up to
// 2^22 tokens (more workgroups than CUs on small inputs), 2^13 above.
constexpr int kChunkLogSmall = 12, kChunkLogLarge = 13;
constexpr uint64_t kSmallChunkMaxN = 1ull << 22;
constexpr int kMaxRounds = 32;              // doubling rounds (n <= 2^26 needs <= 28)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kBufBit = 0x80000000u;   // unit data lives in the alternate buffer
constexpr uint32_t kHeadBit = 0x40000000u;  // SA rounds: every entry's rank is already unit.start + 1
constexpr uint32_t kLenMask = 0x3FFFFFFFu;  // unit length without the flags

// Unit descriptor for the LDS sort: a contiguous slot range sorted by key.
struct Unit {
  uint32_t start;
  uint32_t len;     // low 31 bits length, top bit = alternate buffer
};

// Large unit for MSD bucketing passes.  Units of one list are appended with a
// packed (units << 32 | chunks) atomic, so chunk bases grow with the unit
// index and a chunk finds its unit by binary search.
struct BigUnit {
  uint32_t start;
  uint32_t len;
  uint32_t cbase;   // index of the unit's first chunk (2^chunk_log entries) in its list
  uint32_t meta;    // bits 0-7: key bits still unsorted (from the top);
                    // bit 8: data in the alternate buffer; bit 9: skip scatter
};
constexpr uint32_t kMetaAlt = 1u << 8, kMetaSkip = 1u << 9;

// Device-side counters of one segmented-sort level/round.  Lives in device
// memory; the host reads it back between rounds.
struct SortCounters {
  unsigned long long big_pk[2][kMsdLists];  // large units [list][level]: (units << 32) | chunks
  unsigned long long bulk_pk;       // single-group units of this round, packed likewise
  uint32_t cls_cnt[2][kClasses];    // per class unit counts, [list][class]
  uint32_t act_cnt[2];              // active slot list lengths
  uint32_t err;                     // nonzero: capacity overflow detected on device
  uint32_t lds_elems;               // entries sorted by the LDS path this round
};

// Pointers of one segmented-sort "engine" (arrays of capacity cap elements).
struct SortBufs {
  uint32_t *key[2];     // [0] main, [1] alternate
  uint32_t *val[2];
  Unit *cls[2];         // class lists, [list] each with per-class regions
  uint32_t cls_off[kClasses + 1];   // region offsets (in units) within one list
  BigUnit *big[2][kMsdLists];   // [list][level]
  uint32_t big_cap;
  BigUnit *bulk;
  uint32_t tile_log;    // LDS tile = 2^tile_log entries
  uint32_t digit_bits;  // MSD digit width
  uint32_t chunk_log;   // MSD / bulk chunk = 2^chunk_log entries
  uint32_t *hist;       // big_cap * kBins
  uint32_t *cursor;     // big_cap * kBins
  uint32_t *act[2];     // plain mode: slots still grouped after a level (SA rounds use RankOut::aflag)
  SortCounters *ctr;
  uint64_t cap;
};

// Regroup side effects for suffix-array rounds.
struct RankOut {
  uint32_t *rank;       // rank[pos] = 1 + SA slot of the first suffix of its group
  uint32_t round;
  uint8_t *aflag;       // aflag[slot] = 1 if the slot's suffix is still grouped (replaces the active list)
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
