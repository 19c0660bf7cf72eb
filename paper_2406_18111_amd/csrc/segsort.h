// Host interface of the segmented refine-sort engine (see segsort.hip).
#pragma once
#include "apo_internal.h"

namespace apo {

class SortEngine {
 public:
  // dry_bytes != nullptr: only computes the device bytes alloc would take;
  // ext != nullptr: lays the buffers out in that caller-owned device memory
  // (256-byte aligned, at least bytes_for(capacity)) instead of allocating
  int alloc(uint64_t capacity, size_t *dry_bytes = nullptr, void *ext = nullptr);
  static size_t bytes_for(uint64_t capacity);
  void release();
  SortBufs &bufs() { return b_; }
  uint64_t capacity() const { return cap_; }
  size_t bytes() const { return bytes_; }

  void reset_counters(hipStream_t s);
  void set_params(int tile_log, int digit_bits);
  // chunk size of the MSD and bulk passes for an analysis of n tokens
  void set_chunk_for(uint64_t n);
  int tile_log() const { return (int)b_.tile_log; }
  int digit_bits() const { return (int)b_.digit_bits; }
  void round_begin(int cur, hipStream_t s);
  void round_end(int cur, int r, uint32_t *hist, hipStream_t s);
  // only (nullable): just the ranges w with only[w] != 0
  void init_units(int cur, const uint64_t *d_off, uint32_t nranges, uint32_t base, uint32_t key_bits,
                  hipStream_t s, const uint8_t *only = nullptr);
  // units from runs: run r is [run_start[r], run_start[r+1]) (the last ends at
  // *total_dev); bound: host upper bound of the run count
  void init_runs(int cur, const uint32_t *run_start, const uint32_t *nruns_dev, const uint32_t *total_dev,
                 uint64_t bound, uint32_t key_bits, hipStream_t s);
  // only (nullable): just the slots p with only[wid[p]] != 0, and nothing unless *gate > 0 (gate nullable)
  void gather_identity(const uint32_t *src, uint32_t n, hipStream_t s, const uint32_t *wid = nullptr,
                       const uint8_t *only = nullptr, const uint32_t *gate = nullptr);
  void gather_sa(int cur, const uint32_t *rank, const uint8_t *aflag, const uint32_t *slot_wend, uint32_t n,
                 uint32_t h, uint32_t *hist, int r, hipStream_t s);
  void gather_field(int cur, const uint32_t *field, int stride, const uint32_t *all_dev, int sub,
                    const uint32_t *c_dev, uint32_t c, uint64_t bound, hipStream_t s);
  void iota_val(const uint32_t *n_dev, uint64_t bound, hipStream_t s);
  // slot_base (nullable): digits come from key - slot_base[unit start] (key 0
  // stays 0), so keys that are ranks inside a window need only the window's
  // bits; max_bits counts those bits.
  void msd(int cur, uint64_t work_hint, int max_bits, hipStream_t s, const uint32_t *slot_base = nullptr);
  void lds_sa(int cur, RankOut R, uint32_t next_bits, uint64_t work_hint, hipStream_t s);
  void lds_plain(int cur, uint32_t next_bits, int last_level, uint8_t *keep, uint64_t work_hint,
                 hipStream_t s);
  void bulk_sa(int cur, RankOut R, uint32_t next_bits, uint64_t work_hint, hipStream_t s);
  void bulk_plain(int cur, uint32_t next_bits, int last_level, uint8_t *keep, uint64_t work_hint,
                  hipStream_t s);

 private:
  SortBufs b_{};
  void *mem_ = nullptr;
  bool external_ = false;
  size_t bytes_ = 0;
  uint64_t cap_ = 0;
};

}  // namespace apo
