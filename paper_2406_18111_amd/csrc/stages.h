// Host launch wrappers of the stage kernels (stages.hip).  Counts that are
// produced on the device are passed as device pointers (`*_dev`) together
// with a host upper bound that only sizes the grid.
#pragma once
#include "apo_internal.h"

namespace apo {

constexpr int kMinFan = 16;    // LCP minimum hierarchy: each level holds minima of kMinFan entries below
constexpr int kMinLevels = 8;  // levels 0..7: a top level of at most 16 entries for up to 2^32 positions

void fill_u32(uint32_t *p, uint64_t n, uint32_t v, hipStream_t s);
void fill_u8(uint8_t *p, uint64_t n, uint8_t v, hipStream_t s);
void fill_u8_dev(uint8_t *p, const uint32_t *n_dev, uint64_t bound, uint8_t v, hipStream_t s);
void copy_u32(uint32_t *dst, const uint32_t *src, hipStream_t s);
void copy_n_u32(uint32_t *dst, const uint32_t *src, uint64_t n, hipStream_t s);
void scan_excl(const uint32_t *in, uint32_t *out, const uint32_t *n_dev, uint64_t bound, uint32_t *tile_tmp,
               uint32_t *total, hipStream_t s);

// Table of hc = mask + 1 slots plus one (the token value equal to the empty
// mark has slot mask + 1); hash_clear empties it.
void hash_clear(uint64_t *tab, uint64_t mask, hipStream_t s, const uint32_t *gate = nullptr);
// tok_slot[i] receives the table slot of token i.  With wflag set, only the
// tokens of windows flagged there (window of token i: wid[i]) are inserted
// and get a slot; with gate set, nothing runs unless *gate > 0.
void hash_insert(const uint64_t *tok, uint64_t n, uint64_t *tab, uint64_t mask, uint32_t *dist_idx,
                 uint32_t *dist_slot, uint32_t *nd, uint32_t *tok_slot, hipStream_t s, const uint32_t *wid = nullptr,
                 const uint8_t *wflag = nullptr, const uint32_t *gate = nullptr);
void hash_fields(const uint64_t *tok, const uint32_t *dist_idx, const uint32_t *nd, uint32_t *hi,
                 uint32_t *lo, uint64_t hint, hipStream_t s);
void hash_assign(const uint32_t *sorted_d, const uint32_t *nd, const uint32_t *dist_slot,
                 uint32_t *slot_rank, uint64_t hint, hipStream_t s);
// out[i] = slot_rank[tok_slot[i]] (out may be tok_slot), for the tokens of
// flagged windows only when wflag is set; nothing unless *gate > 0 when set.
void hash_rank(const uint32_t *tok_slot, uint64_t n, const uint32_t *slot_rank, uint32_t *out, hipStream_t s,
               const uint32_t *wid = nullptr, const uint8_t *wflag = nullptr, const uint32_t *gate = nullptr);
// Per-window ranks of a batch (offsets global, ascending): rank[i] = 1 +
// the number of distinct values of i's window below tok[i]; windows with more
// than 4096 distinct values get wflag = 1 and no ranks (else wflag = 0).
// cnt[0] += distinct values per ranked window, cnt[1] = their maximum,
// cnt[2] += 1 per flagged window, cnt[3]: the windows' work counter (all four
// zeroed by the caller).  Windows are taken in the order order[0..nw) (a
// permutation, or null for 0..nw-1; the same for win_pair and win_round0).
void win_rank(const uint64_t *tok, const uint64_t *off, const uint32_t *order, uint32_t nw, uint32_t *rank,
              uint8_t *wflag, uint32_t *cnt, hipStream_t s);
// Per-window ranks of adjacent token pairs: prank[i] = 1 + the number of
// distinct pairs of i's window below (tokrank[i], tokrank[i+1] or 0 past the
// window's end).  A window with wflag set or more than 8192 distinct pairs is
// skipped and counted in cnt[1]; cnt[0]: the windows' work counter (both
// zeroed by the caller).  *act1 += suffixes whose first token occurs twice or
// more in their window (the first round's active count).  With *wcount (the
// windows without ranks of their own) not zero it only counts cnt[1].
void win_pair(const uint64_t *off, const uint32_t *order, uint32_t nw, const uint8_t *wflag, const uint32_t *tokrank,
              uint32_t *prank, uint32_t *cnt, uint32_t *act1, const uint32_t *wcount, hipStream_t s);
// First doubling round of the suffix sort for the windows ranked on their
// own (wflag[w] == 0): suffixes grouped by first token (keyrank = token
// ranks), or with pairs set by first two tokens (keyrank = pair ranks, every
// window unflagged by win_pair), in val[0], ranks (1 + group start slot),
// grouped-slot flags and the groups of two or more as units of the engine's
// list 1, or list 0 for pairs (counters and lists of that list cleared
// before; large units get next_bits key bits).  *wnext: zeroed work counter.
// With pflag set (sync-free runs, both forms launched) the pair form runs
// only when *pflag == 0 and the first-token form only when it is not.  The
// pair form writes *hist0 = *a1 (the first round's active count).
void win_round0(const SortBufs &B, const uint64_t *off, const uint32_t *order, uint32_t nw, const uint8_t *wflag,
                const uint32_t *keyrank, uint32_t *rank, uint8_t *aflag, uint32_t next_bits, uint32_t *wnext, bool pairs,
                const uint32_t *pflag, const uint32_t *a1, uint32_t *hist0, hipStream_t s);
void window_bounds(const uint64_t *off, uint32_t nw, uint32_t *wbeg, uint32_t *wend, uint32_t *wid,
                   hipStream_t s);

// Copy of the rank array after doubling round r into its snapshot level,
// taken only when the round sorted something (*act_dev: slots that entered
// it); *snaps then becomes r + 1.
void snapshot_ranks(const uint32_t *rank, uint32_t *snap_r, uint64_t n, const uint32_t *act_dev, uint32_t *snaps,
                    int r, hipStream_t s);
// LCP of adjacent suffixes.  rank: final ranks of the suffix sort (1 + slot);
// snap: level j at snap + j * n for kSnapFrom <= j < *snaps (and j <= top).
void build_lcp(const uint32_t *sa, const uint32_t *rank, uint64_t n, const uint32_t *wbeg, const uint32_t *wend,
               const uint32_t *snap, const uint32_t *snaps, const uint32_t *key0, int top, uint32_t *lcp,
               hipStream_t s);

// Candidates are written as records of kCandWords words: length, start, ID.
// *cnt counts the records written; a candidate that exactly repeats one of
// the previous pair (both pairs in the disjoint branch with equal LCP: same
// length, same start SA[i], same ID) is not written and counts in *skipped.
constexpr int kCandWords = 3;
void gen_candidates(const uint32_t *sa, const uint32_t *lcp, uint64_t n, const uint32_t *wend,
                    uint32_t min_len, uint32_t *const *levels, int nlev, uint32_t *crec, uint32_t *cnt,
                    uint32_t *skipped, uint32_t *maxl, uint32_t *tile_val, uint32_t *ntiles_dev,
                    uint32_t *tile_tmp, hipStream_t s);

// Stable sort of the candidate records by length, longest first (records in
// suffix-array order come out ordered by (length desc, ID asc)): LSD passes
// over key = *maxl - length, carrying start and ID.  With seg_wid set, the
// records (in suffix-array order, so window by window) are sorted inside each
// of the nseg windows (window of a record = seg_wid of its ID): tiles never
// straddle a window and the histograms are laid out window by window, so
// every pass keeps each window's records together.  With wid set instead, the
// key is (window of the ID << wshift) | (*maxl - length), which orders the
// records window by window through the key.  The result lands in xs = {key,
// start, ID} arrays, the sorted starts also in start_copy (nullable); ys is
// the alternate set; hist holds 256 u32 per tile (tiles of 4096 records,
// plus one per window); hist_n is one device word of scratch; seg holds
// 3 (nseg + 1) + tiles words.
void lsd_sort_candidates(const uint32_t *crec, const uint32_t *maxl_dev, const uint32_t *n_dev, uint64_t bound,
                         int key_bits, uint32_t *const *xs, uint32_t *const *ys, uint32_t *start_copy,
                         uint32_t *hist, uint32_t *hist_n, uint32_t *tile_tmp, hipStream_t s, const uint32_t *wid,
                         int wshift, const uint32_t *seg_wid, uint32_t nseg, uint32_t *seg);
constexpr uint64_t kLsdTileRecords = 4096;
// flag[i] = 1 where (key, p2) differs from position i - 1.
void run_flags(const uint32_t *key, const uint32_t *p2, const uint32_t *n_dev, uint64_t bound, uint8_t *flag,
               hipStream_t s);
// Positions of the set flags, in order; *count receives their number.
void flag_positions(const uint8_t *flag, const uint32_t *n_dev, uint64_t bound, uint32_t *out, uint32_t *count,
                    uint32_t *tile_tmp, hipStream_t s);
// Compaction of the sorted candidates: slot k (keep[k] set) takes position
// order[k] of the length-sorted arrays; length = *maxl - (lkey & lmask).
void compact_sorted_runs(const uint32_t *order, const uint8_t *keep, const uint32_t *m_dev, uint64_t bound,
                         const uint32_t *lkey, const uint32_t *start, const uint32_t *id, const uint32_t *maxl,
                         uint32_t *s_len, uint32_t *s_start, uint32_t *s_id, uint32_t *tile_tmp, uint32_t *total,
                         hipStream_t s, uint32_t lmask = 0xFFFFFFFFu);

void compact_sorted(const uint32_t *order, const uint8_t *keep, const uint32_t *m_dev, uint64_t bound,
                    const uint32_t *crec, uint32_t *s_len, uint32_t *s_start, uint32_t *s_id, uint32_t *tile_tmp,
                    uint32_t *total, hipStream_t s);

// Empties the levels of a selection sparse table that a run can use.
void sel_table_init(uint32_t *T, uint64_t n, const uint32_t *maxl, int top, hipStream_t s);
void sel_init(uint32_t *work, const uint32_t *nlive_dev, uint8_t *state, uint64_t bound, hipStream_t s);
// One selection round: filter by painted positions (r >= 1), then dense
// (sparse table over all positions) or sparse (canonical blocks of the
// working list) evaluation, chosen on the device.  Round 0 works on `work`
// filled by sel_init; undecided candidates go to `pend`, which the next
// round filters back into `work`.  ctree holds 2 * npad words, all
// 0xFFFFFFFF between rounds; mark must be clear before round 0.
void sel_round(const uint32_t *len, const uint32_t *start, uint32_t *Tc, uint32_t *To, int top, uint64_t n,
               uint8_t *state, uint32_t *pend, uint32_t *work, uint32_t *nlive, uint32_t *nwork, uint32_t *undec,
               int r, uint64_t live_hint, const uint32_t *maxl, uint32_t *ctree, uint64_t npad, uint8_t *mark,
               hipStream_t s);
void sel_sequential(uint8_t *state, const uint32_t *len, const uint32_t *start, const uint32_t *m_dev, uint64_t bound,
                    uint8_t *mark, uint64_t n, hipStream_t s);
// Exact greedy over the first k candidates (k <= the candidate count), which
// sets their state and paints the accepted ones into `mark` (zeroed before);
// then round 1's undecided list: pend = k..m-1 and *nlive1 = m - k.
void sel_prefix(const uint32_t *len, const uint32_t *start, uint32_t k, uint8_t *state, uint8_t *mark,
                uint32_t *pend, const uint32_t *m_dev, uint32_t *nlive1, uint64_t bound, hipStream_t s);

// Exact greedy for candidate lists ordered window by window (each window's
// candidates in priority order): one wavefront per window over an LDS bitmap
// of its positions (windows of at most kWinSelMax tokens).  woff: window
// offsets (nwin + 1 entries, the list's positions are relative to woff[0] =
// 0); wid: window of each position (null for one window); state[k]
// receives 1 (accepted) or 2 (rejected).
constexpr uint64_t kWinSelMax = 1ull << 17;
void sel_windows(const uint32_t *len, const uint32_t *start, const uint32_t *m_dev, uint64_t bound,
                 const uint32_t *wid, const uint64_t *woff, uint32_t nwin, uint64_t maxwin, uint8_t *state,
                 hipStream_t s);

void gather_accepted(const uint8_t *state, const uint32_t *m_dev, uint64_t bound, const uint32_t *len,
                     const uint32_t *start, const uint32_t *id, uint32_t *o_len, uint32_t *o_start, uint32_t *o_id,
                     uint32_t *tile_tmp, uint32_t *total, hipStream_t s);
void emit_rows(const uint32_t *order, const uint32_t *a_dev, uint64_t bound, const uint32_t *o_len,
               const uint32_t *o_start, const uint32_t *o_id, const uint32_t *wid, const uint64_t *woff, uint32_t *f,
               uint32_t *rowidx, uint32_t *row_first, void *rows, void *occ, uint32_t *win_rows, uint32_t *tile_tmp,
               uint32_t *nrows, hipStream_t s);
void window_of_occ(const uint32_t *o_start, const uint32_t *wid, const uint32_t *a_dev, uint64_t bound, uint32_t *out,
                   hipStream_t s);
// Per-substring equal-length greedy over sorted candidates: next occurrence
// kept after each one and the chain length from it; tmp holds 3m words.
void interval_counts(const uint32_t *len, const uint32_t *start, const uint32_t *id, uint32_t m, uint32_t *next,
                     uint32_t *count, uint32_t *tmp, hipStream_t s);
void iota_u32(uint32_t *p, const uint32_t *n_dev, uint64_t bound, hipStream_t s);

}  // namespace apo
