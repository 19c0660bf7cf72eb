// Host-side pipeline: workspace ownership and the stage sequence of one
// analysis (a single window or a packed batch of windows).
#pragma once
#include "apo_internal.h"
#include "segsort.h"
#include <vector>

namespace apo {

enum class Stop { SA, LCP, CANDS, FULL };

// HOST: the host reads device counts between stages to size launches and stop
// loops early.  FREE: everything is enqueued with host upper bounds (rounds
// for the longest window, counts from capacities) and one sync at the end.
// CAPTURE: FREE without timing events and without the final sync, for
// recording into a HIP graph.
enum class Mode { HOST, FREE, CAPTURE };
constexpr int kSelFreeRounds = 12;

enum Cnt {
  CNT_ND = 0, CNT_C, CNT_MAXL, CNT_M, CNT_NLIVE0, CNT_NLIVE1, CNT_UNDEC, CNT_A, CNT_NROWS,
  CNT_CSKIP,       // candidates not written because they repeat the previous pair's (counted in the total)
  CNT_RANGE = 10,  // two 64-bit words, 8-byte aligned
  CNT_AUX = 14,    // scratch count of a stage (tile counts, histogram size, runs)
  CNT_SNAPS = 15,  // 1 + last doubling round with a rank snapshot (0: none)
  CNT_NDSUM = 16,  // batches: distinct tokens summed over the windows ranked on their own
  CNT_NDMAX = 17,  // batches: most distinct tokens of one such window
  CNT_WFLAG = 18,  // batches: windows ranked through the shared table instead
  CNT_WNEXT = 19,  // batches: next window for the per-window ranking
  CNT_WNEXT2 = 20, // batches: next window for the per-window first doubling round
  CNT_PNEXT = 21,  // batches: next window for the per-window pair ranks
  CNT_PFLAG = 22,  // batches: windows whose pairs the per-window ranking left alone
  CNT_A1 = 23,     // batches: the first doubling round's active count, from the pair ranking
  CNT_COUNT = 32
};

constexpr int kStages = 7;
// single windows up to this many tokens use the one-wavefront greedy
constexpr uint64_t kWinSelSingle = 1ull << 15;
constexpr int kSelRoundCap = 64;
// Host-driven round-based selection first walks a prefix of kSelPrefixAuto
// candidates exactly when the longest candidate spans at least
// 1/kSelPrefixDiv of the analysis (long intervals decided first then reject
// most of the rest in round 1's filter, instead of all of them being inserted
// into round 0's coverage table).
constexpr uint32_t kSelPrefixAuto = 1024;
constexpr uint64_t kSelPrefixDiv = 64;

struct RunInfo {
  uint64_t n = 0;             // tokens analysed (all windows)
  uint32_t rounds = 0;        // doubling rounds incl. the token sort
  uint64_t active_sum = 0;    // sum over rounds of processed suffixes
  uint32_t sigma = 0;         // distinct tokens (64-bit input)
  uint32_t cands = 0;         // candidates generated (length >= min_len)
  uint32_t cands_dedup = 0;   // after removing exact duplicates
  uint32_t maxl = 0;
  uint32_t sel_rounds = 0;
  uint32_t sel_sequential = 0;
  uint32_t sel_prefix = 0;         // candidates decided by the exact prefix walk
  uint32_t pair_windows = 0;       // windows whose first two doubling rounds came from pair ranks
  uint32_t accepted = 0;
  uint32_t rows = 0;
  double stage_ms[kStages] = {0};
  // live timing of one kernel family (Workspace::ktag), launches with work only
  uint64_t k_launches = 0, k_elems = 0;
  double k_ms = 0;
};

enum KernelTag { KT_NONE = 0, KT_LDS_SA = 1 };
constexpr int kMaxTimed = 64;

struct Workspace {
  uint64_t capN = 0;
  uint32_t capW = 0;
  int nsnap = 0, nT = 0, nlev = 0;
  uint64_t hcap = 0;
  SortEngine eng;
  void *mem = nullptr;
  bool external = false;  // device arrays live in caller-owned memory (attach)
  size_t bytes = 0;

  uint64_t *tok64 = nullptr;
  uint32_t *tokrank = nullptr, *hrank = nullptr, *dist_idx = nullptr, *dist_slot = nullptr;
  uint64_t *htab = nullptr;  // distinct token values (hcap + 1 slots)
  uint32_t *dhi = nullptr, *dlo = nullptr;
  uint64_t *d_off = nullptr;
  uint32_t *d_order = nullptr;  // windows longest first (per-window kernels of sync-free runs take them so)
  std::vector<uint32_t> h_order;  // its host copy, kept alive for the upload
  uint32_t *wbeg = nullptr, *wend = nullptr, *wid = nullptr, *win_rows = nullptr;
  uint32_t *rank = nullptr, *snap = nullptr, *sa = nullptr;
  uint32_t *lcp = nullptr;
  uint32_t *lvl[8] = {nullptr};
  uint32_t *crec = nullptr;  // candidates: records (length, start, ID), three words each
  uint8_t *keep = nullptr;
  uint32_t *s_len = nullptr, *s_start = nullptr, *s_id = nullptr;
  uint32_t *tmp_a = nullptr, *tmp_b = nullptr, *tmp_c = nullptr, *tmp_d = nullptr, *tile_tmp = nullptr;
  uint32_t *T = nullptr, *live[2] = {nullptr, nullptr};
  uint8_t *state = nullptr, *mark = nullptr;
  uint32_t *ctree = nullptr;       // canonical-block tree of sparse selection rounds (2 * capN)
  uint8_t *aflag = nullptr;        // doubling rounds: slot still grouped
  uint8_t *wflag = nullptr;        // batches: window ranked through the shared table
  uint32_t *o_len = nullptr, *o_start = nullptr, *o_id = nullptr;
  void *rows = nullptr, *occ = nullptr;
  uint32_t *row_first = nullptr, *rowidx = nullptr;
  uint32_t *dcnt = nullptr;
  uint32_t *rhist = nullptr;       // per doubling round: active slots, large units after it
  uint32_t *hrhist = nullptr;      // pinned host mirror of rhist
  uint32_t *selcnt = nullptr;      // selection rounds: live counts, undecided counts
  uint32_t *hsel = nullptr;        // pinned host mirror of selcnt
  uint32_t *hcnt = nullptr;        // pinned host mirror of dcnt
  SortCounters *hctr = nullptr;    // pinned host mirror of engine counters
  hipEvent_t ev[kStages + 1] = {};
  int ktag = KT_NONE;              // kernel family timed with events around each launch
  hipEvent_t kev[2 * kMaxTimed] = {};
  int kround[kMaxTimed] = {0};
  int kev_n = 0;
  int sel_cap = kSelRoundCap;      // host-driven selection rounds before the sequential completion
  int sel_prefix = -1;             // exact prefix walk before the rounds: -1 automatic, 0 never, k > 0 k candidates
  uint32_t pair_w = 0;             // windows of the run when it ranked their token pairs (else 0)
  int fail_after = -1;             // test hook: host syncs before one reports a device error (-1: never)
  bool win_greedy = true;          // one-wavefront-per-window greedy where windows are short enough

  // device bytes a workspace of capacity (N, W) holds (exact)
  static size_t bytes_for(uint64_t N, uint32_t W);
  // device bytes held now, and after ensure(N, W)
  size_t held() const { return mem ? bytes + eng.bytes() : 0; }
  size_t bytes_after(uint64_t N, uint32_t W) const;
  // grows (never shrinks) to hold N tokens in W windows; -2 if the grown
  // workspace would exceed `budget` bytes (0: no limit) or allocation fails
  int ensure(uint64_t N, uint32_t W, size_t budget);
  // lays a workspace of capacity (N, W) out in caller-owned device memory
  // (256-byte aligned, ext_bytes >= bytes_for(N, W)); host mirrors and
  // events are still created here.  -2 if it does not fit.
  int attach(void *ext, size_t ext_bytes, uint64_t N, uint32_t W);
  void release();

 private:
  void grow_target(uint64_t N, uint32_t W, uint64_t &wantN, uint32_t &wantW) const;
  int layout(uint64_t N, uint32_t W, size_t *dry_bytes, void *ext = nullptr);

 public:
};

// Uploads a batch's window offsets h_off[0..W] on stream s, and with `order`
// set the order in which the per-window kernels of sync-free and captured
// runs take its windows (longest first, by bit length of the window's size).
int upload_windows(Workspace &w, const uint64_t *h_off, uint32_t W, hipStream_t s, bool order);

// Runs the stages of one analysis on stream s.  d_tok: device tokens of
// `bits` (32/64) bits, windows given by host offsets h_off[0..W] (global,
// ascending, h_off[0] == 0).  Results stay in the workspace.
int run_pipeline(Workspace &w, const void *d_tok, int bits, uint64_t N, const uint64_t *h_off, uint32_t W,
                 uint32_t min_len, Stop stop, hipStream_t s, RunInfo &info, Mode mode = Mode::HOST);
// window_major: the candidate list (and so the accepted occurrences) is
// already ordered window by window.
int emit_output(Workspace &w, uint64_t N, uint32_t W, bool batch, const uint32_t *wid, const uint32_t *wbeg,
                uint64_t m_bound, bool host, hipStream_t s, bool window_major);
// sel_launched: selection rounds enqueued by a sync-free run (-1: host-driven).
// Returns 1 when a sync-free run left candidates undecided (the caller then
// reruns host-driven).
int finish_run(Workspace &w, uint64_t N, uint64_t m_bound, int sel_launched, RunInfo &info, hipStream_t s,
               bool stamps);

}  // namespace apo
