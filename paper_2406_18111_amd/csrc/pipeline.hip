// Stage sequence of one analysis (Section 4.2, Algorithm 2), host side.
#include "pipeline.h"
#include "stages.h"
#include <algorithm>
#include <cstdio>
#include <cstring>

namespace apo {

int hip_fail(hipError_t e, const char *what, const char *file, int line) {
  fprintf(stderr, "[apo] %s failed: %s (%s:%d)\n", what, hipGetErrorString(e), file, line);
  (void)hipGetLastError();
  return e == hipErrorOutOfMemory ? -2 : -4;
}

__global__ void k_set_range(uint64_t *r, const uint32_t *count) {
  if (threadIdx.x == 0) { r[0] = 0; r[1] = *count; }
}

static uint64_t pow2_at_least(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// ---------------------------------------------------------------- layout
struct Layout {
  size_t total = 0;
  size_t take(size_t n) { size_t o = total; total += (n + 255) & ~(size_t)255; return o; }
};

static void plan(uint64_t N, uint32_t W, int &nsnap, int &nT, int &nlev, uint64_t &hcap) {
  nsnap = ceil_log2_u64(N) + 2;
  nT = ceil_log2_u64(N) + 1;
  nlev = 1;
  for (uint64_t sz = N; sz > (uint64_t)kMinFan && nlev < kMinLevels; sz = (sz + kMinFan - 1) / kMinFan) nlev++;
  hcap = pow2_at_least(2 * N);
  (void)W;
}

// Exact device bytes ensure() allocates for capacity (N, W): the workspace
// layout (computed by a dry pass of the layout code) plus the sort engine.
size_t Workspace::bytes_for(uint64_t N, uint32_t W) {
  Workspace probe;
  size_t b = 0;
  probe.layout(N, W, &b);
  return b + SortEngine::bytes_for(2 * N);
}

void Workspace::release() {
  eng.release();
  if (mem && !external) (void)hipFree(mem);
  mem = nullptr;
  external = false;
  if (hcnt) (void)hipHostFree(hcnt);
  hcnt = nullptr;
  if (hctr) (void)hipHostFree(hctr);
  hctr = nullptr;
  if (hrhist) (void)hipHostFree(hrhist);
  hrhist = nullptr;
  if (hsel) (void)hipHostFree(hsel);
  hsel = nullptr;
  for (auto &e : ev)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
  for (auto &e : kev)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
  capN = 0;
  capW = 0;
}

void Workspace::grow_target(uint64_t N, uint32_t W, uint64_t &wantN, uint32_t &wantW) const {
  wantN = std::max<uint64_t>(pow2_at_least(std::max<uint64_t>(N, 1024)), capN);
  wantW = std::max<uint32_t>((uint32_t)pow2_at_least(std::max<uint32_t>(W, 1)), capW);
}

size_t Workspace::bytes_after(uint64_t N, uint32_t W) const {
  if (N <= capN && W <= capW && mem) return held();
  uint64_t wantN;
  uint32_t wantW;
  grow_target(N, W, wantN, wantW);
  return bytes_for(wantN, wantW);
}

int Workspace::ensure(uint64_t N, uint32_t W, size_t budget) {
  if (N <= capN && W <= capW && mem) return 0;
  uint64_t wantN;
  uint32_t wantW;
  grow_target(N, W, wantN, wantW);
  if (budget && bytes_for(wantN, wantW) > budget) return -2;
  release();
  return layout(wantN, wantW, nullptr);
}

int Workspace::attach(void *ext, size_t ext_bytes, uint64_t N, uint32_t W) {
  release();
  if (!ext || ((uintptr_t)ext & 255) || bytes_for(N, W) > ext_bytes) return -2;
  return layout(N, W, nullptr, ext);
}

// Lays out every array of a workspace of capacity (N_, wantW); with
// dry_bytes set only the total is computed (nothing is allocated); with ext
// set the device arrays go into that memory instead of a new allocation.
int Workspace::layout(uint64_t wantN, uint32_t wantW, size_t *dry_bytes, void *ext) {
  plan(wantN, wantW, nsnap, nT, nlev, hcap);
  const uint64_t N_ = wantN, C2 = 2 * wantN;
  Layout L;
  size_t o_tok64 = L.take(N_ * 8), o_tokrank = L.take(N_ * 4), o_htab = L.take((hcap + 1) * 8),
         o_hrank = L.take((hcap + 1) * 4);
  size_t o_di = L.take(N_ * 4), o_ds = L.take(N_ * 4), o_dhi = L.take(N_ * 4), o_dlo = L.take(N_ * 4);
  size_t o_off = L.take((wantW + 1) * 8), o_wb = L.take(N_ * 4), o_we = L.take(N_ * 4), o_wid = L.take(N_ * 4);
  size_t o_wr = L.take((wantW + 1) * 4), o_ord = L.take((wantW + 1) * 4);
  size_t o_wf = L.take(wantW + 1);
  size_t o_rank = L.take(N_ * 4), o_snap = L.take((size_t)nsnap * N_ * 4), o_sa = L.take(N_ * 4);
  size_t o_lcp = L.take(N_ * 4);
  size_t o_lvl[8] = {0};
  {
    uint64_t sz = N_;
    for (int k = 1; k < nlev; k++) { sz = (sz + kMinFan - 1) / kMinFan; o_lvl[k] = L.take(sz * 4 + 4 * kMinFan); }
  }
  size_t o_crec = L.take(C2 * 4 * kCandWords), o_keep = L.take(C2);
  size_t o_sl = L.take(C2 * 4), o_ss = L.take(C2 * 4), o_si = L.take(C2 * 4);
  // tmp_d also holds the candidate sort's digit histograms: 1024 words per 4096 candidates, at least 1024
  size_t o_ta = L.take(C2 * 4), o_tb = L.take(C2 * 4), o_tc = L.take(C2 * 4), o_td = L.take((C2 + 2048) * 4);
  size_t o_tile = L.take((C2 / 4096 + 4) * 4);
  size_t o_T = L.take(2 * (size_t)nT * N_ * 4), o_live0 = L.take(C2 * 4), o_live1 = L.take(C2 * 4);
  size_t o_state = L.take(C2), o_mark = L.take(N_), o_ctree = L.take(2 * N_ * 4), o_aflag = L.take(N_);
  size_t o_ol = L.take(N_ * 4), o_os = L.take(N_ * 4), o_oi = L.take(N_ * 4);
  size_t o_rows = L.take(N_ * 12), o_occ = L.take(N_ * 12), o_rf = L.take(N_ * 4), o_ri = L.take(N_ * 4);
  size_t o_cnt = L.take(CNT_COUNT * 4);
  size_t o_rh = L.take(4 * 64 * 4);
  size_t o_sc = L.take(3 * (kSelRoundCap + 2) * 4);
  if (dry_bytes) {
    *dry_bytes = L.total;
    return 0;
  }
  if (ext) {
    mem = ext;
    external = true;
  } else {
    hipError_t e = hipMalloc(&mem, L.total);
    if (e != hipSuccess) { mem = nullptr; (void)hipGetLastError(); return -2; }
  }
  bytes = L.total;
  char *m = static_cast<char *>(mem);
  tok64 = (uint64_t *)(m + o_tok64);
  tokrank = (uint32_t *)(m + o_tokrank);
  htab = (uint64_t *)(m + o_htab);
  hrank = (uint32_t *)(m + o_hrank);
  dist_idx = (uint32_t *)(m + o_di);
  dist_slot = (uint32_t *)(m + o_ds);
  dhi = (uint32_t *)(m + o_dhi);
  dlo = (uint32_t *)(m + o_dlo);
  d_off = (uint64_t *)(m + o_off);
  wbeg = (uint32_t *)(m + o_wb);
  wend = (uint32_t *)(m + o_we);
  wid = (uint32_t *)(m + o_wid);
  win_rows = (uint32_t *)(m + o_wr);
  d_order = (uint32_t *)(m + o_ord);
  wflag = (uint8_t *)(m + o_wf);
  rank = (uint32_t *)(m + o_rank);
  snap = (uint32_t *)(m + o_snap);
  sa = (uint32_t *)(m + o_sa);
  lcp = (uint32_t *)(m + o_lcp);
  for (int k = 1; k < nlev; k++) lvl[k] = (uint32_t *)(m + o_lvl[k]);
  crec = (uint32_t *)(m + o_crec);
  keep = (uint8_t *)(m + o_keep);
  s_len = (uint32_t *)(m + o_sl);
  s_start = (uint32_t *)(m + o_ss);
  s_id = (uint32_t *)(m + o_si);
  tmp_a = (uint32_t *)(m + o_ta);
  tmp_b = (uint32_t *)(m + o_tb);
  tmp_c = (uint32_t *)(m + o_tc);
  tmp_d = (uint32_t *)(m + o_td);
  tile_tmp = (uint32_t *)(m + o_tile);
  T = (uint32_t *)(m + o_T);
  live[0] = (uint32_t *)(m + o_live0);
  live[1] = (uint32_t *)(m + o_live1);
  state = (uint8_t *)(m + o_state);
  mark = (uint8_t *)(m + o_mark);
  ctree = (uint32_t *)(m + o_ctree);
  aflag = (uint8_t *)(m + o_aflag);
  o_len = (uint32_t *)(m + o_ol);
  o_start = (uint32_t *)(m + o_os);
  o_id = (uint32_t *)(m + o_oi);
  rows = (void *)(m + o_rows);
  occ = (void *)(m + o_occ);
  row_first = (uint32_t *)(m + o_rf);
  rowidx = (uint32_t *)(m + o_ri);
  dcnt = (uint32_t *)(m + o_cnt);
  rhist = (uint32_t *)(m + o_rh);
  selcnt = (uint32_t *)(m + o_sc);
  int rc = eng.alloc(C2, nullptr, ext ? static_cast<char *>(ext) + L.total : nullptr);
  if (rc) { release(); return rc; }
  APO_HIP_TRY(hipHostMalloc((void **)&hcnt, CNT_COUNT * 4, hipHostMallocDefault));
  APO_HIP_TRY(hipHostMalloc((void **)&hctr, sizeof(SortCounters), hipHostMallocDefault));
  APO_HIP_TRY(hipHostMalloc((void **)&hrhist, 4 * 64 * 4, hipHostMallocDefault));
  APO_HIP_TRY(hipHostMalloc((void **)&hsel, 2 * (kSelRoundCap + 2) * 4, hipHostMallocDefault));
  for (auto &ev_ : ev) APO_HIP_TRY(hipEventCreate(&ev_));
  for (auto &ev_ : kev) APO_HIP_TRY(hipEventCreate(&ev_));
  APO_HIP_TRY(hipMemset(dcnt, 0, CNT_COUNT * 4));
  capN = N_;
  capW = wantW;
  return 0;
}

// ------------------------------------------------------------- helpers
static int read_counters(Workspace &w, hipStream_t s) {
  APO_HIP_TRY(hipMemcpyAsync(w.hcnt, w.dcnt, CNT_COUNT * 4, hipMemcpyDeviceToHost, s));
  APO_HIP_TRY(hipMemcpyAsync(w.hctr, w.eng.bufs().ctr, sizeof(SortCounters), hipMemcpyDeviceToHost, s));
  APO_HIP_TRY(hipStreamSynchronize(s));
  if (w.fail_after >= 0 && w.fail_after-- == 0) {  // test hook: this sync reports a device error
    fprintf(stderr, "[apo] injected device error\n");
    return -4;
  }
  if (w.hctr->err) {
    fprintf(stderr, "[apo] device capacity check failed (code %u)\n", w.hctr->err);
    return -4;
  }
  return 0;
}

// Multi-key sort of *count_dev items whose ids are 0..count-1 (bound: host
// upper bound of the count): level k orders by fields[k][id * strides[k]] (c - field when
// subs[k], c read from c_devs[k]) within the groups of level k-1.  The final
// order is left in eng.val[0]; keep[slot] = 0 marks exact duplicates of the
// previous slot at the last level (when keep != nullptr).
static void sort_plain(Workspace &w, const uint32_t *count_dev, uint64_t bound, const uint32_t *const *fields,
                       const int *strides, const int *subs, const uint32_t *const *c_devs, const int *bits,
                       int nlevels, uint8_t *keep, hipStream_t s) {
  SortEngine &E = w.eng;
  int cur = 0;
  E.reset_counters(s);
  E.round_begin(cur, s);
  E.iota_val(count_dev, bound, s);
  E.gather_field(cur, fields[0], strides[0], count_dev, subs[0], c_devs[0], 0, bound, s);
  uint64_t *rng = reinterpret_cast<uint64_t *>(w.dcnt + CNT_RANGE);
  hipLaunchKernelGGL(k_set_range, dim3(1), dim3(64), 0, s, rng, count_dev);
  E.init_units(cur, rng, 1, 0, (uint32_t)bits[0], s);
  if (keep) fill_u8_dev(keep, count_dev, bound, 1, s);
  for (int L = 0; L < nlevels; L++) {
    const int last = (L == nlevels - 1);
    const uint32_t nb = last ? 0u : (uint32_t)bits[L + 1];
    if (bound > (1u << E.tile_log())) E.msd(cur, bound, bits[L], s);
    E.lds_plain(cur, nb, last, keep ? keep : w.keep, bound, s);
    E.bulk_plain(cur, nb, last, keep ? keep : w.keep, bound, s);
    if (!last) {
      cur ^= 1;
      E.round_begin(cur, s);
      E.gather_field(cur, fields[L + 1], strides[L + 1], nullptr, subs[L + 1], c_devs[L + 1], 0, bound, s);
    }
  }
}

static void stamp(Workspace &w, int k, hipStream_t s, bool on) {
  if (on) (void)hipEventRecord(w.ev[k], s);
}

// Reads the device counters of a finished analysis into `info`.
static void fill_info(Workspace &w, uint64_t N, RunInfo &info) {
  info.n = N;
  info.sigma = w.hcnt[CNT_ND] + w.hcnt[CNT_NDSUM];  // shared table + windows ranked on their own
  info.pair_windows = (w.pair_w && w.hcnt[CNT_PFLAG] == 0) ? w.pair_w : 0;
  info.cands = w.hcnt[CNT_C] + w.hcnt[CNT_CSKIP];
  info.maxl = w.hcnt[CNT_MAXL];
  info.cands_dedup = w.hcnt[CNT_M];
  info.accepted = w.hcnt[CNT_A];
  info.rows = w.hcnt[CNT_NROWS];
  info.active_sum = 0;
  for (int k = 0; k < w.nsnap; k++) {
    info.active_sum += (k == 0) ? N : w.hrhist[4 * (k - 1)];
    if (w.hrhist[4 * k] == 0) { info.rounds = (uint32_t)k + 1; break; }
  }
}

int upload_windows(Workspace &w, const uint64_t *h_off, uint32_t W, hipStream_t s, bool order) {
  APO_HIP_TRY(hipMemcpyAsync(w.d_off, h_off, (W + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
  if (!order || !W) return 0;
  // longest first, in buckets of equal bit length (a counting sort): a long
  // window taken last would hold one workgroup while the others are idle
  // (host-driven lanes keep the given order: there other lanes fill the
  // idle compute units, and the step measured slower with it)
  uint32_t cnt[66] = {0};
  for (uint32_t k = 0; k < W; k++) cnt[64 - bit_length_u64(h_off[k + 1] - h_off[k]) + 1]++;
  for (int b = 1; b < 66; b++) cnt[b] += cnt[b - 1];
  w.h_order.resize(W + 1);
  for (uint32_t k = 0; k < W; k++) w.h_order[cnt[64 - bit_length_u64(h_off[k + 1] - h_off[k])]++] = k;
  APO_HIP_TRY(hipMemcpyAsync(w.d_order, w.h_order.data(), W * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  return 0;
}

int run_pipeline(Workspace &w, const void *d_tok, int bits, uint64_t N, const uint64_t *h_off, uint32_t W,
                 uint32_t min_len, Stop stop, hipStream_t s, RunInfo &info, Mode mode) {
  info = RunInfo{};
  SortEngine &E = w.eng;
  E.set_chunk_for(N);
  SortBufs &B = E.bufs();
  int rc;
  const bool host = mode == Mode::HOST;
  const bool stamps = mode != Mode::CAPTURE;
  uint32_t *dc = w.dcnt;
  stamp(w, 0, s, stamps);
  if (mode != Mode::CAPTURE)  // a captured sequence expects d_off (and the order) to be uploaded already
    if ((rc = upload_windows(w, h_off, W, s, !host))) return rc;
  const uint32_t *worder = host ? nullptr : w.d_order;
  const bool batch = W > 1;
  const uint32_t *wbeg = nullptr, *wend = nullptr, *wid = nullptr;
  if (batch) {
    window_bounds(w.d_off, W, w.wbeg, w.wend, w.wid, s);
    wbeg = w.wbeg;
    wend = w.wend;
    wid = w.wid;
  }
  uint64_t maxwin = 0;
  for (uint32_t k = 0; k < W; k++) maxwin = std::max<uint64_t>(maxwin, h_off[k + 1] - h_off[k]);
  fill_u32(dc, CNT_RANGE, 0, s);
  fill_u32(dc + CNT_NDSUM, 8, 0, s);
  fill_u32(dc + CNT_SNAPS, 1, 0, s);
  fill_u32(w.rhist, 4 * (uint64_t)w.nsnap, 0, s);

  // ---- order-preserving token ranks
  const uint32_t *key0;
  uint32_t bits0;
  // batches of 64-bit tokens: the windows ranked on their own also get their
  // first doubling round from a per-window kernel; the engine's first round
  // then only sorts the flagged windows (and is skipped by host-driven runs
  // that have none).  When every window has its own ranks and few distinct
  // token pairs, the first two rounds come from per-window kernels instead
  // (pair ranks, then one counting sort on them): host-driven runs read that
  // from the counters and start the doubling loop at offset 2; sync-free runs
  // launch both forms gated on the device count (pflag) and run the
  // engine's second round empty.
  bool win_r0 = false, skip0 = false, pair0 = false;
  const uint32_t *pflag = nullptr;
  w.pair_w = 0;
  if (bits == 64) {
    const uint64_t *tok = static_cast<const uint64_t *>(d_tok);
    // Batches rank each window on its own first; the shared table then
    // ranks only the windows with too many distinct values for that (a
    // single window always goes through it).  In host-driven runs it is
    // skipped when no window needs it; sync-free runs launch it gated on the
    // device count of such windows.
    const uint32_t *wgate = nullptr;
    const uint8_t *wf = nullptr;
    bool shared = true;
    uint64_t loc_bits = 0;
    if (batch) {
      win_rank(tok, w.d_off, worder, W, w.tokrank, w.wflag, dc + CNT_NDSUM, s);
      wgate = dc + CNT_WFLAG;
      wf = w.wflag;
      win_pair(w.d_off, worder, W, w.wflag, w.tokrank, B.key[1], dc + CNT_PNEXT, dc + CNT_A1, dc + CNT_WFLAG, s);
      w.pair_w = W;
      if (host) {
        if ((rc = read_counters(w, s))) return rc;
        shared = w.hcnt[CNT_WFLAG] > 0;
        pair0 = w.hcnt[CNT_PFLAG] == 0;  // windows counted in CNT_WFLAG count here too
        loc_bits = (uint64_t)bit_length_u64(w.hcnt[CNT_NDMAX]);
      } else {
        pflag = dc + CNT_PFLAG;
      }
    }
    uint64_t nd_bound = N;
    if (shared) {
      const uint64_t hc = pow2_at_least(2 * N);
      hash_clear(w.htab, hc - 1, s, wgate);
      hash_insert(tok, N, w.htab, hc - 1, w.dist_idx, w.dist_slot, dc + CNT_ND, w.tokrank, s, wid, wf, wgate);
      if (host) {
        if ((rc = read_counters(w, s))) return rc;
        nd_bound = w.hcnt[CNT_ND];
      }
      hash_fields(tok, w.dist_idx, dc + CNT_ND, w.dhi, w.dlo, nd_bound, s);
      const uint32_t *f[2] = {w.dhi, w.dlo};
      const int sub[2] = {0, 0};
      const uint32_t *cd[2] = {nullptr, nullptr};
      const int bb[2] = {32, 32};
      const int str[2] = {1, 1};
      sort_plain(w, dc + CNT_ND, nd_bound, f, str, sub, cd, bb, 2, nullptr, s);
      hash_assign(B.val[0], dc + CNT_ND, w.dist_slot, w.hrank, nd_bound, s);
      hash_rank(w.tokrank, N, w.hrank, w.tokrank, s, wid, wf, wgate);  // slots -> ranks in place
    } else {
      nd_bound = 0;
    }
    win_r0 = batch;
    skip0 = batch && !shared;
    key0 = w.tokrank;
    bits0 = (uint32_t)std::max<uint64_t>(bit_length_u64(nd_bound), loc_bits);
  } else {
    key0 = static_cast<const uint32_t *>(d_tok);
    bits0 = 32;
  }
  stamp(w, 1, s, stamps);

  // ---- suffix array by prefix doubling
  // Host-driven: rounds are launched `spec` at a time and the host reads their
  // outcomes once per batch.  Otherwise every round up to the bound for the
  // longest window is launched.  A round launched after the last active suffix
  // became unique finds empty lists everywhere and changes nothing, so extra
  // rounds never alter the result.  Large units only arise from large units
  // of the previous round, so once none are left the MSD passes are skipped.
  const uint32_t rank_bits = (uint32_t)bit_length_u64(N);
  // rounds >= 1 bucket their keys (ranks) relative to the window start:
  // values 0..longest window
  const uint32_t rel_bits = (uint32_t)bit_length_u64(std::max<uint64_t>(maxwin, 1));
  const int r_max = ceil_log2_u64(std::max<uint64_t>(maxwin, 2)) + 1;  // rounds 0..r_max-1 suffice
  int cur = 0;
  E.reset_counters(s);
  E.round_begin(cur, s);
  if (win_r0) {
    if (!skip0) {
      E.gather_identity(key0, (uint32_t)N, s, wid, w.wflag, dc + CNT_WFLAG);
      E.init_units(cur, w.d_off, W, 0, bits0, s, w.wflag);
    }
    // with pairs: the state after round 1 and the lists of round 2 (sync-free
    // runs: the first-token form, which gives way when *pflag == 0)
    if (pair0)
      win_round0(B, w.d_off, worder, W, w.wflag, B.key[1], w.rank, w.aflag, rel_bits, dc + CNT_WNEXT2, true, nullptr,
                 dc + CNT_A1, w.rhist, s);
    else
      win_round0(B, w.d_off, worder, W, w.wflag, key0, w.rank, w.aflag, rel_bits, dc + CNT_WNEXT2, false, pflag, nullptr,
                 nullptr, s);
  } else {
    E.gather_identity(key0, (uint32_t)N, s);
    E.init_units(cur, w.d_off, W, 0, bits0, s);
  }
  bool big = maxwin > (1ull << E.tile_log());
  uint64_t act = N;
  int r = pair0 ? 2 : 0, synced = r, done_round = -1;
  w.kev_n = 0;
  const int spec = host ? 4 : r_max;
  while (done_round < 0) {
    if (r >= w.nsnap) return -4;
    if (r > 0) E.gather_sa(cur, w.rank, w.aflag, wend, (uint32_t)N, 1u << (r - 1), w.rhist, r, s);
    // sync-free runs with pair ranks: the second round's state from them,
    // after that round's gather (which found nothing grouped and cleared
    // the lists it fills), so the round's sort launches find no work
    if (r == 1 && pflag)
      win_round0(B, w.d_off, worder, W, w.wflag, B.key[1], w.rank, w.aflag, rel_bits, dc + CNT_WNEXT2, true, pflag,
                 dc + CNT_A1, w.rhist, s);
    RankOut R{w.rank, (uint32_t)r, w.aflag};
    if (r > 0 || !skip0) {
      if (big) E.msd(cur, act, r == 0 ? (int)bits0 : (int)rel_bits, s, r == 0 ? nullptr : wbeg);
      const bool timed = w.ktag == KT_LDS_SA && w.kev_n < kMaxTimed;
      if (timed) APO_HIP_TRY(hipEventRecord(w.kev[2 * w.kev_n], s));
      E.lds_sa(cur, R, rel_bits, act, s);
      if (timed) {
        APO_HIP_TRY(hipEventRecord(w.kev[2 * w.kev_n + 1], s));
        w.kround[w.kev_n++] = r;
      }
      E.bulk_sa(cur, R, rel_bits, act, s);
    }
    // rounds >= kSnapFrom: the rank array after the round, for the LCP walk
    if (r >= kSnapFrom) snapshot_ranks(w.rank, w.snap + (size_t)r * N, N, w.rhist + 4 * (r - 1), dc + CNT_SNAPS, r, s);
    cur ^= 1;
    r++;
    if (!host) {
      if (r >= r_max) {
        E.round_end(cur ^ 1, r - 1, w.rhist, s);
        done_round = r - 1;  // an upper bound of the last round that did work
      }
      continue;
    }
    if (r - synced >= spec || r >= w.nsnap) {
      E.round_end(cur ^ 1, r - 1, w.rhist, s);
      APO_HIP_TRY(hipMemcpyAsync(w.hrhist, w.rhist, 4 * w.nsnap * 4, hipMemcpyDeviceToHost, s));
      if ((rc = read_counters(w, s))) return rc;
      for (int k = synced; k < r; k++)
        if (w.hrhist[4 * k] == 0) { done_round = k; break; }
      if (done_round < 0) {
        act = w.hrhist[4 * (r - 1)];
        big = w.hrhist[4 * (r - 1) + 1] > 0;
        synced = r;
      }
    }
  }
  r = done_round;
  APO_HIP_TRY(hipMemcpyAsync(w.sa, B.val[0], N * 4, hipMemcpyDeviceToDevice, s));
  stamp(w, 2, s, stamps);
  if (stop == Stop::SA) {
    APO_HIP_TRY(hipMemcpyAsync(w.hrhist, w.rhist, 4 * w.nsnap * 4, hipMemcpyDeviceToHost, s));
    if ((rc = read_counters(w, s))) return rc;
    fill_info(w, N, info);
    return 0;
  }

  // ---- LCP via Phi / PLCP (lifting over the snapshots of the rounds that
  // sorted something, at most r-1)
  build_lcp(w.sa, w.rank, N, wbeg, wend, w.snap, dc + CNT_SNAPS, key0, r - 1, w.lcp, s);
  stamp(w, 3, s, stamps);
  if (stop == Stop::LCP) return read_counters(w, s);

  // ---- candidates
  gen_candidates(w.sa, w.lcp, N, wend, min_len, w.lvl, w.nlev, w.crec, dc + CNT_C, dc + CNT_CSKIP, dc + CNT_MAXL,
                 w.tmp_d, dc + CNT_AUX, w.tile_tmp, s);
  uint64_t c_bound = 2 * N;
  uint64_t maxl_bound = std::max<uint64_t>(maxwin / 2, 1);
  if (host) {
    if ((rc = read_counters(w, s))) return rc;
    c_bound = w.hcnt[CNT_C];
    maxl_bound = std::max<uint32_t>(w.hcnt[CNT_MAXL], 1);
  }
  stamp(w, 4, s, stamps);
  // Greedy by one wavefront per window over an LDS bitmap when every window
  // is short enough: then the candidate list is sorted window by window
  // (window above the length in the sort key), which also leaves the
  // accepted occurrences in the output's (window, priority) order.
  const int lbits = bit_length_u64(maxl_bound);
  const int wbits = batch ? bit_length_u64(W - 1) : 0;
  const bool winsel =
      w.win_greedy && (batch ? (maxwin <= kWinSelMax && lbits + wbits <= 32) : (N <= kWinSelSingle));
  uint64_t m_bound = 0;
  if (c_bound > 0) {
    // Priority order (length desc, ID asc, start asc).  The records are in
    // suffix-array order, where the ID of a fixed length never decreases, so
    // a stable sort by length leaves (length, ID) ordered; runs of equal
    // (length, ID) are then sorted by start as units of the sort engine,
    // whose last level also marks exact duplicates.
    // the sorted starts also go straight into the engine's key buffer (the
    // key of the last level); MSD passes may move them, so the compaction
    // reads its own copy
    uint32_t *xs[3] = {w.tmp_a, w.tmp_b, w.tmp_c};  // length key, start, ID
    uint32_t *ys[3] = {w.s_len, w.s_start, w.s_id};
    // window-major order for the per-window greedy: tiles kept inside
    // windows when the per-window histograms fit the scratch, else the window
    // goes above the length in the key
    const uint64_t seg_tiles = (c_bound + kLsdTileRecords - 1) / kLsdTileRecords + W;
    const bool wseg = winsel && batch && (seg_tiles * 256 <= 2 * w.capN + 2048) && seg_tiles + 3 * (W + 1) <= w.capN;
    const bool wkey = winsel && batch && !wseg;
    lsd_sort_candidates(w.crec, dc + CNT_MAXL, dc + CNT_C, c_bound, lbits + (wkey ? wbits : 0), xs, ys, B.key[0],
                        w.tmp_d, dc + CNT_AUX, w.tile_tmp, s, wkey ? wid : nullptr, lbits, wseg ? wid : nullptr, W,
                        w.o_len);
    E.reset_counters(s);
    E.round_begin(0, s);
    E.iota_val(dc + CNT_C, c_bound, s);
    run_flags(w.tmp_a, w.tmp_c, dc + CNT_C, c_bound, w.keep, s);
    flag_positions(w.keep, dc + CNT_C, c_bound, w.tmp_d, dc + CNT_AUX, w.tile_tmp, s);
    E.init_runs(0, w.tmp_d, dc + CNT_AUX, dc + CNT_C, c_bound, rank_bits, s);
    fill_u8_dev(w.keep, dc + CNT_C, c_bound, 1, s);
    if (c_bound > (1ull << E.tile_log())) E.msd(0, c_bound, (int)rank_bits, s);
    E.lds_plain(0, 0, 1, w.keep, c_bound, s);
    E.bulk_plain(0, 0, 1, w.keep, c_bound, s);
    compact_sorted_runs(B.val[0], w.keep, dc + CNT_C, c_bound, w.tmp_a, w.tmp_b, w.tmp_c, dc + CNT_MAXL, w.s_len,
                        w.s_start, w.s_id, w.tile_tmp, dc + CNT_M, s,
                        wkey ? (uint32_t)((1ull << lbits) - 1) : 0xFFFFFFFFu);
    m_bound = c_bound;
    if (host) {
      if ((rc = read_counters(w, s))) return rc;
      m_bound = w.hcnt[CNT_M];
    }
  }
  stamp(w, 5, s, stamps);
  if (stop == Stop::CANDS) {
    if ((rc = read_counters(w, s))) return rc;
    fill_info(w, N, info);
    return 0;
  }

  // ---- greedy selection
  int sel_done = -1, sel_launched = 0;
  if (m_bound > 0 && winsel) {
    fill_u32(w.selcnt, 3 * (kSelRoundCap + 2), 0, s);  // one round, nothing left undecided after it
    copy_u32(w.selcnt, dc + CNT_M, s);
    sel_windows(w.s_len, w.s_start, dc + CNT_M, m_bound, batch ? wid : nullptr, w.d_off, W, batch ? maxwin : N,
                w.state, s);
    sel_done = 0;
    sel_launched = 1;
  } else if (m_bound > 0) {
    const int top = 63 - __builtin_clzll(maxl_bound);
    uint32_t *Ta = w.T, *Tb = w.T + (size_t)w.nT * w.capN;
    uint32_t *nlive = w.selcnt, *undec = w.selcnt + (kSelRoundCap + 2), *nwork = w.selcnt + 2 * (kSelRoundCap + 2);
    // exact prefix walk (host-driven runs, where the candidate count and the
    // longest length are known): round 0 is then skipped, and its table with it
    uint32_t kpre = 0;
    if (host && w.sel_prefix > 0) kpre = (uint32_t)std::min<uint64_t>((uint64_t)w.sel_prefix, m_bound);
    if (host && w.sel_prefix < 0 && maxl_bound * kSelPrefixDiv >= N)
      kpre = (uint32_t)std::min<uint64_t>(kSelPrefixAuto, m_bound);
    if (!kpre) sel_table_init(Ta, N, dc + CNT_MAXL, top, s);
    fill_u32(w.selcnt, 3 * (kSelRoundCap + 2), 0, s);
    const uint64_t npad = pow2_at_least(N);
    fill_u32(w.ctree, 2 * npad, 0xFFFFFFFFu, s);
    fill_u8(w.mark, N, 0, s);
    copy_u32(nlive, dc + CNT_M, s);
    sel_init(w.live[1], nlive, w.state, m_bound, s);
    const int ahead = host ? 2 : kSelFreeRounds;
    int q0 = 0;
    uint64_t hint = m_bound;
    if (kpre) {
      sel_prefix(w.s_len, w.s_start, kpre, w.state, w.mark, w.live[0], dc + CNT_M, nlive + 1, m_bound, s);
      info.sel_prefix = kpre;
      q0 = 1;  // round 1 filters the candidates after the prefix
      hint = m_bound - kpre;
      sel_launched = 1;
      if (hint == 0) sel_done = 0;
    }
    // host-driven runs stop the rounds at w.sel_cap (kSelRoundCap unless a
    // test lowers it) and finish with the sequential completion
    const int cap = host ? std::max(0, std::min(w.sel_cap, kSelRoundCap)) : kSelRoundCap;
    while (sel_done < 0 && q0 < cap) {
      const int lo = q0, hi = std::min(q0 + ahead, cap);
      for (int q = lo; q < hi; q++)
        sel_round(w.s_len, w.s_start, (q & 1) ? Tb : Ta, (q & 1) ? Ta : Tb, top, N, w.state, w.live[0],
                  w.live[1], nlive, nwork, undec, q, hint, dc + CNT_MAXL, w.ctree, npad, w.mark, s);
      q0 = hi;
      sel_launched = hi;
      if (!host) break;  // checked after the output stage
      APO_HIP_TRY(hipMemcpyAsync(w.hsel, w.selcnt, 2 * (kSelRoundCap + 2) * 4, hipMemcpyDeviceToHost, s));
      if ((rc = read_counters(w, s))) return rc;
      for (int q = lo; q < hi; q++)
        if (w.hsel[q + 1] == 0) { sel_done = q; break; }  // nlive[q + 1]: undecided after round q
      if (sel_done < 0) hint = w.hsel[hi];
    }
    if (host && sel_done < 0) {
      sel_sequential(w.state, w.s_len, w.s_start, dc + CNT_M, m_bound, w.mark, N, s);
      info.sel_sequential = 1;
    }
  }
  stamp(w, 6, s, stamps);

  // ---- accepted occurrences and rows
  int orc = emit_output(w, N, W, batch, wid, wbeg, m_bound, host, s, winsel);
  if (orc) return orc;
  stamp(w, 7, s, stamps);
  if (mode == Mode::CAPTURE) return 0;
  rc = finish_run(w, N, m_bound, host ? -1 : sel_launched, info, s, stamps);
  if (host && sel_done < 0 && m_bound > 0) {
    info.sel_rounds = (uint32_t)sel_launched;
    info.sel_sequential = 1;
  }
  return rc;
}

// Accepted occurrences in priority order, the per-window order of batches,
// rows and their counts.
int emit_output(Workspace &w, uint64_t N, uint32_t W, bool batch, const uint32_t *wid, const uint32_t *wbeg,
                uint64_t m_bound, bool host, hipStream_t s, bool window_major) {
  SortBufs &B = w.eng.bufs();
  uint32_t *dc = w.dcnt;
  int rc;
  fill_u32(dc + CNT_A, 1, 0, s);
  fill_u32(dc + CNT_NROWS, 1, 0, s);
  if (batch) fill_u32(w.win_rows, W + 1, 0, s);
  if (m_bound == 0) return 0;
  gather_accepted(w.state, dc + CNT_M, m_bound, w.s_len, w.s_start, w.s_id, w.o_len, w.o_start, w.o_id, w.tile_tmp,
                  dc + CNT_A, s);
  uint64_t a_bound = std::min<uint64_t>(m_bound, N);
  if (host) {
    if ((rc = read_counters(w, s))) return rc;
    a_bound = w.hcnt[CNT_A];
    if (a_bound == 0) return 0;
  }
  const uint32_t *order = nullptr;
  if (batch && !window_major) {
    window_of_occ(w.o_start, w.wid, dc + CNT_A, a_bound, w.tmp_c, s);
    iota_u32(w.tmp_d, dc + CNT_A, a_bound, s);
    const uint32_t *f[2] = {w.tmp_c, w.tmp_d};
    const int sub[2] = {0, 0};
    const uint32_t *cd[2] = {nullptr, nullptr};
    const int bb[2] = {bit_length_u64(W), bit_length_u64(a_bound)};
    const int str[2] = {1, 1};
    sort_plain(w, dc + CNT_A, a_bound, f, str, sub, cd, bb, 2, nullptr, s);
    order = B.val[0];
  }
  emit_rows(order, dc + CNT_A, a_bound, w.o_len, w.o_start, w.o_id, wid, wbeg ? w.d_off : nullptr, w.tmp_a, w.rowidx, w.row_first, w.rows,
            w.occ, batch ? w.win_rows : nullptr, w.tile_tmp, dc + CNT_NROWS, s);
  return 0;
}

// Final synchronisation of a run (or of a replayed graph): counters, the
// rare selection completion for sync-free runs, stage and kernel timings.
int finish_run(Workspace &w, uint64_t N, uint64_t m_bound, int sel_launched, RunInfo &info, hipStream_t s,
               bool stamps) {
  int rc;
  APO_HIP_TRY(hipMemcpyAsync(w.hrhist, w.rhist, 4 * w.nsnap * 4, hipMemcpyDeviceToHost, s));
  APO_HIP_TRY(hipMemcpyAsync(w.hsel, w.selcnt, 2 * (kSelRoundCap + 2) * 4, hipMemcpyDeviceToHost, s));
  if ((rc = read_counters(w, s))) return rc;
  fill_info(w, N, info);
  info.sel_rounds = 0;
  const int qmax = sel_launched < 0 ? kSelRoundCap : sel_launched;
  for (int q = 0; q < qmax; q++)
    if (w.hsel[q + 1] == 0) { info.sel_rounds = (uint32_t)q + 1; break; }
  // sync-free run whose launched rounds left candidates undecided
  if (sel_launched >= 0 && m_bound > 0 && info.cands_dedup > 0 && info.sel_rounds == 0) return 1;
  if (stamps) {
    for (int k = 0; k < kStages; k++) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, w.ev[k], w.ev[k + 1]) == hipSuccess) info.stage_ms[k] = ms;
      else (void)hipGetLastError();  // a failed query must not linger as the thread's last error
    }
  }
  // timed kernel launches (never inside captured graphs)
  for (int k = 0; k < w.kev_n; k++) {
    const uint32_t elems = w.hrhist[4 * w.kround[k] + 2];
    float ms = 0;
    if (!elems) continue;
    if (hipEventElapsedTime(&ms, w.kev[2 * k], w.kev[2 * k + 1]) == hipSuccess) {
      info.k_launches++;
      info.k_elems += elems;
      info.k_ms += ms;
    } else {
      (void)hipGetLastError();
    }
  }
  return 0;
}

}  // namespace apo
