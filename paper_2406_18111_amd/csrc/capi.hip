// C ABI of libapo (include/apo.h): argument checking, staging of host
// buffers, and the continuous-batching server.
#include "apo.h"
#include "pipeline.h"
#include "stages.h"
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <map>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace apo {

struct Request {
  uint64_t ticket = 0;
  uint32_t stream_id = 0;
  uint32_t min_len = 1;
  std::vector<uint64_t> tokens;
  std::vector<apo_candidate> rows;
  std::chrono::steady_clock::time_point t_submit, t_done;
  int status = 0;
  bool done = false;
  bool discard = false;  // released by the caller: drop the result when done
};

struct Slot {
  Workspace ws;
  hipStream_t stream = nullptr;
  std::thread th;
  uint64_t *pinned = nullptr;  // staging for packed tokens
  uint64_t pinned_cap = 0;
  // admission bookkeeping, guarded by Server::mu: device bytes this slot's
  // workspace holds (or has reserved for the batch it runs), and whether a
  // batch is in flight
  size_t held = 0;
  bool busy = false;
};

// Autotuned kernel parameters per input-size bucket (ceil(log2 n)).
struct TuneTable {
  std::map<int, std::pair<int, int>> best;  // bucket -> (tile_log, digit_bits)
  int fixed_tile = -1, fixed_digit = -1;     // manual override when >= 0
  void pick(uint64_t n, int &tile, int &digit) const {
    tile = kDefaultTileLog;
    digit = kDefaultDigitBits;
    if (fixed_tile >= 0) {
      tile = fixed_tile;
      digit = fixed_digit;
      return;
    }
    if (best.empty()) return;
    const int b = ceil_log2_u64(std::max<uint64_t>(n, 2));
    auto it = best.lower_bound(b);  // nearest tuned bucket
    if (it == best.end()) it = std::prev(best.end());
    else if (it->first != b && it != best.begin()) {
      auto lo = std::prev(it);
      if (b - lo->first < it->first - b) it = lo;
    }
    tile = it->second.first;
    digit = it->second.second;
  }
};

struct Server {
  std::mutex mu;
  std::condition_variable cv_work;
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<std::unique_ptr<Slot>> slots;
  std::condition_variable cv_mem;  // a slot finished a batch (memory may have come free)
  uint64_t next_ticket = 1;
  uint32_t queue_cap = 65536;
  size_t pool = 0;                  // device bytes all slots' workspaces may hold together
  bool stopping = false;
  int device = 0;
  TuneTable tune;
  std::atomic<uint64_t> batches{0}, windows{0};
};

}  // namespace apo

namespace apo {
// A captured batch launch sequence and the shape it was captured for.
struct GraphCache {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const void *tok = nullptr;
  uint64_t total = 0, maxwin = 0;
  uint32_t W = 0, min_len = 0;
  int tile = 0, digit = 0;
  void *mem = nullptr;
  hipStream_t stream = nullptr;
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};
}  // namespace apo

namespace apo {
// Batches on several lanes captured as one graph: every lane's sync-free
// launch sequence is a branch forked from and joined back into the caller's
// stream.  Keyed on the token pointer, min_len, and per lane (first token,
// tokens, windows, longest window, kernel parameters, workspace).
struct LaneGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uint64_t> key;
  std::vector<hipEvent_t> ev;  // fork event + one join event per lane
  void reset() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
};
}  // namespace apo

struct apo_ctx {
  int device = 0;
  size_t budget = 0;
  hipStream_t stream = nullptr;
  apo::Workspace ws;
  apo::RunInfo info;
  apo::TuneTable tune;
  apo::GraphCache gc;
  apo::LaneGraph lg;
  bool graphs = true;         // capture/replay batched launch sequences
  bool lane_graphs = true;    // lanes as branches of one graph (off after a failed capture)
  int sel_cap = apo::kSelRoundCap;  // host-driven selection rounds before the sequential completion
  int sel_prefix = -1;              // exact prefix walk before the selection rounds (-1 automatic)
  bool win_greedy = true;           // per-window greedy where windows are short enough
  uint64_t graph_replays = 0, graph_captures = 0;
  std::unique_ptr<apo::Server> server;
  // Batches are split into `lanes` groups of windows, each analysed on its
  // own stream and workspace concurrently (lane 0: ws and the caller's stream).
  int lanes = 3;
  std::vector<std::unique_ptr<apo::Workspace>> lane_ws;
  std::vector<hipStream_t> lane_stream;
  hipEvent_t lane_ready = nullptr;
  // where the last batch's rows are: workspace, windows, rows (in window order)
  struct LaneOut {
    apo::Workspace *ws;
    uint32_t W, rows;
  };
  std::vector<LaneOut> louts;
};

namespace apo {
// noalloc.hip: the fixed per-device workspace of apo_analyze_window_noalloc
int noalloc_setup(int device);
int noalloc_run(int device, hipStream_t s, int tile_log, int digit_bits, const void *d_tok, int bits, uint32_t n,
                uint32_t min_len, apo_candidate *d_out, uint32_t out_cap, uint32_t *h_out_n, apo_occurrence *d_occ,
                uint32_t occ_cap, uint32_t *h_occ_n, RunInfo &info);
}  // namespace apo

using namespace apo;

static int set_dev(apo_ctx *c) { return hipSetDevice(c->device) == hipSuccess ? APO_OK : APO_EDEVICE; }

extern "C" const char *apo_strerror(int code) {
  switch (code) {
    case APO_OK: return "ok";
    case APO_EINVAL: return "invalid argument";
    case APO_ENOMEM: return "out of device memory or over budget";
    case APO_ERANGE: return "output buffer too small";
    case APO_EDEVICE: return "device error";
    case APO_EAGAIN: return "try again (queue full or result not ready)";
    case APO_ENOTFOUND: return "unknown ticket";
    default: return "unknown error";
  }
}

extern "C" int apo_create(apo_ctx **out, int hip_device, size_t budget) {
  if (!out) return APO_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) {
    (void)hipGetLastError();
    return APO_EDEVICE;
  }
  auto *c = new apo_ctx();
  c->device = hip_device;
  c->budget = budget;
  if (hipSetDevice(hip_device) != hipSuccess || hipStreamCreate(&c->stream) != hipSuccess) {
    delete c;
    return APO_EDEVICE;
  }
  // once per device: the fixed workspace of the no-allocation entry point
  // (its outcome is reported by that entry point)
  (void)noalloc_setup(hip_device);
  *out = c;
  return APO_OK;
}

extern "C" int apo_server_stop(apo_ctx *ctx);

extern "C" int apo_destroy(apo_ctx *ctx) {
  if (!ctx) return APO_OK;
  (void)hipSetDevice(ctx->device);
  apo_server_stop(ctx);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->gc.reset();
  ctx->lg.reset();
  for (auto e : ctx->lg.ev) (void)hipEventDestroy(e);
  ctx->ws.release();
  for (auto &l : ctx->lane_ws) l->release();
  for (auto st : ctx->lane_stream) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  if (ctx->lane_ready) (void)hipEventDestroy(ctx->lane_ready);
  (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return APO_OK;
}

static int map_rc(int rc) {
  if (rc == 0) return APO_OK;
  if (rc == -2) return APO_ENOMEM;
  return APO_EDEVICE;
}

// ---- device memory budget of a context: the sum of the bytes its
// workspaces hold (the main one and the lane workspaces; the server's slots
// draw on their own pool) never exceeds ctx->budget when one is set.
static size_t ctx_held(const apo_ctx *c) {
  size_t b = c->ws.held();
  for (const auto &l : c->lane_ws) b += l->held();
  return b;
}

static void release_lanes_from(apo_ctx *c, size_t first) {
  for (size_t k = first; k < c->lane_ws.size(); k++) {
    (void)hipStreamSynchronize(c->lane_stream[k]);
    c->lane_ws[k]->release();
  }
}

// Grows w to (N, W) within the context's budget; idle lane workspaces give
// their memory back first when they are what stands in the way.
static size_t ctx_limit(const apo_ctx *c);

static int ctx_ensure(apo_ctx *c, Workspace &w, uint64_t N, uint32_t W) {
  if (c->budget) {
    const size_t after = w.bytes_after(N, W), limit = ctx_limit(c);
    if (ctx_held(c) - w.held() + after > limit) {
      if (&w == &c->ws) release_lanes_from(c, 0);
      if (ctx_held(c) - w.held() + after > limit) return -2;
    }
  }
  return w.ensure(N, W, 0);
}

// Runs one analysis on the context workspace, tokens already on the device.
static int run_ctx(apo_ctx *c, const void *d_tok, int bits, uint32_t n, uint32_t min_len, Stop stop,
                   hipStream_t s) {
  int rc = ctx_ensure(c, c->ws, n, 1);
  if (rc) return map_rc(rc);
  c->ws.sel_cap = c->sel_cap;
  c->ws.sel_prefix = c->sel_prefix;
  c->ws.win_greedy = c->win_greedy;
  const uint64_t off[2] = {0, n};
  int tl, db;
  c->tune.pick(n, tl, db);
  c->ws.eng.set_params(tl, db);
  rc = run_pipeline(c->ws, d_tok, bits, n, off, 1, min_len, stop, s, c->info);
  return map_rc(rc);
}

static int analyze_host(apo_ctx *ctx, const void *tokens, int bits, uint32_t n, uint32_t min_len,
                        apo_candidate *out, uint32_t out_cap, uint32_t *out_n, apo_occurrence *occ,
                        uint32_t occ_cap, uint32_t *occ_n) {
  if (!ctx || !out_n || (!tokens && n) || (!out && out_cap) || min_len == 0 || n > APO_MAX_N) return APO_EINVAL;
  if (occ && !occ_n) return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  *out_n = 0;
  if (occ_n) *occ_n = 0;
  ctx->info = RunInfo{};
  if (n < 2) return APO_OK;
  int rc = ctx_ensure(ctx, ctx->ws, n, 1);
  if (rc) return map_rc(rc);
  const size_t bytes = (size_t)n * (bits / 8);
  if (hipMemcpyAsync(ctx->ws.tok64, tokens, bytes, hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
    (void)hipGetLastError();
    return APO_EDEVICE;
  }
  rc = run_ctx(ctx, ctx->ws.tok64, bits, n, min_len, Stop::FULL, ctx->stream);
  if (rc) return rc;
  const uint32_t rows = ctx->info.rows, acc = ctx->info.accepted;
  *out_n = rows;
  if (occ_n) *occ_n = acc;
  if (rows > out_cap || (occ && acc > occ_cap)) return APO_ERANGE;
  if (rows && hipMemcpy(out, ctx->ws.rows, (size_t)rows * sizeof(apo_candidate), hipMemcpyDeviceToHost) != hipSuccess)
    return APO_EDEVICE;
  if (occ && acc &&
      hipMemcpy(occ, ctx->ws.occ, (size_t)acc * sizeof(apo_occurrence), hipMemcpyDeviceToHost) != hipSuccess)
    return APO_EDEVICE;
  return APO_OK;
}

extern "C" int apo_analyze_window(apo_ctx *ctx, const uint64_t *tokens, uint32_t n, uint32_t min_len,
                                  apo_candidate *out, uint32_t out_cap, uint32_t *out_n, apo_occurrence *occ,
                                  uint32_t occ_cap, uint32_t *occ_n) {
  return analyze_host(ctx, tokens, 64, n, min_len, out, out_cap, out_n, occ, occ_cap, occ_n);
}

extern "C" int apo_analyze_window_u32(apo_ctx *ctx, const uint32_t *tokens, uint32_t n, uint32_t min_len,
                                      apo_candidate *out, uint32_t out_cap, uint32_t *out_n, apo_occurrence *occ,
                                      uint32_t occ_cap, uint32_t *occ_n) {
  return analyze_host(ctx, tokens, 32, n, min_len, out, out_cap, out_n, occ, occ_cap, occ_n);
}

static hipStream_t pick_stream(apo_ctx *c, void *s) { return s ? static_cast<hipStream_t>(s) : c->stream; }

extern "C" int apo_analyze_window_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                                      uint32_t min_len, apo_candidate *d_out, uint32_t out_cap, uint32_t *h_out_n,
                                      apo_occurrence *d_occ, uint32_t occ_cap, uint32_t *h_occ_n, void *stream) {
  if (!ctx || !h_out_n || (!d_tokens && n) || (!d_out && out_cap) || min_len == 0 || n > APO_MAX_N ||
      (token_bits != 32 && token_bits != 64) || (d_occ && !h_occ_n))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  *h_out_n = 0;
  if (h_occ_n) *h_occ_n = 0;
  ctx->info = RunInfo{};
  if (n < 2) return APO_OK;
  hipStream_t s = pick_stream(ctx, stream);
  int rc = run_ctx(ctx, d_tokens, token_bits, n, min_len, Stop::FULL, s);
  if (rc) return rc;
  const uint32_t rows = ctx->info.rows, acc = ctx->info.accepted;
  *h_out_n = rows;
  if (h_occ_n) *h_occ_n = acc;
  if (rows > out_cap || (d_occ && acc > occ_cap)) return APO_ERANGE;
  if (rows && hipMemcpyAsync(d_out, ctx->ws.rows, (size_t)rows * 12, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return APO_EDEVICE;
  if (d_occ && acc && hipMemcpyAsync(d_occ, ctx->ws.occ, (size_t)acc * 12, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return APO_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_analyze_window_noalloc(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                                          uint32_t min_len, apo_candidate *d_out, uint32_t out_cap, uint32_t *h_out_n,
                                          apo_occurrence *d_occ, uint32_t occ_cap, uint32_t *h_occ_n, void *stream) {
  if (!ctx || !h_out_n || (!d_tokens && n) || (!d_out && out_cap) || min_len == 0 || n > APO_MAX_N ||
      (token_bits != 32 && token_bits != 64) || (d_occ && !h_occ_n))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  *h_out_n = 0;
  if (h_occ_n) *h_occ_n = 0;
  ctx->info = RunInfo{};
  if (n > APO_NOALLOC_MAX_N) return APO_ENOMEM;
  if (n < 2) return APO_OK;
  int tl, db;
  ctx->tune.pick(n, tl, db);
  return noalloc_run(ctx->device, pick_stream(ctx, stream), tl, db, d_tokens, token_bits, n, min_len, d_out, out_cap,
                     h_out_n, d_occ, occ_cap, h_occ_n, ctx->info);
}

static int check_offsets(const uint64_t *off, uint32_t W, uint64_t &total) {
  if (!off || W == 0) return APO_EINVAL;
  for (uint32_t w = 0; w < W; w++) {
    if (off[w + 1] < off[w]) return APO_EINVAL;
    if (off[w + 1] - off[w] > APO_MAX_N) return APO_EINVAL;
  }
  total = off[W] - off[0];
  if (total >= (1ull << 31)) return APO_EINVAL;
  return APO_OK;
}

// Sums what the per-lane runs counted (maxima for round counts).
static void merge_info(RunInfo &a, const RunInfo &b) {
  a.n += b.n;
  a.rounds = std::max(a.rounds, b.rounds);
  a.active_sum += b.active_sum;
  a.sigma += b.sigma;
  a.cands += b.cands;
  a.cands_dedup += b.cands_dedup;
  a.maxl = std::max(a.maxl, b.maxl);
  a.sel_rounds = std::max(a.sel_rounds, b.sel_rounds);
  a.sel_sequential |= b.sel_sequential;
  a.sel_prefix += b.sel_prefix;
  a.pair_windows += b.pair_windows;
  a.accepted += b.accepted;
  a.rows += b.rows;
  for (int k = 0; k < kStages; k++) a.stage_ms[k] = std::max(a.stage_ms[k], b.stage_ms[k]);
  a.k_launches += b.k_launches;
  a.k_elems += b.k_elems;
  a.k_ms += b.k_ms;
}

// Batch split into L groups of consecutive windows with about equal tokens,
// each run host-driven (exact launch sizes, loops stopped when done) on its
// own stream, workspace and host thread; the streams run concurrently, so one
// lane's host syncs and latency-bound kernels overlap the others' work.
// Results stay per lane (ctx->louts), in window order.
static void lane_groups(const uint64_t *off, uint32_t W, uint64_t total, int L, std::vector<uint32_t> &w0) {
  w0.assign(L + 1, W);
  w0[0] = 0;
  for (int g = 1; g < L; g++) {
    const uint64_t target = off[0] + total * (uint64_t)g / (uint64_t)L;
    const uint32_t w = (uint32_t)(std::lower_bound(off, off + W + 1, target) - off);
    w0[g] = std::max(std::min(w, W), w0[g - 1]);
  }
  // a group of windows without tokens (empty windows only) joins the group
  // with tokens before it (leading ones: the first such group after them):
  // an analysis of no tokens has nothing to launch or capture
  auto has_tokens = [&](int g) { return w0[g + 1] > w0[g] && off[w0[g + 1]] != off[w0[g]]; };
  int first = 0;
  while (first < L && !has_tokens(first)) first++;
  if (first < L)
    for (int k = 1; k <= first; k++) w0[k] = w0[0];
  int last = -1;
  for (int g = 0; g < L; g++) {
    if (w0[g + 1] == w0[g]) continue;
    if (off[w0[g + 1]] != off[w0[g]]) {
      last = g;
      continue;
    }
    if (last >= 0)
      for (int k = last + 1; k <= g; k++) w0[k] = w0[g + 1];
  }
}

// Device bytes the context would hold while running a batch on L lanes
// (lane 0 in ctx->ws, lane g in lane_ws[g-1]; lane workspaces beyond L-1
// keep what they hold).
static size_t lanes_footprint(const apo_ctx *ctx, const uint64_t *off, uint32_t W, uint64_t total, int L) {
  std::vector<uint32_t> w0;
  lane_groups(off, W, total, L, w0);
  size_t b = 0;
  for (int g = 0; g < L; g++) {
    if (w0[g + 1] == w0[g]) continue;
    const uint64_t n = std::max<uint64_t>(off[w0[g + 1]] - off[w0[g]], 2);
    const uint32_t wn = w0[g + 1] - w0[g];
    const Workspace *ws = g == 0 ? &ctx->ws : ((size_t)(g - 1) < ctx->lane_ws.size() ? ctx->lane_ws[g - 1].get() : nullptr);
    if (ws) {
      b += ws->bytes_after(n, wn);
    } else {
      Workspace fresh;
      b += fresh.bytes_after(n, wn);
    }
  }
  for (size_t k = (size_t)std::max(L - 1, 0); k < ctx->lane_ws.size(); k++) b += ctx->lane_ws[k]->held();
  return b;
}

static int batch_lanes(apo_ctx *ctx, const uint64_t *d_tok, const uint64_t *off, uint32_t W, uint32_t min_len,
                       hipStream_t s, uint64_t total, int L) {
  while ((int)ctx->lane_ws.size() < L - 1) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return APO_EDEVICE;
    ctx->lane_stream.push_back(st);
    ctx->lane_ws.emplace_back(new Workspace());
  }
  if (!ctx->lane_ready && hipEventCreateWithFlags(&ctx->lane_ready, hipEventDisableTiming) != hipSuccess)
    return APO_EDEVICE;
  // group g holds windows w0[g] .. w0[g+1]
  std::vector<uint32_t> w0;
  lane_groups(off, W, total, L, w0);
  // the tokens were written on the caller's stream
  if (hipEventRecord(ctx->lane_ready, s) != hipSuccess) return APO_EDEVICE;
  struct Lane {
    Workspace *ws;
    hipStream_t st;
    std::vector<uint64_t> norm;  // window offsets relative to the lane's first token
    uint64_t tok0, total;        // first token (relative to off[0]) and token count
    uint32_t W;
    RunInfo info;
  };
  std::vector<Lane> lanes;
  for (int g = 0; g < L; g++) {
    if (w0[g + 1] == w0[g]) continue;
    Lane ln;
    ln.ws = g == 0 ? &ctx->ws : ctx->lane_ws[g - 1].get();
    ln.st = g == 0 ? s : ctx->lane_stream[g - 1];
    ln.W = w0[g + 1] - w0[g];
    ln.tok0 = off[w0[g]] - off[0];
    ln.total = off[w0[g + 1]] - off[w0[g]];
    ln.norm.resize(ln.W + 1);
    for (uint32_t w = 0; w <= ln.W; w++) ln.norm[w] = off[w0[g] + w] - off[w0[g]];
    const int rc = ln.ws->ensure(std::max<uint64_t>(ln.total, 2), ln.W, 0);  // footprint checked by the caller
    if (rc) return map_rc(rc);
    int tl, db;
    ctx->tune.pick(ln.total, tl, db);
    ln.ws->eng.set_params(tl, db);
    ln.ws->ktag = ctx->ws.ktag;
    ln.ws->sel_cap = ctx->sel_cap;
    ln.ws->sel_prefix = ctx->sel_prefix;
    ln.ws->win_greedy = ctx->win_greedy;
    if (ln.st != s && hipStreamWaitEvent(ln.st, ctx->lane_ready, 0) != hipSuccess) return APO_EDEVICE;
    lanes.push_back(std::move(ln));
  }
  // With graphs on (and no kernel timing, which events inside a capture
  // cannot give), every lane's sync-free sequence is one branch of a single
  // graph, captured once per shape and replayed.
  if (ctx->graphs && ctx->lane_graphs && ctx->ws.ktag == KT_NONE) {
    std::vector<uint64_t> key = {(uint64_t)(uintptr_t)d_tok, min_len, lanes.size(), (uint64_t)ctx->win_greedy,
                                 (uint64_t)(uintptr_t)s};
    for (Lane &ln : lanes) {
      uint64_t mw = 0;
      for (uint32_t w = 0; w < ln.W; w++) mw = std::max<uint64_t>(mw, ln.norm[w + 1] - ln.norm[w]);
      key.insert(key.end(), {ln.tok0, ln.total, ln.W, mw, (uint64_t)ln.ws->eng.tile_log(),
                             (uint64_t)ln.ws->eng.digit_bits(), (uint64_t)(uintptr_t)ln.ws->mem,
                             (uint64_t)(uintptr_t)ln.st});
    }
    LaneGraph &G = ctx->lg;
    // window offsets (and order) of every lane, ahead of the branches that read them
    for (Lane &ln : lanes)
      if (upload_windows(*ln.ws, ln.norm.data(), ln.W, s, true)) return APO_EDEVICE;
    bool ok = true;
    if (!G.exec || G.key != key) {
      G.reset();
      while (G.ev.size() < lanes.size() + 1) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return APO_EDEVICE;
        G.ev.push_back(e);
      }
      ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
      hipGraph_t g = nullptr;
      if (ok) {
        int rc = hipEventRecord(G.ev[0], s) == hipSuccess ? 0 : -4;
        for (size_t i = 0; i < lanes.size() && !rc; i++)
          if (lanes[i].st != s && hipStreamWaitEvent(lanes[i].st, G.ev[0], 0) != hipSuccess) rc = -4;
        for (size_t i = 0; i < lanes.size() && !rc; i++) {
          Lane &ln = lanes[i];
          rc = run_pipeline(*ln.ws, d_tok + ln.tok0, 64, ln.total, ln.norm.data(), ln.W, min_len, Stop::FULL, ln.st,
                            ln.info, Mode::CAPTURE);
        }
        // every lane stream joins back, also after a failure, so that ending
        // the capture releases all of them
        for (size_t i = 0; i < lanes.size(); i++)
          if (lanes[i].st != s && (hipEventRecord(G.ev[i + 1], lanes[i].st) != hipSuccess ||
                                   hipStreamWaitEvent(s, G.ev[i + 1], 0) != hipSuccess))
            rc = -4;
        const hipError_t e = hipStreamEndCapture(s, &g);
        ok = rc == 0 && e == hipSuccess && g != nullptr;
        for (size_t i = 0; i < lanes.size(); i++) {  // a stream the failed capture left capturing ends it
          hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
          if (lanes[i].st != s && hipStreamIsCapturing(lanes[i].st, &cs) == hipSuccess &&
              cs != hipStreamCaptureStatusNone) {
            hipGraph_t lg = nullptr;
            (void)hipStreamEndCapture(lanes[i].st, &lg);
            if (lg) (void)hipGraphDestroy(lg);
            ok = false;
          }
        }
        if (ok && hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0) != hipSuccess) {
          G.exec = nullptr;
          ok = false;
        }
      }
      if (ok) {
        G.graph = g;
        G.key = key;
        ctx->graph_captures++;
      } else {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        fprintf(stderr, "[apo] capture of the lanes failed; lanes run host-driven\n");
        ctx->lane_graphs = false;
      }
    } else {
      ctx->graph_replays++;
    }
    if (ok) {
      if (hipGraphLaunch(G.exec, s) != hipSuccess) return APO_EDEVICE;
      ctx->info = RunInfo{};
      ctx->louts.clear();
      for (Lane &ln : lanes) {
        ln.info = RunInfo{};
        ln.ws->kev_n = 0;
        int rc = finish_run(*ln.ws, ln.total, 2 * ln.total, kSelFreeRounds, ln.info, s, false);
        if (rc == 1)  // greedy rounds left candidates undecided: this lane again, host-driven
          rc = run_pipeline(*ln.ws, d_tok + ln.tok0, 64, ln.total, ln.norm.data(), ln.W, min_len, Stop::FULL, s,
                            ln.info, Mode::HOST);
        if (rc) return map_rc(rc);
        merge_info(ctx->info, ln.info);
        ctx->louts.push_back({ln.ws, ln.W, ln.info.rows});
      }
      return APO_OK;
    }
  }
  // one host thread per lane, so that no lane's launches wait behind another
  // lane's syncs
  std::vector<int> erc(lanes.size(), 0);
  {
    std::vector<std::thread> th;
    for (size_t i = 1; i < lanes.size(); i++)
      th.emplace_back([&, i] {
        Lane &ln = lanes[i];
        if (hipSetDevice(ctx->device) != hipSuccess) { erc[i] = -4; return; }
        erc[i] = run_pipeline(*ln.ws, d_tok + ln.tok0, 64, ln.total, ln.norm.data(), ln.W, min_len, Stop::FULL,
                              ln.st, ln.info, Mode::HOST);
      });
    Lane &l0 = lanes[0];
    erc[0] = run_pipeline(*l0.ws, d_tok + l0.tok0, 64, l0.total, l0.norm.data(), l0.W, min_len, Stop::FULL, l0.st,
                          l0.info, Mode::HOST);
    for (auto &t : th) t.join();
  }
  for (int rc : erc)
    if (rc) return map_rc(rc);
  ctx->info = RunInfo{};
  ctx->louts.clear();
  for (Lane &ln : lanes) {
    merge_info(ctx->info, ln.info);
    ctx->louts.push_back({ln.ws, ln.W, ln.info.rows});
  }
  return APO_OK;
}

// One batched analysis of device tokens.  The launch sequence is sync-free;
// with graphs enabled it is captured once per shape and replayed.  If the
// enqueued selection rounds did not decide every candidate (adversarial
// inputs), the batch is rerun host-driven.
static int batch_single(apo_ctx *ctx, const uint64_t *d_tok, const uint64_t *off, uint32_t W, uint32_t min_len,
                        hipStream_t s, uint64_t total);

static int batch_common(apo_ctx *ctx, const uint64_t *d_tok, const uint64_t *off, uint32_t W, uint32_t min_len,
                        hipStream_t s, uint64_t total) {
  int L = std::min<int>(ctx->lanes, (int)(W / 2));
  if (ctx->budget && L >= 2) {
    // fewer lanes when their workspaces would not fit the budget; lane
    // workspaces left idle by the smaller count give their memory back
    while (L >= 2 && lanes_footprint(ctx, off, W, total, L) > ctx_limit(ctx)) {
      release_lanes_from(ctx, (size_t)(L - 1));
      if (lanes_footprint(ctx, off, W, total, L) <= ctx_limit(ctx)) break;
      L--;
    }
  }
  if (L >= 2) return batch_lanes(ctx, d_tok, off, W, min_len, s, total, L);
  const int rc = batch_single(ctx, d_tok, off, W, min_len, s, total);
  ctx->louts.assign(1, {&ctx->ws, W, ctx->info.rows});
  return rc;
}

static int batch_single(apo_ctx *ctx, const uint64_t *d_tok, const uint64_t *off, uint32_t W, uint32_t min_len,
                        hipStream_t s, uint64_t total) {
  std::vector<uint64_t> norm(W + 1);
  uint64_t maxwin = 0;
  for (uint32_t w = 0; w <= W; w++) norm[w] = off[w] - off[0];
  for (uint32_t w = 0; w < W; w++) maxwin = std::max<uint64_t>(maxwin, norm[w + 1] - norm[w]);
  int rc = ctx_ensure(ctx, ctx->ws, std::max<uint64_t>(total, 2), W);
  if (rc) return map_rc(rc);
  int tl, db;
  ctx->tune.pick(total, tl, db);
  ctx->ws.eng.set_params(tl, db);
  Workspace &w = ctx->ws;
  w.sel_cap = ctx->sel_cap;
  w.sel_prefix = ctx->sel_prefix;
  if (w.win_greedy != ctx->win_greedy) ctx->gc.reset();  // a captured sequence holds the other selection path
  w.win_greedy = ctx->win_greedy;
  // Timed kernel launches are bracketed by events on the stream, which is
  // only reliable outside captured graphs: profiling runs the same sync-free
  // sequence without capture.
  if (!ctx->graphs || w.ktag != 0) {
    rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::FREE);
    if (rc == 1) rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::HOST);
    return map_rc(rc);
  }
  GraphCache &G = ctx->gc;
  const bool hit = G.exec && G.tok == d_tok && G.total == total && G.W == W && G.maxwin == maxwin &&
                   G.min_len == min_len && G.tile == tl && G.digit == db && G.mem == w.mem && G.stream == s;
  if (upload_windows(w, norm.data(), W, s, true) || hipStreamSynchronize(s) != hipSuccess) return APO_EDEVICE;
  if (!hit) {
    G.reset();
    bool ok = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess;
    hipGraph_t g = nullptr;
    if (ok) {
      rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::CAPTURE);
      const hipError_t e = hipStreamEndCapture(s, &g);
      ok = rc == 0 && e == hipSuccess && g != nullptr;
      if (ok && hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0) != hipSuccess) {
        G.exec = nullptr;
        ok = false;
      }
    }
    if (!ok) {
      // capture unavailable: run the same sync-free sequence directly from now on
      if (g) (void)hipGraphDestroy(g);
      (void)hipGetLastError();
      fprintf(stderr, "[apo] graph capture failed; batches run without graphs\n");
      ctx->graphs = false;
      rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::FREE);
      if (rc == 1) rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::HOST);
      return map_rc(rc);
    }
    G.graph = g;
    G.tok = d_tok;
    G.total = total;
    G.W = W;
    G.maxwin = maxwin;
    G.min_len = min_len;
    G.tile = tl;
    G.digit = db;
    G.mem = w.mem;
    G.stream = s;
    ctx->graph_captures++;
  } else {
    ctx->graph_replays++;
  }
  w.kev_n = 0;
  if (hipGraphLaunch(G.exec, s) != hipSuccess) return APO_EDEVICE;
  ctx->info = RunInfo{};
  rc = finish_run(w, total, 2 * total, kSelFreeRounds, ctx->info, s, false);
  if (rc == 1) rc = run_pipeline(w, d_tok, 64, total, norm.data(), W, min_len, Stop::FULL, s, ctx->info, Mode::HOST);
  return map_rc(rc);
}

static int batch_offsets(apo_ctx *ctx, uint32_t W, uint64_t *out_offsets, uint64_t out_cap) {
  std::vector<uint32_t> cnt;
  cnt.reserve(W);
  for (const auto &lo : ctx->louts) {
    std::vector<uint32_t> c(lo.W, 0);
    if (lo.W > 1 && lo.rows) {
      if (hipMemcpy(c.data(), lo.ws->win_rows, lo.W * 4, hipMemcpyDeviceToHost) != hipSuccess) return APO_EDEVICE;
    } else if (lo.W == 1) {
      c[0] = lo.rows;
    }
    cnt.insert(cnt.end(), c.begin(), c.end());
  }
  if (cnt.size() != W) return APO_EDEVICE;
  out_offsets[0] = 0;
  for (uint32_t w = 0; w < W; w++) out_offsets[w + 1] = out_offsets[w] + cnt[w];
  return ctx->info.rows > out_cap ? APO_ERANGE : APO_OK;
}

// Copies the rows of every lane, in window order, to `out` (device or host).
static int batch_rows(apo_ctx *ctx, apo_candidate *out, bool to_host, hipStream_t s) {
  uint64_t at = 0;
  for (const auto &lo : ctx->louts) {
    if (lo.rows) {
      const size_t bytes = (size_t)lo.rows * sizeof(apo_candidate);
      const hipError_t e = to_host ? hipMemcpy(out + at, lo.ws->rows, bytes, hipMemcpyDeviceToHost)
                                   : hipMemcpyAsync(out + at, lo.ws->rows, bytes, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return APO_EDEVICE;
    }
    at += lo.rows;
  }
  return APO_OK;
}

extern "C" int apo_analyze_batch(apo_ctx *ctx, const uint64_t *tokens, const uint64_t *offsets, uint32_t W,
                                 uint32_t min_len, apo_candidate *out, uint64_t out_cap, uint64_t *out_offsets) {
  if (!ctx || !out_offsets || min_len == 0 || (!out && out_cap)) return APO_EINVAL;
  uint64_t total = 0;
  int rc = check_offsets(offsets, W, total);
  if (rc) return rc;
  if (total && !tokens) return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  ctx->info = RunInfo{};
  if (total < 2) {
    for (uint32_t w = 0; w <= W; w++) out_offsets[w] = 0;
    return APO_OK;
  }
  rc = ctx_ensure(ctx, ctx->ws, total, W);
  if (rc) return map_rc(rc);
  if (hipMemcpyAsync(ctx->ws.tok64, tokens + offsets[0], total * 8, hipMemcpyHostToDevice, ctx->stream) !=
      hipSuccess)
    return APO_EDEVICE;
  rc = batch_common(ctx, ctx->ws.tok64, offsets, W, min_len, ctx->stream, total);
  if (rc) return rc;
  rc = batch_offsets(ctx, W, out_offsets, out_cap);
  if (rc) return rc;
  return batch_rows(ctx, out, true, ctx->stream);
}

extern "C" int apo_analyze_batch_dev(apo_ctx *ctx, const uint64_t *d_tokens, const uint64_t *h_offsets, uint32_t W,
                                     uint32_t min_len, apo_candidate *d_out, uint64_t out_cap,
                                     uint64_t *h_out_offsets, void *stream) {
  if (!ctx || !h_out_offsets || min_len == 0 || (!d_out && out_cap)) return APO_EINVAL;
  uint64_t total = 0;
  int rc = check_offsets(h_offsets, W, total);
  if (rc) return rc;
  if (total && !d_tokens) return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  ctx->info = RunInfo{};
  if (total < 2) {
    for (uint32_t w = 0; w <= W; w++) h_out_offsets[w] = 0;
    return APO_OK;
  }
  hipStream_t s = pick_stream(ctx, stream);
  rc = batch_common(ctx, d_tokens + h_offsets[0], h_offsets, W, min_len, s, total);
  if (rc) return rc;
  rc = batch_offsets(ctx, W, h_out_offsets, out_cap);
  if (rc) return rc;
  rc = batch_rows(ctx, d_out, false, s);
  if (rc) return rc;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_suffix_array_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t *d_sa,
                                    uint32_t *h_rounds, void *stream) {
  if (!ctx || !d_tokens || !d_sa || n == 0 || n > APO_MAX_N || (token_bits != 32 && token_bits != 64))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  hipStream_t s = pick_stream(ctx, stream);
  int rc = run_ctx(ctx, d_tokens, token_bits, n, 1, Stop::SA, s);
  if (rc) return rc;
  if (h_rounds) *h_rounds = ctx->info.rounds;
  if (hipMemcpyAsync(d_sa, ctx->ws.sa, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) return APO_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_lcp_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t *d_sa,
                           uint32_t *d_lcp, void *stream) {
  if (!ctx || !d_tokens || !d_lcp || n == 0 || n > APO_MAX_N || (token_bits != 32 && token_bits != 64))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  hipStream_t s = pick_stream(ctx, stream);
  int rc = run_ctx(ctx, d_tokens, token_bits, n, 1, Stop::LCP, s);
  if (rc) return rc;
  if (d_sa && hipMemcpyAsync(d_sa, ctx->ws.sa, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return APO_EDEVICE;
  if (hipMemcpyAsync(d_lcp, ctx->ws.lcp, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
    return APO_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_candidates_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t min_len,
                                  uint32_t *d_len, uint32_t *d_start, uint32_t *d_id, uint32_t cap, uint32_t *h_count,
                                  void *stream) {
  if (!ctx || !d_tokens || !h_count || min_len == 0 || n == 0 || n > APO_MAX_N ||
      (token_bits != 32 && token_bits != 64) || ((!d_len || !d_start || !d_id) && cap))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  *h_count = 0;
  if (n < 2) return APO_OK;
  hipStream_t s = pick_stream(ctx, stream);
  int rc = run_ctx(ctx, d_tokens, token_bits, n, min_len, Stop::CANDS, s);
  if (rc) return rc;
  const uint32_t m = ctx->info.cands_dedup;
  *h_count = m;
  if (m > cap) return APO_ERANGE;
  if (m) {
    if (hipMemcpyAsync(d_len, ctx->ws.s_len, (size_t)m * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_start, ctx->ws.s_start, (size_t)m * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(d_id, ctx->ws.s_id, (size_t)m * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return APO_EDEVICE;
  }
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_interval_counts_dev(apo_ctx *ctx, const uint32_t *d_len, const uint32_t *d_start,
                                       const uint32_t *d_id, uint32_t m, uint32_t *d_next, uint32_t *d_count,
                                       uint32_t *d_tmp, void *stream) {
  if (!ctx || (m && (!d_len || !d_start || !d_id || !d_next || !d_count || !d_tmp)) || m > 2u * APO_MAX_N)
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  if (m == 0) return APO_OK;
  hipStream_t s = pick_stream(ctx, stream);
  apo::interval_counts(d_len, d_start, d_id, m, d_next, d_count, d_tmp, s);
  if (hipGetLastError() != hipSuccess) return APO_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? APO_OK : APO_EDEVICE;
}

extern "C" int apo_last_stage_ms(apo_ctx *ctx, double *ms, int nstages) {
  if (!ctx || !ms || nstages < 0) return APO_EINVAL;
  const int k = std::min(nstages, kStages);
  for (int i = 0; i < k; i++) ms[i] = ctx->info.stage_ms[i];
  return k;
}

extern "C" int apo_last_counters(apo_ctx *ctx, uint64_t *v, int nvals) {
  if (!ctx || !v || nvals < 0) return APO_EINVAL;
  const RunInfo &I = ctx->info;
  const uint64_t all[11] = {I.rounds,     I.cands,          I.cands_dedup, I.sel_rounds,
                            I.accepted,   I.rows,           I.active_sum,  I.sigma,
                            I.sel_sequential, I.sel_prefix, I.pair_windows};
  const int k = std::min(nvals, 11);
  for (int i = 0; i < k; i++) v[i] = all[i];
  return k;
}

extern "C" size_t apo_workspace_bytes(uint64_t n, uint32_t windows) {
  if (n > APO_MAX_N || windows == 0) return 0;
  Workspace fresh;
  return fresh.bytes_after(std::max<uint64_t>(n, 2), windows);
}

extern "C" int apo_inject_device_error(apo_ctx *ctx, int after_syncs) {
  if (!ctx || after_syncs < -1) return APO_EINVAL;
  ctx->ws.fail_after = after_syncs;
  return APO_OK;
}

extern "C" int apo_memory(apo_ctx *ctx, size_t *held, size_t *server_pool, size_t *server_held) {
  if (!ctx || !held) return APO_EINVAL;
  *held = ctx_held(ctx);
  size_t pool = 0, sh = 0;
  if (ctx->server) {
    std::lock_guard<std::mutex> lk(ctx->server->mu);
    pool = ctx->server->pool;
    for (const auto &sl : ctx->server->slots) sh += sl->held;  // an upper bound while a batch grows it
  }
  if (server_pool) *server_pool = pool;
  if (server_held) *server_held = sh;
  return APO_OK;
}

extern "C" int apo_set_window_greedy(apo_ctx *ctx, int on) {
  if (!ctx || on < 0 || on > 1) return APO_EINVAL;
  ctx->win_greedy = on != 0;
  return APO_OK;
}

extern "C" int apo_set_selection_round_cap(apo_ctx *ctx, int rounds) {
  if (!ctx || rounds < 0 || rounds > kSelRoundCap) return APO_EINVAL;
  ctx->sel_cap = rounds;
  return APO_OK;
}

extern "C" int apo_set_selection_prefix(apo_ctx *ctx, int k) {
  if (!ctx || k < -1) return APO_EINVAL;
  ctx->sel_prefix = k;
  return APO_OK;
}

extern "C" int apo_set_lanes(apo_ctx *ctx, int lanes) {
  if (!ctx || lanes < 1 || lanes > 4) return APO_EINVAL;
  ctx->lanes = lanes;
  return APO_OK;
}

extern "C" int apo_set_graphs(apo_ctx *ctx, int on) {
  if (!ctx) return APO_EINVAL;
  ctx->graphs = on != 0;
  if (!ctx->graphs) {
    ctx->gc.reset();
    ctx->lg.reset();
  }
  return APO_OK;
}

extern "C" int apo_graph_stats(apo_ctx *ctx, uint64_t *captures, uint64_t *replays) {
  if (!ctx || !captures || !replays) return APO_EINVAL;
  *captures = ctx->graph_captures;
  *replays = ctx->graph_replays;
  return APO_OK;
}

extern "C" int apo_profile_kernel(apo_ctx *ctx, int tag) {
  if (!ctx || tag < KT_NONE || tag > KT_LDS_SA) return APO_EINVAL;
  ctx->ws.ktag = tag;
  return APO_OK;
}

extern "C" int apo_last_kernel_profile(apo_ctx *ctx, uint64_t *launches, double *total_ms, uint64_t *elems) {
  if (!ctx || !launches || !total_ms || !elems) return APO_EINVAL;
  *launches = ctx->info.k_launches;
  *total_ms = ctx->info.k_ms;
  *elems = ctx->info.k_elems;
  return APO_OK;
}

extern "C" int apo_last_rounds(apo_ctx *ctx, uint32_t *sa_active, uint32_t *n_sa, uint32_t *sel_live,
                               uint32_t *sel_undecided, uint32_t *n_sel, uint32_t cap) {
  if (!ctx || !n_sa || !n_sel || (cap && (!sa_active || !sel_live || !sel_undecided))) return APO_EINVAL;
  const Workspace &w = ctx->ws;
  const RunInfo &I = ctx->info;
  *n_sa = I.rounds;
  *n_sel = I.sel_rounds;
  if (!w.hrhist || !w.hsel) {
    *n_sa = *n_sel = 0;
    return APO_OK;
  }
  for (uint32_t r = 0; r < I.rounds && r < cap; r++)
    sa_active[r] = r == 0 ? (uint32_t)ctx->info.n : w.hrhist[4 * (r - 1)];
  for (uint32_t q = 0; q < I.sel_rounds && q < cap && q < (uint32_t)kSelRoundCap; q++) {
    sel_live[q] = w.hsel[q];
    sel_undecided[q] = w.hsel[q + 1];  // undecided after round q = live entering round q + 1
  }
  return (I.rounds > cap || I.sel_rounds > cap) ? APO_ERANGE : APO_OK;
}

// ================================================================== autotuner
// Times every (LDS tile, digit width) pair on the caller's window and keeps the
// fastest for the window's size bucket.  Results never depend on the choice.
// Batch tuning: times every pair on the caller's whole batch (as
// apo_analyze_batch_dev runs it, lanes included) and keeps the fastest for the
// size bucket of one lane's share.  Results never depend on the choice.
static int batch_common(apo_ctx *ctx, const uint64_t *d_tok, const uint64_t *off, uint32_t W, uint32_t min_len,
                        hipStream_t s, uint64_t total);

extern "C" int apo_tune_batch(apo_ctx *ctx, const uint64_t *d_tokens, const uint64_t *h_offsets, uint32_t W,
                              uint32_t min_len, int reps, int *best_tile_log, int *best_digit_bits, double *best_ms) {
  if (!ctx || !d_tokens || min_len == 0) return APO_EINVAL;
  uint64_t total = 0;
  int rc = check_offsets(h_offsets, W, total);
  if (rc) return rc;
  if (total < 2) return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  reps = std::max(1, std::min(reps, 50));
  const int keep_t = ctx->tune.fixed_tile, keep_d = ctx->tune.fixed_digit;
  double best = 1e30;
  int bt = kDefaultTileLog, bd = kDefaultDigitBits;
  for (int tl = kMinTileLog; tl <= kMaxTileLog && rc == APO_OK; tl++) {
    for (int db : {8, 10, 11, 12}) {
      ctx->tune.fixed_tile = tl;
      ctx->tune.fixed_digit = db;
      std::vector<double> t;
      for (int k = 0; k <= reps; k++) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = batch_common(ctx, d_tokens + h_offsets[0], h_offsets, W, min_len, ctx->stream, total);
        if (rc) break;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (k > 0) t.push_back(ms);
      }
      if (rc) break;
      std::sort(t.begin(), t.end());
      const double med = t[t.size() / 2];
      if (med < best) { best = med; bt = tl; bd = db; }
    }
  }
  ctx->tune.fixed_tile = keep_t;
  ctx->tune.fixed_digit = keep_d;
  if (rc) return rc;
  const int L = std::max(1, std::min<int>(ctx->lanes, (int)(W / 2)));
  ctx->tune.best[ceil_log2_u64(std::max<uint64_t>(total / L, 2))] = {bt, bd};
  if (best_tile_log) *best_tile_log = bt;
  if (best_digit_bits) *best_digit_bits = bd;
  if (best_ms) *best_ms = best;
  return APO_OK;
}

extern "C" int apo_tune(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t min_len, int reps,
                        int *best_tile_log, int *best_digit_bits, double *best_ms) {
  if (!ctx || !d_tokens || n < 2 || n > APO_MAX_N || min_len == 0 || (token_bits != 32 && token_bits != 64))
    return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  reps = std::max(1, std::min(reps, 50));
  int rc = ctx_ensure(ctx, ctx->ws, n, 1);
  if (rc) return map_rc(rc);
  const uint64_t off[2] = {0, n};
  double best = 1e30;
  int bt = kDefaultTileLog, bd = kDefaultDigitBits;
  for (int tl = kMinTileLog; tl <= kMaxTileLog; tl++) {
    for (int db : {8, 10, 11, 12}) {
      ctx->ws.eng.set_params(tl, db);
      std::vector<double> t;
      for (int k = 0; k <= reps; k++) {
        const auto t0 = std::chrono::steady_clock::now();
        rc = map_rc(run_pipeline(ctx->ws, d_tokens, token_bits, n, off, 1, min_len, Stop::FULL, ctx->stream,
                                 ctx->info));
        if (rc) return rc;
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (k > 0) t.push_back(ms);
      }
      std::sort(t.begin(), t.end());
      const double med = t[t.size() / 2];
      if (med < best) { best = med; bt = tl; bd = db; }
    }
  }
  ctx->tune.best[ceil_log2_u64(n)] = {bt, bd};
  if (best_tile_log) *best_tile_log = bt;
  if (best_digit_bits) *best_digit_bits = bd;
  if (best_ms) *best_ms = best;
  return APO_OK;
}

extern "C" int apo_set_params(apo_ctx *ctx, int tile_log, int digit_bits) {
  if (!ctx) return APO_EINVAL;
  if (tile_log < 0 || digit_bits < 0) {
    ctx->tune.fixed_tile = ctx->tune.fixed_digit = -1;
    return APO_OK;
  }
  if (tile_log < kMinTileLog || tile_log > kMaxTileLog || digit_bits < kMinDigitBits || digit_bits > kMaxDigitBits)
    return APO_EINVAL;
  ctx->tune.fixed_tile = tile_log;
  ctx->tune.fixed_digit = digit_bits;
  return APO_OK;
}

extern "C" int apo_tune_save(apo_ctx *ctx, const char *path) {
  if (!ctx || !path) return APO_EINVAL;
  FILE *f = fopen(path, "w");
  if (!f) return APO_EINVAL;
  fprintf(f, "# log2n tile_log digit_bits\n");
  for (auto &kv : ctx->tune.best) fprintf(f, "%d %d %d\n", kv.first, kv.second.first, kv.second.second);
  fclose(f);
  return APO_OK;
}

extern "C" int apo_tune_load(apo_ctx *ctx, const char *path) {
  if (!ctx || !path) return APO_EINVAL;
  FILE *f = fopen(path, "r");
  if (!f) return APO_EINVAL;
  char line[256];
  TuneTable t = ctx->tune;
  t.best.clear();
  while (fgets(line, sizeof line, f)) {
    int b, tl, db;
    if (line[0] == '#') continue;
    if (sscanf(line, "%d %d %d", &b, &tl, &db) == 3 && b >= 1 && b <= 40 && tl >= kMinTileLog &&
        tl <= kMaxTileLog && db >= kMinDigitBits && db <= kMaxDigitBits)
      t.best[b] = {tl, db};
  }
  fclose(f);
  ctx->tune = t;
  return APO_OK;
}

// ===================================================================== server
// Each slot owns a resident workspace and stream.  Admission is by device
// memory: the slots' workspaces together may hold at most the server's pool
// (the context budget, or most of the device memory free at start).  A free
// slot takes the oldest queued request and every later one with the same
// min_len while the grown workspace of the packed batch still fits beside
// what the other slots hold; idle slots hand their workspaces back when a
// batch needs the room, and a batch that does not fit waits (queued) until a
// busy slot finishes.  Windows never interact, so a packed batch gives every
// window its own result.  Slots run concurrently on their streams: requests
// arriving while others are on the GPU are admitted as soon as a slot and
// memory free up, and their work overlaps on the device.

// Device bytes a workspace would hold after growing for `total` tokens in W windows.
static size_t slot_footprint(const Slot *sl, uint64_t total, uint32_t W) {
  return sl->ws.bytes_after(std::max<uint64_t>(total, 2), W);
}

static size_t others_held(const Server *S, const Slot *me) {
  size_t b = 0;
  for (const auto &o : S->slots)
    if (o.get() != me) b += o->held;
  return b;
}

// Under S->mu: frees the workspaces of idle slots (their streams are idle).
static void release_idle_slots(Server *S, Slot *me) {
  for (auto &o : S->slots) {
    if (o.get() == me || o->busy || o->held == 0) continue;
    o->ws.release();
    o->held = 0;
  }
}

// Under S->mu: moves the requests of the next batch from the queue into
// `batch`; returns false when even the oldest request does not fit yet.
static bool take_batch(Server *S, Slot *sl, std::vector<std::shared_ptr<Request>> &batch, size_t &reserve) {
  const uint32_t ml = S->queue.front()->min_len;
  for (int attempt = 0; attempt < 2; attempt++) {
    const size_t avail = S->pool > others_held(S, sl) ? S->pool - others_held(S, sl) : 0;
    uint64_t tot = 0;
    uint32_t W = 0;
    for (auto it = S->queue.begin(); it != S->queue.end();) {
      const uint64_t n = (*it)->tokens.size();
      size_t need;
      if ((*it)->min_len == ml && (need = slot_footprint(sl, tot + n, W + 1)) <= avail) {
        tot += n;
        W++;
        reserve = need;
        batch.push_back(*it);
        it = S->queue.erase(it);
      } else if (batch.empty()) {
        break;  // the oldest request comes first: never overtaken by later ones
      } else {
        ++it;
      }
    }
    if (!batch.empty()) return true;
    release_idle_slots(S, sl);  // make room, then try once more
  }
  return false;
}

static void slot_loop(Server *S, Slot *sl) {
  (void)hipSetDevice(S->device);
  std::vector<std::shared_ptr<Request>> batch;
  std::vector<uint64_t> off;
  std::vector<uint64_t> outoff;
  std::vector<apo_candidate> rows;
  RunInfo info;
  while (true) {
    batch.clear();
    {
      std::unique_lock<std::mutex> lk(S->mu);
      size_t reserve = 0;
      while (true) {
        S->cv_work.wait(lk, [&] { return S->stopping || !S->queue.empty(); });
        if (S->queue.empty() && S->stopping) return;
        if (take_batch(S, sl, batch, reserve)) break;
        // not enough device memory while other slots run: wait for one to finish
        S->cv_mem.wait(lk);
      }
      sl->busy = true;
      sl->held = std::max(sl->held, reserve);
    }
    const uint32_t W = (uint32_t)batch.size();
    off.assign(W + 1, 0);
    for (uint32_t w = 0; w < W; w++) off[w + 1] = off[w] + batch[w]->tokens.size();
    const uint64_t total = off[W];
    int rc = 0;
    if (total > sl->pinned_cap) {
      if (sl->pinned) (void)hipHostFree(sl->pinned);
      sl->pinned = nullptr;
      sl->pinned_cap = 0;
      uint64_t cap = 1;
      while (cap < total) cap <<= 1;
      if (hipHostMalloc((void **)&sl->pinned, cap * 8, hipHostMallocDefault) == hipSuccess) sl->pinned_cap = cap;
      else rc = APO_ENOMEM;
    }
    if (!rc) {
      for (uint32_t w = 0; w < W; w++)
        if (!batch[w]->tokens.empty())
          memcpy(sl->pinned + off[w], batch[w]->tokens.data(), batch[w]->tokens.size() * 8);
      rc = map_rc(sl->ws.ensure(std::max<uint64_t>(total, 2), W, 0));  // admitted against the pool above
    }
    outoff.assign(W + 1, 0);
    if (!rc && total >= 2) {
      if (hipMemcpyAsync(sl->ws.tok64, sl->pinned, total * 8, hipMemcpyHostToDevice, sl->stream) != hipSuccess)
        rc = APO_EDEVICE;
      if (!rc) {
        int tl, db;
        S->tune.pick(total, tl, db);
        sl->ws.eng.set_params(tl, db);
        rc = map_rc(run_pipeline(sl->ws, sl->ws.tok64, 64, total, off.data(), W, batch[0]->min_len, Stop::FULL,
                                 sl->stream, info));
      }
      if (!rc) {
        std::vector<uint32_t> cnt(W, 0);
        if (W > 1 && info.rows) {
          if (hipMemcpy(cnt.data(), sl->ws.win_rows, W * 4, hipMemcpyDeviceToHost) != hipSuccess) rc = APO_EDEVICE;
        } else if (W == 1) {
          cnt[0] = info.rows;
        }
        for (uint32_t w = 0; w < W; w++) outoff[w + 1] = outoff[w] + cnt[w];
        rows.resize(info.rows);
        if (!rc && info.rows &&
            hipMemcpy(rows.data(), sl->ws.rows, (size_t)info.rows * sizeof(apo_candidate), hipMemcpyDeviceToHost) !=
                hipSuccess)
          rc = APO_EDEVICE;
      }
    }
    if (rc) (void)hipGetLastError();
    const auto now = std::chrono::steady_clock::now();
    {
      std::lock_guard<std::mutex> lk(S->mu);
      for (uint32_t w = 0; w < W; w++) {
        Request &R = *batch[w];
        R.status = rc;
        if (!rc && total >= 2) R.rows.assign(rows.begin() + outoff[w], rows.begin() + outoff[w + 1]);
        R.tokens.clear();
        R.tokens.shrink_to_fit();
        R.t_done = now;
        R.done = true;
        if (R.discard) S->tickets.erase(R.ticket);
      }
      sl->busy = false;
      sl->held = sl->ws.held();
    }
    S->cv_mem.notify_all();
    S->cv_work.notify_all();  // requests that waited for memory may fit now
    S->batches++;
    S->windows += W;
  }
}

// What a context's own workspaces may hold: the budget less the server's pool.
static size_t ctx_limit(const apo_ctx *c) {
  const size_t pool = c->server ? c->server->pool : 0;
  return c->budget > pool ? c->budget - pool : 0;
}

extern "C" int apo_server_start(apo_ctx *ctx, uint32_t max_slots, uint32_t queue_cap) {
  if (!ctx || max_slots == 0 || max_slots > 16) return APO_EINVAL;
  if (ctx->server) return APO_EINVAL;
  if (set_dev(ctx)) return APO_EDEVICE;
  auto S = std::make_unique<Server>();
  S->device = ctx->device;
  S->tune = ctx->tune;
  S->queue_cap = queue_cap ? queue_cap : 65536;
  // the slots' memory pool: what the context budget leaves beside the
  // context's own workspaces, else 80% of the device memory free now
  if (ctx->budget) {
    const size_t own = ctx_held(ctx);
    S->pool = ctx->budget > own ? ctx->budget - own : 0;
  } else {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return APO_EDEVICE;
    S->pool = fr / 10 * 8;
  }
  for (uint32_t i = 0; i < max_slots; i++) {
    auto sl = std::make_unique<Slot>();
    if (hipStreamCreate(&sl->stream) != hipSuccess) return APO_EDEVICE;
    S->slots.push_back(std::move(sl));
  }
  Server *raw = S.get();
  for (auto &sl : S->slots) sl->th = std::thread(slot_loop, raw, sl.get());
  ctx->server = std::move(S);
  return APO_OK;
}

extern "C" int apo_submit(apo_ctx *ctx, uint32_t stream_id, const uint64_t *tokens, uint32_t n, uint32_t min_len,
                          uint64_t *ticket) {
  if (!ctx || !ticket || (!tokens && n) || min_len == 0 || n > APO_MAX_N) return APO_EINVAL;
  Server *S = ctx->server.get();
  if (!S) return APO_EINVAL;
  {
    // a window that could never be admitted, even alone on an empty pool
    Workspace fresh;
    if (fresh.bytes_after(std::max<uint32_t>(n, 2), 1) > S->pool) return APO_ENOMEM;
  }
  auto R = std::make_shared<Request>();
  R->stream_id = stream_id;
  R->min_len = min_len;
  R->tokens.assign(tokens, tokens + n);
  R->t_submit = std::chrono::steady_clock::now();
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stopping) return APO_EINVAL;
    if (S->queue.size() >= S->queue_cap) return APO_EAGAIN;
    R->ticket = S->next_ticket++;
    S->tickets[R->ticket] = R;
    S->queue.push_back(R);
    *ticket = R->ticket;
  }
  S->cv_work.notify_one();
  return APO_OK;
}

extern "C" int apo_poll(apo_ctx *ctx, uint64_t ticket, int *done) {
  if (!ctx || !done || !ctx->server) return APO_EINVAL;
  Server *S = ctx->server.get();
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return APO_ENOTFOUND;
  *done = it->second->done ? 1 : 0;
  return APO_OK;
}

extern "C" int apo_fetch(apo_ctx *ctx, uint64_t ticket, apo_candidate *out, uint32_t out_cap, uint32_t *out_n,
                         uint64_t *lat_ns) {
  if (!ctx || !out_n || (!out && out_cap) || !ctx->server) return APO_EINVAL;
  Server *S = ctx->server.get();
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return APO_ENOTFOUND;
  Request &R = *it->second;
  if (!R.done) return APO_EAGAIN;
  if (R.status) {
    const int st = R.status;
    S->tickets.erase(it);
    return st;
  }
  *out_n = (uint32_t)R.rows.size();
  if (R.rows.size() > out_cap) return APO_ERANGE;
  if (!R.rows.empty()) memcpy(out, R.rows.data(), R.rows.size() * sizeof(apo_candidate));
  if (lat_ns)
    *lat_ns = (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(R.t_done - R.t_submit).count();
  S->tickets.erase(it);
  return APO_OK;
}

extern "C" int apo_release(apo_ctx *ctx, uint64_t ticket) {
  if (!ctx || !ctx->server) return APO_EINVAL;
  Server *S = ctx->server.get();
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->tickets.find(ticket);
  if (it == S->tickets.end()) return APO_ENOTFOUND;
  if (it->second->done) S->tickets.erase(it);
  else it->second->discard = true;
  return APO_OK;
}

extern "C" int apo_server_stop(apo_ctx *ctx) {
  if (!ctx) return APO_EINVAL;
  Server *S = ctx->server.get();
  if (!S) return APO_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stopping = true;
  }
  S->cv_work.notify_all();
  S->cv_mem.notify_all();
  for (auto &sl : S->slots) {
    if (sl->th.joinable()) sl->th.join();
    (void)hipSetDevice(S->device);
    (void)hipStreamSynchronize(sl->stream);
    sl->ws.release();
    if (sl->pinned) (void)hipHostFree(sl->pinned);
    (void)hipStreamDestroy(sl->stream);
  }
  ctx->server.reset();
  return APO_OK;
}
