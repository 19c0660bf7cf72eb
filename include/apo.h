/*
 * libapo -- repeated-fragment mining over task-hash token windows on MI355X.
 *
 * Implements FindRepeats, Algorithm 2 ("Non-overlapping repeated
 * sub-strings") of Yadav et al., "Automatic Tracing in Task-Based Runtime
 * Systems", ASPLOS 2025, Section 4.2, including the O(n log n) realisation of
 * the section's implementation paragraph.  A window S of tokens (one hash per
 * issued task, Section 4.1) goes through: order-preserving rank compression,
 * suffix array by prefix doubling, LCP array (Phi/PLCP), candidate generation
 * over adjacent suffix-array pairs, the (length desc, substring asc, start
 * asc) sort, and greedy selection of non-overlapping occurrences.  Every stage
 * runs as HIP kernels on the GPU; there is no CPU fallback.
 *
 * Conventions fixed by this library where the paper is silent:
 *   - tokens compare as unsigned integers, substrings lexicographically, and a
 *     suffix that is a proper prefix of another sorts first;
 *   - candidates shorter than min_len are dropped (min_len >= 1, inclusive);
 *   - an accepted occurrence is (start, length); the result lists one row per
 *     distinct accepted substring -- first accepted start, length, number of
 *     accepted occurrences -- in order of first acceptance, i.e. by length
 *     descending, then substring ascending.
 * The result is a pure function of (tokens, min_len): identical for a window
 * analysed alone, in a batch, or through the server.
 *
 * Ownership: the caller owns every buffer passed in (host or device).  The
 * context owns its device workspace, streams and threads.  Calls on one
 * context must come from one thread, except apo_submit / apo_poll /
 * apo_fetch, which are thread-safe.
 *
 * Errors (all entry points return an int):
 *   APO_OK       success
 *   APO_EINVAL   null pointer, min_len == 0, n > APO_MAX_N, bad offsets
 *   APO_ENOMEM   device memory for the workspace could not be obtained, or
 *                the request exceeds the context's memory budget
 *   APO_ERANGE   an output buffer is too small; the *_n outputs then hold the
 *                required counts and nothing else is written.  floor(n/min_len)
 *                rows and occurrences always suffice.
 *   APO_EDEVICE  a HIP call failed or a device-side capacity check tripped;
 *                the context stays valid and can be destroyed or reused
 *   APO_EAGAIN   server queue full
 *   APO_ENOTFOUND unknown server ticket
 */
#ifndef APO_H
#define APO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define APO_MAX_N (1u << 26)

/* Limits of apo_analyze_window_noalloc: the longest window, and the fixed
 * device array (per GPU, held from the first apo_create on that GPU until
 * the process ends) that is its whole workspace. */
#define APO_NOALLOC_MAX_N (1u << 15)
#define APO_NOALLOC_SCRATCH_BYTES (21u << 20)

enum {
  APO_OK = 0,
  APO_EINVAL = -1,
  APO_ENOMEM = -2,
  APO_ERANGE = -3,
  APO_EDEVICE = -4,
  APO_EAGAIN = -5,
  APO_ENOTFOUND = -6
};

typedef struct apo_ctx apo_ctx;

/* One distinct accepted substring (a candidate trace): first accepted start
 * (relative to its window), length in tokens, number of accepted
 * non-overlapping occurrences. */
typedef struct {
  uint32_t start, length, count;
} apo_candidate;

/* One accepted occurrence, in acceptance order; `cand` indexes the row of
 * its substring in the apo_candidate output. */
typedef struct {
  uint32_t start, length, cand;
} apo_occurrence;

/* Create a context on HIP device `hip_device`.  `device_mem_budget_bytes`
 * caps the device memory the context's workspaces hold together: the
 * single-window workspace, the lane workspaces of batches and the server's
 * slot pool (0 = no cap).  Workspaces grow on demand and stay resident; an
 * analysis whose workspace would not fit returns APO_ENOMEM and leaves the
 * context usable (smaller analyses still run; batches first drop to fewer
 * lanes, and idle lane workspaces are freed, before giving up).  Returns
 * APO_EINVAL for out == NULL, APO_EDEVICE if the device cannot be selected. */
int apo_create(apo_ctx **out, int hip_device, size_t device_mem_budget_bytes);

/* Stops the server if running, frees all device memory.  NULL is a no-op. */
int apo_destroy(apo_ctx *ctx);

/* Static string for an error code. */
const char *apo_strerror(int code);

/* FindRepeats (Section 4.2, Algorithm 2) on one window of host tokens.
 * Blocking.  tokens: n values (n <= APO_MAX_N; n < 2 gives 0 rows).
 * out: room for out_cap rows; *out_n receives the row count.  occ may be
 * NULL; otherwise room for occ_cap occurrences, *occ_n receives their count. */
int apo_analyze_window(apo_ctx *ctx, const uint64_t *tokens, uint32_t n, uint32_t min_len,
                       apo_candidate *out, uint32_t out_cap, uint32_t *out_n,
                       apo_occurrence *occ, uint32_t occ_cap, uint32_t *occ_n);

/* Same for 32-bit tokens. */
int apo_analyze_window_u32(apo_ctx *ctx, const uint32_t *tokens, uint32_t n, uint32_t min_len,
                           apo_candidate *out, uint32_t out_cap, uint32_t *out_n,
                           apo_occurrence *occ, uint32_t occ_cap, uint32_t *occ_n);

/* Device-resident variant: d_tokens is a device array of n tokens of
 * `token_bits` (32 or 64) bits; outputs are device arrays (d_occ may be
 * NULL) and *h_out_n / *h_occ_n are written on the host.  Work is ordered on
 * `hip_stream` (NULL = the context's stream); the call returns when the
 * outputs are complete. */
int apo_analyze_window_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                           uint32_t min_len, apo_candidate *d_out, uint32_t out_cap,
                           uint32_t *h_out_n, apo_occurrence *d_occ, uint32_t occ_cap,
                           uint32_t *h_occ_n, void *hip_stream);

/* For callers that cannot allocate device memory during the call (code
 * around HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): apo_analyze_window_dev with the same arguments, outputs and
 * results, that calls no allocator.  Its workspace is a fixed device array
 * of APO_NOALLOC_SCRATCH_BYTES per GPU, laid out when the first context on
 * that GPU is created.  Windows longer than APO_NOALLOC_MAX_N tokens return
 * APO_ENOMEM (the fixed array is too small).  Every call on a GPU shares
 * that GPU's array: calls on one GPU are serialised by a lock, and each call
 * clears what it needs before use.  The call synchronises `hip_stream`, so
 * it cannot itself be recorded into a graph.  APO_EDEVICE if the array could
 * not be set up on this GPU. */
int apo_analyze_window_noalloc(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                               uint32_t min_len, apo_candidate *d_out, uint32_t out_cap, uint32_t *h_out_n,
                               apo_occurrence *d_occ, uint32_t occ_cap, uint32_t *h_occ_n, void *hip_stream);

/* Many windows at once: window w is tokens[offsets[w] .. offsets[w+1]) of a
 * host array.  Rows of window w are out[out_offsets[w] .. out_offsets[w+1]);
 * out_offsets has num_windows+1 entries.  Each window's rows equal what
 * apo_analyze_window returns for it alone. */
int apo_analyze_batch(apo_ctx *ctx, const uint64_t *tokens, const uint64_t *offsets,
                      uint32_t num_windows, uint32_t min_len, apo_candidate *out,
                      uint64_t out_cap, uint64_t *out_offsets);

/* Device-resident batch: d_tokens (64-bit) and h_offsets (host) as above;
 * d_out device rows, h_out_offsets host. */
int apo_analyze_batch_dev(apo_ctx *ctx, const uint64_t *d_tokens, const uint64_t *h_offsets,
                          uint32_t num_windows, uint32_t min_len, apo_candidate *d_out,
                          uint64_t out_cap, uint64_t *h_out_offsets, void *hip_stream);

/* Batches are split into `lanes` (1..4, default 3) groups of consecutive
 * windows with about equal token counts, analysed concurrently on separate
 * streams, workspaces and host threads (lane 0 uses the caller's stream),
 * each lane host-driven (launches sized from device counts read between
 * stages); results are identical for every value.  With more than one lane,
 * batch calls do not use graph capture.  APO_EINVAL outside 1..4. */
int apo_set_lanes(apo_ctx *ctx, int lanes);

/* Batches on one lane enqueue their whole launch sequence without host
 * synchronisation (round counts bounded by the longest window) and, when
 * enabled (default), record it as a HIP graph that is replayed for later
 * batches of the same shape (same token pointer, total length, window count,
 * longest window, min_len and kernel parameters); window offsets are uploaded
 * outside the graph.  on = 0 disables capture. */
int apo_set_graphs(apo_ctx *ctx, int on);

/* Number of graph captures and replays made by this context. */
int apo_graph_stats(apo_ctx *ctx, uint64_t *captures, uint64_t *replays);

/* ---- stage outputs, for checking each stage against a reference ---- */

/* Suffix array of one device window (Section 4.2, SuffixArray(S)):
 * d_sa[i] = start of the i-th smallest suffix.  *h_rounds (nullable) gets the
 * number of doubling rounds. */
int apo_suffix_array_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                         uint32_t *d_sa, uint32_t *h_rounds, void *hip_stream);

/* Suffix array plus LCP: d_lcp[i] = common prefix of suffixes d_sa[i] and
 * d_sa[i+1] for i < n-1 (the indexing of Algorithm 2's loop); d_lcp[n-1] = 0. */
int apo_lcp_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t *d_sa,
                uint32_t *d_lcp, void *hip_stream);

/* Candidates of length >= min_len after Sort(C), exact duplicates removed:
 * d_len/d_start/d_id (substring ID = suffix-array left boundary of the
 * l-interval of the generating pair).  *h_count gets the count; APO_ERANGE if
 * cap is too small (2n always suffices). */
int apo_candidates_dev(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n,
                       uint32_t min_len, uint32_t *d_len, uint32_t *d_start, uint32_t *d_id,
                       uint32_t cap, uint32_t *h_count, void *hip_stream);

/* Equal-length greedy per substring (Algorithm 2's selection among the
 * occurrences of one substring, Section 4.2): for m candidates on the device
 * in the order apo_candidates_dev returns them (a substring's occurrences
 * are contiguous, by increasing start), d_next[k] = index of the first
 * occurrence of the same substring starting at or after start[k] + len[k]
 * (0xFFFFFFFF if none), and d_count[k] = number of occurrences on the chain
 * k, next[k], next[next[k]], ...; at a substring's first occurrence that is
 * its non-overlapping occurrence count in isolation.  d_tmp: 3m words of
 * scratch.  All buffers are the caller's; synchronous on hip_stream. */
int apo_interval_counts_dev(apo_ctx *ctx, const uint32_t *d_len, const uint32_t *d_start, const uint32_t *d_id,
                            uint32_t m, uint32_t *d_next, uint32_t *d_count, uint32_t *d_tmp, void *hip_stream);

/* Per-stage device times of the last analysis (ms): token ranks, suffix
 * array, LCP, candidates, candidate sort, selection, output.  Returns the
 * number of stages written (<= nstages). */
int apo_last_stage_ms(apo_ctx *ctx, double *stage_ms, int nstages);

/* Counters of the last analysis, in this order: rounds of doubling (the
 * first-token sort included), candidates generated, candidates after dedup,
 * selection rounds, accepted occurrences, rows, sum over rounds of active
 * suffixes (the first-token sort counts every suffix), distinct tokens (for
 * a batch: summed over its windows, except that the windows with more than
 * 4096 distinct tokens, ranked through one shared table, count their union
 * once), 1 if the selection finished with the sequential completion (else
 * 0), the candidates the exact prefix walk decided before the rounds (0: none),
 * and the windows whose first two doubling rounds were taken window by
 * window from ranks of their adjacent token pairs (host-driven batches whose
 * windows all have at most 4096 distinct tokens and 8192 distinct pairs).
 * Writes min(nvals, 11) values and returns that number. */
int apo_last_counters(apo_ctx *ctx, uint64_t *vals, int nvals);

/* Device bytes of the workspace an analysis of n tokens in `windows`
 * windows needs (what a context or a server slot allocates for it; sizes
 * round up to powers of two).  No device is touched.  0 if n > APO_MAX_N or
 * windows == 0. */
size_t apo_workspace_bytes(uint64_t n, uint32_t windows);

/* Device memory of the context: *held = bytes its own workspaces hold (the
 * single-window one and the lane workspaces); *server_pool (nullable) = the
 * running server's pool, 0 without a server; *server_held (nullable) = bytes
 * the server's slots hold or have reserved for the batches they run. */
int apo_memory(apo_ctx *ctx, size_t *held, size_t *server_pool, size_t *server_held);

/* Test hook for the error path: the (after_syncs+1)-th host synchronisation
 * inside the next single-window analysis reports a device error, so that
 * call returns APO_EDEVICE with its work abandoned; the context stays
 * usable and the following calls run normally.  -1 cancels.  APO_EINVAL
 * below -1. */
int apo_inject_device_error(apo_ctx *ctx, int after_syncs);

/* Selection path (Section 4.2, the greedy walk of Algorithm 2): with on = 1
 * (default) windows of at most 2^17 tokens in a batch, and single windows of
 * at most 2^15 tokens, are decided by one wavefront per window walking the
 * window's candidates in priority order over an on-chip bitmap; longer
 * windows use the round-based evaluation.  on = 0 sends every analysis
 * through the rounds.  Results are identical either way.  APO_EINVAL
 * unless on is 0 or 1. */
int apo_set_window_greedy(apo_ctx *ctx, int on);

/* Test hook: host-driven analyses stop the round-based greedy selection
 * after `rounds` rounds (0..64, default 64) and decide the rest with the
 * sequential completion, which gives the same result (Section 4.2, the
 * greedy walk of Algorithm 2).  APO_EINVAL outside 0..64. */
int apo_set_selection_round_cap(apo_ctx *ctx, int rounds);

/* Host-driven analyses that use the round-based greedy selection may first
 * decide a prefix of the priority order exactly (one workgroup walks the
 * longest candidates in order over the mark array, Section 4.2, the greedy
 * walk of Algorithm 2), then run the rounds from round 1 on the rest, whose
 * filter rejects every candidate the prefix covers.  k = -1 (default): a
 * prefix of 1024 candidates when the longest candidate spans at least 1/64 of
 * the analysed tokens; k = 0: never; k > 0: always a prefix of k candidates
 * (a test hook).  Results are identical either way.  APO_EINVAL if k < -1. */
int apo_set_selection_prefix(apo_ctx *ctx, int k);

/* Per-round sizes of the last analysis (diagnostic): sa_active[r] = suffixes
 * entering doubling round r (r < *n_sa); sel_live[q] / sel_undecided[q] =
 * candidates live at the start of selection round q and still undecided
 * after it (q < *n_sel).  APO_ERANGE if cap is below either count (the
 * first cap entries are written). */
int apo_last_rounds(apo_ctx *ctx, uint32_t *sa_active, uint32_t *n_sa, uint32_t *sel_live, uint32_t *sel_undecided,
                    uint32_t *n_sel, uint32_t cap);

/* Live timing of one kernel family with HIP events around each of its
 * launches (on the stream the kernel runs on): tag 1 = the LDS sort-and-regroup
 * kernel of the suffix-array doubling rounds; 0 = off.  Costs one event pair
 * per timed launch. */
int apo_profile_kernel(apo_ctx *ctx, int tag);

/* For the last analysis: number of timed launches that had work, their total
 * device time (ms) and the number of entries they processed. */
int apo_last_kernel_profile(apo_ctx *ctx, uint64_t *launches, double *total_ms, uint64_t *elems);

/* ---- autotuning of kernel parameters ---- */

/* Times every (LDS sort tile 2^11..2^13, MSD digit width 8/10/11/12) pair on
 * the device window d_tokens (median of `reps` runs after one warm-up) and
 * keeps the fastest for windows of the same size bucket (ceil(log2 n)); later
 * analyses, batches and server slots use the nearest tuned bucket.  Outputs
 * (nullable) receive the chosen pair and its median time in ms.  Parameters
 * change speed only, never results. */
int apo_tune(apo_ctx *ctx, const void *d_tokens, int token_bits, uint32_t n, uint32_t min_len, int reps,
             int *best_tile_log, int *best_digit_bits, double *best_ms);

/* Tunes on a whole batch of device windows (offsets as in
 * apo_analyze_batch_dev), timing each pair as the batch call runs it
 * (lanes included), and keeps the fastest for the size of one lane's share.
 * Same outputs as apo_tune.  APO_EINVAL for fewer than 2 tokens. */
int apo_tune_batch(apo_ctx *ctx, const uint64_t *d_tokens, const uint64_t *h_offsets, uint32_t num_windows,
                   uint32_t min_len, int reps, int *best_tile_log, int *best_digit_bits, double *best_ms);

/* Fix the pair for all sizes (tile_log 11..13, digit_bits 8..12); negative
 * values return to the tuned table. */
int apo_set_params(apo_ctx *ctx, int tile_log, int digit_bits);

/* Persist / restore the tuned table (text: "log2n tile_log digit_bits" lines). */
int apo_tune_save(apo_ctx *ctx, const char *path);
int apo_tune_load(apo_ctx *ctx, const char *path);

/* ---- continuous-batching server ---- */

/* Start the server: up to max_slots (1..16) batches in flight on the device
 * at once, each slot with a resident workspace and its own stream.
 * Admission is by device memory: the slots' workspaces together hold at most
 * the server's pool (the context budget less what the context's own
 * workspaces hold at start, or 80% of the device memory free at start when
 * there is no budget).  A free slot takes the oldest queued request and every
 * later one with the same min_len while the packed batch's workspace still
 * fits beside the other slots' (idle slots give theirs back first); if even
 * the oldest does not fit, it stays queued until a busy slot finishes.
 * queue_cap bounds waiting requests (0 = 65536).  APO_EINVAL if a server
 * runs already or max_slots is out of range. */
int apo_server_start(apo_ctx *ctx, uint32_t max_slots, uint32_t queue_cap);

/* Enqueue a window (tokens are copied before return).  *ticket identifies it.
 * A window that fits the pool waits in the queue until memory frees up;
 * APO_ENOMEM only for a window whose workspace alone exceeds the pool,
 * APO_EAGAIN when the queue is full, APO_EINVAL without a running server. */
int apo_submit(apo_ctx *ctx, uint32_t stream_id, const uint64_t *tokens, uint32_t n,
               uint32_t min_len, uint64_t *ticket);

/* *done = 1 once the result of `ticket` is ready. */
int apo_poll(apo_ctx *ctx, uint64_t ticket, int *done);

/* Copy the rows of a finished ticket and release it.  APO_EAGAIN if not done;
 * APO_ERANGE (with *out_n set, ticket kept) if out_cap is too small.
 * *lat_ns (nullable) gets submit-to-ready latency in ns. */
int apo_fetch(apo_ctx *ctx, uint64_t ticket, apo_candidate *out, uint32_t out_cap,
              uint32_t *out_n, uint64_t *lat_ns);

/* Give up a ticket: its result is dropped now if ready, else when it is. */
int apo_release(apo_ctx *ctx, uint64_t ticket);

/* Drain in-flight work, stop the server threads. */
int apo_server_stop(apo_ctx *ctx);

/* ---- trace finder: history buffer + ruler-function sampling ---- */

/* Section 4.4: after the i-th block (i >= 1) of block_tokens tokens, the
 * analysed slice is the last block_tokens * 2^v(i) tokens, v(i) the number of
 * trailing zero bits of i, capped at `capacity`.  Returns that length (0 for
 * i == 0). */
uint64_t apo_ruler_slice(uint64_t block_index, uint32_t block_tokens, uint64_t capacity);

typedef struct apo_tracer apo_tracer;

/* A trace finder for one task stream (Algorithm 1's TraceFinder): keeps the
 * last `capacity` tokens and, after every block of `block_tokens` new tokens,
 * submits the ruler slice of the history to ctx's server (apo_server_start
 * must have been called) as an asynchronous FindRepeats with min_len. */
int apo_tracer_create(apo_ctx *ctx, uint32_t stream_id, uint32_t block_tokens, uint32_t capacity,
                      uint32_t min_len, apo_tracer **out);

/* Appends n tokens (copied); *submitted (nullable) gets the number of
 * analyses submitted.  Errors of apo_submit are passed through. */
int apo_tracer_push(apo_tracer *t, const uint64_t *tokens, uint32_t n, uint32_t *submitted);

/* Oldest finished analysis in submission order: slice start (in stream
 * positions) and length, and its rows (start relative to the slice).  If
 * slice_tokens is not NULL it receives the slice's tokens (room for
 * `capacity` tokens).  APO_EAGAIN if it is not ready or none is pending;
 * APO_ERANGE (result kept, *out_n = rows) if out_cap is too small. */
int apo_tracer_poll(apo_tracer *t, uint64_t *slice_begin, uint64_t *slice_len, apo_candidate *out,
                    uint32_t out_cap, uint32_t *out_n, uint64_t *slice_tokens);

/* Frees the tracer (results still queued are dropped). */
int apo_tracer_destroy(apo_tracer *t);

/* ---- trace replayer (Section 4.3; Algorithm 1's TraceReplayer) ---- */

typedef struct apo_replayer apo_replayer;

/* Issued task range [begin, end) (task indices since creation); trace is the
 * id of the replayed candidate trace, or -1 for tasks issued untraced. */
typedef struct {
  uint64_t begin, end;
  int64_t trace;
} apo_replay_event;

/* Host-side replayer.  Candidates are scored length * min(count, count_cap) *
 * decay^(tasks since last seen) * (1 + replay_bonus if replayed before)
 * (Section 4.3 names these factors, not their constants).  APO_EINVAL for
 * count_cap == 0, decay outside (0, 1], replay_bonus < 0 or out == NULL. */
int apo_replayer_create(uint32_t count_cap, double decay, double replay_bonus, apo_replayer **out);

/* Adds the rows of a FindRepeats result over tokens[0..n) as candidate
 * traces (the row's substring; a trace already known keeps the larger
 * count).  APO_EINVAL if a row lies outside tokens. */
int apo_replayer_ingest(apo_replayer *r, const uint64_t *tokens, uint64_t n, const apo_candidate *rows,
                        uint32_t nrows);

/* Issues n tasks with the given tokens, in order: active pointers advance
 * in the candidate trie, a completed candidate (best score, ties to the
 * lower id) is replayed with the pending tasks before it issued untraced,
 * and pending tasks no pointer covers are issued untraced. */
int apo_replayer_step(apo_replayer *r, const uint64_t *tokens, uint64_t n);

/* Issues every pending task untraced. */
int apo_replayer_flush(apo_replayer *r);

/* Moves the events issued so far to out; *n gets their number.  APO_ERANGE
 * (events kept) if out_cap is too small. */
int apo_replayer_events(apo_replayer *r, apo_replay_event *out, uint32_t out_cap, uint32_t *n);

/* Tasks seen, tasks issued inside replayed traces, replays, known traces. */
int apo_replayer_stats(apo_replayer *r, uint64_t *tasks, uint64_t *traced, uint64_t *replays, uint64_t *traces);

int apo_replayer_destroy(apo_replayer *r);

/* Section 6.2's maximum trace length: each row longer than max_len becomes
 * consecutive pieces of max_len tokens (the last one shorter), each with the
 * row's count; pieces shorter than min_len are dropped.  *out_n gets the
 * number of pieces; APO_ERANGE if more than out_cap. */
int apo_split_rows(const apo_candidate *rows, uint32_t n, uint32_t max_len, uint32_t min_len, apo_candidate *out,
                   uint32_t out_cap, uint32_t *out_n);

/* ---- Algorithm 1 end to end, with deterministic ingestion (Section 5.1) ---- */

typedef struct apo_agree apo_agree;

/* Agreement among `nodes` (1..64) replicas of one task stream.  timeout_ms
 * bounds each vote's wait for the other nodes (0 = wait indefinitely). */
int apo_agree_create(uint32_t nodes, uint32_t timeout_ms, apo_agree **out);

/* Collective for analysis j: every node calls it once with whether it had
 * to wait for that analysis; all get *any_waited = OR over the nodes.
 * Blocks until all nodes voted; APO_EAGAIN (vote withdrawn) on timeout,
 * APO_EINVAL for a bad node or a second vote. */
int apo_agree_vote(apo_agree *a, uint32_t node, uint64_t j, int waited, int *any_waited);

int apo_agree_destroy(apo_agree *a);

typedef struct {
  uint32_t block_tokens;   /* trace finder block (ruler unit), e.g. 250 or 500 */
  uint32_t capacity;       /* history buffer, e.g. 5000 */
  uint32_t min_len;        /* minimum trace length, e.g. 25 */
  uint32_t max_trace_len;  /* recorded traces are split into pieces of at most this, e.g. 200 */
  uint64_t lag0;           /* tasks between an analysis' submission and its ingestion, initially */
  uint32_t count_cap;      /* replayer score parameters (apo_replayer_create) */
  double decay, replay_bonus;
} apo_auto_params;

/* One ingested analysis: tasks seen at submission and at ingestion, the
 * analysed slice, pieces ingested, whether this node waited and whether any
 * node did (which grew the lag). */
typedef struct {
  uint64_t submitted_at, ingested_at, slice_begin, slice_len;
  uint32_t pieces, waited, any_waited;
} apo_auto_ingest;

typedef struct apo_auto apo_auto;

/* Algorithm 1 over one task stream on ctx's server (apo_server_start must
 * have been called): trace finder + trace replayer.  Analysis j is ingested
 * before the task at which submitted_at + lag tasks have been seen (waiting
 * for it if needed); when any node waited the lag becomes
 * max(2 * lag, block_tokens).  agree (nullable) is shared by the replicas;
 * node is this replica's index. */
int apo_auto_create(apo_ctx *ctx, uint32_t stream_id, const apo_auto_params *p, apo_agree *agree, uint32_t node,
                    apo_auto **out);

/* ExecuteTask for n tasks with the given tokens (task hashes). */
int apo_auto_execute(apo_auto *a, const uint64_t *tokens, uint64_t n);

/* The replayer inside (events, stats, flush); owned by the apo_auto. */
int apo_auto_replayer(apo_auto *a, apo_replayer **out);

/* Ingestion log so far; APO_ERANGE (with *n set) if out_cap is too small. */
int apo_auto_ingests(apo_auto *a, apo_auto_ingest *out, uint32_t out_cap, uint32_t *n);

/* Current lag and number of analyses this node waited for. */
int apo_auto_lag(apo_auto *a, uint64_t *lag, uint64_t *waits);

int apo_auto_destroy(apo_auto *a);

#ifdef __cplusplus
}
#endif

#endif /* APO_H */
