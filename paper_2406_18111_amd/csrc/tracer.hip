// Trace finder over one task stream (Section 4.2 / 4.4 of the paper): a
// history buffer of the last `capacity` tokens and ruler-function sampling of
// the slices analysed.  After the i-th block of `block` tokens the analysed
// slice is the last block * 2^v(i) tokens (v(i) = number of trailing zero bits
// of i), capped at the history capacity; every slice goes to the context's
// server as an asynchronous FindRepeats request.
#include "apo.h"
#include <algorithm>
#include <deque>
#include <mutex>
#include <vector>

struct apo_tracer {
  apo_ctx *ctx = nullptr;
  uint32_t stream_id = 0, block = 0, min_len = 1;
  uint64_t capacity = 0;
  std::vector<uint64_t> hist;     // ring of the last `capacity` tokens
  uint64_t total = 0;             // tokens pushed so far
  uint64_t blocks = 0;            // completed blocks
  uint32_t in_block = 0;
  struct Pending {
    uint64_t ticket, begin, len;
    std::vector<uint64_t> tokens;  // the slice as submitted
  };
  std::deque<Pending> pending;
  std::mutex mu;
};

extern "C" uint64_t apo_ruler_slice(uint64_t block_index, uint32_t block_tokens, uint64_t capacity) {
  if (block_index == 0 || block_tokens == 0) return 0;
  const int v = __builtin_ctzll(block_index);
  uint64_t len = (uint64_t)block_tokens;
  for (int k = 0; k < v && len < capacity; k++) len <<= 1;
  return std::min<uint64_t>(len, capacity);
}

extern "C" int apo_tracer_create(apo_ctx *ctx, uint32_t stream_id, uint32_t block_tokens, uint32_t capacity,
                                 uint32_t min_len, apo_tracer **out) {
  if (!ctx || !out || block_tokens == 0 || capacity < block_tokens || capacity > APO_MAX_N || min_len == 0)
    return APO_EINVAL;
  auto *t = new apo_tracer();
  t->ctx = ctx;
  t->stream_id = stream_id;
  t->block = block_tokens;
  t->capacity = capacity;
  t->min_len = min_len;
  t->hist.assign(capacity, 0);
  *out = t;
  return APO_OK;
}

extern "C" int apo_tracer_destroy(apo_tracer *t) {
  if (!t) return APO_OK;
  for (auto &p : t->pending) (void)apo_release(t->ctx, p.ticket);
  delete t;
  return APO_OK;
}

// Appends tokens; whenever a block completes, submits its ruler slice.
extern "C" int apo_tracer_push(apo_tracer *t, const uint64_t *tokens, uint32_t n, uint32_t *submitted) {
  if (!t || (!tokens && n)) return APO_EINVAL;
  std::lock_guard<std::mutex> lk(t->mu);
  uint32_t sub = 0;
  std::vector<uint64_t> slice;
  for (uint32_t k = 0; k < n; k++) {
    t->hist[t->total % t->capacity] = tokens[k];
    t->total++;
    if (++t->in_block < t->block) continue;
    t->in_block = 0;
    t->blocks++;
    const uint64_t len = std::min<uint64_t>(apo_ruler_slice(t->blocks, t->block, t->capacity), t->total);
    const uint64_t begin = t->total - len;
    slice.resize(len);
    for (uint64_t i = 0; i < len; i++) slice[i] = t->hist[(begin + i) % t->capacity];
    uint64_t ticket = 0;
    const int rc = apo_submit(t->ctx, t->stream_id, slice.data(), (uint32_t)len, t->min_len, &ticket);
    if (rc != APO_OK) {
      if (submitted) *submitted = sub;
      return rc;
    }
    t->pending.push_back({ticket, begin, len, slice});
    sub++;
  }
  if (submitted) *submitted = sub;
  return APO_OK;
}

// Oldest finished analysis (in submission order): the slice it covered in
// stream coordinates, optionally its tokens, and its rows.  APO_EAGAIN if the
// oldest is not ready or none is pending.  On APO_ERANGE *out_n holds the row
// count and the result stays queued.
extern "C" int apo_tracer_poll(apo_tracer *t, uint64_t *slice_begin, uint64_t *slice_len, apo_candidate *out,
                               uint32_t out_cap, uint32_t *out_n, uint64_t *slice_tokens) {
  if (!t || !slice_begin || !slice_len || !out_n || (!out && out_cap)) return APO_EINVAL;
  std::lock_guard<std::mutex> lk(t->mu);
  if (t->pending.empty()) return APO_EAGAIN;
  const auto &p = t->pending.front();
  const int rc = apo_fetch(t->ctx, p.ticket, out, out_cap, out_n, nullptr);
  if (rc != APO_OK) return rc;
  *slice_begin = p.begin;
  *slice_len = p.len;
  if (slice_tokens) std::copy(p.tokens.begin(), p.tokens.end(), slice_tokens);
  t->pending.pop_front();
  return APO_OK;
}
