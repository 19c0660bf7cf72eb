// Test stand-in for the library's analysis server, for sanitizer builds of
// the host-only sources (tracer, replayer, Algorithm 1 driver) without a GPU.
// apo_submit queues the window; a result becomes ready on the second fetch
// attempt, so callers also take their not-ready paths.  The rows are not an
// analysis: for a window of n tokens and minimum length m they name the
// substrings [0, m) and, when it fits, [m, 2m) -- rows inside the window,
// which is all the host code under test relies on.
#include "apo.h"
#include <map>
#include <mutex>
#include <vector>

struct apo_ctx {
  int unused;
};

namespace {
struct Pending {
  std::vector<apo_candidate> rows;
  int polls = 0;
};
std::mutex g_mu;
std::map<uint64_t, Pending> g_tickets;
uint64_t g_next = 1;
}  // namespace

extern "C" int apo_submit(apo_ctx *ctx, uint32_t stream_id, const uint64_t *tokens, uint32_t n, uint32_t min_len,
                          uint64_t *ticket) {
  (void)stream_id;
  if (!ctx || !ticket || (!tokens && n) || min_len == 0) return APO_EINVAL;
  Pending p;
  if (n >= 2 * min_len) p.rows.push_back({0, min_len, 2});
  if (n >= 4 * min_len) p.rows.push_back({2 * min_len, min_len, 1});
  std::lock_guard<std::mutex> lk(g_mu);
  *ticket = g_next++;
  g_tickets[*ticket] = std::move(p);
  return APO_OK;
}

extern "C" int apo_fetch(apo_ctx *ctx, uint64_t ticket, apo_candidate *out, uint32_t out_cap, uint32_t *out_n,
                         uint64_t *lat_ns) {
  if (!ctx || !out_n || (!out && out_cap)) return APO_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_tickets.find(ticket);
  if (it == g_tickets.end()) return APO_ENOTFOUND;
  if (it->second.polls++ == 0) return APO_EAGAIN;
  *out_n = (uint32_t)it->second.rows.size();
  if (it->second.rows.size() > out_cap) return APO_ERANGE;
  for (size_t k = 0; k < it->second.rows.size(); k++) out[k] = it->second.rows[k];
  if (lat_ns) *lat_ns = 0;
  g_tickets.erase(it);
  return APO_OK;
}

extern "C" int apo_release(apo_ctx *ctx, uint64_t ticket) {
  if (!ctx) return APO_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_tickets.erase(ticket) ? APO_OK : APO_ENOTFOUND;
}

// the driver's context
apo_ctx *fake_ctx() {
  static apo_ctx c{0};
  return &c;
}
