// The dynamic analysis of Algorithm 1 over one task stream: every issued
// task's token goes to the trace finder (ruler-sampled asynchronous
// FindRepeats on the context's server) and then to the trace replayer.
// Finished analyses are ingested at a deterministic point: analysis j is
// ingested before the task at which (tasks seen when it was submitted) + lag
// tasks have been seen, waiting for it if it is not done yet.  Whenever an
// analysis had to be waited for, the lag for the following analyses grows
// (Section 5.1).  With an agreement object several replicas of the stream
// ("nodes") vote at every ingestion and all take the same next lag, so they
// ingest the same results at the same tasks and make the same decisions.
#include "apo.h"
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

struct apo_agree {
  uint32_t nodes = 1;
  uint32_t timeout_ms = 0;
  std::mutex mu;
  std::condition_variable cv;
  struct Vote {
    uint64_t voted = 0, left = 0;  // node bitmasks
    bool waited = false;
    bool done = false;
  };
  std::map<uint64_t, Vote> votes;  // analysis index -> vote
};

extern "C" int apo_agree_create(uint32_t nodes, uint32_t timeout_ms, apo_agree **out) {
  if (!out || nodes == 0 || nodes > 64) return APO_EINVAL;
  auto *a = new apo_agree();
  a->nodes = nodes;
  a->timeout_ms = timeout_ms;
  *out = a;
  return APO_OK;
}

extern "C" int apo_agree_destroy(apo_agree *a) {
  delete a;
  return APO_OK;
}

// Collective over all nodes for analysis j: *any_waited = OR of the votes.
extern "C" int apo_agree_vote(apo_agree *a, uint32_t node, uint64_t j, int waited, int *any_waited) {
  if (!a || !any_waited || node >= a->nodes) return APO_EINVAL;
  const uint64_t bit = 1ull << node;
  const uint64_t all = a->nodes == 64 ? ~0ull : (1ull << a->nodes) - 1;
  std::unique_lock<std::mutex> lk(a->mu);
  auto &V = a->votes[j];
  if (V.voted & bit) return APO_EINVAL;  // voted twice
  V.voted |= bit;
  V.waited = V.waited || waited != 0;
  if (V.voted == all) {
    V.done = true;
    a->cv.notify_all();
  } else {
    auto ready = [&] { return a->votes[j].done; };
    if (a->timeout_ms) {
      if (!a->cv.wait_for(lk, std::chrono::milliseconds(a->timeout_ms), ready)) {
        a->votes[j].voted &= ~bit;  // withdraw, so the call can be repeated
        return APO_EAGAIN;
      }
    } else {
      a->cv.wait(lk, ready);
    }
  }
  auto &W = a->votes[j];
  *any_waited = W.waited ? 1 : 0;
  W.left |= bit;
  if (W.left == all) a->votes.erase(j);
  return APO_OK;
}

struct apo_auto {
  apo_ctx *ctx = nullptr;
  apo_tracer *tr = nullptr;
  apo_replayer *rp = nullptr;
  apo_agree *ag = nullptr;
  uint32_t node = 0;
  apo_auto_params p{};
  uint64_t lag = 0;
  uint64_t seen = 0;
  std::deque<uint64_t> submitted_at;  // per pending analysis: tasks seen at submission
  uint64_t next_j = 0;                // index of the next analysis to ingest
  std::vector<apo_auto_ingest> log;
  std::vector<apo_candidate> rows, pieces;
  std::vector<uint64_t> slice;
  uint64_t waits = 0;
};

extern "C" int apo_auto_create(apo_ctx *ctx, uint32_t stream_id, const apo_auto_params *p, apo_agree *agree,
                               uint32_t node, apo_auto **out) {
  if (!ctx || !p || !out || p->block_tokens == 0 || p->capacity < p->block_tokens || p->min_len == 0 ||
      p->max_trace_len < p->min_len || (agree && node >= agree->nodes))
    return APO_EINVAL;
  auto *a = new apo_auto();
  int rc = apo_tracer_create(ctx, stream_id, p->block_tokens, p->capacity, p->min_len, &a->tr);
  if (rc == APO_OK) rc = apo_replayer_create(p->count_cap, p->decay, p->replay_bonus, &a->rp);
  if (rc != APO_OK) {
    if (a->tr) apo_tracer_destroy(a->tr);
    delete a;
    return rc;
  }
  a->ctx = ctx;
  a->ag = agree;
  a->node = node;
  a->p = *p;
  a->lag = p->lag0;
  a->slice.resize(p->capacity);
  *out = a;
  return APO_OK;
}

extern "C" int apo_auto_destroy(apo_auto *a) {
  if (!a) return APO_OK;
  apo_tracer_destroy(a->tr);
  apo_replayer_destroy(a->rp);
  delete a;
  return APO_OK;
}

static int ingest_next(apo_auto *a) {
  bool waited = false;
  uint64_t begin = 0, len = 0;
  uint32_t n = 0;
  int rc;
  for (;;) {
    rc = apo_tracer_poll(a->tr, &begin, &len, a->rows.data(), (uint32_t)a->rows.size(), &n, a->slice.data());
    if (rc == APO_ERANGE) {
      a->rows.resize(n);
      continue;
    }
    if (rc != APO_EAGAIN) break;
    waited = true;
    std::this_thread::sleep_for(std::chrono::microseconds(50));
  }
  if (rc != APO_OK) return rc;
  // recorded traces longer than the maximum are replayed in pieces
  uint32_t m = 0;
  rc = apo_split_rows(a->rows.data(), n, a->p.max_trace_len, a->p.min_len, a->pieces.data(),
                      (uint32_t)a->pieces.size(), &m);
  if (rc == APO_ERANGE) {
    a->pieces.resize(m);
    rc = apo_split_rows(a->rows.data(), n, a->p.max_trace_len, a->p.min_len, a->pieces.data(), m, &m);
  }
  if (rc != APO_OK) return rc;
  rc = apo_replayer_ingest(a->rp, a->slice.data(), len, a->pieces.data(), m);
  if (rc != APO_OK) return rc;
  int any = waited ? 1 : 0;
  if (a->ag && (rc = apo_agree_vote(a->ag, a->node, a->next_j, any, &any)) != APO_OK) return rc;
  a->log.push_back(apo_auto_ingest{a->submitted_at.front(), a->seen, begin, len, m, waited ? 1u : 0u,
                                   any ? 1u : 0u});
  a->submitted_at.pop_front();
  a->next_j++;
  if (waited) a->waits++;
  if (any) a->lag = std::max<uint64_t>(2 * a->lag, a->p.block_tokens);
  return APO_OK;
}

// ExecuteTask for n tasks: TraceFinder(H), then TraceReplayer(T, H), whose
// first step ingests the analyses that are due.
extern "C" int apo_auto_execute(apo_auto *a, const uint64_t *tokens, uint64_t n) {
  if (!a || (!tokens && n)) return APO_EINVAL;
  for (uint64_t k = 0; k < n; k++) {
    uint32_t sub = 0;
    int rc = apo_tracer_push(a->tr, &tokens[k], 1, &sub);
    if (rc != APO_OK) return rc;
    a->seen++;
    for (uint32_t i = 0; i < sub; i++) a->submitted_at.push_back(a->seen);
    while (!a->submitted_at.empty() && a->submitted_at.front() + a->lag <= a->seen)
      if ((rc = ingest_next(a)) != APO_OK) return rc;
    if ((rc = apo_replayer_step(a->rp, &tokens[k], 1)) != APO_OK) return rc;
  }
  return APO_OK;
}

extern "C" int apo_auto_replayer(apo_auto *a, apo_replayer **out) {
  if (!a || !out) return APO_EINVAL;
  *out = a->rp;
  return APO_OK;
}

extern "C" int apo_auto_ingests(apo_auto *a, apo_auto_ingest *out, uint32_t cap, uint32_t *n) {
  if (!a || !n || (!out && cap)) return APO_EINVAL;
  *n = (uint32_t)a->log.size();
  if (a->log.size() > cap) return APO_ERANGE;
  std::copy(a->log.begin(), a->log.end(), out);
  return APO_OK;
}

extern "C" int apo_auto_lag(apo_auto *a, uint64_t *lag, uint64_t *waits) {
  if (!a || !lag || !waits) return APO_EINVAL;
  *lag = a->lag;
  *waits = a->waits;
  return APO_OK;
}
