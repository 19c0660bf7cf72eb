// Trace replayer (Section 4.3; TraceReplayer of Algorithm 1) and the
// max-trace-length split of recorded traces (Section 6.2, "auto-200").
//
// Candidate traces (token sequences found by FindRepeats) are kept in a trie.
// For every issued task the replayer starts a pointer at the trie's root,
// steps every pointer down by the task's token, drops the pointers that
// cannot step, and collects the pointers that sit on the end of a candidate.
// When some candidate completed, the best one by score is replayed: the
// pending tasks before it are issued untraced, the candidate is issued as one
// replayed trace, and all pointers are dropped (their tasks are consumed).
// Pending tasks that no pointer covers any more are issued untraced at once.
//
// Score: length x min(count, cap) x (1 + bonus if replayed before), where
// count is the appearance count decayed by decay^(tasks since the previous
// appearance) and then incremented at each appearance.  Section 4.3 names
// these factors but not their constants, so they are parameters.
#include "apo.h"
#include <algorithm>
#include <cmath>
#include <unordered_map>
#include <vector>

namespace {

struct Node {
  std::unordered_map<uint64_t, uint32_t> child;
  int64_t trace = -1;  // candidate ending here
};

struct TraceInfo {
  uint32_t length = 0;
  double count = 0;        // decayed appearance count as of last_seen
  uint64_t last_seen = 0;  // task count at its last appearance (or ingestion)
  bool replayed = false;
};

struct Ptr {
  uint32_t node;
  uint64_t start;  // task index of the first task of the partial match
};

}  // namespace

struct apo_replayer {
  std::vector<Node> nodes{1};
  std::vector<TraceInfo> traces;
  std::vector<Ptr> active;
  uint64_t next_task = 0;     // index of the next task
  uint64_t issued = 0;        // tasks before this index have been issued
  std::vector<apo_replay_event> events;
  uint32_t count_cap = 8;
  double decay = 0.999, bonus = 0.1;
  uint64_t traced = 0, replays = 0;

  void emit(uint64_t b, uint64_t e, int64_t trace) {
    if (e <= b) return;
    if (trace < 0 && !events.empty() && events.back().trace < 0 && events.back().end == b) {
      events.back().end = e;
      return;
    }
    events.push_back(apo_replay_event{b, e, trace});
  }

  // one more appearance ending with task index `task`
  void appeared(TraceInfo &I, uint64_t task) {
    I.count = I.count * std::pow(decay, (double)(task + 1 - I.last_seen)) + 1.0;
    I.last_seen = task + 1;
  }

  double score(int64_t t) const {
    const TraceInfo &I = traces[(size_t)t];
    return (double)I.length * std::min<double>(I.count, (double)count_cap) * (I.replayed ? 1.0 + bonus : 1.0);
  }
};

extern "C" int apo_replayer_create(uint32_t count_cap, double decay, double replay_bonus, apo_replayer **out) {
  if (!out || count_cap == 0 || !(decay > 0.0 && decay <= 1.0) || replay_bonus < 0.0) return APO_EINVAL;
  auto *r = new apo_replayer();
  r->count_cap = count_cap;
  r->decay = decay;
  r->bonus = replay_bonus;
  *out = r;
  return APO_OK;
}

extern "C" int apo_replayer_destroy(apo_replayer *r) {
  delete r;
  return APO_OK;
}

// IngestCandidates: rows come from FindRepeats over `tokens`; each row's
// substring tokens[start .. start+length) becomes a candidate trace.
extern "C" int apo_replayer_ingest(apo_replayer *r, const uint64_t *tokens, uint64_t n, const apo_candidate *rows,
                                   uint32_t nrows) {
  if (!r || (!tokens && n) || (!rows && nrows)) return APO_EINVAL;
  for (uint32_t k = 0; k < nrows; k++) {
    const apo_candidate &c = rows[k];
    if (c.length == 0 || (uint64_t)c.start + c.length > n) return APO_EINVAL;
    uint32_t node = 0;
    for (uint32_t i = 0; i < c.length; i++) {
      const uint64_t tok = tokens[c.start + i];
      auto it = r->nodes[node].child.find(tok);
      if (it == r->nodes[node].child.end()) {
        r->nodes.push_back(Node{});
        const uint32_t nn = (uint32_t)r->nodes.size() - 1;
        r->nodes[node].child.emplace(tok, nn);
        node = nn;
      } else {
        node = it->second;
      }
    }
    int64_t t = r->nodes[node].trace;
    if (t < 0) {
      t = (int64_t)r->traces.size();
      r->nodes[node].trace = t;
      TraceInfo I;
      I.length = c.length;
      I.count = c.count;
      I.last_seen = r->next_task;
      r->traces.push_back(I);
    } else {
      TraceInfo &I = r->traces[(size_t)t];
      I.count = std::max<double>(I.count, c.count);
    }
  }
  return APO_OK;
}

// Issues n tasks with the given tokens.
extern "C" int apo_replayer_step(apo_replayer *r, const uint64_t *tokens, uint64_t n) {
  if (!r || (!tokens && n)) return APO_EINVAL;
  std::vector<Ptr> nxt;
  std::vector<int64_t> done;
  for (uint64_t k = 0; k < n; k++) {
    const uint64_t tok = tokens[k];
    const uint64_t task = r->next_task++;
    // AdvanceActiveCandidates (+ a new pointer at the root) and FilterInvalid
    nxt.clear();
    r->active.push_back(Ptr{0, task});
    for (const Ptr &p : r->active) {
      auto it = r->nodes[p.node].child.find(tok);
      if (it != r->nodes[p.node].child.end()) nxt.push_back(Ptr{it->second, p.start});
    }
    r->active.swap(nxt);
    // FilterCompleted
    done.clear();
    for (const Ptr &p : r->active) {
      const int64_t t = r->nodes[p.node].trace;
      if (t >= 0) {
        r->appeared(r->traces[(size_t)t], task);
        done.push_back(t);
      }
    }
    if (!done.empty()) {
      // SelectReplayTrace + ExecuteAndReplay
      int64_t best = done[0];
      double bs = r->score(best);
      for (size_t i = 1; i < done.size(); i++) {
        const double sc = r->score(done[i]);
        if (sc > bs || (sc == bs && done[i] < best)) { bs = sc; best = done[i]; }
      }
      TraceInfo &I = r->traces[(size_t)best];
      const uint64_t b = task + 1 - I.length;
      r->emit(r->issued, b, -1);
      r->emit(b, task + 1, best);
      r->issued = task + 1;
      r->traced += I.length;
      r->replays++;
      I.replayed = true;
      r->active.clear();
      continue;
    }
    // pending tasks no pointer can still cover are issued untraced
    uint64_t keep_from = task + 1;
    for (const Ptr &p : r->active) keep_from = std::min(keep_from, p.start);
    if (keep_from > r->issued) {
      r->emit(r->issued, keep_from, -1);
      r->issued = keep_from;
    }
  }
  return APO_OK;
}

// Issues every pending task untraced (end of the stream).
extern "C" int apo_replayer_flush(apo_replayer *r) {
  if (!r) return APO_EINVAL;
  r->emit(r->issued, r->next_task, -1);
  r->issued = r->next_task;
  r->active.clear();
  return APO_OK;
}

// Drains the issued events: [begin, end) task ranges, trace id or -1.
extern "C" int apo_replayer_events(apo_replayer *r, apo_replay_event *out, uint32_t cap, uint32_t *n) {
  if (!r || !n || (!out && cap)) return APO_EINVAL;
  *n = (uint32_t)r->events.size();
  if (r->events.size() > cap) return APO_ERANGE;
  std::copy(r->events.begin(), r->events.end(), out);
  r->events.clear();
  return APO_OK;
}

extern "C" int apo_replayer_stats(apo_replayer *r, uint64_t *tasks, uint64_t *traced, uint64_t *replays,
                                  uint64_t *traces) {
  if (!r || !tasks || !traced || !replays || !traces) return APO_EINVAL;
  *tasks = r->next_task;
  *traced = r->traced;
  *replays = r->replays;
  *traces = r->traces.size();
  return APO_OK;
}

// max_trace_length: every row longer than max_len becomes consecutive pieces
// of max_len (the last one shorter); pieces shorter than min_len are dropped.
// Each piece keeps the row's count (every occurrence splits the same way).
extern "C" int apo_split_rows(const apo_candidate *rows, uint32_t n, uint32_t max_len, uint32_t min_len,
                              apo_candidate *out, uint32_t cap, uint32_t *out_n) {
  if ((!rows && n) || !out_n || (!out && cap) || max_len == 0 || min_len == 0) return APO_EINVAL;
  uint32_t m = 0;
  for (uint32_t k = 0; k < n; k++) {
    for (uint32_t off = 0; off < rows[k].length; off += max_len) {
      const uint32_t len = std::min(max_len, rows[k].length - off);
      if (len < min_len) continue;
      if (m < cap) out[m] = apo_candidate{rows[k].start + off, len, rows[k].count};
      m++;
    }
  }
  *out_n = m;
  return m > cap ? APO_ERANGE : APO_OK;
}
