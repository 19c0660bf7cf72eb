// Exercises the host-only library code (trace replayer, max-trace-length
// split, agreement, trace finder, Algorithm 1 driver) for a sanitizer build;
// the analysis server is the stand-in of fake_server.cpp.  Exits non-zero
// when a call returns something other than what its contract says.
#include "apo.h"
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

apo_ctx *fake_ctx();

#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "check failed: %s (line %d)\n", #cond, __LINE__); \
      exit(1);                                                         \
    }                                                                  \
  } while (0)

static std::vector<uint64_t> loop_stream(uint64_t seed, size_t n, size_t period) {
  std::vector<uint64_t> body(period), t(n);
  uint64_t x = seed;
  for (auto &b : body) b = (x = x * 6364136223846793005ull + 1442695040888963407ull) >> 20;
  for (size_t i = 0; i < n; i++) {
    t[i] = body[i % period];
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    if ((x >> 58) == 0) t[i] = x;  // about 1.6% substitutions
  }
  return t;
}

static void replayer_and_split() {
  apo_replayer *r = nullptr;
  CHECK(apo_replayer_create(0, 0.99, 0.1, &r) == APO_EINVAL);
  CHECK(apo_replayer_create(8, 0.999, 0.1, &r) == APO_OK);
  const auto t = loop_stream(3, 6000, 37);
  std::vector<apo_candidate> rows = {{0, 37, 3}, {5, 30, 2}, {0, 74, 1}, {100, 12, 4}};
  CHECK(apo_replayer_ingest(r, t.data(), t.size(), rows.data(), (uint32_t)rows.size()) == APO_OK);
  apo_candidate bad = {5990, 20, 1};
  CHECK(apo_replayer_ingest(r, t.data(), t.size(), &bad, 1) == APO_EINVAL);
  for (size_t k = 0; k < t.size(); k += 97) CHECK(apo_replayer_step(r, t.data() + k, std::min<size_t>(97, t.size() - k)) == APO_OK);
  CHECK(apo_replayer_flush(r) == APO_OK);
  uint32_t ne = 0;
  apo_replay_event one[1];
  const int rc = apo_replayer_events(r, one, 1, &ne);
  CHECK(rc == APO_OK || rc == APO_ERANGE);
  std::vector<apo_replay_event> ev(ne + 1);
  CHECK(apo_replayer_events(r, ev.data(), (uint32_t)ev.size(), &ne) == APO_OK);
  uint64_t covered = 0;
  for (uint32_t k = 0; k < ne; k++) covered += ev[k].end - ev[k].begin;
  uint64_t tasks = 0, traced = 0, replays = 0, traces = 0;
  CHECK(apo_replayer_stats(r, &tasks, &traced, &replays, &traces) == APO_OK);
  CHECK(tasks == t.size() && covered == tasks && traced <= tasks);
  CHECK(apo_replayer_destroy(r) == APO_OK);

  std::vector<apo_candidate> in = {{0, 450, 2}, {10, 200, 3}, {7, 9, 5}, {3, 201, 1}};
  uint32_t n = 0;
  apo_candidate small[2];
  CHECK(apo_split_rows(in.data(), (uint32_t)in.size(), 200, 10, small, 2, &n) == APO_ERANGE);
  std::vector<apo_candidate> out(n);
  CHECK(apo_split_rows(in.data(), (uint32_t)in.size(), 200, 10, out.data(), n, &n) == APO_OK);
  for (const auto &p : out) CHECK(p.length <= 200 && p.length >= 10);
}

static void agreement() {
  apo_agree *a = nullptr;
  CHECK(apo_agree_create(0, 0, &a) == APO_EINVAL);
  CHECK(apo_agree_create(3, 0, &a) == APO_OK);
  int any[3] = {0, 0, 0};
  std::vector<std::thread> th;
  for (uint32_t node = 0; node < 3; node++)
    th.emplace_back([&, node] {
      for (uint64_t j = 0; j < 50; j++) {
        int aw = 0;
        CHECK(apo_agree_vote(a, node, j, (int)((j + node) % 7 == 0), &aw) == APO_OK);
        any[node] += aw;
      }
    });
  for (auto &x : th) x.join();
  CHECK(any[0] == any[1] && any[1] == any[2]);
  int aw = 0;
  CHECK(apo_agree_vote(a, 7, 0, 0, &aw) == APO_EINVAL);
  CHECK(apo_agree_destroy(a) == APO_OK);
  CHECK(apo_agree_create(2, 20, &a) == APO_OK);  // the other node never votes: timeout
  CHECK(apo_agree_vote(a, 0, 0, 1, &aw) == APO_EAGAIN);
  CHECK(apo_agree_destroy(a) == APO_OK);
}

static void tracer() {
  apo_tracer *t = nullptr;
  CHECK(apo_tracer_create(fake_ctx(), 1, 0, 100, 4, &t) == APO_EINVAL);
  CHECK(apo_tracer_create(fake_ctx(), 1, 50, 400, 4, &t) == APO_OK);
  const auto s = loop_stream(5, 3000, 23);
  uint32_t sub = 0, total = 0;
  for (size_t k = 0; k < s.size(); k += 130) {
    CHECK(apo_tracer_push(t, s.data() + k, (uint32_t)std::min<size_t>(130, s.size() - k), &sub) == APO_OK);
    total += sub;
  }
  CHECK(total == s.size() / 50);
  std::vector<uint64_t> toks(400);
  uint32_t got = 0;
  int guard = 0;
  while (got < total && guard++ < 100000) {
    uint64_t b = 0, l = 0;
    uint32_t n = 0;
    apo_candidate rows[1];
    int rc = apo_tracer_poll(t, &b, &l, rows, 0, &n, toks.data());
    if (rc == APO_EAGAIN) continue;
    if (rc == APO_ERANGE) {
      std::vector<apo_candidate> big(n);
      rc = apo_tracer_poll(t, &b, &l, big.data(), n, &n, toks.data());
    }
    CHECK(rc == APO_OK);
    CHECK(l <= 400 && b + l <= s.size());
    for (uint64_t i = 0; i < l; i++) CHECK(toks[i] == s[b + i]);
    got++;
  }
  CHECK(got == total);
  // results still queued are dropped on destroy
  CHECK(apo_tracer_push(t, s.data(), 200, &sub) == APO_OK);
  CHECK(apo_tracer_destroy(t) == APO_OK);
}

static void algorithm1() {
  apo_auto_params p{};
  p.block_tokens = 50;
  p.capacity = 500;
  p.min_len = 5;
  p.max_trace_len = 40;
  p.lag0 = 60;
  p.count_cap = 8;
  p.decay = 0.999;
  p.replay_bonus = 0.1;
  apo_agree *ag = nullptr;
  CHECK(apo_agree_create(2, 0, &ag) == APO_OK);
  const auto s = loop_stream(9, 8000, 31);
  std::vector<std::thread> th;
  uint64_t tasks[2] = {0, 0}, nevents[2] = {0, 0};
  for (uint32_t node = 0; node < 2; node++)
    th.emplace_back([&, node] {
      apo_auto *a = nullptr;
      CHECK(apo_auto_create(fake_ctx(), node, &p, ag, node, &a) == APO_OK);
      for (size_t k = 0; k < s.size(); k += 333) CHECK(apo_auto_execute(a, s.data() + k, std::min<size_t>(333, s.size() - k)) == APO_OK);
      uint32_t n = 0;
      apo_auto_ingest one[1];
      const int rc = apo_auto_ingests(a, one, 1, &n);
      CHECK(rc == APO_OK || rc == APO_ERANGE);
      std::vector<apo_auto_ingest> ing(n + 1);
      CHECK(apo_auto_ingests(a, ing.data(), (uint32_t)ing.size(), &n) == APO_OK);
      uint64_t lag = 0, waits = 0;
      CHECK(apo_auto_lag(a, &lag, &waits) == APO_OK);
      apo_replayer *r = nullptr;
      CHECK(apo_auto_replayer(a, &r) == APO_OK);
      CHECK(apo_replayer_flush(r) == APO_OK);
      uint64_t t = 0, tr = 0, rp = 0, tc = 0;
      CHECK(apo_replayer_stats(r, &t, &tr, &rp, &tc) == APO_OK);
      tasks[node] = t;
      std::vector<apo_replay_event> ev(t + 1);
      uint32_t ne = 0;
      CHECK(apo_replayer_events(r, ev.data(), (uint32_t)ev.size(), &ne) == APO_OK);
      nevents[node] = ne;
      CHECK(apo_auto_destroy(a) == APO_OK);
    });
  for (auto &x : th) x.join();
  CHECK(tasks[0] == s.size() && tasks[1] == s.size());
  CHECK(nevents[0] == nevents[1]);
  CHECK(apo_agree_destroy(ag) == APO_OK);
}

int main() {
  replayer_and_split();
  agreement();
  tracer();
  algorithm1();
  printf("host driver ok\n");
  return 0;
}
