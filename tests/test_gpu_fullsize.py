"""Full-size parity of the benchmark configurations against the oracle.

* config3 (4096 windows, 48.8 M tokens): every window's rows, batched on three
  lanes and on one lane (graph replay), against the C oracle run over all
  windows on a pool of host threads;
* config2 (n = 2^24): the whole suffix and LCP arrays against the SHA-256
  digests of the oracle's arrays stored by tests/golden/make_config_golden.py;
* config4 (serving trace, windows up to 2^20): every served result against the
  oracle and against the window analysed alone;
* the per-round active suffix counts a_r of the doubling rounds against the
  oracle's (the counts the byte model of the measurement is built on);
* the sequential completion of the greedy selection, forced by a round cap.
"""
import concurrent.futures as cf
import hashlib
import json
import os
import time

import numpy as np
import pytest

import oracle
from paper_2406_18111_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "config_results.json")
POOL = max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_18111_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(t):
    import torch
    t = np.ascontiguousarray(t)
    return torch.from_numpy(t.view(np.int64) if t.dtype == np.uint64 else t.view(np.int32)).cuda()


def _rows_ref(t, m):
    r = oracle.find_repeats(t, m)
    return np.stack([r["row_start"], r["row_len"], r["row_count"]], 1).astype(np.int64).reshape(-1, 3)


def _as3(rows):
    return np.stack([rows["start"], rows["length"], rows["count"]], 1).astype(np.int64).reshape(-1, 3)


def _pack(wins):
    off = np.zeros(len(wins) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(w) for w in wins])
    return np.concatenate(wins).astype(np.uint64), off


def _oracle_active_sum(t):
    _sa, act = oracle.suffix_array(t, return_active=True)
    return int(act.sum())


@pytest.fixture(scope="module")
def config3_ref():
    """Oracle rows and active suffix counts of all 4096 windows (host pool)."""
    wins, m = synth.config3()
    t0 = time.time()
    order = sorted(range(len(wins)), key=lambda w: -len(wins[w]))
    with cf.ThreadPoolExecutor(max_workers=POOL) as ex:
        rows = dict(zip(order, ex.map(lambda w: _rows_ref(wins[w], m), order)))
        act = dict(zip(order, ex.map(lambda w: _oracle_active_sum(wins[w]), order)))
    print("oracle over %d windows: %.1f s on %d threads" % (len(wins), time.time() - t0, POOL), flush=True)
    return wins, m, rows, act


@pytest.mark.parametrize("lanes,graphs", [(3, True), (3, False), (1, True), (1, False)])
def test_config3_every_window(config3_ref, lanes, graphs):
    """All 4096 windows in one batch call: every window's rows equal the
    oracle's, and the doubling rounds processed exactly the oracle's active
    suffixes (plus one first-token sort of every suffix).  Three lanes
    without graphs are the host-driven lanes the benchmark times."""
    import torch
    from paper_2406_18111_amd import Context
    wins, m, ref, act = config3_ref
    toks, off = _pack(wins)
    dev = _dev(toks)
    print("config3 lanes", lanes, "graphs", graphs, flush=True)
    with Context(0) as g:
        g.set_lanes(lanes)
        g.set_graphs(graphs)
        for rep in range(2 if graphs else 1):  # capture, then replay
            rows, oo = g.analyze_batch_dev(dev, off, m)
            rows = rows.cpu().numpy().astype(np.int64)
            bad = [w for w in range(len(wins)) if not np.array_equal(rows[int(oo[w]):int(oo[w + 1])], ref[w])]
            assert not bad, (rep, bad[:10], len(bad))
            c = g.counters()
            assert c["active_sum"] - len(toks) == sum(act.values())
        if graphs:
            assert g.graph_stats()["replays"] >= 1


SINGLE = [("config0", lambda: synth.config0()), ("config1", lambda: synth.config1()),
          ("config1_2^16", lambda: synth.config1(n=1 << 16)),
          ("const_5000", lambda: (np.full(5000, 3, np.uint64), 8)),
          ("periodic_7x9000", lambda: (np.tile(np.arange(7, dtype=np.uint64), 9000), 4)),
          ("random_a4_30000", lambda: (np.random.default_rng(5).integers(0, 4, 30000).astype(np.uint64), 4))]


@pytest.mark.parametrize("name,gen", SINGLE, ids=[s[0] for s in SINGLE])
def test_active_counts_per_round(ctx, name, gen):
    """Suffixes entering each doubling round r >= 1 (after the first-token
    sort) equal the oracle's a_r, round by round."""
    t, m = gen()
    _sa, act = oracle.suffix_array(t, return_active=True)
    ctx.analyze_dev(_dev(t), m)
    got = [a for a in ctx.rounds()["sa_active"][1:] if a]
    assert got == [int(a) for a in act if a], name
    assert ctx.counters()["active_sum"] - len(t) == int(act.sum())


def test_config2_whole_arrays(ctx):
    """n = 2^24 adversarial window: the complete suffix array and LCP array
    (little-endian uint32, LCP of length n-1) hash to the digests of the
    oracle's arrays, and every round's active count matches."""
    g = json.load(open(GOLDEN))["configs"]["config2_n2^24_u32"]
    t, m = synth.config2()
    sa, lcp = ctx.lcp_dev(_dev(t))
    sa = sa.cpu().numpy().view(np.uint32)
    lcp = lcp.cpu().numpy().view(np.uint32)
    assert hashlib.sha256(sa.astype("<u4").tobytes()).hexdigest() == g["sa_sha256"]
    assert hashlib.sha256(lcp[: len(t) - 1].astype("<u4").tobytes()).hexdigest() == g["lcp_sha256"]
    ctx.analyze_dev(_dev(t), m)
    got = [a for a in ctx.rounds()["sa_active"][1:] if a]
    assert got == g["active_per_round"]


def test_server_config4_windows_up_to_2_20(ctx):
    """Requests of the serving trace (64 nested-loop streams, windows
    log-uniform in [1024, 2^20]) submitted at once to a three-slot server:
    every result equals the oracle's and the window's own analysis."""
    from paper_2406_18111_amd import Context
    reqs = synth.config4_requests(duration=10.0, max_requests=40, threads=POOL)
    assert max(len(r.tokens) for r in reqs) > (1 << 19)
    with cf.ThreadPoolExecutor(max_workers=POOL) as ex:
        fut = [ex.submit(_rows_ref, r.tokens, 16) for r in reqs]
        with Context(0) as srv:
            srv.server_start(slots=3)
            tickets = [srv.submit(r.tokens, 16, r.stream) for r in reqs]
            got = [None] * len(reqs)
            deadline = time.time() + 100
            while any(x is None for x in got) and time.time() < deadline:
                for i, tk in enumerate(tickets):
                    if got[i] is None:
                        r = srv.fetch(tk)
                        if r is not None:
                            got[i] = _as3(r[0])
                time.sleep(0.002)
            srv.server_stop()
        ref = [f.result() for f in fut]
    assert all(x is not None for x in got)
    for i, r in enumerate(reqs):
        assert np.array_equal(got[i], ref[i]), (i, len(r.tokens))
        assert np.array_equal(got[i], _as3(ctx.analyze(r.tokens, 16))), i


@pytest.mark.parametrize("cap", [0, 1, 2, 5])
def test_sequential_selection_completion(ctx, cap):
    """With the greedy rounds capped, the sequential completion decides the
    rest: the result is still the oracle's, and the counters say the
    completion ran."""
    blocks = []
    for k in range(1, 300):
        blocks += [0] * k + [1]
    assert len(blocks) > (1 << 15)  # above the single-window size of the one-wavefront greedy
    cases = [(np.array(blocks, dtype=np.uint64), 1), synth.config1(n=1 << 16), synth.config0()]
    try:
        ctx.set_selection_round_cap(cap)
        ctx.set_selection_prefix(0)  # the rounds and the completion alone
        ctx.set_window_greedy(False)  # config0 through the rounds as well
        for k, (t, m) in enumerate(cases):
            rows, occ = ctx.analyze(t, m, occurrences=True)
            ref = oracle.find_repeats(t, m)
            assert np.array_equal(_as3(rows), np.stack([ref["row_start"], ref["row_len"], ref["row_count"]], 1))
            assert np.array_equal(occ["start"].astype(np.int64), ref["occ_start"])
            assert np.array_equal(occ["length"].astype(np.int64), ref["occ_len"])
            c = ctx.counters()
            if k == 0 or cap == 0:
                # the block family needs far more than 5 greedy rounds
                assert c["selection_sequential"] == 1, (cap, c)
            assert c["selection_sequential"] == 1 or c["selection_rounds"] <= cap
    finally:
        ctx.set_selection_round_cap(64)
        ctx.set_selection_prefix(-1)
        ctx.set_window_greedy(True)
    ctx.analyze(cases[1][0], cases[1][1])
    assert ctx.counters()["selection_sequential"] == 0
