"""Batched and served analyses: each window's result is identical alone, in a
batch, and in the server mix (exact, integer results), and matches the oracle."""
import time

import numpy as np
import pytest

import oracle
from paper_2406_18111_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_18111_amd import Context
    c = Context(0)
    yield c
    c.close()


def _rows_ref(t, m):
    r = oracle.find_repeats(t, m)
    return np.stack([r["row_start"], r["row_len"], r["row_count"]], 1).astype(np.int64).reshape(-1, 3)


def _as3(rows):
    return np.stack([rows["start"], rows["length"], rows["count"]], 1).astype(np.int64).reshape(-1, 3)


def _pack(wins):
    off = np.zeros(len(wins) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(w) for w in wins])
    toks = np.concatenate(wins).astype(np.uint64) if wins else np.zeros(0, np.uint64)
    return toks, off


def _mixed_windows(seed, count):
    rng = np.random.default_rng(seed)
    wins = []
    for k in range(count):
        kind = k % 5
        L = int(rng.choice([0, 1, 2, 3, 100, 4095, 4096, 4097, 9000, 30000]))
        if kind == 0:
            w = rng.integers(0, 3, L)
        elif kind == 1:
            w = np.full(L, 5)
        elif kind == 2:
            w = synth.loop_stream(int(rng.integers(1 << 30)), L, int(rng.integers(10, 60)), 64, 0.05) if L else np.zeros(0)
        elif kind == 3:
            w = np.tile(np.arange(7), L // 7 + 1)[:L]
        else:
            w = rng.integers(0, 1 << 40, L)
        wins.append(np.asarray(w, dtype=np.uint64))
    return wins


def test_batch_equals_alone_and_oracle(ctx):
    wins = _mixed_windows(5, 40)
    toks, off = _pack(wins)
    for m in (1, 4, 8):
        print("batch min_len", m, flush=True)
        rows, oo = ctx.analyze_batch(toks, off, m)
        for w, win in enumerate(wins):
            got = _as3(rows[int(oo[w]):int(oo[w + 1])])
            alone = _as3(ctx.analyze(win, m))
            assert np.array_equal(got, alone), (w, len(win))
            assert np.array_equal(got, _rows_ref(win, m)), (w, len(win))


def _distinct_window(rng, d, with_max):
    """A window of exactly d distinct values (plus 2^64-1 when asked), each
    value at least twice, with repeated runs."""
    vals = np.unique(rng.integers(0, np.iinfo(np.uint64).max, 3 * d + 8, dtype=np.uint64))[:d]
    assert len(vals) == d
    rng.shuffle(vals)
    parts = [vals, vals[rng.permutation(d)], np.tile(vals[: min(d, 9)], 20)]
    if with_max:
        parts.append(np.full(3, np.iinfo(np.uint64).max, dtype=np.uint64))
    w = np.concatenate(parts)
    return w.astype(np.uint64)


def test_batch_window_ranks(ctx):
    """Batches rank each window's tokens on their own unless the window has
    more than 4096 distinct values (the shared table ranks those): windows at
    and around that bound, some holding the largest value 2^64-1, give the
    oracle's rows with host-driven lanes, with lanes as branches of one graph
    and in one sync-free lane (graphs on and off); with no window over the
    bound the distinct-token counter is the sum over windows."""
    rng = np.random.default_rng(21)
    small = [_distinct_window(rng, d, mx) for d, mx in ((1, False), (2, True), (700, False), (4095, True),
                                                       (4096, False), (4096, True))]
    big = [_distinct_window(rng, d, mx) for d, mx in ((4097, False), (6000, True))]
    for wins in (small, small + big, big[::-1] + small[:2]):
        toks, off = _pack(wins)
        refs = [_rows_ref(w, 2) for w in wins]
        for lanes, graphs in ((3, True), (3, False), (1, False), (1, True)):
            print("windows", len(wins), "lanes", lanes, "graphs", graphs, flush=True)
            try:
                ctx.set_lanes(lanes)
                ctx.set_graphs(graphs)
                for rep in range(2):
                    rows, oo = ctx.analyze_batch(toks, off, 2)
                    for w in range(len(wins)):
                        assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), refs[w]), (w, len(wins[w]))
                    if wins is small:
                        assert ctx.counters()["sigma"] == sum(len(np.unique(x)) for x in wins)
            finally:
                ctx.set_lanes(3)
                ctx.set_graphs(True)


def _pairs_window(rng, npairs):
    """A window over 200 symbols whose adjacent token pairs, with the pair of
    its last token and the window's end, are exactly npairs distinct ones."""
    t = rng.integers(1, 201, 4 * npairs).astype(np.uint64)
    key = t[:-1] * 256 + t[1:]
    _, first = np.unique(key, return_index=True)
    fresh = np.zeros(len(key), np.int64)
    fresh[first] = 1
    seen = np.cumsum(fresh)  # seen[i]: distinct pairs among key[:i+1]
    i = int(np.searchsorted(seen, npairs - 1))  # window t[:i+2]: npairs - 1 inner pairs + the end pair
    assert seen[i] == npairs - 1
    w = t[: i + 2]
    inner = len(np.unique(w[:-1] * 256 + w[1:]))
    assert inner + 1 == npairs
    return w


def _oracle_active(t):
    _sa, act = oracle.suffix_array(t, return_active=True)
    return int(act.sum())


def _pair_lane_windows(wins, lanes, over):
    """Windows that take pair ranks: a batch runs as min(lanes, W // 2) lanes
    of consecutive windows with about equal tokens (one lane below two), and
    a lane takes them when it holds two windows or more, none of them
    `over`."""
    W = len(wins)
    L = max(min(lanes, W // 2), 1)
    off = np.cumsum([0] + [len(w) for w in wins])
    w0 = [0]
    for g in range(1, L):
        w0.append(max(min(int(np.searchsorted(off, off[-1] * g // L, side="left")), W), w0[-1]))
    w0.append(W)
    return sum(w0[g + 1] - w0[g] for g in range(L)
               if w0[g + 1] - w0[g] >= 2 and not any(wins[k] is over for k in range(w0[g], w0[g + 1])))


def test_batch_pair_ranks_bound(ctx):
    """Batches take the first two doubling rounds window by window when every
    window of a lane has at most 8192 distinct adjacent token pairs (the pair
    of the last token and the window's end included), and the engine's second
    round otherwise: windows at 8192 and 8193 distinct pairs beside loop
    streams give the oracle's rows and the oracle's active suffix counts on
    either path, in host-driven lanes (the host picks the path), in one
    sync-free lane and in graphs (both forms launched, the device count picks
    one), each graph replayed once."""
    rng = np.random.default_rng(33)
    at, over = _pairs_window(rng, 8192), _pairs_window(rng, 8193)
    loops = [synth.loop_stream(40 + k, n, body, 64, 0.05) for k, (n, body) in
             enumerate(((3000, 17), (9000, 250), (700, 11), (5000, 40), (12000, 90), (1500, 300)))]
    m = 3
    seen = set()
    for wins in (loops + [at], loops + [over], loops[:3] + [over] + loops[3:] + [at], [over, at]):
        toks, off = _pack(wins)
        refs = [_rows_ref(w, m) for w in wins]
        act = sum(_oracle_active(w) for w in wins)
        for lanes, graphs in ((3, False), (2, False), (1, False), (3, True), (1, True)):
            print("windows", [len(w) for w in wins], "lanes", lanes, "graphs", graphs, flush=True)
            try:
                ctx.set_lanes(lanes)
                ctx.set_graphs(graphs)
                for rep in range(2 if graphs else 1):
                    rows, oo = ctx.analyze_batch(toks, off, m)
                    for w in range(len(wins)):
                        assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), refs[w]), (rep, w, len(wins[w]))
                    c = ctx.counters()
                    assert c["active_sum"] - len(toks) == act
                    assert c["pair_windows"] == _pair_lane_windows(wins, lanes, over), c
                    seen.add((lanes > 1 and not graphs, c["pair_windows"] == len(wins)))
            finally:
                ctx.set_lanes(3)
                ctx.set_graphs(True)
    assert seen == {(a, b) for a in (True, False) for b in (True, False)}  # both paths, host- and device-picked


def _pair_mix_windows(seed, count):
    """Windows whose tokens mostly fit the per-window ranks (small alphabets,
    loop streams, periodic runs, the value 2^64-1 sprinkled in, lengths 1 to
    20000), so that whole lanes take the pair ranks or just miss them."""
    rng = np.random.default_rng(seed)
    top = np.uint64(np.iinfo(np.uint64).max)
    wins = []
    for k in range(count):
        L = int(rng.choice([1, 2, 3, 7, 64, 65, 500, 2047, 2048, 2049, 5000, 9000, 20000]))
        kind = k % 4
        if kind == 0:
            w = synth.loop_stream(int(rng.integers(1 << 30)), L, int(rng.integers(3, 500)),
                                  int(rng.integers(8, 4000)), float(rng.choice([0.0, 0.01, 0.05, 0.1])))
        elif kind == 1:
            w = rng.integers(0, int(rng.choice([2, 3, 16, 90])), L).astype(np.uint64)
        elif kind == 2:
            w = np.tile(rng.integers(0, 1 << 62, int(rng.integers(1, 50))).astype(np.uint64), L // 2 + 1)[:L]
        else:
            w = rng.integers(0, 4000, L).astype(np.uint64)
        w = np.asarray(w, dtype=np.uint64).copy()
        if L and rng.random() < 0.4:
            w[rng.integers(0, L, max(1, L // 50))] = top
        wins.append(w)
    return wins


def _distinct_pairs(w):
    """Distinct adjacent pairs of a window, the pair of its last token and its end included."""
    if len(w) == 0:
        return 0
    return len(np.unique(np.stack([w[:-1], w[1:]], 1), axis=0)) + 1


@pytest.mark.parametrize("seed,keep_over", [(5, True), (6, True), (7, False)])
def test_batch_pair_ranks_random(ctx, seed, keep_over):
    """Random batches of windows around the per-window ranking bounds (distinct
    tokens and distinct pairs, tiny windows, the largest token value): rows
    equal the oracle's and the active suffix counts the oracle's, in
    host-driven lanes (the host picks the path), in one sync-free lane and
    replayed from a graph (the device picks it); one batch without windows
    over 8192 distinct pairs, so that every path takes the pair ranks."""
    wins = _pair_mix_windows(seed, 16)
    if not keep_over:
        wins = [w for w in wins if _distinct_pairs(w) <= 8192]
    toks, off = _pack(wins)
    m = 3
    refs = [_rows_ref(w, m) for w in wins]
    act = sum(_oracle_active(w) for w in wins)
    pairs = 0
    for lanes, graphs in ((3, False), (1, False), (1, True)):
        print("seed", seed, "lanes", lanes, "graphs", graphs, flush=True)
        try:
            ctx.set_lanes(lanes)
            ctx.set_graphs(graphs)
            for rep in range(2 if graphs else 1):
                rows, oo = ctx.analyze_batch(toks, off, m)
                for w in range(len(wins)):
                    assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), refs[w]), (rep, w, len(wins[w]))
                c = ctx.counters()
                assert c["active_sum"] - len(toks) == act
                if not keep_over and lanes == 1:
                    assert c["pair_windows"] == len(wins), c
                pairs += c["pair_windows"]
        finally:
            ctx.set_lanes(3)
            ctx.set_graphs(True)
    print("windows with pair ranks over the runs:", pairs, flush=True)


def test_batch_long_windows(ctx):
    """Windows longer than 2^16 tokens beside short ones: the doubling rounds'
    window-relative bucketing digits then need more than 16 bits, and the
    windows finish their doubling after very different numbers of rounds
    (rank snapshots exist for some and not for others).  Host-driven lanes,
    one sync-free lane (rounds bounded by the longest window) and its graph."""
    rng = np.random.default_rng(21)
    wins = [np.tile(np.arange(7, dtype=np.uint64), 100000 // 7 + 1)[:100000],
            rng.integers(0, 1 << 40, 70000).astype(np.uint64),
            np.full(80000, 5, dtype=np.uint64),
            synth.loop_stream(77, 5000, 40, 64, 0.05).astype(np.uint64),
            rng.integers(0, 4, 66000).astype(np.uint64),
            np.array([1, 2, 1, 2, 1], dtype=np.uint64)]
    toks, off = _pack(wins)
    for m in (2, 8):
        refs = [_rows_ref(win, m) for win in wins]
        alone = [_as3(ctx.analyze(win, m)) for win in wins]
        for lanes, graphs in ((3, False), (1, False), (1, True)):
            print("long-window batch min_len", m, "lanes", lanes, "graphs", graphs, flush=True)
            try:
                ctx.set_lanes(lanes)
                ctx.set_graphs(graphs)
                rows, oo = ctx.analyze_batch(toks, off, m)
                for w, win in enumerate(wins):
                    got = _as3(rows[int(oo[w]):int(oo[w + 1])])
                    assert np.array_equal(got, alone[w]), (w, len(win))
                    assert np.array_equal(got, refs[w]), (w, len(win))
            finally:
                ctx.set_lanes(3)
                ctx.set_graphs(True)


def test_batch_windows_past_the_slot_bitmap(ctx):
    """Windows of more than 2^17 tokens with few distinct values (the
    per-window first rounds then find grouped slots by searching the group
    starts instead of the singleton bitmap) beside short ones, with and
    without other windows over the per-window bounds: the oracle's rows and
    active suffix counts in host-driven lanes, one sync-free lane and a graph."""
    big = [np.tile(np.arange(7, dtype=np.uint64), 140000 // 7 + 1)[:140000],
           synth.loop_stream(91, 150000, 37, 200, 0.02).astype(np.uint64)]
    small = [synth.loop_stream(92 + k, n, 23, 64, 0.05).astype(np.uint64) for k, n in enumerate((3000, 900, 12000))]
    m = 8
    for wins in (big + small, small[:1] + big[::-1] + small[1:]):
        toks, off = _pack(wins)
        refs = [_rows_ref(w, m) for w in wins]
        act = sum(_oracle_active(w) for w in wins)
        for lanes, graphs in ((3, False), (2, False), (1, False), (1, True)):
            print("windows", [len(w) for w in wins], "lanes", lanes, "graphs", graphs, flush=True)
            try:
                ctx.set_lanes(lanes)
                ctx.set_graphs(graphs)
                rows, oo = ctx.analyze_batch(toks, off, m)
                for w in range(len(wins)):
                    assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), refs[w]), (w, len(wins[w]))
                assert ctx.counters()["active_sum"] - len(toks) == act
            finally:
                ctx.set_lanes(3)
                ctx.set_graphs(True)


def test_lanes_never_get_only_empty_windows(ctx):
    """Lanes split a batch by tokens, and a lane of empty windows only (here
    the trailing empty windows) would be an analysis of no tokens, which a
    captured graph cannot hold: such windows join their neighbour lane.  The
    oracle's rows (none for the empty windows) with host-driven lanes and
    with the lanes captured as one graph, replayed."""
    rng = np.random.default_rng(44)
    heads = [synth.loop_stream(70 + k, n, 13, 64, 0.05).astype(np.uint64) for k, n in enumerate((17, 100, 2047))]
    e = np.zeros(0, np.uint64)
    batches = [heads + [e],
               heads + [e] * 5,
               [rng.integers(0, 3, 3000).astype(np.uint64)] + [e] * 7,
               # the last lane's first boundary lands past the big window: an
               # empty group between it and the trailing empty windows
               [heads[0][:5], heads[0][:3], heads[2], heads[0][:1], heads[1], rng.integers(0, 9, 30000).astype(np.uint64), e]]
    m = 3
    for wins in batches:
        toks, off = _pack(wins)
        refs = [_rows_ref(w, m) for w in wins]
        for lanes, graphs in ((3, False), (3, True), (2, True)):
            print("windows", [len(w) for w in wins], "lanes", lanes, "graphs", graphs, flush=True)
            try:
                ctx.set_lanes(lanes)
                ctx.set_graphs(graphs)
                replays = ctx.graph_stats()["replays"]
                for rep in range(2 if graphs else 1):
                    rows, oo = ctx.analyze_batch(toks, off, m)
                    for w in range(len(wins)):
                        assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), refs[w]), (rep, w, len(wins[w]))
                if graphs:  # captured (a failed capture would have fallen back to host-driven lanes)
                    assert ctx.graph_stats()["replays"] > replays
            finally:
                ctx.set_lanes(3)
                ctx.set_graphs(True)


def test_batch_device_api(ctx):
    import torch
    wins, m = synth.config3(num_windows=24)
    toks, off = _pack(wins)
    dev = torch.from_numpy(toks.view(np.int64)).cuda()
    rows_d, oo_d = ctx.analyze_batch_dev(dev, off, m)
    rows_h, oo_h = ctx.analyze_batch(toks, off, m)
    assert np.array_equal(oo_d, oo_h)
    assert np.array_equal(rows_d.cpu().numpy().astype(np.int64), _as3(rows_h))
    for w, win in enumerate(wins):
        assert np.array_equal(_as3(rows_h[int(oo_h[w]):int(oo_h[w + 1])]), _rows_ref(win, m))


def test_config3_full_batch_sampled(ctx):
    """All 4096 windows of the batched workload in one call; 48 sampled windows
    checked against the oracle and against their own single-window analysis."""
    wins, m = synth.config3()
    toks, off = _pack(wins)
    print("config3 tokens", len(toks), flush=True)
    rows, oo = ctx.analyze_batch(toks, off, m)
    rng = np.random.default_rng(11)
    sample = sorted(set(rng.integers(0, len(wins), 44).tolist()) | {0, len(wins) - 1,
                    int(np.argmax([len(w) for w in wins])), int(np.argmin([len(w) for w in wins]))})
    for w in sample:
        got = _as3(rows[int(oo[w]):int(oo[w + 1])])
        assert np.array_equal(got, _rows_ref(wins[w], m)), w
        assert np.array_equal(got, _as3(ctx.analyze(wins[w], m))), w


def test_server_mix_equals_alone(ctx):
    from paper_2406_18111_amd import Context
    reqs = list(synth.config4_trace(duration=0.03, hi=1 << 16))
    reqs += [synth.Request(0.0, 0, np.zeros(0, np.uint64)), synth.Request(0.0, 0, np.array([3], np.uint64))]
    with Context(0) as srv:
        srv.server_start(slots=3)
        tickets = []
        for i, r in enumerate(reqs):
            m = 16 if i % 3 else 8  # two min lengths in flight at once
            tickets.append((srv.submit(r.tokens, m, r.stream), r.tokens, m))
        results = []
        deadline = time.time() + 120
        pending = list(tickets)
        while pending and time.time() < deadline:
            nxt = []
            for tk, toks, m in pending:
                got = srv.fetch(tk)
                if got is None:
                    nxt.append((tk, toks, m))
                else:
                    results.append((got[0], toks, m, got[1]))
            pending = nxt
            time.sleep(0.002)
        assert not pending
        srv.server_stop()
    for rows, toks, m, lat in results:
        assert lat >= 0
        assert np.array_equal(_as3(rows), _as3(ctx.analyze(toks, m)))
    for rows, toks, m, _ in results[:10]:
        assert np.array_equal(_as3(rows), _rows_ref(toks, m))


def test_server_errors(ctx):
    from paper_2406_18111_amd import ApoError, Context
    from paper_2406_18111_amd import _lib
    with Context(0) as srv:
        with pytest.raises(ApoError):
            srv.submit(np.arange(10, dtype=np.uint64), 2)  # server not started
        srv.server_start(slots=1)
        with pytest.raises(ApoError) as e:
            srv.fetch(987654)
        assert e.value.code == _lib.APO_ENOTFOUND
        tk = srv.submit(np.tile(np.arange(5, dtype=np.uint64), 400), 2)
        t0 = time.time()
        got = None
        while got is None and time.time() - t0 < 60:
            got = srv.fetch(tk, cap=0)  # too small at first: binding retries with the needed size
            time.sleep(0.001)
        assert got is not None and len(got[0]) >= 1
        srv.server_stop()
        with pytest.raises(ApoError):
            srv.submit(np.arange(10, dtype=np.uint64), 2)


def _same_shape_batches(seed):
    """Two window layouts with the same window count, total length and longest window."""
    rng = np.random.default_rng(seed)
    lens_a = [3000, 700, 9000, 1, 0, 4200, 2500]
    lens_b = [9000, 2600, 3000, 700, 4100, 1, 0]
    assert sum(lens_a) == sum(lens_b) and max(lens_a) == max(lens_b)
    out = []
    for lens in (lens_a, lens_b):
        wins = [synth.loop_stream(int(rng.integers(1 << 30)), L, int(rng.integers(10, 80)), 64, 0.05) if L > 1
                else np.full(L, 7, np.uint64) for L in lens]
        out.append(wins)
    return out


def test_graph_capture_and_replay(ctx):
    """The batched launch sequence is captured once and replayed: results of
    every replay equal the per-window results, with eager work between
    replays, tokens rewritten in place, and a new layout of the same shape."""
    import torch
    from paper_2406_18111_amd import Context
    wins_a, wins_b = _same_shape_batches(21)
    with Context(0) as g:
        g.set_graphs(True)
        g.set_lanes(1)  # graphs record single-stream batches
        toks_a, off_a = _pack(wins_a)
        dev = torch.from_numpy(toks_a.view(np.int64)).cuda()
        for rep in range(3):
            rows, oo = g.analyze_batch_dev(dev, off_a, 4)
            rows = rows.cpu().numpy().astype(np.int64)
            for w, win in enumerate(wins_a):
                assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 4)), (rep, w)
            # eager work between replays on the same context
            assert np.array_equal(_as3(g.analyze(wins_a[0], 4)), _rows_ref(wins_a[0], 4))
        st = g.graph_stats()
        assert st["captures"] == 1 and st["replays"] == 2
        # same pointer and shape, other tokens and window boundaries
        toks_b, off_b = _pack(wins_b)
        dev.copy_(torch.from_numpy(toks_b.view(np.int64)))
        rows, oo = g.analyze_batch_dev(dev, off_b, 4)
        rows = rows.cpu().numpy().astype(np.int64)
        for w, win in enumerate(wins_b):
            assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 4)), w
        assert g.graph_stats()["replays"] == 3


def test_lane_graph_capture_and_replay():
    """Three lanes captured as branches of one graph: every replay (tokens
    rewritten in place, other window boundaries of the same shape, eager work
    in between) equals the oracle; a new shape is captured anew."""
    import torch
    from paper_2406_18111_amd import Context
    wins_a, wins_b = _same_shape_batches(33)
    with Context(0) as g:
        g.set_graphs(True)
        g.set_lanes(3)
        toks_a, off_a = _pack(wins_a)
        dev = torch.from_numpy(toks_a.view(np.int64)).cuda()
        for rep in range(3):
            rows, oo = g.analyze_batch_dev(dev, off_a, 4)
            rows = rows.cpu().numpy().astype(np.int64)
            for w, win in enumerate(wins_a):
                assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 4)), (rep, w)
            assert np.array_equal(_as3(g.analyze(wins_a[1], 4)), _rows_ref(wins_a[1], 4))
        st = g.graph_stats()
        assert st["captures"] == 1 and st["replays"] == 2
        toks_b, off_b = _pack(wins_b)
        dev.copy_(torch.from_numpy(toks_b.view(np.int64)))
        rows, oo = g.analyze_batch_dev(dev, off_b, 4)
        rows = rows.cpu().numpy().astype(np.int64)
        for w, win in enumerate(wins_b):
            assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 4)), w
        # a different shape: captured again, still exact
        wins_c = wins_a[:5]
        toks_c, off_c = _pack(wins_c)
        rows, oo = g.analyze_batch_dev(torch.from_numpy(toks_c.view(np.int64)).cuda(), off_c, 4)
        rows = rows.cpu().numpy().astype(np.int64)
        for w, win in enumerate(wins_c):
            assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 4)), w
        assert g.graph_stats()["captures"] >= 2


@pytest.mark.parametrize("lanes", [1, 2, 3, 4])
@pytest.mark.parametrize("window_greedy", [True, False])
def test_lanes_give_identical_results(lanes, window_greedy):
    """Concurrent window groups on separate streams: every lane count gives
    the rows of the single-stream batch and of the oracle, with the
    per-window greedy and with the round-based selection."""
    import torch
    from paper_2406_18111_amd import Context
    wins = _mixed_windows(17, 23) + [np.zeros(0, np.uint64)] * 3
    toks, off = _pack(wins)
    dev = torch.from_numpy(toks.view(np.int64)).cuda()
    with Context(0) as g:
        g.set_lanes(lanes)
        g.set_window_greedy(window_greedy)
        for m in (2, 8):
            rows, oo = g.analyze_batch_dev(dev, off, m)
            rows = rows.cpu().numpy().astype(np.int64)
            hrows, hoo = g.analyze_batch(toks, off, m)
            assert np.array_equal(oo, hoo)
            assert np.array_equal(rows, _as3(hrows))
            for w, win in enumerate(wins):
                assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, m)), (lanes, m, w)
    with pytest.raises(Exception):
        Context(0).set_lanes(5)


def test_batch_tuning_keeps_results():
    """The batch autotuner times all 12 (tile, digit) pairs on the batch; the
    chosen pair is used afterwards and results stay those of the oracle."""
    import torch
    from paper_2406_18111_amd import Context
    wins, m = synth.config3(num_windows=30)
    toks, off = _pack(wins)
    dev = torch.from_numpy(toks.view(np.int64)).cuda()
    with Context(0) as g:
        tl, db, ms = g.tune_batch(dev, off, m, reps=1)
        assert 11 <= tl <= 13 and db in (8, 10, 11, 12) and ms > 0
        rows, oo = g.analyze_batch_dev(dev, off, m)
        rows = rows.cpu().numpy().astype(np.int64)
        for w, win in enumerate(wins):
            assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, m)), w


def test_sync_free_batch_without_graphs(ctx):
    import torch
    from paper_2406_18111_amd import Context
    wins, m = synth.config3(num_windows=40)
    toks, off = _pack(wins)
    with Context(0) as g:
        g.set_graphs(False)
        rows, oo = g.analyze_batch_dev(torch.from_numpy(toks.view(np.int64)).cuda(), off, m)
        rows = rows.cpu().numpy().astype(np.int64)
        for w, win in enumerate(wins):
            assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, m)), w
        assert g.graph_stats()["captures"] == 0


def test_batch_needing_many_selection_rounds(ctx):
    """Block families need more greedy rounds than a sync-free batch enqueues;
    the batch then completes host-driven with the same result."""
    import torch
    blocks = []
    for k in range(1, 60):
        blocks += [0] * k + [1]
    wins = [np.array(blocks, dtype=np.uint64), synth.config0()[0]]
    toks, off = _pack(wins)
    rows, oo = ctx.analyze_batch_dev(torch.from_numpy(toks.view(np.int64)).cuda(), off, 1)
    rows = rows.cpu().numpy().astype(np.int64)
    for w, win in enumerate(wins):
        assert np.array_equal(rows[int(oo[w]):int(oo[w + 1])], _rows_ref(win, 1)), w


def test_tracer_ruler_slices(ctx):
    """Trace finder: after every block of 250 tokens the ruler slice of the
    last <= 5000 tokens is analysed asynchronously; each result equals the
    single-window analysis of that slice of the stream."""
    from paper_2406_18111_amd import Context, _lib
    src = synth.NestedLoopSource(77, alphabet=1 << 10)
    stream = src.take(12000)
    with Context(0) as srv:
        srv.server_start(slots=2)
        tr = _lib.Tracer(srv, block_tokens=250, capacity=5000, min_len=8, stream_id=3)
        submitted = 0
        for k in range(0, len(stream), 700):
            submitted += tr.push(stream[k:k + 700])
        assert submitted == len(stream) // 250
        results = []
        t0 = time.time()
        while len(results) < submitted and time.time() - t0 < 120:
            got = tr.poll()
            if got is None:
                time.sleep(0.002)
            else:
                results.append(got)
        assert len(results) == submitted
        for i, (b, ln, rows) in enumerate(results, start=1):
            assert ln == min(_lib.ruler_slice(i, 250, 5000), 250 * i)
            assert b + ln == 250 * i
            assert np.array_equal(_as3(rows), _as3(ctx.analyze(stream[b:b + ln], 8))), i
        tr.close()
        srv.server_stop()
