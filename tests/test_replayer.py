"""Trace replayer (Section 4.3) and max-trace-length split (Section 6.2):
the native host implementation against the plain reference in
``oracle.replayer`` and against hand-derived outcomes of the scoring rules."""
import numpy as np
import pytest

import oracle
from oracle.replayer import ReplayerRef, split_rows as split_ref
from paper_2406_18111_amd import _lib, synth


def _rows(lst):
    return np.array([tuple(r) for r in lst], dtype=_lib.ROW_DTYPE)


def _events(ev):
    return [(int(b), int(e), int(t)) for b, e, t in ev]


def _check_partition(events, tokens, cands):
    """Events tile [0, n) in order; every replayed range holds its trace."""
    pos = 0
    for b, e, t in events:
        assert b == pos and e > b
        if t >= 0:
            assert tuple(tokens[b:e]) == cands[t]
        pos = e
    return pos


# ---- max trace length -------------------------------------------------------

def test_split_rows_pins():
    # 450 tokens with a 200 cap: 200 + 200 + 50 (Section 6.2's auto-200 reading)
    got = _lib.split_rows(_rows([(10, 450, 3)]), 200, 25)
    assert [tuple(map(int, r)) for r in got] == [(10, 200, 3), (210, 200, 3), (410, 50, 3)]
    got = _lib.split_rows(_rows([(10, 450, 3)]), 200, 60)
    assert [tuple(map(int, r)) for r in got] == [(10, 200, 3), (210, 200, 3)]
    # rows at or below the cap pass unchanged; an exact multiple has no tail
    got = _lib.split_rows(_rows([(0, 200, 2), (5, 30, 9), (0, 400, 4)]), 200, 25)
    assert [tuple(map(int, r)) for r in got] == [(0, 200, 2), (5, 30, 9), (0, 200, 4), (200, 200, 4)]
    assert len(_lib.split_rows(_rows([]), 200, 25)) == 0


def test_split_rows_matches_reference():
    rng = np.random.default_rng(3)
    rows = [(int(rng.integers(0, 1000)), int(rng.integers(1, 2000)), int(rng.integers(2, 50))) for _ in range(300)]
    for max_len, min_len in ((200, 25), (1, 1), (7, 3), (5000, 25)):
        got = [tuple(map(int, r)) for r in _lib.split_rows(_rows(rows), max_len, min_len)]
        assert got == split_ref(rows, max_len, min_len)
        # pieces never exceed the cap and cover each row's prefix of full pieces
        assert all(min_len <= ln <= max_len for _, ln, _ in got)


def test_split_rows_errors():
    lib = _lib.load()
    import ctypes
    n = ctypes.c_uint32(0)
    assert lib.apo_split_rows(None, 0, 0, 1, None, 0, ctypes.byref(n)) == _lib.APO_EINVAL
    assert lib.apo_split_rows(None, 0, 5, 0, None, 0, ctypes.byref(n)) == _lib.APO_EINVAL
    r = _rows([(0, 10, 2)])
    assert lib.apo_split_rows(_lib._np_ptr(r), 1, 3, 1, None, 0, ctypes.byref(n)) == _lib.APO_ERANGE
    assert n.value == 4


# ---- replayer: hand-derived outcomes ------------------------------------------

def _run(cands, counts, stream, **kw):
    toks = np.concatenate([np.asarray(c, np.uint64) for c in cands])
    rows, off = [], 0
    for c, k in zip(cands, counts):
        rows.append((off, len(c), k))
        off += len(c)
    r = _lib.Replayer(**kw)
    r.ingest(toks, _rows(rows))
    r.step(np.asarray(stream, np.uint64))
    r.flush()
    ev = _events(r.events())
    st = r.stats()
    r.close()
    _check_partition(ev, list(stream), [tuple(c) for c in cands])
    return ev, st


def test_replay_pure_repetition():
    ev, st = _run([(1, 2, 3, 4)], [2], [1, 2, 3, 4] * 5 + [9])
    assert ev == [(4 * i, 4 * i + 4, 0) for i in range(5)] + [(20, 21, -1)]
    assert st == {"tasks": 21, "traced": 20, "replays": 5, "traces": 1}


def test_untraced_prefix_then_replay():
    # 5 1 2 is pending while the match 1 2 ... lives; 5 goes out at once
    ev, _ = _run([(1, 2, 3)], [2], [5, 1, 2, 1, 2, 3, 7])
    assert ev == [(0, 3, -1), (3, 6, 0), (6, 7, -1)]


def test_longer_trace_wins_same_count():
    # both end at the 4: (9 2 3 4) scores 4 * 3, (2 3 4) scores 3 * 3
    ev, _ = _run([(2, 3, 4), (9, 2, 3, 4)], [2, 2], [9, 2, 3, 4], decay=1.0)
    assert ev == [(0, 4, 1)]


def test_count_cap():
    # (3 4 5) seen 100 times vs (1 2 3 4 5) twice: cap 8 -> 3*8 = 24 > 5*3 = 15;
    # cap 2 -> 3*2 = 6 < 5*2 = 10
    cands, counts, stream = [(3, 4, 5), (1, 2, 3, 4, 5)], [100, 2], [1, 2, 3, 4, 5]
    assert _run(cands, counts, stream, count_cap=8, decay=1.0)[0] == [(0, 2, -1), (2, 5, 0)]
    assert _run(cands, counts, stream, count_cap=2, decay=1.0)[0] == [(0, 5, 1)]


def test_replay_bonus():
    # (2 3 4) is replayed once alone; then both complete with base score 12:
    # the bonus picks the one replayed before, without it the tie goes to id 0
    cands, counts = [(9, 2, 3, 4), (2, 3, 4)], [2, 2]
    stream = [7, 2, 3, 4, 9, 2, 3, 4]
    ev, _ = _run(cands, counts, stream, count_cap=100, decay=1.0, replay_bonus=0.1)
    assert ev == [(0, 1, -1), (1, 4, 1), (4, 5, -1), (5, 8, 1)]
    ev, _ = _run(cands, counts, stream, count_cap=100, decay=1.0, replay_bonus=0.0)
    assert ev == [(0, 1, -1), (1, 4, 1), (4, 8, 0)]


def test_decay():
    # (2 3 4) recurs every 4 tasks (count saturates at the cap of 3, replayed:
    # 3*3*1.1 = 9.9); (7 8 9 2 3 4) was ingested 506 tasks earlier with count 2:
    # without decay 6*3 = 18 wins, with decay 0.99 its count is
    # 2*0.99^506 + 1 ~ 1.012 and 6*1.012 < 9.9.
    cands, counts = [(2, 3, 4), (7, 8, 9, 2, 3, 4)], [2, 2]
    stream = [2, 3, 4, 0] * 125 + [7, 8, 9, 2, 3, 4]
    ev, _ = _run(cands, counts, stream, count_cap=3, decay=1.0)
    assert ev[-1] == (500, 506, 1)
    ev, _ = _run(cands, counts, stream, count_cap=3, decay=0.99)
    assert ev[-1] == (503, 506, 0) and ev[-2] == (499, 503, -1) and ev[-3] == (496, 499, 0)


def test_replayer_errors():
    import ctypes
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.apo_replayer_create(0, 0.9, 0.1, ctypes.byref(h)) == _lib.APO_EINVAL
    assert lib.apo_replayer_create(8, 0.0, 0.1, ctypes.byref(h)) == _lib.APO_EINVAL
    assert lib.apo_replayer_create(8, 1.5, 0.1, ctypes.byref(h)) == _lib.APO_EINVAL
    assert lib.apo_replayer_create(8, 0.9, -1.0, ctypes.byref(h)) == _lib.APO_EINVAL
    r = _lib.Replayer()
    with pytest.raises(_lib.ApoError):
        r.ingest(np.arange(5, dtype=np.uint64), _rows([(3, 5, 2)]))  # row outside the tokens
    with pytest.raises(_lib.ApoError):
        r.ingest(np.arange(5, dtype=np.uint64), _rows([(3, 0, 2)]))  # empty row
    r.step(np.zeros(0, np.uint64))
    r.flush()
    assert len(r.events()) == 0
    # many events: the binding retries with the needed capacity
    r.ingest(np.array([1, 2], np.uint64), _rows([(0, 2, 2)]))
    r.step(np.tile(np.array([1, 2, 5], np.uint64), 1000))
    ev = r.events()
    assert len(ev) == 2000 and int(ev[-1]["end"]) == 3000
    r.close()


# ---- replayer vs the plain reference on FindRepeats output --------------------------

@pytest.mark.parametrize("seed", range(6))
def test_replayer_matches_reference(seed):
    rng = np.random.default_rng(100 + seed)
    kw = dict(count_cap=int(rng.integers(1, 10)), decay=float(rng.choice([1.0, 0.999, 0.95])),
              replay_bonus=float(rng.choice([0.0, 0.1, 0.5])))
    period = int(rng.integers(5, 30))
    stream = synth.loop_stream(seed, 3000, period, 12, float(rng.choice([0.0, 0.02, 0.1])))
    ref, nat = ReplayerRef(**kw), _lib.Replayer(**kw)
    pos, hist, next_ingest = 0, 600, 600
    while pos < len(stream):
        if pos >= next_ingest:
            next_ingest += hist
            # candidate traces from the history so far, min_len as the trace finder would use
            window = stream[pos - hist:pos]
            res = oracle.find_repeats(window, 4)
            rows = list(zip(res["row_start"].tolist(), res["row_len"].tolist(), res["row_count"].tolist()))
            rows = split_ref(rows, 40, 4)
            ref.ingest(window, rows)
            nat.ingest(window, _rows(rows))
        k = int(rng.integers(0, 97))
        chunk = stream[pos:pos + k]
        ref.step(chunk)
        nat.step(chunk)
        pos += len(chunk)
    ref.flush()
    nat.flush()
    ev = _events(nat.events())
    assert ev == ref.events
    n = _check_partition(ev, [int(x) for x in stream], ref.cands)
    assert n == len(stream)
    st = nat.stats()
    assert st["traces"] == len(ref.cands) > 0 and st["tasks"] == len(stream) and st["replays"] > 0
    assert st["traced"] == sum(e - b for b, e, t in ev if t >= 0)
    nat.close()


def test_periodic_stream_mostly_traced():
    """A loop repeating one 20-task body: after one analysis of 200 tasks
    nearly every later task is issued inside a replayed trace."""
    body = np.arange(100, 120, dtype=np.uint64)
    stream = np.tile(body, 60)
    hist = stream[:200]
    res = oracle.find_repeats(hist, 5)
    rows = _rows(zip(res["row_start"].tolist(), res["row_len"].tolist(), res["row_count"].tolist()))
    r = _lib.Replayer()
    r.ingest(hist, rows)
    r.step(stream[200:])
    r.flush()
    st = r.stats()
    assert st["traced"] >= 0.95 * (len(stream) - 200)
    r.close()
