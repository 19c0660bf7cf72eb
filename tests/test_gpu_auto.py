"""Algorithm 1 end to end on the GPU: ruler-sampled FindRepeats on the server,
deterministic ingestion, max-trace-length split and trace replay.  The event
stream must equal the plain reference driven by the same ingestion schedule
(analyses computed by the oracle), and replicas sharing an agreement object
must take identical decisions."""
import threading

import numpy as np
import pytest

import oracle
from oracle.replayer import ReplayerRef, split_rows as split_ref
from paper_2406_18111_amd import _lib, synth

pytestmark = pytest.mark.gpu

P = dict(block_tokens=250, capacity=5000, min_len=25, max_trace_len=200, count_cap=8, decay=0.999,
         replay_bonus=0.1)


def _reference(stream, log):
    ref = ReplayerRef(P["count_cap"], P["decay"], P["replay_bonus"])
    by_task = {}
    for rec in log:
        by_task.setdefault(int(rec["ingested_at"]) - 1, []).append(rec)
    for t, tok in enumerate(stream):
        for rec in by_task.get(t, []):
            b, ln = int(rec["slice_begin"]), int(rec["slice_len"])
            sl = stream[b:b + ln]
            res = oracle.find_repeats(sl, P["min_len"])
            rows = list(zip(res["row_start"].tolist(), res["row_len"].tolist(), res["row_count"].tolist()))
            pieces = split_ref(rows, P["max_trace_len"], P["min_len"])
            assert len(pieces) == int(rec["pieces"])
            ref.ingest(sl, pieces)
        ref.step([tok])
    ref.flush()
    return ref


def _check_schedule(log, lag0):
    """Ingestion points follow from submission points and the lag rule."""
    lag, prev = lag0, 0
    for j, rec in enumerate(log):
        assert int(rec["submitted_at"]) == (j + 1) * P["block_tokens"]
        assert int(rec["slice_len"]) == min(_lib.ruler_slice(j + 1, P["block_tokens"], P["capacity"]),
                                            int(rec["submitted_at"]))
        assert int(rec["slice_begin"]) + int(rec["slice_len"]) == int(rec["submitted_at"])
        assert int(rec["ingested_at"]) == max(int(rec["submitted_at"]) + lag, prev)
        prev = int(rec["ingested_at"])
        if rec["any_waited"]:
            lag = max(2 * lag, P["block_tokens"])
    return lag


@pytest.fixture(scope="module")
def srv():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_18111_amd import Context
    c = Context(0)
    c.server_start(slots=2)
    yield c
    c.server_stop()
    c.close()


@pytest.mark.parametrize("lag0", [0, 1000])
def test_auto_single_node_matches_reference(srv, lag0):
    src = synth.NestedLoopSource(91, alphabet=1 << 12)
    stream = src.take(12000)
    a = _lib.Auto(srv, stream_id=1, lag0=lag0, **P)
    for k in range(0, len(stream), 997):
        a.execute(stream[k:k + 997])
    rp = a.replayer
    rp.flush()
    ev = [(int(b), int(e), int(t)) for b, e, t in rp.events()]
    log = a.ingests()
    lag, waits = a.lag()
    print("analyses", len(log), "lag", lag, "waits", waits, "stats", rp.stats(), flush=True)
    assert len(log) >= len(stream) // P["block_tokens"] - (lag // P["block_tokens"]) - 1
    assert _check_schedule(log, lag0) == lag
    ref = _reference([int(x) for x in stream], log)
    assert ev == ref.events
    half = len(stream) // 2
    late = sum(e - max(b, half) for b, e, t in ev if t >= 0 and e > half)
    assert late > 0.4 * (len(stream) - half)  # a noisy loop stream, mostly replayed once traces are known
    a.close()


def test_auto_replicas_agree(srv):
    """Two replicas of one stream, each with its own analyses, ingest at the
    same tasks and replay the same traces."""
    src = synth.NestedLoopSource(5, alphabet=1 << 12)
    stream = src.take(8000)
    ag = _lib.Agreement(2, timeout_ms=60000)
    nodes = [_lib.Auto(srv, stream_id=10 + k, lag0=0, agreement=ag, node=k, **P) for k in range(2)]
    err = []

    def run(k):
        try:
            step = 331 if k == 0 else 977  # the replicas advance in different chunks
            for i in range(0, len(stream), step):
                nodes[k].execute(stream[i:i + step])
        except Exception as e:
            err.append(e)

    th = [threading.Thread(target=run, args=(k,)) for k in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(300)
    assert not err, err
    logs = [n.ingests() for n in nodes]
    keys = ["submitted_at", "ingested_at", "slice_begin", "slice_len", "pieces", "any_waited"]
    assert all(np.array_equal(logs[0][k], logs[1][k]) for k in keys)
    evs = []
    for n in nodes:
        n.replayer.flush()
        evs.append([(int(b), int(e), int(t)) for b, e, t in n.replayer.events()])
    assert evs[0] == evs[1]
    for n in nodes:
        n.close()
    ag.close()
