"""Ingestion agreement (Section 5.1) on the CPU: host threads stand in for the
nodes of a replicated runtime."""
import threading

import pytest

from paper_2406_18111_amd import _lib


def _run_nodes(ag, nodes, rounds, waits):
    """Every node votes on every analysis; waits[j] = set of nodes that waited."""
    out = [[None] * rounds for _ in range(nodes)]
    err = []

    def node(k):
        try:
            for j in range(rounds):
                out[k][j] = ag.vote(k, j, k in waits.get(j, ()))
        except Exception as e:  # surfaced in the main thread
            err.append(e)

    th = [threading.Thread(target=node, args=(k,)) for k in range(nodes)]
    for t in th:
        t.start()
    for t in th:
        t.join(60)
    assert not err, err
    return out


def test_vote_is_an_or_over_nodes():
    ag = _lib.Agreement(4, timeout_ms=20000)
    waits = {1: {2}, 3: {0, 3}, 6: {1}}
    out = _run_nodes(ag, 4, 8, waits)
    want = [j in waits for j in range(8)]
    for k in range(4):
        assert out[k] == want
    ag.close()


def test_single_node_vote_returns_own_flag():
    ag = _lib.Agreement(1)
    assert ag.vote(0, 0, True) is True
    assert ag.vote(0, 1, False) is False
    ag.close()


def test_missing_node_times_out_and_vote_can_be_repeated():
    ag = _lib.Agreement(2, timeout_ms=50)
    with pytest.raises(_lib.ApoError) as e:
        ag.vote(0, 0, True)
    assert e.value.code == _lib.APO_EAGAIN
    # the withdrawn vote can be cast again once the other node shows up
    res = {}
    t = threading.Thread(target=lambda: res.setdefault(1, ag.vote(1, 0, False)))
    t.start()
    import time
    time.sleep(0.01)
    got = None
    for _ in range(100):
        try:
            got = ag.vote(0, 0, True)
            break
        except _lib.ApoError as err:
            assert err.code == _lib.APO_EAGAIN
    t.join(10)
    assert got is True and res[1] is True
    ag.close()


def test_vote_errors():
    ag = _lib.Agreement(2, timeout_ms=10)
    with pytest.raises(_lib.ApoError):
        ag.vote(2, 0, False)          # no such node
    lib = _lib.load()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.apo_agree_create(0, 0, ctypes.byref(h)) == _lib.APO_EINVAL
    assert lib.apo_agree_create(65, 0, ctypes.byref(h)) == _lib.APO_EINVAL
    ag.close()


def test_many_nodes_many_rounds():
    ag = _lib.Agreement(16, timeout_ms=30000)
    waits = {j: {j % 16} for j in range(0, 200, 7)}
    out = _run_nodes(ag, 16, 200, waits)
    want = [j in waits for j in range(200)]
    assert all(o == want for o in out)
    ag.close()
