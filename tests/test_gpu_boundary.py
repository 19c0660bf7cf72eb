"""Error conventions of the C ABI, called through ctypes on the GPU:

* APO_ERANGE when an output buffer is too small: the required count is
  returned and nothing is written;
* APO_ENOMEM when a workspace would exceed the context's device-memory
  budget: the context stays usable, batches fall back to fewer lanes, and the
  bytes held never exceed the budget;
* the server queues windows that fit its memory pool until memory frees up
  and refuses (APO_ENOMEM) only a window that could never fit;
* a device error reported inside an analysis returns APO_EDEVICE and leaves
  the context usable.
"""
import ctypes
import threading
import time

import numpy as np
import pytest

import oracle
from paper_2406_18111_amd import _lib, synth

pytestmark = pytest.mark.gpu


def _rows_ref(t, m):
    r = oracle.find_repeats(t, m)
    return np.stack([r["row_start"], r["row_len"], r["row_count"]], 1).astype(np.int64).reshape(-1, 3)


def _as3(rows):
    return np.stack([rows["start"], rows["length"], rows["count"]], 1).astype(np.int64).reshape(-1, 3)


def _pack(wins):
    off = np.zeros(len(wins) + 1, dtype=np.uint64)
    off[1:] = np.cumsum([len(w) for w in wins])
    return np.concatenate(wins).astype(np.uint64), off


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_18111_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_erange_host_window(ctx):
    """Too small a row or occurrence buffer: APO_ERANGE, *out_n / *occ_n hold
    the required counts, and the buffers are left untouched."""
    lib = _lib.load()
    t, m = synth.config0()
    ref = oracle.find_repeats(t, m)
    need_rows, need_occ = len(ref["row_start"]), len(ref["occ_start"])
    assert need_rows > 2
    for cap_rows, cap_occ in ((need_rows - 1, need_occ), (need_rows, need_occ - 1), (0, 0)):
        rows = np.full(max(cap_rows, 1), 0xAB, dtype=_lib.ROW_DTYPE)
        occ = np.full(max(cap_occ, 1), 0xCD, dtype=_lib.OCC_DTYPE)
        before_r, before_o = rows.copy(), occ.copy()
        rn, on = ctypes.c_uint32(0), ctypes.c_uint32(0)
        rc = lib.apo_analyze_window(ctx._h, _lib._np_ptr(t), len(t), m, _lib._np_ptr(rows), cap_rows,
                                    ctypes.byref(rn), _lib._np_ptr(occ), cap_occ, ctypes.byref(on))
        assert rc == _lib.APO_ERANGE
        assert rn.value == need_rows and on.value == need_occ
        assert np.array_equal(rows, before_r) and np.array_equal(occ, before_o)
    # exactly the required sizes succeed
    rows = np.zeros(need_rows, dtype=_lib.ROW_DTYPE)
    rn = ctypes.c_uint32(0)
    assert lib.apo_analyze_window(ctx._h, _lib._np_ptr(t), len(t), m, _lib._np_ptr(rows), need_rows,
                                  ctypes.byref(rn), None, 0, None) == _lib.APO_OK
    assert np.array_equal(_as3(rows), _rows_ref(t, m))


def test_erange_device_window_and_batch(ctx):
    import torch
    lib = _lib.load()
    t, m = synth.config0()
    need = len(_rows_ref(t, m))
    dev = torch.from_numpy(t.view(np.int64)).cuda()
    out = torch.full((need, 3), -7, dtype=torch.int32, device="cuda")
    rn = ctypes.c_uint32(0)
    rc = lib.apo_analyze_window_dev(ctx._h, _lib._dev_ptr(dev), 64, len(t), m, _lib._dev_ptr(out), need - 1,
                                    ctypes.byref(rn), None, 0, None, None)
    assert rc == _lib.APO_ERANGE and rn.value == need
    assert bool((out == -7).all())
    # batch: the required total is in out_offsets[W]; no row is written
    wins = [synth.loop_stream(s, 3000, 40, 64, 0.05) for s in (1, 2, 3)]
    toks, off = _pack(wins)
    total_rows = sum(len(_rows_ref(w, 8)) for w in wins)
    rows = np.full(total_rows, 0x5A, dtype=_lib.ROW_DTYPE)
    before = rows.copy()
    oo = np.zeros(len(wins) + 1, dtype=np.uint64)
    rc = lib.apo_analyze_batch(ctx._h, _lib._np_ptr(toks), _lib._np_ptr(off), len(wins), 8, _lib._np_ptr(rows),
                               total_rows - 1, _lib._np_ptr(oo))
    assert rc == _lib.APO_ERANGE and int(oo[-1]) == total_rows
    assert np.array_equal(rows, before)


def test_enomem_small_budget_context_stays_usable():
    """A 64 MiB budget: a 2^20-token window does not fit (APO_ENOMEM); the
    same context then analyses small windows and a small batch exactly, and
    never holds more than its budget."""
    from paper_2406_18111_amd import ApoError, Context
    budget = 64 << 20
    with Context(0, budget_bytes=budget) as c:
        t1, m1 = synth.config1()
        with pytest.raises(ApoError) as e:
            c.analyze(t1, m1)
        assert e.value.code == _lib.APO_ENOMEM
        assert c.memory()["held"] <= budget
        t0, m0 = synth.config0()
        assert np.array_equal(_as3(c.analyze(t0, m0)), _rows_ref(t0, m0))
        wins, m = synth.config3(num_windows=12, hi=4096)
        toks, off = _pack(wins)
        rows, oo = c.analyze_batch(toks, off, m)
        for w, win in enumerate(wins):
            assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), _rows_ref(win, m)), w
        assert 0 < c.memory()["held"] <= budget


def test_budget_caps_lane_workspaces():
    """Batches split into lanes keep the sum of all workspaces within the
    budget: with room for about one full-batch workspace the batch runs on
    fewer lanes, with the same rows."""
    from paper_2406_18111_amd import Context
    wins, m = synth.config3(num_windows=40, hi=1 << 14)
    toks, off = _pack(wins)
    total = int(off[-1])
    with Context(0) as probe:
        probe.set_lanes(1)
        probe.analyze_batch(toks, off, m)
        one = probe.memory()["held"]
    budget = int(one * 1.3)
    with Context(0, budget_bytes=budget) as c:
        c.set_lanes(3)
        for rep in range(2):
            rows, oo = c.analyze_batch(toks, off, m)
            assert c.memory()["held"] <= budget, (rep, c.memory(), budget, total)
            for w, win in enumerate(wins):
                assert np.array_equal(_as3(rows[int(oo[w]):int(oo[w + 1])]), _rows_ref(win, m)), (rep, w)
        # the device-pointer batch API under the same budget
        import torch
        dev = torch.from_numpy(toks.view(np.int64)).cuda()
        rows_d, oo_d = c.analyze_batch_dev(dev, off, m)
        assert np.array_equal(oo_d, oo)
        assert c.memory()["held"] <= budget


def test_server_queues_until_memory_frees():
    """A server whose pool holds one 2^17-token workspace but not two: eight
    such windows submitted at once on three slots all complete exactly (they
    wait in the queue for memory instead of failing), the slots never hold
    more than the pool, and only a window that could never fit is refused
    with APO_ENOMEM."""
    from paper_2406_18111_amd import ApoError, Context
    n = 1 << 17
    with Context(0) as probe:
        probe.analyze(synth.config1(n=n)[0], 16)
        one = probe.memory()["held"]
    budget = int(one * 1.5)
    wins = [synth.NestedLoopSource(300 + k).take(n) for k in range(8)]
    refs = [_rows_ref(w, 16) for w in wins]
    with Context(0, budget_bytes=budget) as srv:
        srv.server_start(slots=3)
        pool = srv.memory()["server_pool"]
        assert one <= pool <= budget
        with pytest.raises(ApoError) as e:
            srv.submit(synth.config1(n=1 << 20)[0], 16)
        assert e.value.code == _lib.APO_ENOMEM
        seen = []
        stop = threading.Event()

        def watch():
            while not stop.is_set():
                seen.append(srv.memory()["server_held"])
                time.sleep(0.001)

        th = threading.Thread(target=watch)
        th.start()
        tickets = [srv.submit(w, 16, k) for k, w in enumerate(wins)]
        got = [None] * len(wins)
        deadline = time.time() + 100
        while any(g is None for g in got) and time.time() < deadline:
            for i, tk in enumerate(tickets):
                if got[i] is None:
                    r = srv.fetch(tk)
                    if r is not None:
                        got[i] = _as3(r[0])
            time.sleep(0.002)
        stop.set()
        th.join()
        srv.server_stop()
    assert all(g is not None for g in got)
    for i in range(len(wins)):
        assert np.array_equal(got[i], refs[i]), i
    assert max(seen) <= pool


def test_injected_device_error_leaves_context_usable(ctx):
    """A device error reported at a host synchronisation inside an analysis
    surfaces as APO_EDEVICE; the next analyses on the same context are exact."""
    from paper_2406_18111_amd import ApoError
    t, m = synth.config1(n=1 << 16)
    ref = _rows_ref(t, m)
    for after in (0, 1, 3):
        ctx.inject_device_error(after)
        with pytest.raises(ApoError) as e:
            ctx.analyze(t, m)
        assert e.value.code == _lib.APO_EDEVICE, after
        assert np.array_equal(_as3(ctx.analyze(t, m)), ref), after
    ctx.inject_device_error(-1)
    assert np.array_equal(_as3(ctx.analyze(t, m)), ref)


_LIB_BEFORE_TORCH = r"""
import ctypes, sys
sys.path.insert(0, sys.argv[1])
from paper_2406_18111_amd import Context
c = Context(0)
import torch
x = torch.arange(8, device="cuda", dtype=torch.int64)
print("torch", int(x.sum().item()), flush=True)
c.close()
"""


def test_context_before_torch_cuda():
    """A context opened before the program touches PyTorch's GPU runtime
    leaves that runtime usable (PyTorch ships its own HIP runtime, which finds
    no device once another runtime holds the GPU, so the binding sets it up
    first).  Runs in a fresh process, since this one has PyTorch running."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", _LIB_BEFORE_TORCH, root], capture_output=True, text=True, timeout=180)
    assert p.returncode == 0, p.stderr[-2000:]
    assert "torch 28" in p.stdout
