"""apo_analyze_window_noalloc (the entry point whose workspace is a fixed
device array, for callers that cannot allocate) against
apo_analyze_window_dev on the same inputs, through the C ABI: identical rows
and occurrences, bit for bit, on consecutive calls that reuse the array with
a smaller input second, at the size limit, and a clear refusal above it."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2406_18111_amd import _lib, synth

pytestmark = pytest.mark.gpu

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "apo.h")


def _limit():
    m = re.search(r"#define APO_NOALLOC_MAX_N \(1u << (\d+)\)", open(HEADER).read())
    return 1 << int(m.group(1))


def _call(lib, fn, ctx, dev, bits, n, m, cap):
    import torch
    rows = torch.full((max(cap, 1), 3), -1, dtype=torch.int32, device="cuda")
    occ = torch.full((max(cap, 1), 3), -1, dtype=torch.int32, device="cuda")
    rn, on = ctypes.c_uint32(0), ctypes.c_uint32(0)
    rc = getattr(lib, fn)(ctx, ctypes.c_void_p(dev.data_ptr()), bits, n, m, ctypes.c_void_p(rows.data_ptr()), cap,
                          ctypes.byref(rn), ctypes.c_void_p(occ.data_ptr()), cap, ctypes.byref(on), None)
    return rc, rows[: rn.value].cpu().numpy(), occ[: on.value].cpu().numpy()


def _dev(t):
    import torch
    t = np.ascontiguousarray(t)
    return torch.from_numpy(t.view(np.int64) if t.dtype == np.uint64 else t.view(np.int32)).cuda()


def test_noalloc_matches_device_entry_point():
    import torch
    assert torch.cuda.is_available()
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.apo_create(ctypes.byref(h), 0, 0) == _lib.APO_OK
    try:
        nmax = _limit()
        rng = np.random.default_rng(99)
        cases = [synth.config0(),                                           # 4096 tokens
                 (synth.loop_stream(7, 1500, 30, 64, 0.05), 4),              # smaller, right after
                 (synth.config1(n=nmax)[0], 16),                             # at the limit
                 (rng.integers(0, 3, 20000).astype(np.uint64), 2),
                 (np.full(3000, 9, np.uint64), 8),
                 (rng.integers(0, 4, 12000).astype(np.uint32), 3),           # 32-bit tokens
                 (synth.loop_stream(8, 700, 20, 16, 0.0), 5)]
        for t, m in cases:
            dev = _dev(t)
            bits = 64 if t.dtype == np.uint64 else 32
            cap = max(len(t) // m, 1)
            rc_n, rows_n, occ_n = _call(lib, "apo_analyze_window_noalloc", h, dev, bits, len(t), m, cap)
            rc_d, rows_d, occ_d = _call(lib, "apo_analyze_window_dev", h, dev, bits, len(t), m, cap)
            assert rc_n == _lib.APO_OK and rc_d == _lib.APO_OK, (len(t), rc_n, rc_d)
            assert np.array_equal(rows_n, rows_d), len(t)
            assert np.array_equal(occ_n, occ_d), len(t)
            ref = oracle.find_repeats(t, m)
            assert np.array_equal(rows_n[:, 0].astype(np.int64), ref["row_start"])
            assert np.array_equal(rows_n[:, 2].astype(np.int64), ref["row_count"])
        # above the limit: refused, nothing written
        t = synth.config1(n=nmax + 1)[0]
        rc, rows, _ = _call(lib, "apo_analyze_window_noalloc", h, _dev(t), 64, len(t), 16, 4096)
        assert rc == _lib.APO_ENOMEM and len(rows) == 0
        # too small an output buffer: the required count, nothing written
        t, m = synth.config0()
        dev = _dev(t)
        need = len(oracle.find_repeats(t, m)["row_start"])
        out = torch.full((need, 3), -5, dtype=torch.int32, device="cuda")
        rn = ctypes.c_uint32(0)
        rc = lib.apo_analyze_window_noalloc(h, ctypes.c_void_p(dev.data_ptr()), 64, len(t), m,
                                            ctypes.c_void_p(out.data_ptr()), need - 1, ctypes.byref(rn), None, 0,
                                            None, None)
        assert rc == _lib.APO_ERANGE and rn.value == need and bool((out == -5).all())
    finally:
        lib.apo_destroy(h)
