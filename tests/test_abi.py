"""The C-ABI library loads and exports every entry point include/apo.h declares
(no GPU needed; no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apo.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apo_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for must in ("apo_create", "apo_destroy", "apo_analyze_window", "apo_analyze_batch", "apo_server_start",
                 "apo_submit", "apo_poll", "apo_fetch", "apo_server_stop", "apo_suffix_array_dev", "apo_lcp_dev",
                 "apo_candidates_dev"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2406_18111_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, name


def test_argument_errors_without_device():
    from paper_2406_18111_amd import _lib
    lib = _lib.load()
    assert lib.apo_create(None, 0, 0) == _lib.APO_EINVAL
    assert lib.apo_destroy(None) == _lib.APO_OK
    assert lib.apo_strerror(_lib.APO_ERANGE) == b"output buffer too small"
    out_n = ctypes.c_uint32(7)
    # null context is rejected before any device work
    assert lib.apo_analyze_window(None, None, 0, 1, None, 0, ctypes.byref(out_n), None, 0, None) == _lib.APO_EINVAL
    assert lib.apo_analyze_batch(None, None, None, 0, 1, None, 0, None) == _lib.APO_EINVAL
    assert lib.apo_submit(None, 0, None, 0, 1, None) == _lib.APO_EINVAL


def test_no_cpu_fallback_when_library_missing(monkeypatch, tmp_path):
    from paper_2406_18111_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError):
        _lib.load()


def test_ruler_slices():
    """Section 4.4: slices 1,2,1,4 on a buffer of four (block of one token);
    with a block of 250 and a buffer of 5000 the slices are 250 * 2^v(i),
    capped."""
    from paper_2406_18111_amd import _lib
    assert [_lib.ruler_slice(i, 1, 4) for i in range(1, 9)] == [1, 2, 1, 4, 1, 2, 1, 4]
    got = [_lib.ruler_slice(i, 250, 5000) for i in range(1, 33)]
    assert got[:8] == [250, 500, 250, 1000, 250, 500, 250, 2000]
    assert got[15] == 4000 and got[31] == 5000 and max(got) == 5000
    assert _lib.ruler_slice(0, 250, 5000) == 0
    # total work over K blocks: c * sum 2^v(i) = c * (K/2) * (log2 K + 2) for K a power of two (uncapped)
    K = 1024
    tot = sum(_lib.ruler_slice(i, 1, 1 << 30) for i in range(1, K + 1))
    assert tot == (K // 2) * (10 + 2)


def test_noalloc_scratch_holds_its_workspace():
    """The fixed array of the no-allocation entry point is large enough for
    the workspace of its longest window (checked without a device)."""
    from paper_2406_18111_amd import _lib
    src = open(HEADER).read()
    max_n = 1 << int(re.search(r"#define APO_NOALLOC_MAX_N \(1u << (\d+)\)", src).group(1))
    scratch = int(re.search(r"#define APO_NOALLOC_SCRATCH_BYTES \((\d+)u << 20\)", src).group(1)) << 20
    need = _lib.workspace_bytes(max_n, 1)
    assert 0 < need <= scratch, (need, scratch)
    assert _lib.workspace_bytes(max_n + 1, 1) > scratch  # the next size up would not fit
