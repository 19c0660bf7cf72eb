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
