"""CPU oracle for FindRepeats -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and has
no CPU fallback.

Two independent implementations of Algorithm 2 (Yadav et al., ASPLOS'25,
Section 4.2):

* :mod:`oracle.naive` -- literal pure Python, small inputs;
* ``findrepeats_ref.c`` -- the same algorithm in plain C with the textbook
  O(n log n) pieces the paper names (suffix array, Kasai LCP, ID-keyed sort,
  mark-array greedy), wrapped here with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "findrepeats_ref.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc into oracle/_build/liboracle.so."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.ref_token_ranks.argtypes = [p, i64, p]
        lib.ref_token_ranks.restype = i64
        lib.ref_suffix_array.argtypes = [p, i64, p, p]
        lib.ref_suffix_array.restype = i64
        lib.ref_lcp.argtypes = [p, i64, p, p]
        lib.ref_lcp.restype = ctypes.c_int
        lib.ref_find_repeats.argtypes = [p, i64, i64, p, p, p, p, p, p, p, p, p]
        lib.ref_find_repeats.restype = ctypes.c_int
        lib.ref_sorted_candidates.argtypes = [p, i64, i64, p, p, p, p]
        lib.ref_sorted_candidates.restype = i64
        _lib = lib
    return _lib


def _tokens(tokens) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(tokens))
    if t.dtype != np.uint64:
        if t.dtype.kind == "i" and t.size and t.min() < 0:
            raise ValueError("tokens must be non-negative")
        t = t.astype(np.uint64)
    return np.ascontiguousarray(t)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def token_ranks(tokens) -> np.ndarray:
    t = _tokens(tokens)
    r = np.zeros(len(t), dtype=np.int64)
    _load().ref_token_ranks(_ptr(t), len(t), _ptr(r))
    return r


def suffix_array(tokens, return_active: bool = False):
    t = _tokens(tokens)
    n = len(t)
    sa = np.zeros(max(n, 1), dtype=np.int64)
    act = np.zeros(64, dtype=np.int64)
    rounds = _load().ref_suffix_array(_ptr(t), n, _ptr(sa), _ptr(act))
    if rounds < 0:
        raise MemoryError("oracle suffix array")
    sa = sa[:n]
    if return_active:
        return sa, act[: min(int(rounds), 64)]
    return sa


def lcp(tokens, sa) -> np.ndarray:
    t = _tokens(tokens)
    sa = np.ascontiguousarray(np.asarray(sa, dtype=np.int64))
    out = np.zeros(max(len(t) - 1, 1), dtype=np.int64)
    if _load().ref_lcp(_ptr(t), len(t), _ptr(sa), _ptr(out)) != 0:
        raise MemoryError("oracle lcp")
    return out[: max(len(t) - 1, 0)]


def sorted_candidates(tokens, min_len: int):
    """Candidates with length >= min_len in the Sort(C) order, duplicates kept.

    Returns a structured dict of int64 arrays: len, id, start, pair.
    """
    t = _tokens(tokens)
    n = len(t)
    cap = max(2 * n, 1)
    arrs = {k: np.zeros(cap, dtype=np.int64) for k in ("len", "id", "start", "pair")}
    m = _load().ref_sorted_candidates(_ptr(t), n, int(min_len), _ptr(arrs["len"]),
                                      _ptr(arrs["id"]), _ptr(arrs["start"]), _ptr(arrs["pair"]))
    if m < 0:
        raise MemoryError("oracle candidates")
    return {k: v[:m] for k, v in arrs.items()}


STAT_NAMES = ("candidates", "rounds", "active_sum", "coverage", "occurrences", "rows",
              "max_lcp", "sigma")


def find_repeats(tokens, min_len: int, with_stats: bool = False):
    """FindRepeats(S) with minimum length.

    Returns dict with numpy int64 arrays: occ_start, occ_len, occ_row (acceptance
    order) and row_start, row_len, row_count (first-acceptance order).
    """
    if min_len < 1:
        raise ValueError("min_len must be >= 1")
    t = _tokens(tokens)
    n = len(t)
    cap = max(n, 1)
    o = {k: np.zeros(cap, dtype=np.int64) for k in
         ("occ_start", "occ_len", "occ_row", "row_start", "row_len", "row_count")}
    no = ctypes.c_int64(0)
    nr = ctypes.c_int64(0)
    st = np.zeros(8, dtype=np.int64)
    rc = _load().ref_find_repeats(_ptr(t), n, int(min_len), _ptr(o["occ_start"]), _ptr(o["occ_len"]),
                                  _ptr(o["occ_row"]), ctypes.byref(no), _ptr(o["row_start"]),
                                  _ptr(o["row_len"]), _ptr(o["row_count"]), ctypes.byref(nr), _ptr(st))
    if rc == -1:
        raise ValueError("bad arguments")
    if rc != 0:
        raise MemoryError("oracle find_repeats")
    res = {k: (v[: no.value] if k.startswith("occ") else v[: nr.value]) for k, v in o.items()}
    if with_stats:
        res["stats"] = dict(zip(STAT_NAMES, (int(x) for x in st)))
    return res


def interval_counts(length, start, ident):
    """Equal-length greedy per substring over a sorted candidate list
    (Algorithm 2's selection restricted to the occurrences of one substring,
    Section 4.2).  Candidates with equal (length, ID) form one substring,
    listed by increasing start.  Returns (next, count): next[k] = index of the
    first later occurrence of the same substring starting at or after
    start[k] + length[k] (-1 if none); count[k] = number of occurrences on the
    chain k, next[k], ... .  Plain loops."""
    m = len(length)
    nxt = np.full(m, -1, dtype=np.int64)
    cnt = np.zeros(m, dtype=np.int64)
    for k in range(m):
        j = k + 1
        while j < m and length[j] == length[k] and ident[j] == ident[k]:
            if start[j] >= start[k] + length[k]:
                nxt[k] = j
                break
            j += 1
    for k in range(m - 1, -1, -1):
        cnt[k] = 1 + (cnt[nxt[k]] if nxt[k] >= 0 else 0)
    return nxt, cnt
