"""ctypes binding of libapo (include/apo.h): argument marshalling only.

Every step of the analysis runs in the HIP library.  If the library is not
built, :func:`load` raises; there is no fallback path.  PyTorch is used only to
hand over device memory (``tensor.data_ptr()``) and streams.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libapo.so")

APO_OK, APO_EINVAL, APO_ENOMEM, APO_ERANGE, APO_EDEVICE, APO_EAGAIN, APO_ENOTFOUND = 0, -1, -2, -3, -4, -5, -6
APO_MAX_N = 1 << 26

ROW_DTYPE = np.dtype([("start", "<u4"), ("length", "<u4"), ("count", "<u4")])
OCC_DTYPE = np.dtype([("start", "<u4"), ("length", "<u4"), ("cand", "<u4")])
EVENT_DTYPE = np.dtype([("begin", "<u8"), ("end", "<u8"), ("trace", "<i8")])
INGEST_DTYPE = np.dtype([("submitted_at", "<u8"), ("ingested_at", "<u8"), ("slice_begin", "<u8"),
                         ("slice_len", "<u8"), ("pieces", "<u4"), ("waited", "<u4"), ("any_waited", "<u4"),
                         ("_pad", "<u4")])


class AutoParams(ctypes.Structure):
    _fields_ = [("block_tokens", ctypes.c_uint32), ("capacity", ctypes.c_uint32), ("min_len", ctypes.c_uint32),
                ("max_trace_len", ctypes.c_uint32), ("lag0", ctypes.c_uint64), ("count_cap", ctypes.c_uint32),
                ("decay", ctypes.c_double), ("replay_bonus", ctypes.c_double)]

STAGES = ("token_rank", "suffix_array", "lcp", "candidates", "candidate_sort", "selection", "output")
COUNTERS = ("rounds", "candidates", "candidates_dedup", "selection_rounds", "accepted", "rows",
            "active_sum", "sigma", "selection_sequential", "selection_prefix", "pair_windows")

# name -> (restype, argtypes); mirrors include/apo.h
_P, _U32, _U64, _I, _SZ = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_size_t
SIGNATURES = {
    "apo_create": (_I, [ctypes.POINTER(_P), _I, _SZ]),
    "apo_destroy": (_I, [_P]),
    "apo_strerror": (ctypes.c_char_p, [_I]),
    "apo_analyze_window": (_I, [_P, _P, _U32, _U32, _P, _U32, _P, _P, _U32, _P]),
    "apo_analyze_window_u32": (_I, [_P, _P, _U32, _U32, _P, _U32, _P, _P, _U32, _P]),
    "apo_analyze_window_dev": (_I, [_P, _P, _I, _U32, _U32, _P, _U32, _P, _P, _U32, _P, _P]),
    "apo_analyze_window_noalloc": (_I, [_P, _P, _I, _U32, _U32, _P, _U32, _P, _P, _U32, _P, _P]),
    "apo_analyze_batch": (_I, [_P, _P, _P, _U32, _U32, _P, _U64, _P]),
    "apo_analyze_batch_dev": (_I, [_P, _P, _P, _U32, _U32, _P, _U64, _P, _P]),
    "apo_set_graphs": (_I, [_P, _I]),
    "apo_set_lanes": (_I, [_P, _I]),
    "apo_set_selection_round_cap": (_I, [_P, _I]),
    "apo_set_selection_prefix": (_I, [_P, _I]),
    "apo_set_window_greedy": (_I, [_P, _I]),
    "apo_inject_device_error": (_I, [_P, _I]),
    "apo_memory": (_I, [_P, _P, _P, _P]),
    "apo_workspace_bytes": (_SZ, [_U64, _U32]),
    "apo_graph_stats": (_I, [_P, _P, _P]),
    "apo_suffix_array_dev": (_I, [_P, _P, _I, _U32, _P, _P, _P]),
    "apo_lcp_dev": (_I, [_P, _P, _I, _U32, _P, _P, _P]),
    "apo_candidates_dev": (_I, [_P, _P, _I, _U32, _U32, _P, _P, _P, _U32, _P, _P]),
    "apo_interval_counts_dev": (_I, [_P, _P, _P, _P, _U32, _P, _P, _P, _P]),
    "apo_last_stage_ms": (_I, [_P, _P, _I]),
    "apo_last_rounds": (_I, [_P, _P, _P, _P, _P, _P, _U32]),
    "apo_last_counters": (_I, [_P, _P, _I]),
    "apo_profile_kernel": (_I, [_P, _I]),
    "apo_last_kernel_profile": (_I, [_P, _P, _P, _P]),
    "apo_tune": (_I, [_P, _P, _I, _U32, _U32, _I, _P, _P, _P]),
    "apo_set_params": (_I, [_P, _I, _I]),
    "apo_tune_batch": (_I, [_P, _P, _P, _U32, _U32, _I, _P, _P, _P]),
    "apo_tune_save": (_I, [_P, ctypes.c_char_p]),
    "apo_tune_load": (_I, [_P, ctypes.c_char_p]),
    "apo_server_start": (_I, [_P, _U32, _U32]),
    "apo_submit": (_I, [_P, _U32, _P, _U32, _U32, _P]),
    "apo_poll": (_I, [_P, _U64, _P]),
    "apo_fetch": (_I, [_P, _U64, _P, _U32, _P, _P]),
    "apo_server_stop": (_I, [_P]),
    "apo_release": (_I, [_P, _U64]),
    "apo_ruler_slice": (_U64, [_U64, _U32, _U64]),
    "apo_tracer_create": (_I, [_P, _U32, _U32, _U32, _U32, ctypes.POINTER(_P)]),
    "apo_tracer_push": (_I, [_P, _P, _U32, _P]),
    "apo_tracer_poll": (_I, [_P, _P, _P, _P, _U32, _P, _P]),
    "apo_tracer_destroy": (_I, [_P]),
    "apo_replayer_create": (_I, [_U32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_P)]),
    "apo_replayer_ingest": (_I, [_P, _P, _U64, _P, _U32]),
    "apo_replayer_step": (_I, [_P, _P, _U64]),
    "apo_replayer_flush": (_I, [_P]),
    "apo_replayer_events": (_I, [_P, _P, _U32, _P]),
    "apo_replayer_stats": (_I, [_P, _P, _P, _P, _P]),
    "apo_replayer_destroy": (_I, [_P]),
    "apo_split_rows": (_I, [_P, _U32, _U32, _U32, _P, _U32, _P]),
    "apo_agree_create": (_I, [_U32, _U32, ctypes.POINTER(_P)]),
    "apo_agree_vote": (_I, [_P, _U32, _U64, _I, _P]),
    "apo_agree_destroy": (_I, [_P]),
    "apo_auto_create": (_I, [_P, _U32, _P, _P, _U32, ctypes.POINTER(_P)]),
    "apo_auto_execute": (_I, [_P, _P, _U64]),
    "apo_auto_replayer": (_I, [_P, ctypes.POINTER(_P)]),
    "apo_auto_ingests": (_I, [_P, _P, _U32, _P]),
    "apo_auto_lag": (_I, [_P, _P, _P]),
    "apo_auto_destroy": (_I, [_P]),
}

_lib = None


class ApoError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        msg = _lib.apo_strerror(code).decode() if _lib is not None else str(code)
        super().__init__("%s: %s (%d)" % (what, msg, code))


def _torch_first():
    """With PyTorch present, its GPU context is set up before the library's:
    PyTorch brings its own HIP runtime, and once the library's runtime holds
    the GPU, PyTorch's later initialisation finds no device (the other order
    works).  Without PyTorch, or without a GPU, nothing happens."""
    try:
        import torch
    except ImportError:
        return
    if torch.cuda.is_available():
        torch.cuda.init()


def load() -> ctypes.CDLL:
    """Load libapo.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libapo.so is not built (%s); run python -m paper_2406_18111_amd.build" % LIB_PATH)
        _torch_first()
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(rc: int, what: str):
    if rc != APO_OK:
        raise ApoError(rc, what)


def _np_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dev_ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream) -> Optional[ctypes.c_void_p]:
    if stream is None:
        return None
    return ctypes.c_void_p(stream.cuda_stream)


def _host_tokens(tokens):
    t = np.ascontiguousarray(np.asarray(tokens))
    if t.dtype == np.uint32:
        return t, 32
    if t.dtype != np.uint64:
        if t.dtype.kind == "i" and t.size and int(t.min()) < 0:
            raise ValueError("tokens must be non-negative")
        t = np.ascontiguousarray(t.astype(np.uint64))
    return t, 64


class Context:
    """One libapo context on a HIP device (owns a device workspace and stream)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        lib = load()
        h = ctypes.c_void_p()
        _check(lib.apo_create(ctypes.byref(h), int(device), int(budget_bytes)), "apo_create")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.apo_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ---------------------------------------------------------- host API
    def analyze(self, tokens, min_len: int, occurrences: bool = False):
        """FindRepeats on one host window.  Returns rows (ROW_DTYPE) and, if
        asked, occurrences (OCC_DTYPE)."""
        t, bits = _host_tokens(tokens)
        n = len(t)
        cap = max(n // max(int(min_len), 1), 1) if min_len > 0 else 1
        rows = np.zeros(cap, dtype=ROW_DTYPE)
        occ = np.zeros(cap, dtype=OCC_DTYPE) if occurrences else None
        rn, on = ctypes.c_uint32(0), ctypes.c_uint32(0)
        fn = self._lib.apo_analyze_window if bits == 64 else self._lib.apo_analyze_window_u32
        rc = fn(self._h, _np_ptr(t) if n else None, n, int(min_len), _np_ptr(rows), cap, ctypes.byref(rn),
                _np_ptr(occ) if occurrences else None, cap if occurrences else 0,
                ctypes.byref(on) if occurrences else None)
        _check(rc, "apo_analyze_window")
        rows = rows[: rn.value].copy()
        return (rows, occ[: on.value].copy()) if occurrences else rows

    def analyze_batch(self, tokens, offsets, min_len: int):
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        W = len(off) - 1
        total = int(off[-1] - off[0]) if W >= 1 else 0
        cap = max(total // max(int(min_len), 1), 1)
        rows = np.zeros(cap, dtype=ROW_DTYPE)
        oo = np.zeros(W + 1, dtype=np.uint64)
        rc = self._lib.apo_analyze_batch(self._h, _np_ptr(t) if len(t) else None, _np_ptr(off), W, int(min_len),
                                         _np_ptr(rows), cap, _np_ptr(oo))
        _check(rc, "apo_analyze_batch")
        return rows[: int(oo[-1])].copy(), oo

    # -------------------------------------------------------- device API
    def analyze_dev(self, tokens, min_len: int, stream=None, occurrences: bool = False):
        """tokens: 1-D torch tensor on the GPU (uint64 as int64 view, or int32/uint32 bits).
        Returns (rows_u32[k,3] tensor, occ_u32[m,3] tensor or None)."""
        import torch
        bits = 64 if tokens.element_size() == 8 else 32
        n = tokens.numel()
        cap = max(n // max(int(min_len), 1), 1)
        rows = torch.empty((cap, 3), dtype=torch.int32, device=tokens.device)
        occ = torch.empty((cap, 3), dtype=torch.int32, device=tokens.device) if occurrences else None
        rn, on = ctypes.c_uint32(0), ctypes.c_uint32(0)
        rc = self._lib.apo_analyze_window_dev(self._h, _dev_ptr(tokens), bits, n, int(min_len), _dev_ptr(rows), cap,
                                              ctypes.byref(rn), _dev_ptr(occ) if occurrences else None,
                                              cap if occurrences else 0,
                                              ctypes.byref(on) if occurrences else None, _stream_ptr(stream))
        _check(rc, "apo_analyze_window_dev")
        return rows[: rn.value], (occ[: on.value] if occurrences else None)

    def analyze_batch_dev(self, tokens, offsets, min_len: int, stream=None):
        import torch
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        W = len(off) - 1
        total = int(off[-1] - off[0])
        cap = max(total // max(int(min_len), 1), 1)
        rows = torch.empty((cap, 3), dtype=torch.int32, device=tokens.device)
        oo = np.zeros(W + 1, dtype=np.uint64)
        rc = self._lib.apo_analyze_batch_dev(self._h, _dev_ptr(tokens), _np_ptr(off), W, int(min_len),
                                             _dev_ptr(rows), cap, _np_ptr(oo), _stream_ptr(stream))
        _check(rc, "apo_analyze_batch_dev")
        return rows[: int(oo[-1])], oo

    def set_lanes(self, lanes: int):
        """Concurrent window groups per batch (1..4)."""
        _check(self._lib.apo_set_lanes(self._h, int(lanes)), "apo_set_lanes")

    def set_window_greedy(self, on: bool):
        """Per-window one-wavefront greedy for short windows (default on); off: round-based selection only."""
        _check(self._lib.apo_set_window_greedy(self._h, int(bool(on))), "apo_set_window_greedy")

    def set_selection_round_cap(self, rounds: int):
        """Test hook: stop host-driven greedy rounds after `rounds` (0..64)."""
        _check(self._lib.apo_set_selection_round_cap(self._h, int(rounds)), "apo_set_selection_round_cap")

    def set_selection_prefix(self, k: int):
        """Exact prefix walk before the selection rounds: -1 automatic, 0 never, k > 0 always k candidates."""
        _check(self._lib.apo_set_selection_prefix(self._h, int(k)), "apo_set_selection_prefix")

    def inject_device_error(self, after_syncs: int):
        """Test hook: a host sync of the next single-window analysis reports a device error."""
        _check(self._lib.apo_inject_device_error(self._h, int(after_syncs)), "apo_inject_device_error")

    def memory(self):
        """Device bytes held: the context's own workspaces, the server pool and what its slots hold."""
        h, p, sh = ctypes.c_size_t(0), ctypes.c_size_t(0), ctypes.c_size_t(0)
        _check(self._lib.apo_memory(self._h, ctypes.byref(h), ctypes.byref(p), ctypes.byref(sh)), "apo_memory")
        return {"held": h.value, "server_pool": p.value, "server_held": sh.value}

    def set_graphs(self, on: bool):
        _check(self._lib.apo_set_graphs(self._h, int(bool(on))), "apo_set_graphs")

    def graph_stats(self):
        c, r = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(self._lib.apo_graph_stats(self._h, ctypes.byref(c), ctypes.byref(r)), "apo_graph_stats")
        return {"captures": c.value, "replays": r.value}

    def suffix_array_dev(self, tokens, stream=None):
        import torch
        bits = 64 if tokens.element_size() == 8 else 32
        n = tokens.numel()
        sa = torch.empty(n, dtype=torch.int32, device=tokens.device)
        rounds = ctypes.c_uint32(0)
        _check(self._lib.apo_suffix_array_dev(self._h, _dev_ptr(tokens), bits, n, _dev_ptr(sa), ctypes.byref(rounds),
                                              _stream_ptr(stream)), "apo_suffix_array_dev")
        return sa, rounds.value

    def lcp_dev(self, tokens, stream=None):
        import torch
        bits = 64 if tokens.element_size() == 8 else 32
        n = tokens.numel()
        sa = torch.empty(n, dtype=torch.int32, device=tokens.device)
        lcp = torch.empty(n, dtype=torch.int32, device=tokens.device)
        _check(self._lib.apo_lcp_dev(self._h, _dev_ptr(tokens), bits, n, _dev_ptr(sa), _dev_ptr(lcp),
                                     _stream_ptr(stream)), "apo_lcp_dev")
        return sa, lcp

    def candidates_dev(self, tokens, min_len: int, stream=None):
        import torch
        bits = 64 if tokens.element_size() == 8 else 32
        n = tokens.numel()
        cap = max(2 * n, 1)
        ln = torch.empty(cap, dtype=torch.int32, device=tokens.device)
        st = torch.empty(cap, dtype=torch.int32, device=tokens.device)
        ids = torch.empty(cap, dtype=torch.int32, device=tokens.device)
        cnt = ctypes.c_uint32(0)
        _check(self._lib.apo_candidates_dev(self._h, _dev_ptr(tokens), bits, n, int(min_len), _dev_ptr(ln),
                                            _dev_ptr(st), _dev_ptr(ids), cap, ctypes.byref(cnt), _stream_ptr(stream)),
               "apo_candidates_dev")
        m = cnt.value
        return {"len": ln[:m], "start": st[:m], "id": ids[:m]}

    def interval_counts_dev(self, cands, stream=None):
        """Per-substring equal-length greedy over sorted candidates (dict of
        device tensors as candidates_dev returns): next index and chain count."""
        import torch
        ln, st, ids = (cands[k].contiguous() for k in ("len", "start", "id"))
        m = ln.numel()
        nxt = torch.empty(max(m, 1), dtype=torch.int32, device=ln.device)
        cnt = torch.empty(max(m, 1), dtype=torch.int32, device=ln.device)
        tmp = torch.empty(max(3 * m, 1), dtype=torch.int32, device=ln.device)
        _check(self._lib.apo_interval_counts_dev(self._h, _dev_ptr(ln), _dev_ptr(st), _dev_ptr(ids), m,
                                                 _dev_ptr(nxt), _dev_ptr(cnt), _dev_ptr(tmp), _stream_ptr(stream)),
               "apo_interval_counts_dev")
        return nxt[:m], cnt[:m]

    # ------------------------------------------------------ diagnostics
    def stage_ms(self):
        a = (ctypes.c_double * len(STAGES))()
        k = self._lib.apo_last_stage_ms(self._h, a, len(STAGES))
        return dict(zip(STAGES[:k], list(a)[:k]))

    def counters(self):
        a = (ctypes.c_uint64 * len(COUNTERS))()
        k = self._lib.apo_last_counters(self._h, a, len(COUNTERS))
        return dict(zip(COUNTERS[:k], list(a)[:k]))

    def rounds(self):
        """Per-round sizes of the last analysis: suffixes entering each doubling
        round; live and undecided candidates of each selection round."""
        cap = 128
        a, l, u = (ctypes.c_uint32 * cap)(), (ctypes.c_uint32 * cap)(), (ctypes.c_uint32 * cap)()
        ns, nq = ctypes.c_uint32(0), ctypes.c_uint32(0)
        rc = self._lib.apo_last_rounds(self._h, a, ctypes.byref(ns), l, u, ctypes.byref(nq), cap)
        if rc not in (APO_OK, APO_ERANGE):
            _check(rc, "apo_last_rounds")
        ns, nq = min(ns.value, cap), min(nq.value, cap)
        return {"sa_active": list(a)[:ns], "sel_live": list(l)[:nq], "sel_undecided": list(u)[:nq]}

    def profile_kernel(self, tag: int):
        """Time one kernel family with HIP events (1: LDS sort of the doubling rounds; 0: off)."""
        _check(self._lib.apo_profile_kernel(self._h, int(tag)), "apo_profile_kernel")

    def kernel_profile(self):
        la, ms, el = ctypes.c_uint64(0), ctypes.c_double(0), ctypes.c_uint64(0)
        _check(self._lib.apo_last_kernel_profile(self._h, ctypes.byref(la), ctypes.byref(ms), ctypes.byref(el)),
               "apo_last_kernel_profile")
        return {"launches": la.value, "ms": ms.value, "elems": el.value}

    # ------------------------------------------------------- autotuner
    def tune(self, tokens, min_len: int, reps: int = 3):
        """Autotune (LDS tile, digit width) on a device window; returns (tile_log, digit_bits, ms)."""
        bits = 64 if tokens.element_size() == 8 else 32
        t, d, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        _check(self._lib.apo_tune(self._h, _dev_ptr(tokens), bits, tokens.numel(), int(min_len), int(reps),
                                  ctypes.byref(t), ctypes.byref(d), ctypes.byref(ms)), "apo_tune")
        return t.value, d.value, ms.value

    def tune_batch(self, tokens, offsets, min_len: int, reps: int = 1):
        """Autotune on a batch of device windows; returns (tile_log, digit_bits, ms)."""
        off = np.ascontiguousarray(np.asarray(offsets, dtype=np.uint64))
        t, d, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0)
        _check(self._lib.apo_tune_batch(self._h, _dev_ptr(tokens), _np_ptr(off), len(off) - 1, int(min_len),
                                        int(reps), ctypes.byref(t), ctypes.byref(d), ctypes.byref(ms)),
               "apo_tune_batch")
        return t.value, d.value, ms.value

    def set_params(self, tile_log: int, digit_bits: int):
        _check(self._lib.apo_set_params(self._h, int(tile_log), int(digit_bits)), "apo_set_params")

    def tune_save(self, path: str):
        _check(self._lib.apo_tune_save(self._h, path.encode()), "apo_tune_save")

    def tune_load(self, path: str):
        _check(self._lib.apo_tune_load(self._h, path.encode()), "apo_tune_load")

    # ---------------------------------------------------------- server
    def server_start(self, slots: int = 2, queue_cap: int = 0):
        _check(self._lib.apo_server_start(self._h, int(slots), int(queue_cap)), "apo_server_start")

    def submit(self, tokens, min_len: int, stream_id: int = 0) -> int:
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        tk = ctypes.c_uint64(0)
        rc = self._lib.apo_submit(self._h, int(stream_id), _np_ptr(t) if len(t) else None, len(t), int(min_len),
                                  ctypes.byref(tk))
        _check(rc, "apo_submit")
        return tk.value

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int(0)
        _check(self._lib.apo_poll(self._h, ctypes.c_uint64(ticket), ctypes.byref(d)), "apo_poll")
        return bool(d.value)

    def fetch(self, ticket: int, cap: int = 1 << 16):
        """Rows of a finished ticket and its submit-to-ready latency (s); None if not ready."""
        while True:
            rows = np.zeros(max(cap, 1), dtype=ROW_DTYPE)
            n = ctypes.c_uint32(0)
            lat = ctypes.c_uint64(0)
            rc = self._lib.apo_fetch(self._h, ctypes.c_uint64(ticket), _np_ptr(rows), len(rows), ctypes.byref(n),
                                     ctypes.byref(lat))
            if rc == APO_EAGAIN:
                return None
            if rc == APO_ERANGE:
                cap = n.value
                continue
            _check(rc, "apo_fetch")
            return rows[: n.value].copy(), lat.value * 1e-9

    def server_stop(self):
        _check(self._lib.apo_server_stop(self._h), "apo_server_stop")


def workspace_bytes(n: int, windows: int = 1) -> int:
    """Device bytes of the workspace for n tokens in `windows` windows."""
    return int(load().apo_workspace_bytes(int(n), int(windows)))


def ruler_slice(block_index: int, block_tokens: int, capacity: int) -> int:
    """Length of the slice analysed after block `block_index` (Section 4.4)."""
    return int(load().apo_ruler_slice(int(block_index), int(block_tokens), int(capacity)))


class Tracer:
    """Trace finder for one task stream on a Context whose server is running."""

    def __init__(self, ctx: Context, block_tokens: int = 500, capacity: int = 5000, min_len: int = 25,
                 stream_id: int = 0):
        h = ctypes.c_void_p()
        _check(ctx._lib.apo_tracer_create(ctx._h, int(stream_id), int(block_tokens), int(capacity), int(min_len),
                                          ctypes.byref(h)), "apo_tracer_create")
        self._h, self._ctx = h, ctx

    def push(self, tokens) -> int:
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        sub = ctypes.c_uint32(0)
        _check(self._ctx._lib.apo_tracer_push(self._h, _np_ptr(t) if len(t) else None, len(t), ctypes.byref(sub)),
               "apo_tracer_push")
        return sub.value

    def poll(self, cap: int = 1 << 14):
        """(slice_begin, slice_len, rows) of the oldest finished analysis, or None."""
        while True:
            rows = np.zeros(max(cap, 1), dtype=ROW_DTYPE)
            b, ln, n = ctypes.c_uint64(0), ctypes.c_uint64(0), ctypes.c_uint32(0)
            rc = self._ctx._lib.apo_tracer_poll(self._h, ctypes.byref(b), ctypes.byref(ln), _np_ptr(rows), len(rows),
                                                ctypes.byref(n), None)
            if rc == APO_EAGAIN:
                return None
            if rc == APO_ERANGE:
                cap = n.value
                continue
            _check(rc, "apo_tracer_poll")
            return b.value, ln.value, rows[: n.value].copy()

    def close(self):
        if getattr(self, "_h", None):
            self._ctx._lib.apo_tracer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def split_rows(rows: np.ndarray, max_len: int, min_len: int = 1) -> np.ndarray:
    """Rows cut into pieces of at most max_len tokens (Section 6.2)."""
    lib = load()
    rows = np.ascontiguousarray(rows, dtype=ROW_DTYPE)
    cap = max(1, len(rows))
    while True:
        out = np.zeros(cap, dtype=ROW_DTYPE)
        n = ctypes.c_uint32(0)
        rc = lib.apo_split_rows(_np_ptr(rows) if len(rows) else None, len(rows), int(max_len), int(min_len),
                                _np_ptr(out), cap, ctypes.byref(n))
        if rc == APO_ERANGE:
            cap = n.value
            continue
        _check(rc, "apo_split_rows")
        return out[: n.value].copy()


class Replayer:
    """Trace replayer over a task stream (Section 4.3), host-side."""

    def __init__(self, count_cap: int = 8, decay: float = 0.999, replay_bonus: float = 0.1, _borrow=None):
        self._lib = load()
        self._owned = _borrow is None
        if _borrow is not None:
            self._h = _borrow
            return
        h = ctypes.c_void_p()
        _check(self._lib.apo_replayer_create(int(count_cap), float(decay), float(replay_bonus), ctypes.byref(h)),
               "apo_replayer_create")
        self._h = h

    def ingest(self, tokens, rows):
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        r = np.ascontiguousarray(rows, dtype=ROW_DTYPE)
        _check(self._lib.apo_replayer_ingest(self._h, _np_ptr(t) if len(t) else None, len(t),
                                             _np_ptr(r) if len(r) else None, len(r)), "apo_replayer_ingest")

    def step(self, tokens):
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        _check(self._lib.apo_replayer_step(self._h, _np_ptr(t) if len(t) else None, len(t)), "apo_replayer_step")

    def flush(self):
        _check(self._lib.apo_replayer_flush(self._h), "apo_replayer_flush")

    def events(self) -> np.ndarray:
        cap = 256
        while True:
            out = np.zeros(cap, dtype=EVENT_DTYPE)
            n = ctypes.c_uint32(0)
            rc = self._lib.apo_replayer_events(self._h, _np_ptr(out), cap, ctypes.byref(n))
            if rc == APO_ERANGE:
                cap = n.value
                continue
            _check(rc, "apo_replayer_events")
            return out[: n.value].copy()

    def stats(self) -> dict:
        v = [ctypes.c_uint64(0) for _ in range(4)]
        _check(self._lib.apo_replayer_stats(self._h, *[ctypes.byref(x) for x in v]), "apo_replayer_stats")
        return dict(zip(("tasks", "traced", "replays", "traces"), [x.value for x in v]))

    def close(self):
        if getattr(self, "_h", None):
            if self._owned:
                self._lib.apo_replayer_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Agreement:
    """Ingestion agreement among replicas of one task stream (Section 5.1)."""

    def __init__(self, nodes: int, timeout_ms: int = 0):
        self._lib = load()
        h = ctypes.c_void_p()
        _check(self._lib.apo_agree_create(int(nodes), int(timeout_ms), ctypes.byref(h)), "apo_agree_create")
        self._h = h

    def vote(self, node: int, j: int, waited: bool) -> bool:
        out = ctypes.c_int(0)
        _check(self._lib.apo_agree_vote(self._h, int(node), int(j), int(bool(waited)), ctypes.byref(out)),
               "apo_agree_vote")
        return bool(out.value)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.apo_agree_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Auto:
    """Algorithm 1 over one task stream: trace finder on ctx's server + replayer."""

    def __init__(self, ctx: Context, stream_id: int = 0, block_tokens: int = 250, capacity: int = 5000,
                 min_len: int = 25, max_trace_len: int = 200, lag0: int = 0, count_cap: int = 8,
                 decay: float = 0.999, replay_bonus: float = 0.1, agreement: Optional[Agreement] = None,
                 node: int = 0):
        self._lib = ctx._lib
        self.params = AutoParams(block_tokens, capacity, min_len, max_trace_len, lag0, count_cap, decay, replay_bonus)
        h = ctypes.c_void_p()
        _check(self._lib.apo_auto_create(ctx._h, int(stream_id), ctypes.byref(self.params),
                                         agreement._h if agreement is not None else None, int(node), ctypes.byref(h)),
               "apo_auto_create")
        self._h, self._ctx = h, ctx
        r = ctypes.c_void_p()
        _check(self._lib.apo_auto_replayer(self._h, ctypes.byref(r)), "apo_auto_replayer")
        self.replayer = Replayer(_borrow=r)

    def execute(self, tokens):
        t = np.ascontiguousarray(np.asarray(tokens, dtype=np.uint64))
        _check(self._lib.apo_auto_execute(self._h, _np_ptr(t) if len(t) else None, len(t)), "apo_auto_execute")

    def ingests(self) -> np.ndarray:
        cap = 64
        while True:
            out = np.zeros(cap, dtype=INGEST_DTYPE)
            n = ctypes.c_uint32(0)
            rc = self._lib.apo_auto_ingests(self._h, _np_ptr(out), cap, ctypes.byref(n))
            if rc == APO_ERANGE:
                cap = n.value
                continue
            _check(rc, "apo_auto_ingests")
            return out[: n.value].copy()

    def lag(self):
        lag, waits = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(self._lib.apo_auto_lag(self._h, ctypes.byref(lag), ctypes.byref(waits)), "apo_auto_lag")
        return lag.value, waits.value

    def close(self):
        if getattr(self, "_h", None):
            self.replayer._h = None
            self._lib.apo_auto_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
