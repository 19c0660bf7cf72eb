"""GPU parity: every stage of the HIP path against the CPU oracle (exact).

Integer results, so the bar is bit-exactness: suffix array, LCP array, the
sorted and de-duplicated candidate list (length, start, substring ID), and the
final rows and occurrences.  Inputs are seeded and synthetic; sizes span one
or several LDS tiles (4096) with ragged tails, the MSD bucketing path (units
longer than a tile), and the degenerate cases of the method.
"""
import json
import os
import random

import numpy as np
import pytest

import oracle
from paper_2406_18111_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN_DIR = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    from paper_2406_18111_amd import Context
    c = Context(0)
    yield c
    c.close()


def _dev(tokens):
    import torch
    t = np.ascontiguousarray(tokens)
    if t.dtype == np.uint64:
        return torch.from_numpy(t.view(np.int64)).cuda()
    if t.dtype == np.uint32:
        return torch.from_numpy(t.view(np.int32)).cuda()
    raise TypeError(t.dtype)


def _u64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def _cases_small():
    rng = random.Random(1234)
    cases = []
    for s in ([0, 0, 1, 2, 1, 2, 1, 0, 0], [0, 1, 0, 1, 0, 1], [0, 1, 2, 3, 1, 4] * 2, [5, 5], [7]):
        cases.append(("paper_" + "".join(map(str, s[:6])), _u64(s)))
    for n in (2, 3, 63, 64, 65, 127, 129, 1000, 4095, 4096, 4097, 8191, 12289):
        a = rng.choice([1, 2, 3, 4, 16, 1 << 20])
        cases.append(("rand_n%d_a%d" % (n, a), _u64([rng.randrange(a) for _ in range(n)])))
    for n in (5000, 70000):
        cases.append(("const_%d" % n, _u64([9] * n)))
    cases.append(("periodic_3x5000", _u64(list(range(3)) * 5000)))
    cases.append(("big_tokens", np.array([2 ** 64 - 1, 0, 2 ** 63, 2 ** 64 - 1, 0, 2 ** 63] * 700, dtype=np.uint64)))
    fib = [0]
    a, b = [0], [0, 1]
    while len(b) < 20000:
        a, b = b, b + a
    cases.append(("fibonacci_20000", _u64(b[:20000])))
    cases.append(("thue_morse_16384", _u64([bin(i).count("1") % 2 for i in range(16384)])))
    blocks = []
    for k in range(1, 40):
        blocks += [0] * k + [1]
    cases.append(("a^k_b_blocks", _u64(blocks)))
    t0, _ = synth.config0()
    cases.append(("config0", t0))
    return cases


CASES = _cases_small()


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
def test_suffix_array_and_lcp(ctx, name, tokens):
    print("case", name, len(tokens), flush=True)
    sa_ref = oracle.suffix_array(tokens)
    lcp_ref = oracle.lcp(tokens, sa_ref)
    sa, lcp = ctx.lcp_dev(_dev(tokens))
    sa = sa.cpu().numpy().astype(np.int64)
    lcp = lcp.cpu().numpy().astype(np.int64)
    assert np.array_equal(sa, sa_ref)
    assert np.array_equal(lcp[: len(tokens) - 1], lcp_ref)
    assert lcp[-1] == 0


def _dedup(c):
    """Oracle candidate list with exact (length, start) duplicates removed."""
    keep = np.ones(len(c["len"]), dtype=bool)
    keep[1:] = (c["len"][1:] != c["len"][:-1]) | (c["start"][1:] != c["start"][:-1])
    return {k: v[keep] for k, v in c.items()}


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("min_len", [1, 3, 8])
def test_candidates_sorted(ctx, name, tokens, min_len):
    print("case", name, min_len, flush=True)
    ref = _dedup(oracle.sorted_candidates(tokens, min_len))
    got = ctx.candidates_dev(_dev(tokens), min_len)
    for k in ("len", "start", "id"):
        g = got[k].cpu().numpy().astype(np.int64)
        assert np.array_equal(g, ref[k]), k


def test_candidates_one_long_run(ctx):
    """One token followed by 50 000 distinct tokens: the 1-interval of that
    token has 50 000 children, so about 100 000 candidates share (length 1,
    ID) and the start-level sort takes the multi-level bucketing path."""
    rng = np.random.default_rng(13)
    n = 100000
    t = np.empty(n, np.uint64)
    t[0::2] = 0x1234567
    t[1::2] = rng.integers(1 << 40, 1 << 62, n // 2, dtype=np.uint64)
    for min_len in (1, 2):
        ref = _dedup(oracle.sorted_candidates(t, min_len))
        got = ctx.candidates_dev(_dev(t), min_len)
        for k in ("len", "start", "id"):
            g = got[k].cpu().numpy().astype(np.int64)
            assert np.array_equal(g, ref[k]), (min_len, k)
    _check_full(ctx, t, 1)


def _check_full(ctx, tokens, min_len):
    ref = oracle.find_repeats(tokens, min_len)
    rows, occ = ctx.analyze(tokens, min_len, occurrences=True)
    assert np.array_equal(rows["start"].astype(np.int64), ref["row_start"])
    assert np.array_equal(rows["length"].astype(np.int64), ref["row_len"])
    assert np.array_equal(rows["count"].astype(np.int64), ref["row_count"])
    assert np.array_equal(occ["start"].astype(np.int64), ref["occ_start"])
    assert np.array_equal(occ["length"].astype(np.int64), ref["occ_len"])
    assert np.array_equal(occ["cand"].astype(np.int64), ref["occ_row"])
    return ref


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("min_len", [1, 2, 8, 25])
def test_find_repeats(ctx, name, tokens, min_len):
    print("case", name, min_len, flush=True)
    _check_full(ctx, tokens, min_len)


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("min_len", [1, 8])
def test_find_repeats_both_selection_paths(ctx, name, tokens, min_len):
    """The round-based selection and the one-wavefront-per-window greedy give
    the oracle's result on every case (short windows take the wavefront
    greedy by default; the switch sends them through the rounds)."""
    print("case", name, min_len, flush=True)
    try:
        ctx.set_window_greedy(False)
        _check_full(ctx, tokens, min_len)
    finally:
        ctx.set_window_greedy(True)
    _check_full(ctx, tokens, min_len)


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("k", [1, 100, 5000])
def test_find_repeats_selection_prefix(ctx, name, tokens, k):
    """An exact prefix walk of k candidates before the selection rounds (the
    rest from round 1, whose filter rejects what the prefix covers) gives the
    oracle's result; the counters report the candidates it decided."""
    print("case", name, k, flush=True)
    try:
        ctx.set_window_greedy(False)
        ctx.set_selection_prefix(k)
        for min_len in (1, 8):
            _check_full(ctx, tokens, min_len)
            c = ctx.counters()
            assert c["selection_prefix"] == min(k, c["candidates_dedup"]), c
    finally:
        ctx.set_selection_prefix(-1)
        ctx.set_window_greedy(True)


def test_selection_prefix_long_runs(ctx):
    """Inputs whose longest candidates span much of the window (a long
    constant run, then other text) take the automatic prefix walk; the result
    is the oracle's, and equals the rounds alone."""
    rng = np.random.default_rng(11)
    cases = []
    for n, run in ((1 << 16, 1 << 15), (100003, 40000), (70000, 70000)):
        t = rng.integers(0, 4, n).astype(np.uint32)
        t[:run] = 0
        cases.append(t)
    a = [0] * 30000 + [1] + [0] * 20000 + [2, 3] * 5000
    cases.append(np.array(a, dtype=np.uint64))
    for t in cases:
        for m in (1, 32):
            ref = _check_full(ctx, t, m)
            c = ctx.counters()
            assert c["selection_prefix"] > 0, c
            try:
                ctx.set_selection_prefix(0)
                rows = ctx.analyze(t, m)
                assert ctx.counters()["selection_prefix"] == 0
                assert np.array_equal(rows["start"].astype(np.int64), ref["row_start"])
                assert np.array_equal(rows["length"].astype(np.int64), ref["row_len"])
                assert np.array_equal(rows["count"].astype(np.int64), ref["row_count"])
            finally:
                ctx.set_selection_prefix(-1)


def test_golden_examples(ctx):
    g = json.load(open(os.path.join(GOLDEN_DIR, "worked_examples.json")))
    for case in g["cases"]:
        for run in case["runs"]:
            rows, occ = ctx.analyze(_u64(case["tokens"]), run["min_len"], occurrences=True)
            assert [[int(a), int(b)] for a, b in zip(occ["start"], occ["length"])] == run["occurrences"]
            assert [list(map(int, r)) for r in rows.tolist()] == run["rows"]


def test_u32_input_matches_u64(ctx):
    rng = np.random.default_rng(3)
    t = rng.integers(0, 5, 30000).astype(np.uint32)
    r32 = ctx.analyze(t, 4)
    r64 = ctx.analyze(t.astype(np.uint64), 4)
    assert np.array_equal(r32, r64)
    _check_full(ctx, t, 4)


def test_device_api_matches_host_api(ctx):
    t, m = synth.config0()
    rows_h = ctx.analyze(t, m)
    rows_d, _ = ctx.analyze_dev(_dev(t), m)
    assert np.array_equal(rows_d.cpu().numpy().astype(np.int64),
                          np.stack([rows_h["start"], rows_h["length"], rows_h["count"]], 1).astype(np.int64))


def test_trivial_and_errors(ctx):
    from paper_2406_18111_amd import ApoError
    assert len(ctx.analyze(_u64([]), 1)) == 0
    assert len(ctx.analyze(_u64([4]), 1)) == 0
    with pytest.raises(ApoError):
        ctx.analyze(_u64([1, 2, 3]), 0)
    # distinct tokens: no repeats
    assert len(ctx.analyze(np.arange(5000, dtype=np.uint64) * np.uint64(7919), 1)) == 0


def test_repeatable(ctx):
    t, m = synth.config1(n=1 << 16)
    a = ctx.analyze(t, m, occurrences=True)
    b = ctx.analyze(t, m, occurrences=True)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_config1_full_size(ctx):
    """n = 2^20 nested-loop stream, min length 16: full oracle parity."""
    t, m = synth.config1()
    _check_full(ctx, t, m)


def test_config2_full_size(ctx):
    """n = 2^24 adversarial input (half constant run, half uniform over 4
    symbols), min length 32: result against the stored oracle run; suffix
    array checked as a permutation and on sampled adjacent pairs by direct
    comparison; LCP checked on the same samples."""
    g = json.load(open(os.path.join(GOLDEN_DIR, "config_results.json")))["configs"]["config2_n2^24_u32"]
    t, m = synth.config2()
    rows, occ = ctx.analyze(t, m, occurrences=True)
    assert [[int(a), int(b)] for a, b in zip(occ["start"], occ["length"])] == g["occurrences"]
    assert [list(map(int, r)) for r in rows.tolist()] == g["rows"]
    assert ctx.counters()["candidates"] == g["stats"]["candidates"]
    assert ctx.counters()["selection_prefix"] > 0  # the longest candidates span half the window
    sa, lcp = ctx.lcp_dev(_dev(t))
    sa = sa.cpu().numpy().astype(np.int64)
    lcp = lcp.cpu().numpy().astype(np.int64)
    n = len(t)
    assert np.array_equal(np.sort(sa), np.arange(n))
    rng = np.random.default_rng(7)
    for i in np.concatenate([rng.integers(0, n - 1, 300), [0, n // 2 - 1, n // 2, n - 2]]):
        a, b = int(sa[i]), int(sa[i + 1])
        la, lb = n - a, n - b
        k = min(la, lb)
        x, y = t[a:a + k], t[b:b + k]
        neq = np.flatnonzero(x != y)
        p = int(neq[0]) if len(neq) else k
        assert lcp[i] == p
        # strictly increasing suffixes
        if p < k:
            assert x[p] < y[p]
        else:
            assert la < lb


@pytest.mark.parametrize("tile_log", [11, 12, 13])
@pytest.mark.parametrize("digit_bits", [8, 10, 11, 12])
def test_kernel_params_do_not_change_results(ctx, tile_log, digit_bits):
    """Every LDS tile / MSD digit width gives the oracle's result (units longer
    than the tile exercise the MSD path)."""
    ctx.set_params(tile_log, digit_bits)
    try:
        rng = np.random.default_rng(tile_log * 100 + digit_bits)
        cases = [rng.integers(0, 3, 20000).astype(np.uint64), _u64([4] * 9000 + [1, 2] * 3000),
                 synth.config1(n=1 << 15)[0]]
        for t in cases:
            for m in (2, 16):
                _check_full(ctx, t, m)
        sa, _ = ctx.suffix_array_dev(_dev(cases[1]))
        assert np.array_equal(sa.cpu().numpy().astype(np.int64), oracle.suffix_array(cases[1]))
    finally:
        ctx.set_params(-1, -1)


def test_tune_table_roundtrip(ctx, tmp_path):
    t, m = synth.config1(n=1 << 14)
    tl, db, ms = ctx.tune(_dev(t), m, reps=1)
    assert 11 <= tl <= 13 and db in (8, 10, 11, 12) and ms > 0
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    assert open(path).read().split("\n")[1].split() == ["14", str(tl), str(db)]
    ctx.tune_load(path)
    _check_full(ctx, t, m)


@pytest.mark.parametrize("name,tokens", CASES, ids=[c[0] for c in CASES])
def test_interval_counts(ctx, name, tokens):
    """Per-substring equal-length greedy (next occurrence kept, chain counts)
    on the sorted candidate list, against the oracle on its own list."""
    print("case", name, flush=True)
    ref = _dedup(oracle.sorted_candidates(tokens, 2))
    rnxt, rcnt = oracle.interval_counts(ref["len"], ref["start"], ref["id"])
    got = ctx.candidates_dev(_dev(tokens), 2)
    nxt, cnt = ctx.interval_counts_dev(got)
    g = nxt.cpu().numpy().astype(np.int64)  # int32 view: "none" reads as -1
    assert np.array_equal(np.where(g < 0, -1, g), rnxt)
    assert np.array_equal(cnt.cpu().numpy().astype(np.int64), rcnt)


def test_interval_counts_synthetic_lists(ctx):
    """Seeded candidate lists built directly (groups of equal length and ID,
    starts ascending; many members per group, long chains)."""
    import torch
    rng = np.random.default_rng(23)
    for trial in range(6):
        L, S, I = [], [], []
        lens = sorted(rng.integers(1, 40, int(rng.integers(1, 50))).tolist(), reverse=True)
        for g, l in enumerate(lens):
            st = np.unique(rng.integers(0, 20000, int(rng.integers(1, 3000))))
            L += [l] * len(st)
            S += st.tolist()
            I += [g] * len(st)
        rnxt, rcnt = oracle.interval_counts(L, S, I)
        d = {k: torch.tensor(np.array(v, dtype=np.int64).astype(np.int32)).cuda()
             for k, v in (("len", L), ("start", S), ("id", I))}
        nxt, cnt = ctx.interval_counts_dev(d)
        g = nxt.cpu().numpy().astype(np.int64)
        assert np.array_equal(np.where(g < 0, -1, g), rnxt), trial
        assert np.array_equal(cnt.cpu().numpy().astype(np.int64), rcnt), trial
