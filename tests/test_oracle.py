"""Pins for the CPU oracle (no GPU).

The oracle is checked against things other than itself:
* hand-derived runs on the paper's own example strings (tests/golden);
* closed forms for periodic strings, a^n and all-distinct strings;
* brute-force suffix order (Python list comparison) and direct LCPs;
* invariants every result of Algorithm 2 must satisfy;
* the literal pure-Python oracle against the C oracle, exhaustively on small
  strings and on random and adversarial families;
* planted mistakes in the literal oracle that these pins must catch.
"""
import itertools
import json
import os
import random

import numpy as np
import pytest

import oracle
import oracle.naive as nv
from paper_2406_18111_amd import synth

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")))


def _c_result(tokens, min_len):
    r = oracle.find_repeats(tokens, min_len)
    occ = list(zip(r["occ_start"].tolist(), r["occ_len"].tolist()))
    rows = list(zip(r["row_start"].tolist(), r["row_len"].tolist(), r["row_count"].tolist()))
    return occ, rows


# ----------------------------------------------------------------- golden

@pytest.mark.parametrize("case", GOLDEN["cases"], ids=[c["name"] for c in GOLDEN["cases"]])
def test_golden_sa_lcp(case):
    t = case["tokens"]
    assert nv.suffix_array(t) == case["sa"]
    assert nv.lcp_array(t, case["sa"]) == case["lcp"]
    sa = oracle.suffix_array(t)
    assert sa.tolist() == case["sa"]
    assert oracle.lcp(t, sa).tolist() == case["lcp"]


@pytest.mark.parametrize("case", GOLDEN["cases"], ids=[c["name"] for c in GOLDEN["cases"]])
def test_golden_selection(case):
    for run in case["runs"]:
        occ, rows = nv.find_repeats(case["tokens"], run["min_len"])
        assert [list(x) for x in occ] == run["occurrences"]
        assert [list(x) for x in rows] == run["rows"]
        occ2, rows2 = _c_result(case["tokens"], run["min_len"])
        assert [list(x) for x in occ2] == run["occurrences"]
        assert [list(x) for x in rows2] == run["rows"]


def test_golden_candidate_list_aabcbcbaa():
    """The per-pair candidates written out in the fixture's derivation."""
    t = [0, 0, 1, 2, 1, 2, 1, 0, 0]
    sa = nv.suffix_array(t)
    cands = nv.candidates(t, sa, nv.lcp_array(t, sa))
    got = [(l, s) for (l, _r, s) in cands]
    assert got == [(1, 8), (1, 7), (2, 7), (2, 0), (1, 0), (1, 1), (0, 1), (0, 6),
                   (1, 6), (1, 4), (2, 2), (2, 4), (0, 2), (0, 5), (2, 5), (2, 3)]
    c = oracle.sorted_candidates(t, 1)
    assert list(zip(c["len"].tolist(), c["start"].tolist())) == [
        (2, 0), (2, 7), (2, 2), (2, 4), (2, 3), (2, 5), (1, 0), (1, 1), (1, 7), (1, 8), (1, 4), (1, 6)]


# ----------------------------------------------------------- closed forms

@pytest.mark.parametrize("P", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_periodic_closed_form(P, k):
    """body^k with P distinct body tokens, min_len <= P: the pair (P, 0) has the
    longest LCP P(k-1) and takes the overlap branch with d=P, giving
    l = P*floor(k/2) at 0 and at l; an odd k leaves one body copy at the end,
    taken by a length-P candidate.  k=1 has no repeat."""
    s = list(range(P)) * k
    h = P * (k // 2)
    exp = [] if k == 1 else [(0, h), (h, h)] + ([(P * (k - 1), P)] if k % 2 == 1 else [])
    for m in sorted({1, P}):
        occ, _ = nv.find_repeats(s, m)
        assert occ == exp
        assert _c_result(s, m)[0] == exp


@pytest.mark.parametrize("n", list(range(2, 40)) + [257, 1000])
def test_constant_run(n):
    """a^n: SA = n-1..0, LCP[i] = i+1; selection (0,n/2),(n/2,n/2) (+ (n-1,1) if odd)."""
    s = [7] * n
    sa = oracle.suffix_array(s)
    assert sa.tolist() == list(range(n - 1, -1, -1))
    assert oracle.lcp(s, sa).tolist() == list(range(1, n))
    h = n // 2
    exp = [(0, h), (h, h)] + ([(n - 1, 1)] if n % 2 else [])
    assert _c_result(s, 1)[0] == exp


def test_all_distinct():
    rng = np.random.default_rng(5)
    t = rng.permutation(1000).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    sa = oracle.suffix_array(t)
    assert sa.tolist() == np.argsort(t, kind="stable").tolist()
    assert not oracle.lcp(t, sa).any()
    occ, rows = _c_result(t, 1)
    assert occ == [] and rows == []


def test_token_order_is_unsigned():
    """Reading: tokens compare as unsigned 64-bit integers."""
    big = np.array([2 ** 63 + 5, 3, 2 ** 64 - 1, 3], dtype=np.uint64)
    assert oracle.suffix_array(big).tolist() == nv.suffix_array([int(x) for x in big])
    assert oracle.suffix_array(big).tolist() == [3, 1, 0, 2]


def test_trivial_sizes_and_errors():
    for n in (0, 1):
        assert _c_result([1] * n, 1) == ([], [])
        assert nv.find_repeats([1] * n, 1) == ([], [])
    assert _c_result([5, 5], 1)[0] == [(0, 1), (1, 1)]
    with pytest.raises(ValueError):
        oracle.find_repeats([1, 2, 3], 0)
    with pytest.raises(ValueError):
        nv.find_repeats([1, 2, 3], 0)


# ----------------------------------------------------------- brute force

def _brute_longest_nonoverlapping_repeat(s):
    n = len(s)
    best = 0
    for L in range(1, n // 2 + 1):
        seen = {}
        found = False
        for i in range(n - L + 1):
            key = tuple(s[i:i + L])
            if key in seen and seen[key] + L <= i:
                found = True
                break
            seen.setdefault(key, i)
        if found:
            best = L
    return best


def _check_invariants(s, min_len, occ, rows):
    n = len(s)
    # disjoint, long enough, in range
    cover = [0] * n
    for st, l in occ:
        assert l >= min_len and 0 <= st and st + l <= n
        for x in range(st, st + l):
            assert cover[x] == 0
            cover[x] = 1
    assert len(occ) <= n // min_len
    # rows: counts add up, every occurrence equals its row's string
    assert sum(r[2] for r in rows) == len(occ)
    strings = {}
    for st, l in occ:
        strings.setdefault(tuple(s[st:st + l]), 0)
        strings[tuple(s[st:st + l])] += 1
    assert sorted(strings.values()) == sorted(r[2] for r in rows)
    for (st, l, c) in rows:
        assert strings[tuple(s[st:st + l])] == c
    # first selected length <= longest non-overlapping repeat
    if occ:
        assert occ[0][1] <= _brute_longest_nonoverlapping_repeat(s)
    # maximality: every candidate not chosen meets an earlier chosen interval
    sa = nv.suffix_array(s)
    cands = sorted((c for c in nv.candidates(s, sa, nv.lcp_array(s, sa)) if c[0] >= min_len),
                   key=lambda c: (-c[0], c[1], c[2]))
    key = {}
    for c in cands:
        key.setdefault((c[2], c[0]), (-c[0], c[1], c[2]))
    for c in cands:
        if (c[2], c[0]) in set(occ):
            continue
        kc = (-c[0], c[1], c[2])
        assert any(key[(a, b)] <= kc and not (c[2] + c[0] <= a or a + b <= c[2]) for a, b in occ)


def test_brute_force_suffix_order_and_lcp():
    rng = random.Random(11)
    for _ in range(300):
        n = rng.randint(1, 60)
        a = rng.randint(1, 4)
        s = [rng.randrange(a) for _ in range(n)]
        sa = oracle.suffix_array(s).tolist()
        assert sorted(sa) == list(range(n))
        for i in range(n - 1):
            assert s[sa[i]:] < s[sa[i + 1]:]
        lc = oracle.lcp(s, sa).tolist()
        for i in range(n - 1):
            assert lc[i] == nv.common_prefix(s, sa[i], sa[i + 1])


def test_overlap_branch_invariants():
    """d <= l, base+2l <= n, and the two emitted copies are equal strings."""
    rng = random.Random(12)
    for _ in range(300):
        n = rng.randint(2, 80)
        s = [rng.randrange(rng.randint(1, 3)) for _ in range(n)]
        sa = nv.suffix_array(s)
        lc = nv.lcp_array(s, sa)
        for i in range(n - 1):
            s1, s2, p = sa[i], sa[i + 1], lc[i]
            lo, hi = min(s1, s2), max(s1, s2)
            if lo + p > hi:
                d = hi - lo
                l = (p + d) // 2
                l -= l % d
                assert d <= l and lo + 2 * l <= n
                assert s[lo:lo + l] == s[lo + l:lo + 2 * l]


def test_invariants_random():
    rng = random.Random(13)
    for _ in range(150):
        n = rng.randint(2, 70)
        s = [rng.randrange(rng.randint(1, 4)) for _ in range(n)]
        m = rng.randint(1, 4)
        occ, rows = _c_result(s, m)
        _check_invariants(s, m, occ, rows)


def test_min_len_filter_before_or_after():
    """Filtering short candidates before the greedy equals running the greedy
    with everything and dropping short selections afterwards (longer
    candidates always come first in the order)."""
    rng = random.Random(14)
    for _ in range(200):
        n = rng.randint(2, 60)
        s = [rng.randrange(rng.randint(1, 3)) for _ in range(n)]
        m = rng.randint(2, 5)
        occ_all, _ = nv.find_repeats(s, 1)
        assert nv.find_repeats(s, m)[0] == [o for o in occ_all if o[1] >= m]


# ------------------------------------------------ literal vs C, exhaustive

def test_exhaustive_binary():
    for n in range(1, 13):
        for s in itertools.product(range(2), repeat=n):
            for m in (1, 2, 3):
                assert _c_result(s, m) == nv.find_repeats(s, m), (s, m)


def test_exhaustive_ternary():
    for n in range(1, 8):
        for s in itertools.product(range(3), repeat=n):
            for m in (1, 2):
                assert _c_result(s, m) == nv.find_repeats(s, m), (s, m)


def _fib(n):
    a, b = [0], [0, 1]
    while len(b) < n:
        a, b = b, b + a
    return b[:n]


def _thue_morse(n):
    return [bin(i).count("1") % 2 for i in range(n)]


def test_families_and_random_vs_literal():
    rng = random.Random(15)
    cases = [_fib(300), _thue_morse(256), ([0] * 7 + [1]) * 20, [0] * 150 + [1, 2] * 40]
    for _ in range(60):
        n = rng.randint(50, 400)
        a = rng.randint(1, 8)
        cases.append([rng.randrange(a) for _ in range(n)])
    for s in cases:
        for m in (1, 2, 5, 8):
            assert _c_result(s, m) == nv.find_repeats(s, m)


# ------------------------------------------------- planted mistakes caught

def _planted(monkeypatch, fn):
    monkeypatch.setattr(nv, "candidates", fn)


def test_planted_mistake_no_modulo_is_caught(monkeypatch):
    orig = nv.candidates

    def bad(s, sa, lcp):
        out = []
        for i in range(len(sa) - 1):
            s1, s2, p = sa[i], sa[i + 1], lcp[i]
            lo, hi = min(s1, s2), max(s1, s2)
            if lo + p <= hi:
                r = tuple(s[s1:s1 + p])
                out += [(p, r, s1), (p, r, s2)]
            else:
                d = hi - lo
                ln = (p + d) // 2  # remainder step dropped
                r = tuple(s[lo:lo + ln])
                out += [(ln, r, lo), (ln, r, lo + ln)]
        return out

    _planted(monkeypatch, bad)
    case = [c for c in GOLDEN["cases"] if c["name"] == "ababab"][0]
    assert [list(x) for x in nv.find_repeats(case["tokens"], 1)[0]] != case["runs"][0]["occurrences"]
    monkeypatch.setattr(nv, "candidates", orig)


def test_planted_mistake_wrong_base_is_caught(monkeypatch):
    def bad(s, sa, lcp):
        out = []
        for i in range(len(sa) - 1):
            s1, s2, p = sa[i], sa[i + 1], lcp[i]
            lo, hi = min(s1, s2), max(s1, s2)
            if lo + p <= hi:
                r = tuple(s[s1:s1 + p])
                out += [(p, r, s1), (p, r, s2)]
            else:
                d = hi - lo
                ln = (p + d) // 2
                ln -= ln % d
                r = tuple(s[hi:hi + ln])  # base taken at the larger start
                out += [(ln, r, hi), (ln, r, hi + ln)]
        return out

    _planted(monkeypatch, bad)
    ok = True
    for P, k in ((3, 3), (2, 5), (1, 9)):
        s = list(range(P)) * k
        h = P * (k // 2)
        exp = [(0, h), (h, h), (P * (k - 1), P)]
        if nv.find_repeats(s, 1)[0] != exp:
            ok = False
    assert not ok


def test_planted_mistake_sort_order_is_caught(monkeypatch):
    """Sorting by increasing length instead of decreasing breaks the golden runs."""
    orig_sorted = sorted

    case = [c for c in GOLDEN["cases"] if c["name"] == "aabcbcbaa"][0]
    s = case["tokens"]
    sa = nv.suffix_array(s)
    cands = [c for c in nv.candidates(s, sa, nv.lcp_array(s, sa)) if c[0] >= 1]
    cands = orig_sorted(cands, key=lambda c: (c[0], c[1], c[2]))
    acc = []
    for (l, r, st) in cands:
        if all(st + l <= a or a + b <= st for (a, b) in acc):
            acc.append((st, l))
    assert [list(x) for x in acc] != case["runs"][0]["occurrences"]


# ---- per-substring equal-length greedy (interval counts) -----------------------

def test_interval_counts_hand_example():
    # one substring of length 4 at starts 0, 2, 4, 6 (e.g. "abab" in "ababababab"):
    # 0 -> 4 -> none; 2 -> 6 -> none
    nxt, cnt = oracle.interval_counts([4, 4, 4, 4], [0, 2, 4, 6], [7, 7, 7, 7])
    assert nxt.tolist() == [2, 3, -1, -1] and cnt.tolist() == [2, 2, 1, 1]
    # a second substring never continues the first one's chain
    nxt, cnt = oracle.interval_counts([4, 4, 3, 3], [0, 9, 0, 3], [7, 7, 1, 1])
    assert nxt.tolist() == [1, -1, 3, -1] and cnt.tolist() == [2, 1, 2, 1]


def _max_disjoint(starts, l):
    best = 0
    n = len(starts)
    for mask in range(1 << n):
        sel = sorted(starts[i] for i in range(n) if mask >> i & 1)
        if all(b >= a + l for a, b in zip(sel, sel[1:])):
            best = max(best, len(sel))
    return best


def test_interval_counts_head_is_maximum_disjoint_set():
    """Earliest-start greedy over equal-length intervals is optimal (interval
    scheduling), so the count at a substring's first occurrence equals the
    largest set of pairwise disjoint occurrences, found by brute force."""
    rng = np.random.default_rng(17)
    for _ in range(300):
        groups = []
        for g in range(int(rng.integers(1, 4))):
            l = int(rng.integers(1, 6))
            starts = sorted(set(rng.integers(0, 30, int(rng.integers(1, 11))).tolist()))
            groups.append((l, g, starts))
        groups.sort(key=lambda x: (-x[0], x[1]))
        L = [l for l, g, st in groups for _ in st]
        S = [s for l, g, st in groups for s in st]
        I = [g for l, g, st in groups for _ in st]
        nxt, cnt = oracle.interval_counts(L, S, I)
        k = 0
        for l, g, st in groups:
            assert cnt[k] == _max_disjoint(st, l)
            k += len(st)


@pytest.mark.parametrize("seed", range(4))
def test_interval_counts_on_real_candidates(seed):
    """On FindRepeats' own candidate lists: chains stay inside a substring and
    every link is the first non-overlapping later occurrence."""
    t = synth.loop_stream(seed, 3000, 17 + seed, 16, 0.03)
    c = oracle.sorted_candidates(t, 4)
    nxt, cnt = oracle.interval_counts(c["len"], c["start"], c["id"])
    for k in range(len(nxt)):
        j = nxt[k]
        if j >= 0:
            assert c["len"][j] == c["len"][k] and c["id"][j] == c["id"][k]
            assert c["start"][j] >= c["start"][k] + c["len"][k]
            assert all(c["start"][i] < c["start"][k] + c["len"][k] for i in range(k + 1, j))
            assert cnt[k] == cnt[j] + 1
        else:
            assert cnt[k] == 1


# ------------------------------------------- per-round active suffix counts

def _active_by_brute_force(s):
    """a_r for r = 1, 2, ...: the suffixes whose 2^(r-1)-prefix is shared with
    a suffix-array neighbour, i.e. #{k : max(LCP[k-1], LCP[k]) >= 2^(r-1)},
    from suffixes sorted by Python list comparison and direct common prefixes
    (none of the oracle's own arrays)."""
    n = len(s)
    sa = sorted(range(n), key=lambda i: s[i:])
    lc = [nv.common_prefix(s, sa[k], sa[k + 1]) for k in range(n - 1)]
    near = [max(lc[k - 1] if k > 0 else 0, lc[k] if k < n - 1 else 0) for k in range(n)]
    out = []
    h = 1
    while True:
        a = sum(1 for v in near if v >= h)
        if a == 0:
            return out
        out.append(a)
        h *= 2


def _check_active(s):
    _sa, act = oracle.suffix_array(s, return_active=True)
    assert act.tolist() == _active_by_brute_force(s), s


def test_active_counts_exhaustive_binary():
    """The oracle's doubling-round counts (the a_r of the byte model) equal
    the brute-force counts on every binary string of length <= 10."""
    for n in range(1, 11):
        for s in itertools.product((0, 1), repeat=n):
            _check_active(list(s))


def test_active_counts_random_and_families():
    rng = random.Random(31)
    for _ in range(200):
        n = rng.randint(1, 300)
        a = rng.randint(1, 5)
        _check_active([rng.randrange(a) for _ in range(n)])
    for n in (1, 2, 3, 17, 64, 100):
        _check_active([7] * n)                      # a^n: LCP[k] = k+1
    _check_active(list(range(50)))                  # all distinct: no round
    _check_active([0, 1, 2, 3, 4] * 20)             # body^k
    _check_active(synth.loop_stream(5, 2000, 40, 16, 0.05).tolist())


def test_active_counts_closed_form_constant_run():
    """a^n: the suffix array is n-1..0 with LCP[k] = k+1, so slot k's larger
    neighbour LCP is k+1 (k < n-1) or n-1 (last slot): a_r = n - 2^(r-1) + 1
    for 2^(r-1) <= n-1, and no round after that."""
    for n in (2, 5, 16, 33, 100):
        _sa, act = oracle.suffix_array([3] * n, return_active=True)
        want = []
        h = 1
        while h <= n - 1:
            want.append(n - h + 1)
            h *= 2
        assert act.tolist() == want, n
