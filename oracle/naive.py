"""Literal pure-Python FindRepeats -- TEST INFRASTRUCTURE ONLY (small inputs).

Follows Algorithm 2 of Yadav et al. (ASPLOS'25, Section 4.2) step by step with
no implementation tricks, so that it can be read against the paper:

* the suffix array is ``sorted`` over the suffixes themselves (Python list
  comparison: element-wise, a proper prefix sorts first);
* LCP values are measured by comparing the two suffixes directly;
* each candidate carries the repeated substring itself (a tuple of tokens);
* the sort key is (-length, substring, start), compared as Python tuples;
* the selection loop tests every accepted interval for intersection;
* deduplication keeps the first acceptance of each distinct substring.

Quadratic or worse; meant for n up to a few hundred.  The product path never
imports this module.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple


def suffix_array(s: Sequence[int]) -> List[int]:
    """Suffix start positions in lexicographic order of the suffixes (Sec. 4.2)."""
    s = list(s)
    return sorted(range(len(s)), key=lambda i: s[i:])


def common_prefix(s: Sequence[int], a: int, b: int) -> int:
    k = 0
    n = len(s)
    while a + k < n and b + k < n and s[a + k] == s[b + k]:
        k += 1
    return k


def lcp_array(s: Sequence[int], sa: Sequence[int]) -> List[int]:
    """LCP[i] = common prefix length of suffixes SA[i] and SA[i+1] (Alg. 2 loop)."""
    return [common_prefix(s, sa[i], sa[i + 1]) for i in range(len(sa) - 1)]


def candidates(s: Sequence[int], sa: Sequence[int], lcp: Sequence[int]):
    """Candidate tuples (length, substring, start) from every adjacent SA pair.

    Disjoint branch: both occurrences of the common prefix.  Overlap branch:
    with d the distance of the starts, take floor((p+d)/2), drop the remainder
    modulo d, and emit the two back-to-back copies starting at the smaller start.
    """
    s = list(s)
    out = []
    for i in range(len(sa) - 1):
        s1, s2, p = sa[i], sa[i + 1], lcp[i]
        r1 = set(range(s1, s1 + p))
        r2 = set(range(s2, s2 + p))
        if not (r1 & r2):
            r = tuple(s[s1:s1 + p])
            out.append((p, r, s1))
            out.append((p, r, s2))
        else:
            lo, hi = min(s1, s2), max(s1, s2)
            d = hi - lo
            ln = (p + d) // 2
            ln = ln - (ln % d)
            r = tuple(s[lo:lo + ln])
            out.append((ln, r, lo))
            out.append((ln, r, lo + ln))
    return out


def find_repeats(s: Sequence[int], min_len: int = 1):
    """Algorithm 2 with a minimum length (candidates shorter than min_len dropped).

    Returns (occurrences, rows): occurrences = [(start, length)] in acceptance
    order; rows = [(first start, length, count)] per distinct substring, in
    order of first acceptance.
    """
    if min_len < 1:
        raise ValueError("min_len must be >= 1")
    s = list(s)
    if len(s) < 2:
        return [], []
    sa = suffix_array(s)
    lcp = lcp_array(s, sa)
    cands = [c for c in candidates(s, sa, lcp) if c[0] >= min_len]
    cands.sort(key=lambda c: (-c[0], c[1], c[2]))
    accepted: List[Tuple[int, int]] = []
    strings = []
    for (l, r, st) in cands:
        if all(st + l <= a or a + b <= st for (a, b) in accepted):
            accepted.append((st, l))
            strings.append(r)
    rows = []
    index = {}
    for (st, l), r in zip(accepted, strings):
        if r not in index:
            index[r] = len(rows)
            rows.append([st, l, 0])
        rows[index[r]][2] += 1
    return accepted, [tuple(x) for x in rows]
