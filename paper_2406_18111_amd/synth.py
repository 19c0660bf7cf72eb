"""Seeded synthetic task-hash streams (input generators only).

These stand in for the task streams of the applications the paper evaluates
(Section 6), which need Legion and the applications themselves.  They are
loop-structured token streams with the scale the paper quotes: traces of
thousands of tasks (Section 4.2) and a history buffer of thousands of tokens
(Section 6 set-up).  The module holds no part of the repeat-finding method:
it is shared by the tests, the benchmark and the smoke check, and both the
oracle and the GPU library only ever receive its output arrays.

Randomness: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; constants as published by Vigna), used in
counter mode: draw k of stream (seed, tag) is mix64(base + (k+1)*GOLDEN)
with base = mix64(seed*GOLDEN ^ tag).  Uniform integers in [0, m) use the
multiply-high range reduction floor(x*m / 2^64); Bernoulli(p) compares the top
53 bits, scaled to [0,1), against p.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Iterator, List, Tuple

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
MASK64 = (1 << 64) - 1


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def _mix_int(x: int) -> int:
    return int(mix64(np.array([x & MASK64], dtype=np.uint64))[0])


class Stream:
    """Counter-based SplitMix64 stream identified by (seed, tag)."""

    def __init__(self, seed: int, tag: int):
        self.base = _mix_int(((seed * 0x9E3779B97F4A7C15) ^ tag) & MASK64)
        self.pos = 0

    def raw(self, count: int) -> np.ndarray:
        k = np.arange(self.pos + 1, self.pos + 1 + count, dtype=np.uint64)
        self.pos += count
        with np.errstate(over="ignore"):
            return mix64(np.uint64(self.base) + k * GOLDEN)

    def raw_at(self, offsets: np.ndarray, count: int) -> np.ndarray:
        """The draws at `offsets` (0-based, relative to the current position)
        of the next `count` draws, then skips all `count`: equal to
        raw(count)[offsets] without computing the other draws."""
        k = np.asarray(offsets, dtype=np.uint64) + np.uint64(self.pos + 1)
        self.pos += count
        with np.errstate(over="ignore"):
            return mix64(np.uint64(self.base) + k * GOLDEN)

    def below(self, m: int, count: int) -> np.ndarray:
        """Uniform integers in [0, m), m < 2^32."""
        assert 0 < m < (1 << 32)
        x = self.raw(count)
        mm = np.uint64(m)
        with np.errstate(over="ignore"):
            hi = (x >> np.uint64(32)) * mm
            lo = ((x & np.uint64(0xFFFFFFFF)) * mm) >> np.uint64(32)
            return ((hi + lo) >> np.uint64(32)).astype(np.int64)

    def unit(self, count: int) -> np.ndarray:
        return (self.raw(count) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))

    def bern(self, p: float, count: int) -> np.ndarray:
        # unit < p on the top 53 bits i: i * 2^-53 < p  <=>  i < ceil(p * 2^53)
        # (both sides exact in binary64), compared as integers
        thr = np.uint64(min(math.ceil(p * float(1 << 53)), 1 << 53))
        return (self.raw(count) >> np.uint64(11)) < thr


# stream tags
_T_ALPHA, _T_BODY, _T_SUBMASK, _T_FRESH, _T_INSMASK, _T_INSFRESH, _T_LEN, _T_SYM = range(1, 9)


def loop_stream(seed: int, n: int, body_len: int = 50, alphabet: int = 64, p_sub: float = 0.05) -> np.ndarray:
    """A loop body of `body_len` tokens drawn from an alphabet of `alphabet`
    random hashes, repeated end to end; each position is independently
    replaced by a fresh random hash with probability p_sub.  uint64[n]."""
    alpha = Stream(seed, _T_ALPHA).raw(alphabet)
    body = alpha[Stream(seed, _T_BODY).below(alphabet, body_len)]
    t = body[np.arange(n) % body_len].copy()
    sub = Stream(seed, _T_SUBMASK).bern(p_sub, n)
    fresh = Stream(seed, _T_FRESH).raw(n)
    t[sub] = fresh[sub]
    return t


def config0(seed: int = 0) -> Tuple[np.ndarray, int]:
    """n=4096, loop body 50 tokens from an alphabet of 64, 5% substitutions; min length 8."""
    return loop_stream(seed, 4096, 50, 64, 0.05), 8


class NestedLoopSource:
    """Endless nested-loop task stream.

    One outer iteration is outer[0:100] + inner*10 + outer[100:200] (500
    tokens), with outer (200 tokens) and inner (30 tokens) drawn from an
    alphabet of 2^16 random hashes.  For every clean token: with probability
    0.005 a fresh hash is inserted first, then the token is emitted, replaced
    by a fresh hash with probability 0.01.
    """

    def __init__(self, seed: int, alphabet: int = 1 << 16, p_sub: float = 0.01, p_ins: float = 0.005):
        alpha = Stream(seed, _T_ALPHA).raw(alphabet)
        pick = Stream(seed, _T_BODY).below(alphabet, 230)
        outer, inner = alpha[pick[:200]], alpha[pick[200:]]
        self.period = np.concatenate([outer[:100], np.tile(inner, 10), outer[100:]])
        self.s_sub = Stream(seed, _T_SUBMASK)
        self.s_fresh = Stream(seed, _T_FRESH)
        self.s_ins = Stream(seed, _T_INSMASK)
        self.s_insf = Stream(seed, _T_INSFRESH)
        self.p_sub, self.p_ins = p_sub, p_ins
        self.clean_pos = 0
        self.buf = np.zeros(0, dtype=np.uint64)

    def _produce(self, clean: int) -> np.ndarray:
        # every draw is indexed by the clean token's position, so the output
        # does not depend on how the stream is cut into _produce calls; fresh
        # hashes are computed only where a substitution or insertion happens
        k = np.arange(self.clean_pos, self.clean_pos + clean)
        self.clean_pos += clean
        tok = self.period[k % len(self.period)]
        sub = np.flatnonzero(self.s_sub.bern(self.p_sub, clean))
        tok[sub] = self.s_fresh.raw_at(sub, clean)
        ins = self.s_ins.bern(self.p_ins, clean)
        insi = np.flatnonzero(ins)
        insv = self.s_insf.raw_at(insi, clean)
        out = np.empty(clean + len(insi), dtype=np.uint64)
        slot = np.arange(clean) + np.cumsum(ins)  # position of each clean token
        out[slot] = tok
        out[slot[insi] - 1] = insv
        return out

    def take(self, count: int) -> np.ndarray:
        while len(self.buf) < count:
            self.buf = np.concatenate([self.buf, self._produce(max(count - len(self.buf), 4096))])
        out, self.buf = self.buf[:count].copy(), self.buf[count:]
        return out


def config1(seed: int = 1, n: int = 1 << 20) -> Tuple[np.ndarray, int]:
    """n=2^20 nested-loop stream (alphabet 2^16, 1% substitutions, 0.5% insertions); min length 16."""
    return NestedLoopSource(seed).take(n), 16


def config2(seed: int = 2, n: int = 1 << 24) -> Tuple[np.ndarray, int]:
    """n=2^24 uint32 tokens: first half the token 0, second half uniform over {0,1,2,3}; min length 32."""
    t = np.zeros(n, dtype=np.uint32)
    half = n // 2
    t[half:] = Stream(seed, _T_SYM).below(4, n - half).astype(np.uint32)
    return t, 32


def config3(num_windows: int = 4096, lo: int = 256, hi: int = 65536, seed0: int = 1000):
    """Batched windows: window w uses seed seed0+w, length floor(exp(U(ln lo, ln hi))),
    loop-body length uniform in [10, 500], alphabet 2^12, 5% substitutions.
    Returns (list of uint64 arrays, min length 8)."""
    wins = []
    for w in range(num_windows):
        s = seed0 + w
        st = Stream(s, _T_LEN)
        u = st.unit(1)[0]
        L = int(math.floor(math.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))))
        L = max(lo, min(hi, L))
        body = 10 + int(st.below(491, 1)[0])
        wins.append(loop_stream(s, L, body, 1 << 12, 0.05))
    return wins, 8


@dataclass
class Request:
    arrival: float  # seconds from the start of the trace
    stream: int
    tokens: np.ndarray


def config4_trace(duration: float = 10.0, rate: float = 2000.0, streams: int = 64,
                  lo: int = 1024, hi: int = 1 << 20, seed: int = 4242, stream_seed0: int = 2000,
                  max_requests: int | None = None) -> Iterator[Request]:
    """Serving trace: Poisson arrivals at `rate`/s; each request picks one of
    `streams` nested-loop streams (seed stream_seed0+k) and a window length
    log-uniform in [lo, hi]; its window is the next W tokens of that stream.
    Yields requests lazily (min length 16)."""
    sa = Stream(seed, _T_LEN)
    srcs: List[NestedLoopSource | None] = [None] * streams
    t = 0.0
    count = 0
    while True:
        gap, us, uw = sa.unit(3)
        t += -math.log(1.0 - gap) / rate
        if t > duration or (max_requests is not None and count >= max_requests):
            return
        k = min(streams - 1, int(us * streams))
        W = int(math.floor(math.exp(math.log(lo) + uw * (math.log(hi) - math.log(lo)))))
        W = max(lo, min(hi, W))
        if srcs[k] is None:
            srcs[k] = NestedLoopSource(stream_seed0 + k)
        count += 1
        yield Request(t, k, srcs[k].take(W))


def config4_requests(duration: float = 10.0, threads: int = 8, **kw) -> List[Request]:
    """The requests of config4_trace(duration, **kw) as a list, identical to
    the lazy trace, with each stream's tokens generated on a pool of threads
    (a stream's windows are consecutive pieces of that stream)."""
    import concurrent.futures as cf
    rate = kw.get("rate", 2000.0)
    streams = kw.get("streams", 64)
    lo, hi = kw.get("lo", 1024), kw.get("hi", 1 << 20)
    seed, stream_seed0 = kw.get("seed", 4242), kw.get("stream_seed0", 2000)
    max_requests = kw.get("max_requests")
    sa = Stream(seed, _T_LEN)
    plan = []
    t = 0.0
    while True:
        gap, us, uw = sa.unit(3)
        t += -math.log(1.0 - gap) / rate
        if t > duration or (max_requests is not None and len(plan) >= max_requests):
            break
        k = min(streams - 1, int(us * streams))
        W = int(math.floor(math.exp(math.log(lo) + uw * (math.log(hi) - math.log(lo)))))
        plan.append((t, k, max(lo, min(hi, W))))
    per_stream = {}
    for i, (_, k, W) in enumerate(plan):
        per_stream.setdefault(k, []).append(i)

    def gen(k):
        idx = per_stream[k]
        whole = NestedLoopSource(stream_seed0 + k).take(sum(plan[i][2] for i in idx))
        out, at = [], 0
        for i in idx:
            out.append((i, whole[at: at + plan[i][2]]))
            at += plan[i][2]
        return out

    toks: List[np.ndarray | None] = [None] * len(plan)
    with cf.ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        for part in ex.map(gen, sorted(per_stream)):
            for i, a in part:
                toks[i] = a
    return [Request(a, k, toks[i]) for i, (a, k, _) in enumerate(plan)]


CONFIG_MIN_LEN = {0: 8, 1: 16, 2: 32, 3: 8, 4: 16}
