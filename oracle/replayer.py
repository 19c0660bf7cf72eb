"""Plain reference of the trace replayer (Section 4.3, TraceReplayer of
Algorithm 1) and of the max-trace-length split (Section 6.2) -- TEST
INFRASTRUCTURE ONLY, like the rest of ``oracle``.

No trie: a pending match is the task index where it began plus the list of
candidates whose first tokens equal the tokens issued since then (filtered
token by token).  A match completes a candidate when it has matched all of
the candidate's tokens, and it dies when no candidate is left.  The decisions
follow the order of the algorithm:

1. add the task to the pending list P and start a match at it;
2. keep the matches whose tokens are still a prefix of a candidate;
3. take the completed ones (D); if D is not empty, pick the one with the best
   score (ties to the candidate ingested first), issue the pending tasks
   before it untraced, issue it as a replay, and drop every match;
4. otherwise issue untraced the pending tasks that no live match covers.

Scoring (Section 4.3 names the factors, not the constants): each appearance
decays the previous count by decay^(tasks since the previous appearance, or
since ingestion) and adds one; score = length * min(count, cap), times
(1 + bonus) once the candidate has been replayed.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple


def split_rows(rows: Sequence[Tuple[int, int, int]], max_len: int, min_len: int = 1):
    """Section 6.2: recorded traces longer than max_len are cut into pieces
    of max_len tokens (the last one shorter); pieces below min_len go."""
    out = []
    for start, length, count in rows:
        off = 0
        while off < length:
            piece = min(max_len, length - off)
            if piece >= min_len:
                out.append((start + off, piece, count))
            off += max_len
    return out


class ReplayerRef:
    def __init__(self, count_cap: int = 8, decay: float = 0.999, replay_bonus: float = 0.1):
        self.cap, self.decay, self.bonus = count_cap, decay, replay_bonus
        self.cands: List[tuple] = []           # candidate id -> token tuple
        self.index: Dict[tuple, int] = {}
        self.count: List[float] = []
        self.last: List[int] = []
        self.replayed: List[bool] = []
        self.tokens: List[int] = []            # every task's token
        self.issued = 0                        # tasks before this index are issued
        # live matches: [start task, ids of the candidates that begin with tokens[start:now]]
        self.matches: List[list] = []
        self.events: List[Tuple[int, int, int]] = []

    def ingest(self, tokens, rows):
        for start, length, count in rows:
            key = tuple(int(x) for x in tokens[start:start + length])
            if key in self.index:
                c = self.index[key]
                self.count[c] = max(self.count[c], float(count))
                continue
            c = len(self.cands)
            self.index[key] = c
            self.cands.append(key)
            self.count.append(float(count))
            self.last.append(len(self.tokens))
            self.replayed.append(False)
            # live matches continue into the new candidate where it agrees with them
            now = len(self.tokens)
            for m in self.matches:
                if len(key) > now - m[0] and key[:now - m[0]] == tuple(self.tokens[m[0]:now]):
                    m[1].append(c)

    def _emit(self, b: int, e: int, trace: int):
        if e <= b:
            return
        if trace < 0 and self.events and self.events[-1][2] < 0 and self.events[-1][1] == b:
            self.events[-1] = (self.events[-1][0], e, -1)
        else:
            self.events.append((b, e, trace))

    def _score(self, c: int) -> float:
        s = len(self.cands[c]) * min(self.count[c], float(self.cap))
        return s * (1.0 + self.bonus) if self.replayed[c] else s

    def step(self, tokens):
        for tok in tokens:
            tok = int(tok)
            self.tokens.append(tok)
            now = len(self.tokens)             # tasks seen, including this one
            self.matches.append([now - 1, list(range(len(self.cands)))])
            done, alive = [], []
            for b, ids in self.matches:
                pos = now - 1 - b              # index of this token inside the candidates
                ids = [c for c in ids if len(self.cands[c]) > pos and self.cands[c][pos] == tok]
                for c in ids:
                    if len(self.cands[c]) == pos + 1:
                        self.count[c] = self.count[c] * self.decay ** (now - self.last[c]) + 1.0
                        self.last[c] = now
                        done.append(c)
                ids = [c for c in ids if len(self.cands[c]) > pos + 1]
                if ids:
                    alive.append([b, ids])
            self.matches = alive
            if done:
                best = done[0]
                for c in done[1:]:
                    if self._score(c) > self._score(best) or (self._score(c) == self._score(best) and c < best):
                        best = c
                begin = now - len(self.cands[best])
                self._emit(self.issued, begin, -1)
                self._emit(begin, now, best)
                self.issued = now
                self.replayed[best] = True
                self.matches = []
                continue
            keep = min(m[0] for m in self.matches) if self.matches else now
            if keep > self.issued:
                self._emit(self.issued, keep, -1)
                self.issued = keep

    def flush(self):
        self._emit(self.issued, len(self.tokens), -1)
        self.issued = len(self.tokens)
        self.matches = []
