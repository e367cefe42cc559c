"""Brute-force references used to pin the oracle (tests only).

Everything here is written from the paper's definitions or from textbook
algorithms, independently of ``oracle/``:

* neighbourhoods Gamma(e), triangles, C(t*) (Sec. 2);
* the exact law of one NBSI estimator (Claim 1): P(f1 = e) = 1/m,
  P(f2 = f | f1 = e) = 1/|Gamma(e)|, P(triangle t found) = 1/(m C(t));
  hence E[X] = tau (Lemma 1) and E[X^2] = m * sum_t C(t);
* a per-edge neighbourhood sampler (batch size 1: the textbook reservoir of
  Sec. 4.2 plus the level-2 reservoir over Gamma(f1)), with its own copy of
  the counter-based random protocol written in Python integers.
"""
from __future__ import annotations

from collections import defaultdict

EMPTY = (1 << 64) - 1
_M = (1 << 64) - 1
_GOLD = 0x9E3779B97F4A7C15


def canon(a: int, b: int) -> int:
    lo, hi = (a, b) if a < b else (b, a)
    return (lo << 32) | hi


def ends(e: int) -> tuple[int, int]:
    return e >> 32, e & 0xFFFFFFFF


def stream_codes(edges) -> list[int]:
    return [canon(int(a), int(b)) for a, b in edges]


def gamma(codes: list[int], i: int) -> list[int]:
    """Indices j > i whose edge shares exactly one vertex with edge i."""
    a, b = ends(codes[i])
    out = []
    for j in range(i + 1, len(codes)):
        x, y = ends(codes[j])
        if len({a, b} & {x, y}) == 1:
            out.append(j)
    return out


def triangles(codes: list[int]) -> list[tuple[int, int, int]]:
    """All triangles as sorted triples of stream indices."""
    pos = {e: i for i, e in enumerate(codes)}
    adj = defaultdict(set)
    for e in codes:
        a, b = ends(e)
        adj[a].add(b)
        adj[b].add(a)
    out = []
    for e in codes:
        a, b = ends(e)
        for c in adj[a] & adj[b]:
            if c > b:  # a < b < c: each triangle once
                out.append(tuple(sorted((pos[canon(a, b)], pos[canon(a, c)],
                                         pos[canon(b, c)]))))
    return out


def exact_moments(codes: list[int]):
    """(tau, E[X^2]) of one estimator over the whole stream (Claim 1)."""
    tris = triangles(codes)
    m = len(codes)
    second = 0
    for t in tris:
        second += m * len(gamma(codes, t[0]))
    return len(tris), second


def closing(f1: int, f2: int) -> int:
    a, b = ends(f1)
    x, y = ends(f2)
    s = {a, b} & {x, y}
    if f1 == f2 or len(s) != 1:
        return EMPTY
    (z,) = s
    t = a if b == z else b
    f = x if y == z else y
    return canon(t, f)


# -- random protocol, re-derived in Python integers -------------------------

def _mix(z: int) -> int:
    z &= _M
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M
    z ^= z >> 31
    return z


def draw(seed: int, est: int, batch: int, purpose: int, n: int) -> int:
    """Uniform integer in [0, n): keyed splitmix64 finalizer + Lemire."""
    k = _mix(_mix(_mix(seed ^ _GOLD) ^ est) ^ batch)
    attempt = 0
    while True:
        x = _mix(k ^ ((purpose * _GOLD + attempt) & _M))
        p = x * n
        lo = p & _M
        if lo < n and lo < (1 << 64) % n:
            attempt += 1
            continue
        return p >> 64


def per_edge_sampler(codes: list[int], r: int, seed: int):
    """Neighbourhood sampling one edge at a time (batch size 1).

    Edge t (1-based) replaces f1 with probability 1/t; an edge adjacent to f1
    raises chi by one and replaces f2 with probability 1/chi; an edge equal
    to the wedge's closing edge, arriving after f2, closes it.  Every coin
    uses the same key as the bulk update would with one edge per batch.
    """
    r1 = [EMPTY] * r
    r2 = [EMPTY] * r
    c = [0] * r
    closed = [0] * r
    for t, e in enumerate(codes, start=1):
        batch = t - 1
        for i in range(r):
            if draw(seed, i, batch, 1, t) == t - 1:
                r1[i], r2[i], c[i], closed[i] = e, EMPTY, 0, 0
                continue
            if len(set(ends(e)) & set(ends(r1[i]))) == 1:
                c[i] += 1
                if draw(seed, i, batch, 2, c[i]) == c[i] - 1:
                    r2[i], closed[i] = e, 0
                    continue
            if r2[i] != EMPTY and not closed[i] and e == closing(r1[i], r2[i]):
                closed[i] = 1
    return r1, r2, c, closed


def check_invariants(codes: list[int], r1, r2, c, closed):
    """Deterministic NBSI facts after a prefix `codes` of the stream
    (Invariant 1 items 2-4); returns a list of violations."""
    pos = {e: i for i, e in enumerate(codes)}
    bad = []
    for i in range(len(r1)):
        e1 = int(r1[i])
        if e1 not in pos:
            bad.append((i, "f1 not in stream"))
            continue
        g = gamma(codes, pos[e1])
        if int(c[i]) != len(g):
            bad.append((i, f"chi {int(c[i])} != |Gamma(f1)| {len(g)}"))
        e2 = int(r2[i])
        if e2 == EMPTY:
            if g:
                bad.append((i, "f2 empty but Gamma(f1) non-empty"))
            if closed[i]:
                bad.append((i, "closed without f2"))
            continue
        if e2 not in pos or pos[e2] not in g:
            bad.append((i, "f2 not in Gamma(f1)"))
            continue
        q = closing(e1, e2)
        want = int(q in pos and pos[q] > pos[e2])
        if int(closed[i]) != want:
            bad.append((i, f"closed {int(closed[i])} != {want}"))
    return bad
