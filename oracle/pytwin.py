"""Pure-Python twin of the C oracle, for tiny graphs only (test infrastructure).

Written separately from ``rrr_oracle.c`` so that a slip in either one shows up
as a disagreement.  Same definitions: Definition 2 (RRR set = vertices with a
live path to the start), Philox4x32-10 (SC 2011) as the keyed coin, the
threshold rule for fp32 probabilities, canonical edge ids by (dst, src) rank.
"""

from __future__ import annotations

from collections import deque

import numpy as np

MASK32 = 0xFFFFFFFF
_M = (0xD2511F53, 0xCD9E8D57)
_W = (0x9E3779B9, 0xBB67AE85)


def philox4x32_10(ctr, key):
    x = [int(c) & MASK32 for c in ctr]
    k = [int(key[0]) & MASK32, int(key[1]) & MASK32]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + _W[0]) & MASK32, (k[1] + _W[1]) & MASK32]
        prod_a = _M[0] * x[0]
        prod_b = _M[1] * x[2]
        x = [
            (prod_b >> 32) ^ x[1] ^ k[0],
            prod_b & MASK32,
            (prod_a >> 32) ^ x[3] ^ k[1],
            prod_a & MASK32,
        ]
    return tuple(x)


def _key(seed):
    return (seed & MASK32, (seed >> 32) & MASK32)


def coin_word(seed, s, e):
    block = philox4x32_10((e >> 2, s & MASK32, s >> 32, 0), _key(seed))
    return block[e % 4]


def start_vertex(seed, s, n):
    block = philox4x32_10(((s >> 2) & MASK32, s >> 34, 0, 1), _key(seed))
    return (block[s % 4] * n) >> 32


def thr32(p):
    p = float(np.float32(p))
    if p >= 1.0:
        return MASK32
    return int(p * 4294967296.0)


class TinyGraph:
    def __init__(self, n, src, dst, prob):
        edges = sorted(zip((int(d) for d in dst), (int(s) for s in src),
                           (float(np.float32(p)) for p in prob)))
        for a, b in zip(edges, edges[1:]):
            if a[0] == b[0] and a[1] == b[1]:
                raise ValueError("repeated edge")
        self.n = n
        self.incoming = [[] for _ in range(n)]   # v -> [(u, canonical id, thr)]
        for eid, (d, s, p) in enumerate(edges):
            self.incoming[d].append((s, eid, thr32(p)))

    def rrr(self, seed, s):
        start = start_vertex(seed, s, self.n)
        depth = {start: 0}
        todo = deque([start])
        while todo:
            v = todo.popleft()
            for u, eid, t in self.incoming[v]:
                if u in depth:
                    continue
                if t == MASK32 or coin_word(seed, s, eid) < t:
                    depth[u] = depth[v] + 1
                    todo.append(u)
        return sorted(depth), depth
