"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only *draws* inputs: directed edge lists and their fp32 edge
probabilities.  It holds none of the sampling method's arithmetic (no
thresholds, no random-number keying, no traversal), so both sides of every
parity check can take their inputs from here without sharing any of the code
that is being checked.

Workloads (Section 6, Table 1 lists the paper's SNAP inputs: 0.69-4.85 M
vertices, average degree 11.7-76.3; those files are not available here, so
R-MAT graphs of the same order stand in for them):

* ``er_graph``      - Erdos-Renyi style directed graph with exactly ``m``
                      distinct non-loop edges, drawn uniformly.
* ``rmat_graph``    - R-MAT (recursive matrix) power-law graph; duplicates and
                      self-loops dropped.
* ``lfr_graph``     - LFR benchmark graph (power-law degrees and community
                      sizes; the paper's synthetic fusion analysis, Section 3.2),
                      drawn by NetworkX, each undirected edge taken both ways.
* ``uniform_prob``  - one fixed probability for every edge (the paper sweeps a
                      fixed traversal probability, Section 7).
* ``wc_prob``       - weighted cascade: p(u->v) = 1/indeg(v) in fp32.
"""

from __future__ import annotations

import hashlib

import numpy as np

__all__ = [
    "er_graph",
    "rmat_graph",
    "lfr_graph",
    "uniform_prob",
    "wc_prob",
    "edges_sha256",
    "random_small_graph",
]


def er_graph(n: int, m: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Directed graph on ``n`` vertices with ``m`` distinct edges u->v, u != v.

    Pairs are drawn uniformly with a seeded PCG64 stream; self-loops and
    repeats are rejected in draw order until ``m`` distinct pairs exist.
    Returns ``(src, dst)`` as uint32 arrays in draw order.
    """
    if m > n * (n - 1):
        raise ValueError("m exceeds the number of possible non-loop edges")
    rng = np.random.Generator(np.random.PCG64(seed))
    seen: set[int] = set()
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    k = 0
    while k < m:
        draw = max(1024, 2 * (m - k))
        u = rng.integers(0, n, size=draw, dtype=np.uint64)
        v = rng.integers(0, n, size=draw, dtype=np.uint64)
        for a, b in zip(u.tolist(), v.tolist()):
            if a == b:
                continue
            key = a * n + b
            if key in seen:
                continue
            seen.add(key)
            src[k] = a
            dst[k] = b
            k += 1
            if k == m:
                break
    return src, dst


def rmat_graph(scale: int, edge_factor: int, a: float, b: float, c: float,
               seed: int) -> tuple[np.ndarray, np.ndarray]:
    """R-MAT graph with 2**scale vertices and edge_factor * 2**scale draws.

    Each draw picks, bit by bit from the most significant, one quadrant of the
    adjacency matrix: (src bit, dst bit) = (0,0) with probability a, (0,1)
    with b, (1,0) with c and (1,1) with d = 1-a-b-c (a uniform 32-bit draw per
    bit, compared with the cumulative thresholds).  No noise, no relabelling.
    Self-loops and duplicate (src, dst) pairs are dropped; the surviving edges
    are returned sorted by (src, dst) as uint32 arrays.
    """
    n_draw = edge_factor << scale
    rng = np.random.Generator(np.random.PCG64(seed))
    t_a = np.uint32(min(int(round(a * 2**32)), 2**32 - 1))
    t_ab = np.uint32(min(int(round((a + b) * 2**32)), 2**32 - 1))
    t_abc = np.uint32(min(int(round((a + b + c) * 2**32)), 2**32 - 1))
    keys = []
    chunk = 1 << 20
    for lo in range(0, n_draw, chunk):
        k = min(chunk, n_draw - lo)
        src = np.zeros(k, dtype=np.uint32)
        dst = np.zeros(k, dtype=np.uint32)
        for level in range(scale):
            bit = np.uint32(1 << (scale - 1 - level))
            r = rng.integers(0, 2**32, size=k, dtype=np.uint32)
            src_bit = r >= t_ab                                # quadrants c, d
            dst_bit = ((r >= t_a) & (r < t_ab)) | (r >= t_abc)  # quadrants b, d
            src |= src_bit.astype(np.uint32) * bit
            dst |= dst_bit.astype(np.uint32) * bit
        keep = src != dst
        keys.append((src[keep].astype(np.uint64) << np.uint64(32)) | dst[keep].astype(np.uint64))
    key = np.unique(np.concatenate(keys))
    del keys
    out_src = (key >> np.uint64(32)).astype(np.uint32)
    out_dst = (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)
    return out_src, out_dst


def lfr_graph(n: int, average_degree: float, seed: int, tau1: float = 3.0, tau2: float = 1.5,
              mu: float = 0.1, min_community: int = 20, max_community: int = 1000) -> tuple[np.ndarray, np.ndarray]:
    """LFR benchmark graph (Lancichinetti, Fortunato, Radicchi 2008) as drawn by
    NetworkX's ``LFR_benchmark_graph``: power-law degrees (exponent ``tau1``)
    and community sizes (``tau2``), mixing ``mu``.  The graph is undirected;
    every edge {u, v} becomes the two directed edges u->v and v->u, so each
    vertex's out-degree is its LFR degree.  Sorted by (src, dst).  Not every
    seed converges (NetworkX raises ExceededMaxIterations); seeds 2, 3 and 4
    do for n = 10,000 at average degrees 4, 11 and 16."""
    from networkx.generators.community import LFR_benchmark_graph
    g = LFR_benchmark_graph(n, tau1, tau2, mu, average_degree=average_degree, min_community=min_community,
                            max_community=max_community, seed=seed, max_iters=1000)
    e = np.array(list(g.edges()), dtype=np.uint64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    key = np.unique(np.concatenate([(e[:, 0] << np.uint64(32)) | e[:, 1], (e[:, 1] << np.uint64(32)) | e[:, 0]]))
    return (key >> np.uint64(32)).astype(np.uint32), (key & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def uniform_prob(m: int, p: float) -> np.ndarray:
    """fp32 probability ``p`` on each of ``m`` edges."""
    return np.full(m, np.float32(p), dtype=np.float32)


def wc_prob(n: int, dst: np.ndarray) -> np.ndarray:
    """Weighted-cascade probabilities p(u->v) = 1/indeg(v), computed in fp32."""
    indeg = np.bincount(dst, minlength=n).astype(np.float32)
    return (np.float32(1.0) / indeg[dst]).astype(np.float32)


def edges_sha256(n: int, src: np.ndarray, dst: np.ndarray, prob: np.ndarray) -> str:
    """Digest of an input graph, recorded beside results."""
    h = hashlib.sha256()
    h.update(np.uint64(n).tobytes())
    h.update(np.ascontiguousarray(src, dtype=np.uint32).tobytes())
    h.update(np.ascontiguousarray(dst, dtype=np.uint32).tobytes())
    h.update(np.ascontiguousarray(prob, dtype=np.float32).tobytes())
    return h.hexdigest()


def random_small_graph(n: int, m: int, seed: int, p_choices=None,
                       allow_self_loops: bool = False):
    """Tiny random graph with per-edge probabilities drawn from ``p_choices``
    (or U(0,1) in fp32 when None).  Used by property and parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs: list[tuple[int, int]] = []
    seen: set[tuple[int, int]] = set()
    limit = n * n if allow_self_loops else n * (n - 1)
    m = min(m, limit)
    while len(pairs) < m:
        u = int(rng.integers(0, n))
        v = int(rng.integers(0, n))
        if u == v and not allow_self_loops:
            continue
        if (u, v) in seen:
            continue
        seen.add((u, v))
        pairs.append((u, v))
    src = np.array([p[0] for p in pairs], dtype=np.uint32)
    dst = np.array([p[1] for p in pairs], dtype=np.uint32)
    if p_choices is None:
        prob = rng.random(m, dtype=np.float32)
    else:
        prob = np.array(p_choices, dtype=np.float32)[rng.integers(0, len(p_choices), size=m)]
    return src, dst, prob.astype(np.float32)
