"""CPU oracle for RRR-set sampling (test infrastructure only).

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library never links, loads or calls it,
and it imports nothing from the GPU library.

``rrr_oracle.c`` is the plain C reference (one textbook reverse BFS per
sample, Definition 2); this module loads it with ctypes, and adds the
work-accounting formulas of Section 3.1/3.2 in numpy.  ``pytwin`` is a second,
pure-Python implementation for tiny graphs.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rrr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OR_OK = 0
OR_EINVAL = -1
OR_ENOMEM = -2


def build(force: bool = True) -> str:
    """Compile the C oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = ctypes.CDLL(_LIB)
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    vp = ctypes.c_void_p
    lib.or_thr32.argtypes = [ctypes.c_float]
    lib.or_thr32.restype = u32
    lib.or_philox4x32_10.argtypes = [vp, vp, vp]
    lib.or_philox4x32_10.restype = None
    lib.or_coin_word.argtypes = [u64, u64, u64]
    lib.or_coin_word.restype = u32
    lib.or_edge_live.argtypes = [u64, u64, u64, u32]
    lib.or_edge_live.restype = i32
    lib.or_start_vertex.argtypes = [u64, u64, u32]
    lib.or_start_vertex.restype = u32
    lib.or_graph_build.argtypes = [u32, u64, vp, vp, vp, ctypes.POINTER(i32)]
    lib.or_graph_build.restype = vp
    lib.or_graph_free.argtypes = [vp]
    lib.or_graph_free.restype = None
    lib.or_graph_n.argtypes = [vp]
    lib.or_graph_n.restype = u32
    lib.or_graph_m.argtypes = [vp]
    lib.or_graph_m.restype = u64
    lib.or_graph_export.argtypes = [vp, vp, vp, vp]
    lib.or_graph_export.restype = None
    lib.or_sample_ids.argtypes = [vp, u64, vp, u64, i32, ctypes.POINTER(i32)]
    lib.or_sample_ids.restype = vp
    lib.or_result_free.argtypes = [vp]
    lib.or_result_free.restype = None
    lib.or_result_count.argtypes = [vp]
    lib.or_result_count.restype = u64
    lib.or_result_total.argtypes = [vp]
    lib.or_result_total.restype = u64
    lib.or_result_export.argtypes = [vp, vp, vp, vp, vp]
    lib.or_result_export.restype = None
    lib.or_quad_accounting.argtypes = [vp, u64, vp, vp, vp, i32, vp, vp, vp]
    lib.or_quad_accounting.restype = None
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def thr32(p: float) -> int:
    """Threshold of an fp32 probability (0xFFFFFFFF = always live)."""
    return int(_load().or_thr32(float(np.float32(p))))


def philox4x32_10(ctr, key) -> tuple[int, int, int, int]:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return tuple(int(x) for x in out)


def coin_word(seed: int, s: int, e: int) -> int:
    return int(_load().or_coin_word(seed, s, e))


def edge_live(seed: int, s: int, e: int, thr: int) -> bool:
    return bool(_load().or_edge_live(seed, s, e, thr))


def start_vertex(seed: int, s: int, n: int) -> int:
    return int(_load().or_start_vertex(seed, s, n))


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


@dataclass
class RRRSets:
    """Sampled sets in CSR form plus per-member BFS distance and per-sample TE."""
    sample_ids: np.ndarray   # uint64[count]
    offsets: np.ndarray      # uint64[count+1]
    members: np.ndarray      # uint32[total], ascending within each set
    dist: np.ndarray         # int32[total]
    te: np.ndarray           # uint64[count], sum of member in-degrees

    def set_of(self, i: int) -> np.ndarray:
        return self.members[self.offsets[i]:self.offsets[i + 1]]

    def __len__(self) -> int:
        return len(self.sample_ids)


class Graph:
    """Oracle-side graph: canonical incoming adjacency built from an edge list."""

    def __init__(self, n: int, src, dst, prob):
        lib = _load()
        self._src = np.ascontiguousarray(src, dtype=np.uint32)
        self._dst = np.ascontiguousarray(dst, dtype=np.uint32)
        self._prob = np.ascontiguousarray(prob, dtype=np.float32)
        m = len(self._src)
        if len(self._dst) != m or len(self._prob) != m:
            raise ValueError("src, dst and prob must have equal length")
        st = ctypes.c_int(0)
        h = lib.or_graph_build(n, m, _ptr(self._src) if m else None, _ptr(self._dst) if m else None,
                               _ptr(self._prob) if m else None, ctypes.byref(st))
        if not h:
            raise OracleError(st.value)
        self._h = h
        self.n = int(n)
        self.m = int(m)
        self._adj = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().or_graph_free(h)
            self._h = None

    def incoming(self):
        """(in_begin uint64[n+1], in_src uint32[m], in_thr uint32[m]) in canonical order."""
        if self._adj is None:
            b = np.zeros(self.n + 1, dtype=np.uint64)
            s = np.zeros(max(self.m, 1), dtype=np.uint32)
            t = np.zeros(max(self.m, 1), dtype=np.uint32)
            _load().or_graph_export(self._h, _ptr(b), _ptr(s), _ptr(t))
            self._adj = (b, s[: self.m], t[: self.m])
        return self._adj

    def indegree(self) -> np.ndarray:
        b = self.incoming()[0]
        return (b[1:] - b[:-1]).astype(np.uint64)

    def sample_ids(self, seed: int, ids, nthreads: int = 1) -> RRRSets:
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        lib = _load()
        st = ctypes.c_int(0)
        r = lib.or_sample_ids(self._h, seed, _ptr(ids) if len(ids) else None, len(ids),
                              int(nthreads), ctypes.byref(st))
        if not r:
            raise OracleError(st.value)
        try:
            count = int(lib.or_result_count(r))
            total = int(lib.or_result_total(r))
            offsets = np.zeros(count + 1, dtype=np.uint64)
            members = np.zeros(max(total, 1), dtype=np.uint32)
            dist = np.zeros(max(total, 1), dtype=np.int32)
            te = np.zeros(max(count, 1), dtype=np.uint64)
            lib.or_result_export(r, _ptr(offsets), _ptr(members), _ptr(dist), _ptr(te))
        finally:
            lib.or_result_free(r)
        return RRRSets(ids, offsets, members[:total], dist[:total], te[:count])

    def sample(self, seed: int, n_samples: int, first_sample: int = 0,
               nthreads: int = 1) -> RRRSets:
        ids = np.arange(first_sample, first_sample + n_samples, dtype=np.uint64)
        return self.sample_ids(seed, ids, nthreads)


def _batch_pairs(sets: RRRSets, idx: np.ndarray) -> np.ndarray:
    """Distinct (vertex, BFS level) pairs reached by the samples ``idx`` of ``sets``."""
    lo, hi = sets.offsets[idx].astype(np.int64), sets.offsets[idx + 1].astype(np.int64)
    pos = np.concatenate([np.arange(a, b) for a, b in zip(lo.tolist(), hi.tolist())]) if len(idx) else \
        np.zeros(0, dtype=np.int64)
    v = sets.members[pos].astype(np.uint64)
    d = sets.dist[pos].astype(np.uint64)
    return np.unique((v << np.uint64(32)) | d)


def fused_edge_accesses(graph: Graph, sets: RRRSets, colors: int, order: np.ndarray | None = None) -> int:
    """Edge accesses of a level-synchronous fused traversal (Section 3.2).

    Samples are grouped into batches of ``colors`` consecutive entries of
    ``sets`` (which must hold consecutive sample ids starting at a batch
    boundary), or, when ``order`` is given, of ``order`` (positions in
    ``sets``; batch b is order[b*colors : (b+1)*colors]).  Within a batch, a
    vertex v is expanded once per distinct BFS level at which any colour of
    the batch reaches it, and each expansion examines all indeg(v) incoming
    edges.  With colors == 1 this equals the total TE of unfused traversals
    (Theorem 1 holds with equality).
    """
    indeg = graph.indegree()
    total = 0
    count = len(sets)
    if order is not None:
        order = np.asarray(order, dtype=np.int64)
        for b0 in range(0, count, colors):
            pairs = _batch_pairs(sets, order[b0:b0 + colors])
            total += int(indeg[(pairs >> np.uint64(32)).astype(np.int64)].sum())
        return total
    for b0 in range(0, count, colors):
        b1 = min(count, b0 + colors)
        lo, hi = int(sets.offsets[b0]), int(sets.offsets[b1])
        v = sets.members[lo:hi].astype(np.uint64)
        d = sets.dist[lo:hi].astype(np.uint64)
        pairs = np.unique((v << np.uint64(32)) | d)
        verts = (pairs >> np.uint64(32)).astype(np.int64)
        total += int(indeg[verts].sum())
    return total


def _rows_one_threshold(graph: Graph) -> bool:
    """True when every in-edge of a vertex has the same threshold (a uniform
    probability, or one that depends only on the destination as in weighted
    cascade): then one stored threshold per row tells whether any of its
    coins can be live."""
    b, _, thr = graph.incoming()
    if graph.m < 2:
        return True
    row = np.repeat(np.arange(graph.n, dtype=np.int64), np.diff(b).astype(np.int64))
    return bool(np.all((thr[1:] == thr[:-1]) | (row[1:] != row[:-1])))


def coin_blocks(graph: Graph, sets: RRRSets) -> tuple[np.ndarray, np.ndarray]:
    """Per-set Philox block counts under the keyed coin layout: coin (s, e)
    is word e & 3 of one block keyed on (e >> 2, s), so a block serves the
    four edges of a "quad" 4q .. 4q+3 of one sample.

    Returns (all, listing), uint64 per set:
      all      quads met by the rows of the set's members: the blocks a
               traversal evaluates when it draws the coins of every in-edge of
               each expanded (vertex, sample) before looking at the source
               (rows that can never be live are skipped when each row has one
               threshold, and rows without in-edges have no quad);
      listing  of those, the quads holding an edge u -> v whose source u is
               not in the set at a depth <= depth(v): the only coins Listing 1
               can need, since it masks each edge's colours with
               ~visited[u] and such a source is visited before v's level is
               expanded.
    """
    count = len(sets)
    all_ = np.zeros(max(count, 1), dtype=np.uint64)
    listing = np.zeros(max(count, 1), dtype=np.uint64)
    if count:
        dist = np.full(graph.n, -1, dtype=np.int32)
        members = np.ascontiguousarray(sets.members, dtype=np.uint32)
        mdist = np.ascontiguousarray(sets.dist, dtype=np.int32)
        offsets = np.ascontiguousarray(sets.offsets, dtype=np.uint64)
        _load().or_quad_accounting(graph._h, count, _ptr(offsets), _ptr(members) if len(members) else None,
                                   _ptr(mdist) if len(mdist) else None, int(_rows_one_threshold(graph)),
                                   _ptr(dist), _ptr(all_), _ptr(listing))
    return all_[:count], listing[:count]


def philox_blocks(graph: Graph, sets: RRRSets) -> int:
    """Total Philox blocks of a flip-before-gather traversal of ``sets`` (the
    ``all`` column of :func:`coin_blocks`).  Fusing does not change it: every
    (member, sample) pair draws its own coins."""
    return int(coin_blocks(graph, sets)[0].sum())


def listing_blocks(graph: Graph, sets: RRRSets) -> int:
    """Total Philox blocks Listing 1's visited mask leaves needed (the
    ``listing`` column of :func:`coin_blocks`)."""
    return int(coin_blocks(graph, sets)[1].sum())


def sorted_start_order(sets: RRRSets, rank: np.ndarray | None = None) -> np.ndarray:
    """Positions of ``sets`` ordered by start vertex (the member at BFS level
    0), or by ``rank[start]`` when a vertex ranking is given; ties keep
    sample order (Section 5: batches of traversals with nearby starts)."""
    starts = sets.members[sets.dist == 0].astype(np.int64)
    assert len(starts) == len(sets)
    key = starts if rank is None else np.asarray(rank, dtype=np.int64)[starts]
    return np.argsort(key, kind="stable")


def fused_frontier_entries(sets: RRRSets, colors: int, order: np.ndarray | None = None) -> int:
    """Number of (batch, level, vertex) frontier entries of the same traversal."""
    if order is not None:
        order = np.asarray(order, dtype=np.int64)
        return sum(len(_batch_pairs(sets, order[b0:b0 + colors])) for b0 in range(0, len(sets), colors))
    total = 0
    count = len(sets)
    for b0 in range(0, count, colors):
        b1 = min(count, b0 + colors)
        lo, hi = int(sets.offsets[b0]), int(sets.offsets[b1])
        v = sets.members[lo:hi].astype(np.uint64)
        d = sets.dist[lo:hi].astype(np.uint64)
        total += len(np.unique((v << np.uint64(32)) | d))
    return total


def greedy_max_cover(offsets: np.ndarray, members: np.ndarray, n: int, k: int) -> tuple[np.ndarray, np.ndarray]:
    """Influence-maximization seed selection over RRR sets (Section 2: with
    reverse influence sampling, choosing k seeds is a maximum k-coverage over
    the sets, and the greedy choice gives a 1 - 1/e approximation).

    k greedy steps; each takes the vertex, among those not chosen yet, that
    lies in the most sets no chosen vertex covers yet (the lowest id on ties,
    also when that count is 0), then marks its sets covered.  Returns the seeds
    and, per step, the number of sets newly covered (int64).  Counts are kept
    exactly: a vertex's count drops by one for every newly covered set that
    holds it.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    members = np.asarray(members, dtype=np.int64)
    S = len(offsets) - 1
    set_of = np.repeat(np.arange(S, dtype=np.int64), np.diff(offsets))
    count = np.bincount(members, minlength=n).astype(np.int64)
    by_vertex = np.argsort(members, kind="stable")   # positions of each vertex's memberships
    vstart = np.searchsorted(members[by_vertex], np.arange(n + 1))
    covered = np.zeros(S, dtype=bool)
    chosen = np.zeros(n, dtype=bool)
    seeds = np.zeros(k, dtype=np.int64)
    gains = np.zeros(k, dtype=np.int64)
    for step in range(k):
        cand = np.where(chosen, -1, count)
        v = int(np.argmax(cand))                      # first maximum: the lowest id
        seeds[step], gains[step] = v, count[v]
        chosen[v] = True
        sets_v = set_of[by_vertex[vstart[v]:vstart[v + 1]]]
        new = sets_v[~covered[sets_v]]
        covered[new] = True
        if len(new):
            lo, hi = offsets[new], offsets[new + 1]
            idx = np.concatenate([np.arange(a, b) for a, b in zip(lo.tolist(), hi.tolist())])
            count -= np.bincount(members[idx], minlength=n)
    return seeds, gains
