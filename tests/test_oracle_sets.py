"""Pins of the oracle's RRR sets against what Definition 2 and the IC model fix.

Each check is independent of the oracle's own BFS:
  * p = 1: the set is the exact reverse-reachable set (scipy / networkx).
  * p = 0: the set is the start alone.
  * Exact enumeration over all 2^m live-edge worlds on graphs with m <= 10
    edges: per-vertex inclusion probabilities (5 sigma, Bonferroni) and the
    whole-set distribution (chi-square) given the start.
  * Closed forms: in-star (E|R| = 1 + k p) and path (P = p^d).
  * RIS identity sigma({u}) = n P(u in R), with sigma from a forward IC
    simulation, which pins the edge direction.
  * Certificate: closure under live in-edges and reachability inside the set.
  * Canonical edge ids: input order does not change the result.
  * Theorem 1: fused edge accesses <= unfused, equal at one colour.
"""

import itertools
import random
from collections import Counter, deque

import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import breadth_first_order
from scipy.stats import chisquare

import graphgen
import oracle
from oracle import pytwin


def _sets(g, seed, n_samples, threads=4):
    return g.sample(seed, n_samples, nthreads=threads)


def test_p1_is_exact_reverse_reachability():
    for gseed in range(6):
        n = 60
        src, dst, _ = graphgen.random_small_graph(n, 150, gseed)
        prob = np.ones(len(src), dtype=np.float32)
        g = oracle.Graph(n, src, dst, prob)
        res = _sets(g, seed=gseed, n_samples=100)
        # transpose adjacency: row v lists u for every edge u -> v
        A_T = sp.csr_matrix((np.ones(len(src)), (dst, src)), shape=(n, n))
        G = nx.DiGraph()
        G.add_nodes_from(range(n))
        G.add_edges_from(zip(src.tolist(), dst.tolist()))
        for i in range(len(res)):
            start = oracle.start_vertex(gseed, i, n)
            want = np.sort(breadth_first_order(A_T, start, directed=True, return_predecessors=False))
            got = res.set_of(i)
            assert np.array_equal(got, want)
            assert set(got.tolist()) == nx.ancestors(G, start) | {start}


def test_p0_gives_singletons():
    src, dst = graphgen.rmat_graph(10, 8, 0.57, 0.19, 0.19, seed=3)
    n = 1 << 10
    g = oracle.Graph(n, src, dst, graphgen.uniform_prob(len(src), 0.0))
    res = _sets(g, 11, 500)
    for i in range(len(res)):
        assert res.set_of(i).tolist() == [oracle.start_vertex(11, i, n)]
        assert res.dist[res.offsets[i]] == 0


def _reach_back(n, live_edges, v):
    """Vertices with a path to v using the given (u -> w) edges."""
    back = [[] for _ in range(n)]
    for u, w in live_edges:
        back[w].append(u)
    seen = {v}
    todo = [v]
    while todo:
        x = todo.pop()
        for u in back[x]:
            if u not in seen:
                seen.add(u)
                todo.append(u)
    return frozenset(seen)


def _enumerate(n, src, dst, prob):
    """Exact distribution of the RRR set given each start, over all 2^m worlds."""
    m = len(src)
    p = [float(np.float32(x)) for x in prob]
    dist = {v: Counter() for v in range(n)}
    for world in itertools.product((0, 1), repeat=m):
        w = 1.0
        live = []
        for k in range(m):
            if world[k]:
                w *= p[k]
                live.append((int(src[k]), int(dst[k])))
            else:
                w *= 1.0 - p[k]
        if w == 0.0:
            continue
        for v in range(n):
            dist[v][_reach_back(n, live, v)] += w
    return dist


@pytest.mark.parametrize("gseed", [0, 1, 2])
def test_exact_enumeration_small_graphs(gseed):
    n, m = 5, 9
    src, dst, prob = graphgen.random_small_graph(n, m, 100 + gseed,
                                                 p_choices=[0.2, 0.5, 0.7, 0.9, 1.0],
                                                 allow_self_loops=(gseed == 2))
    exact = _enumerate(n, src, dst, prob)
    g = oracle.Graph(n, src, dst, prob)
    N = 150_000
    seed = 1000 + gseed
    res = _sets(g, seed, N)
    starts = np.array([oracle.start_vertex(seed, s, n) for s in range(N)])
    observed = {v: Counter() for v in range(n)}
    for i in range(N):
        observed[int(starts[i])][frozenset(res.set_of(i).tolist())] += 1
    n_tests = n * n
    z = 5.0 + np.log(n_tests) / 4  # Bonferroni-widened 5 sigma
    for v in range(n):
        Nv = sum(observed[v].values())
        assert Nv > 20_000
        for u in range(n):
            P = min(1.0, max(0.0, sum(w for S, w in exact[v].items() if u in S)))
            f = sum(c for S, c in observed[v].items() if u in S) / Nv
            sd = max((P * (1 - P) / Nv) ** 0.5, 1e-12)
            assert abs(f - P) <= z * sd + 1e-12, (v, u, f, P)
        # whole-set distribution given the start
        support = sorted(exact[v], key=lambda S: sorted(S))
        assert set(observed[v]) <= set(support)
        exp = np.array([exact[v][S] * Nv for S in support])
        obs = np.array([observed[v][S] for S in support], dtype=float)
        keep = exp >= 5
        if keep.sum() >= 2:
            e2 = np.append(exp[keep], exp[~keep].sum())
            o2 = np.append(obs[keep], obs[~keep].sum())
            if e2[-1] == 0:
                e2, o2 = e2[:-1], o2[:-1]
            e2 = e2 * o2.sum() / e2.sum()
            assert chisquare(o2, e2).pvalue > 1e-6


def test_closed_form_in_star():
    """k leaves each with one edge into the centre: given start = centre,
    |R| - 1 ~ Binomial(k, p), so E|R| = 1 + k p."""
    k, p = 12, 0.25
    n = k + 1
    src = np.arange(1, n, dtype=np.uint32)
    dst = np.zeros(k, dtype=np.uint32)
    g = oracle.Graph(n, src, dst, graphgen.uniform_prob(k, p))
    N = 120_000
    res = _sets(g, 77, N)
    sizes = np.diff(res.offsets).astype(float)
    starts = np.array([oracle.start_vertex(77, s, n) for s in range(N)])
    c = sizes[starts == 0]
    assert abs(c.mean() - (1 + k * p)) < 5 * np.sqrt(k * p * (1 - p) / len(c))
    assert np.all(sizes[starts != 0] == 1)


def test_closed_form_path():
    """Path 0 -> 1 -> ... -> L: from start L, vertex L-d is in R with prob p^d."""
    L, p = 6, 0.7
    n = L + 1
    src = np.arange(0, L, dtype=np.uint32)
    dst = np.arange(1, L + 1, dtype=np.uint32)
    g = oracle.Graph(n, src, dst, graphgen.uniform_prob(L, p))
    N = 140_000
    res = _sets(g, 5, N)
    starts = np.array([oracle.start_vertex(5, s, n) for s in range(N)])
    idx = np.nonzero(starts == L)[0]
    for d in range(1, L + 1):
        hits = sum(1 for i in idx if (L - d) in set(res.set_of(i).tolist()))
        P = p ** d
        assert abs(hits / len(idx) - P) < 5 * np.sqrt(P * (1 - P) / len(idx))
    # distances equal the path length
    for i in idx[:200]:
        members = res.set_of(i).tolist()
        dists = res.dist[res.offsets[i]:res.offsets[i + 1]].tolist()
        for u, d in zip(members, dists):
            assert d == L - u


def test_ris_identity_forward_ic():
    """sigma({u}) from forward IC cascades equals n * P(u in RRR set)."""
    n = 6
    src = np.array([0, 0, 1, 2, 3, 4, 5, 2], dtype=np.uint32)
    dst = np.array([1, 2, 3, 3, 4, 5, 0, 4], dtype=np.uint32)
    prob = np.array([0.8, 0.3, 0.6, 0.9, 0.5, 0.4, 0.2, 0.7], dtype=np.float32)
    g = oracle.Graph(n, src, dst, prob)
    N = 200_000
    res = _sets(g, 31, N)
    freq = np.bincount(res.members.astype(np.int64), minlength=n) / N
    out = [[] for _ in range(n)]
    for u, v, p in zip(src.tolist(), dst.tolist(), prob.tolist()):
        out[u].append((v, p))
    rnd = random.Random(4)
    R = 60_000
    for u in range(n):
        spread = 0
        for _ in range(R):
            active = {u}
            todo = deque([u])
            while todo:
                x = todo.popleft()
                for y, p in out[x]:
                    if y not in active and rnd.random() < p:
                        active.add(y)
                        todo.append(y)
            spread += len(active)
        sigma = spread / R
        est = n * freq[u]
        sd = n * np.sqrt(freq[u] * (1 - freq[u]) / N) + np.sqrt(n * n / 4 / R)
        assert abs(sigma - est) < 5 * sd, (u, sigma, est)


def _certificate(graph: oracle.Graph, seed, s, members):
    """(closure) every live in-edge of a member comes from a member;
    (reachability) a search from the start inside the set over live edges
    reaches every member.  Together they fix the set uniquely."""
    b, srcs, thr = graph.incoming()
    mem = set(members)
    start = pytwin.start_vertex(seed, s, graph.n)
    if start not in mem:
        return False
    for w in members:
        for e in range(int(b[w]), int(b[w + 1])):
            if pytwin.coin_word(seed, s, e) < thr[e] or thr[e] == 0xFFFFFFFF:
                if int(srcs[e]) not in mem:
                    return False
    seen = {start}
    todo = [start]
    while todo:
        w = todo.pop()
        for e in range(int(b[w]), int(b[w + 1])):
            u = int(srcs[e])
            if u in mem and u not in seen and (thr[e] == 0xFFFFFFFF or pytwin.coin_word(seed, s, e) < thr[e]):
                seen.add(u)
                todo.append(u)
    return seen == mem


def test_certificate_on_random_graphs():
    src, dst = graphgen.rmat_graph(8, 6, 0.57, 0.19, 0.19, seed=8)
    n = 256
    prob = graphgen.wc_prob(n, dst) * np.float32(1.5)
    prob = np.minimum(prob, np.float32(1.0)).astype(np.float32)
    g = oracle.Graph(n, src, dst, prob)
    res = _sets(g, 9, 120)
    assert res.offsets[-1] > 120  # not all singletons
    for i in range(len(res)):
        assert _certificate(g, 9, i, res.set_of(i).tolist())


def test_pytwin_agrees_with_c_oracle():
    for gseed in range(5):
        n = 40
        src, dst, prob = graphgen.random_small_graph(n, 160, 500 + gseed)
        g = oracle.Graph(n, src, dst, prob)
        tg = pytwin.TinyGraph(n, src, dst, prob)
        res = g.sample(gseed, 64, first_sample=2**32 - 20)
        for i, s in enumerate(res.sample_ids.tolist()):
            members, depth = tg.rrr(gseed, s)
            assert res.set_of(i).tolist() == members
            assert res.dist[res.offsets[i]:res.offsets[i + 1]].tolist() == [depth[u] for u in members]
            indeg = g.indegree()
            assert res.te[i] == sum(int(indeg[u]) for u in members)


def test_input_order_does_not_matter():
    src, dst = graphgen.rmat_graph(9, 8, 0.57, 0.19, 0.19, seed=12)
    n = 512
    prob = graphgen.wc_prob(n, dst)
    a = oracle.Graph(n, src, dst, prob).sample(3, 300)
    perm = np.random.Generator(np.random.PCG64(1)).permutation(len(src))
    b = oracle.Graph(n, src[perm], dst[perm], prob[perm]).sample(3, 300)
    assert np.array_equal(a.offsets, b.offsets)
    assert np.array_equal(a.members, b.members)
    assert np.array_equal(a.dist, b.dist)


def test_theorem1_fused_accesses_bounded_by_unfused():
    src, dst = graphgen.rmat_graph(10, 16, 0.57, 0.19, 0.19, seed=21)
    n = 1024
    g = oracle.Graph(n, src, dst, graphgen.uniform_prob(len(src), 0.08))
    res = g.sample(4, 1024, nthreads=4)
    te = int(res.te.sum())
    ea1 = oracle.fused_edge_accesses(g, res, 1)
    assert ea1 == te
    prev = ea1
    for c in (2, 4, 16, 64, 256, 1024):
        ea = oracle.fused_edge_accesses(g, res, c)
        assert ea <= prev  # batches of 2c are unions of batches of c
        prev = ea
    assert prev < te  # this graph is dense enough that fusing saves work
    assert oracle.fused_frontier_entries(res, 1) == int(res.offsets[-1])


def test_invalid_inputs_rejected():
    ok_src = np.array([0, 1], dtype=np.uint32)
    ok_dst = np.array([1, 2], dtype=np.uint32)
    ok_p = np.array([0.5, 0.5], dtype=np.float32)
    oracle.Graph(3, ok_src, ok_dst, ok_p)
    bad = [
        (3, np.array([0, 0], np.uint32), np.array([1, 1], np.uint32), ok_p),        # repeated edge
        (3, ok_src, np.array([1, 3], np.uint32), ok_p),                             # vertex out of range
        (3, ok_src, ok_dst, np.array([0.5, np.nan], np.float32)),                   # NaN
        (3, ok_src, ok_dst, np.array([0.5, 1.5], np.float32)),                      # > 1
        (3, ok_src, ok_dst, np.array([-0.1, 0.5], np.float32)),                     # < 0
        (0, np.array([], np.uint32), np.array([], np.uint32), np.array([], np.float32)),  # n = 0
    ]
    for n, s, d, p in bad:
        with pytest.raises(oracle.OracleError) as ei:
            oracle.Graph(n, s, d, p)
        assert ei.value.status == oracle.OR_EINVAL


def test_empty_graph_and_zero_samples():
    g = oracle.Graph(5, np.array([], np.uint32), np.array([], np.uint32), np.array([], np.float32))
    res = g.sample(1, 10)
    assert np.array_equal(np.diff(res.offsets), np.ones(10, dtype=np.uint64))
    assert len(g.sample(1, 0)) == 0


def test_ordered_batches_accounting():
    """The batch-order form of the fused accounting agrees with the id-order
    form on the identity order, stays within Theorem 1 for any order, and the
    sorted-start order sorts by the level-0 member."""
    import graphgen
    n = 1000
    src, dst = graphgen.er_graph(n, 10_000, seed=42)
    og = oracle.Graph(n, src, dst, graphgen.uniform_prob(len(src), 0.1))
    ref = og.sample(3, 700, nthreads=4)
    ident = np.arange(len(ref))
    for c in (1, 8, 64):
        assert oracle.fused_edge_accesses(og, ref, c, ident) == oracle.fused_edge_accesses(og, ref, c)
        assert oracle.fused_frontier_entries(ref, c, ident) == oracle.fused_frontier_entries(ref, c)
    te = int(ref.te.sum())
    order = oracle.sorted_start_order(ref)
    starts = np.array([oracle.start_vertex(3, s, n) for s in range(len(ref))])
    assert np.array_equal(order, np.argsort(starts, kind="stable"))
    rng = np.random.Generator(np.random.PCG64(1))
    for o in (order, rng.permutation(len(ref))):
        assert oracle.fused_edge_accesses(og, ref, 1, o) == te
        assert oracle.fused_edge_accesses(og, ref, 64, o) <= te
    rank = rng.permutation(n)
    o2 = oracle.sorted_start_order(ref, rank)
    assert np.all(np.diff(rank[starts[o2]]) >= 0)
