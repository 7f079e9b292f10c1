"""Hand-worked pins of the oracle's work accounting (no GPU).

The fused accounting of Section 3.2 (a level-synchronous traversal expands a
vertex once per distinct BFS level at which any colour of its batch reaches it,
and scans all of its in-edges each time), the Philox-block count of the keyed
coin layout, the blocks Listing 1's visited mask leaves needed, and the
sorted-start batch order of Section 5 are each checked here against values
worked out by hand on graphs small enough to follow on paper.  None of the
expected numbers is computed by the code under test.

Fixture graph (edges u -> v; an RRR set walks them backwards), n = 6:

    5 -> 0,  0 -> 1,  1 -> 2,  2 -> 3,  4 -> 3,  0 -> 4

Canonical edge ids (rank of (dst, src)): e0 = 5->0, e1 = 0->1, e2 = 1->2,
e3 = 2->3, e4 = 4->3, e5 = 0->4.  In-degrees: v0 1, v1 1, v2 1, v3 2, v4 1,
v5 0.  Rows (edge ranges) and the 4-edge quads they meet: v0 [0,1) {q0};
v1 [1,2) {q0}; v2 [2,3) {q0}; v3 [3,5) {q0, q1}; v4 [5,6) {q1}; v5 empty.

With p = 1 every edge is live.  Philox seed 157 puts the starts of samples
0, 1, 2 at vertices 3, 2, 3 (checked below with the start mapping, which
test_oracle_rng pins against ATen's and rocRAND's Philox).  By hand:

    sample 0 (start 3): 3@0, 2@1, 4@1, 1@2, 0@2, 5@3        (vertex@depth)
    sample 1 (start 2): 2@0, 1@1, 0@2, 5@3
    sample 2 (start 3): as sample 0

    TE = (2+1+1+1+1+0) + (1+1+1+0) + 6 = 6 + 3 + 6 = 15

Batch {0, 1} (C = 2): distinct (vertex, depth) pairs are 3@0 2@1 4@1 1@2 0@2
5@3 from sample 0 plus 2@0 1@1 from sample 1 (0@2 and 5@3 are shared): 8
frontier entries, EA = 2+1+1+1+1+0 + 1+1 = 8.  Grouping by vertex alone would
give 6 entries and EA = 6.
"""

import numpy as np

import oracle

N6 = 6
SRC6 = np.array([5, 0, 1, 2, 4, 0], dtype=np.uint32)
DST6 = np.array([0, 1, 2, 3, 3, 4], dtype=np.uint32)
SEED = 157


def _fixture():
    g = oracle.Graph(N6, SRC6, DST6, np.ones(6, dtype=np.float32))
    return g, g.sample(SEED, 3)


def test_fixture_sets_are_the_hand_worked_ones():
    g, res = _fixture()
    assert [oracle.start_vertex(SEED, s, N6) for s in range(3)] == [3, 2, 3]
    want = [({0: 2, 1: 2, 2: 1, 3: 0, 4: 1, 5: 3}), ({0: 2, 1: 1, 2: 0, 5: 3}), ({0: 2, 1: 2, 2: 1, 3: 0, 4: 1, 5: 3})]
    for i, d in enumerate(want):
        lo, hi = int(res.offsets[i]), int(res.offsets[i + 1])
        assert res.members[lo:hi].tolist() == sorted(d)
        assert res.dist[lo:hi].tolist() == [d[v] for v in sorted(d)]
    assert res.te.tolist() == [6, 3, 6]
    b, src, _ = g.incoming()
    assert b.tolist() == [0, 1, 2, 3, 5, 6, 6]
    assert src.tolist() == [5, 0, 1, 2, 4, 0]


def test_fused_accounting_hand_worked():
    g, res = _fixture()
    # one colour per batch: every (sample, member) pair is an entry (Theorem 1 equality)
    assert oracle.fused_frontier_entries(res, 1) == 6 + 4 + 6
    assert oracle.fused_edge_accesses(g, res, 1) == 15
    # batch {0, 1} then batch {2}: 8 + 6 entries; EA 8 + 6
    assert oracle.fused_frontier_entries(res, 2) == 14
    assert oracle.fused_edge_accesses(g, res, 2) == 14
    # one batch {0, 1, 2}: sample 2 repeats sample 0's pairs exactly
    assert oracle.fused_frontier_entries(res, 4) == 8
    assert oracle.fused_edge_accesses(g, res, 4) == 8
    # the same batches through the explicit-order form
    order = np.array([0, 1, 2])
    assert oracle.fused_frontier_entries(res, 2, order) == 14
    assert oracle.fused_edge_accesses(g, res, 2, order) == 14
    # order (0, 2 | 1): samples 0 and 2 share every pair
    order = np.array([0, 2, 1])
    assert oracle.fused_frontier_entries(res, 2, order) == 6 + 4
    assert oracle.fused_edge_accesses(g, res, 2, order) == 6 + 3


def test_coin_blocks_hand_counted():
    """Quads met per member: v0 1, v1 1, v2 1, v3 2, v4 1, v5 0, so sample 0
    evaluates 6 blocks, sample 1 3 and sample 2 6.  Listing 1 needs a block
    unless every edge of it in the row comes from a source at depth <= the
    member's depth.  Sample 0: v3@0 needs q0 (e3 from 2@1) and q1 (e4 from
    4@1); v2@1 needs q0 (e2 from 1@2); v4@1 needs q1 (e5 from 0@2); v1@2 does
    not (e1 from 0@2, same depth); v0@2 needs q0 (e0 from 5@3): 5.  Sample 1:
    v2@0, v1@1, v0@2 each need their one quad: 3."""
    g, res = _fixture()
    all_, listing = oracle.coin_blocks(g, res)
    assert all_.tolist() == [6, 3, 6]
    assert listing.tolist() == [5, 3, 5]
    assert oracle.philox_blocks(g, res) == 15
    assert oracle.listing_blocks(g, res) == 13


def test_coin_blocks_rows_across_quads_and_dead_rows():
    """Rows that straddle quad boundaries, and rows whose threshold is 0.

    n = 8; in-edges of v7 from 0..6 (7 edges), of v6 from 0..4 (5), nothing
    else.  Canonical ids: v6's row is [0, 5) (quads q0, q1), v7's row is
    [5, 12) (quads q1, q2).  A set {6, 7} with both at depth 0 meets 2 + 2
    quads.  With per-destination probabilities (one threshold per row) a row
    whose probability is 0 is skipped; with one row of several thresholds
    (some non-zero) every row counts, dead or not."""
    src = np.array([0, 1, 2, 3, 4, 0, 1, 2, 3, 4, 5, 6], dtype=np.uint32)
    dst = np.array([6] * 5 + [7] * 7, dtype=np.uint32)
    sets = oracle.RRRSets(np.array([0], np.uint64), np.array([0, 2], np.uint64),
                          np.array([6, 7], np.uint32), np.array([0, 0], np.int32), np.array([12], np.uint64))
    both = np.full(12, 0.5, np.float32)
    g = oracle.Graph(8, src, dst, both)
    assert oracle.coin_blocks(g, sets)[0].tolist() == [4]
    # every quad holds a source outside the set (6 -> 7, edge 11, shares q2 with 3, 4, 5)
    assert oracle.coin_blocks(g, sets)[1].tolist() == [4]
    row_dead = np.where(dst == 6, np.float32(0.0), np.float32(0.5)).astype(np.float32)
    g = oracle.Graph(8, src, dst, row_dead)
    assert oracle.coin_blocks(g, sets)[0].tolist() == [2]
    mixed = both.copy()
    mixed[:5] = 0.0
    mixed[11] = 0.25  # v7's row now has two thresholds: per-edge storage, no row is skipped
    g = oracle.Graph(8, src, dst, mixed)
    assert oracle.coin_blocks(g, sets)[0].tolist() == [4]
    # depths decide which quads Listing 1 needs: {0..4 @1, 5 @2, 6 @0, 7 @1}.
    # v6 @0: its sources 0..4 are deeper, both quads needed.  v7 @1: q1 (edges
    # 5..7 from 0..2 @1) is not needed; q2 (edges 8..11 from 3 @1, 4 @1, 5 @2,
    # 6 @0) is, for 5 @2.  Sources 0..5 have no in-edges.
    members = np.arange(8, dtype=np.uint32)
    d = np.array([1, 1, 1, 1, 1, 2, 0, 1], np.int32)
    s2 = oracle.RRRSets(np.array([0], np.uint64), np.array([0, 8], np.uint64), members, d, np.array([12], np.uint64))
    g = oracle.Graph(8, src, dst, both)
    a, l = oracle.coin_blocks(g, s2)
    assert a.tolist() == [4] and l.tolist() == [3]


def test_sorted_start_order_literal():
    """Section 5 batches samples by start vertex, ties in sample order.  Six
    sets with starts 3, 1, 3, 0, 2, 1 (the member at depth 0; other members
    at depth 1) sort to positions 3, 1, 5, 4, 0, 2.  Under the vertex ranking
    rank = (2, 0, 3, 1) the keys are 1, 0, 1, 2, 3, 0 and the order is
    1, 5, 0, 2, 3, 4."""
    starts = [3, 1, 3, 0, 2, 1]
    others = [[0], [], [1, 2], [3], [], [0, 2]]
    members, dist, offsets = [], [], [0]
    for st, ot in zip(starts, others):
        pairs = sorted([(st, 0)] + [(v, 1) for v in ot])
        members += [v for v, _ in pairs]
        dist += [d for _, d in pairs]
        offsets.append(len(members))
    sets = oracle.RRRSets(np.arange(6, dtype=np.uint64), np.array(offsets, np.uint64),
                          np.array(members, np.uint32), np.array(dist, np.int32), np.zeros(6, np.uint64))
    assert oracle.sorted_start_order(sets).tolist() == [3, 1, 5, 4, 0, 2]
    assert oracle.sorted_start_order(sets, np.array([2, 0, 3, 1])).tolist() == [1, 5, 0, 2, 3, 4]
