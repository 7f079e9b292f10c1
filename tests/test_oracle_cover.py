"""Pins of the oracle's greedy maximum coverage (the influence-maximization
query over RRR sets, Section 2): against a from-scratch recount of the greedy
choice, the 1 - 1/e guarantee against brute-force optima, submodularity of the
gains, and RRR sets of a real sampling run."""

import itertools
import math

import numpy as np
import pytest

import graphgen
import oracle


def random_sets(n, S, max_size, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    sets = [np.unique(rng.integers(0, n, int(rng.integers(1, max_size + 1)))) for _ in range(S)]
    offsets = np.zeros(S + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(x) for x in sets])
    return offsets, np.concatenate(sets).astype(np.int64), sets


def recount_greedy(sets, n, k):
    """The greedy choice written out: every step recounts, for every vertex
    not chosen yet, the uncovered sets that hold it."""
    covered = [False] * len(sets)
    chosen, gains = [], []
    for _ in range(k):
        best, best_c = None, -1
        for v in range(n):
            if v in chosen:
                continue
            c = sum(1 for i, s in enumerate(sets) if not covered[i] and v in s)
            if c > best_c:
                best, best_c = v, c
        chosen.append(best)
        gains.append(best_c)
        for i, s in enumerate(sets):
            if best in s:
                covered[i] = True
    return chosen, gains


@pytest.mark.parametrize("seed", range(6))
def test_greedy_matches_recount(seed):
    n, S, k = 30, 80, 8
    offsets, members, sets = random_sets(n, S, 6, seed)
    seeds, gains = oracle.greedy_max_cover(offsets, members, n, k)
    want_seeds, want_gains = recount_greedy([set(x.tolist()) for x in sets], n, k)
    assert seeds.tolist() == want_seeds and gains.tolist() == want_gains


def test_ties_and_exhaustion():
    # vertices 3 and 1 each cover two sets: the lowest id wins; once every set
    # is covered the remaining seeds are the lowest unchosen ids with gain 0
    offsets = np.array([0, 2, 4, 5])
    members = np.array([1, 3, 1, 3, 4])
    seeds, gains = oracle.greedy_max_cover(offsets, members, 6, 4)
    assert seeds.tolist() == [1, 4, 0, 2] and gains.tolist() == [2, 1, 0, 0]


@pytest.mark.parametrize("seed", range(5))
def test_one_minus_one_over_e(seed):
    n, S = 9, 40
    offsets, members, sets = random_sets(n, S, 4, 100 + seed)
    sets = [set(x.tolist()) for x in sets]
    for k in (1, 2, 3):
        _, gains = oracle.greedy_max_cover(offsets, members, n, k)
        opt = max(sum(1 for s in sets if s & set(c)) for c in itertools.combinations(range(n), k))
        assert gains.sum() >= (1 - 1 / math.e) * opt - 1e-9
        if k == 1:
            assert gains.sum() == opt  # one greedy step is optimal


def test_gains_non_increasing_on_rrr_sets():
    n = 1000
    src, dst = graphgen.er_graph(n, 10_000, seed=42)
    ref = oracle.Graph(n, src, dst, graphgen.uniform_prob(len(src), 0.1)).sample(42, 2000, nthreads=4)
    seeds, gains = oracle.greedy_max_cover(ref.offsets, ref.members, n, 50)
    assert np.all(np.diff(gains) <= 0)                 # submodular: marginal gains never grow
    assert len(set(seeds.tolist())) == 50
    # the first seed is the vertex in the most sets
    assert gains[0] == np.bincount(ref.members.astype(np.int64), minlength=n).max()
    # coverage of the seed set, recounted directly
    sset = set(seeds.tolist())
    covered = sum(1 for i in range(len(ref)) if sset & set(ref.set_of(i).tolist()))
    assert covered == gains.sum()
