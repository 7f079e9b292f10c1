"""Host-side logic without a GPU: the seeded input generators are
deterministic and well formed, the benchmark's instance draw respects its
stated bounds, and bench.py refuses more than one GPU."""

import os
import subprocess
import sys

import numpy as np

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _well_formed(n, src, dst):
    assert src.dtype == np.uint32 and dst.dtype == np.uint32
    assert len(src) == len(dst) and np.all(src < n) and np.all(dst < n)
    assert np.all(src != dst)
    key = (src.astype(np.uint64) << np.uint64(32)) | dst
    assert len(np.unique(key)) == len(key)


def test_generators_deterministic_and_well_formed():
    a = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=3)
    b = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=3)
    c = graphgen.rmat_graph(12, 8, 0.57, 0.19, 0.19, seed=4)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not (len(a[0]) == len(c[0]) and np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1]))
    _well_formed(1 << 12, *a)
    e = graphgen.er_graph(500, 4000, seed=1)
    assert len(e[0]) == 4000
    _well_formed(500, *e)


def test_lfr_graph_symmetric_and_deterministic():
    s1, d1 = graphgen.lfr_graph(10_000, 4, 2)
    s2, d2 = graphgen.lfr_graph(10_000, 4, 2)
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    _well_formed(10_000, s1, d1)
    fwd = set(zip(s1.tolist(), d1.tolist()))
    assert all((v, u) in fwd for u, v in fwd)          # every edge in both directions
    assert 3.0 < len(s1) / 10_000 < 6.0                 # mean out-degree near the requested 4


def test_probabilities():
    _, dst = graphgen.rmat_graph(10, 8, 0.57, 0.19, 0.19, seed=1)
    p = graphgen.wc_prob(1 << 10, dst)
    indeg = np.bincount(dst, minlength=1 << 10)
    assert p.dtype == np.float32 and np.allclose(p, (1.0 / indeg[dst]).astype(np.float32))
    assert np.all(graphgen.uniform_prob(7, 0.25) == np.float32(0.25))


def test_mix_draw_within_bounds():
    sys.path.insert(0, ROOT)
    import bench
    w = bench.WORKLOADS["rmat-mix32"]
    a, b = bench.mix_instances(w), bench.mix_instances(w)
    assert a == b and len(a) == w["instances"]
    for k in a:
        assert w["scale_lo"] <= k["scale"] <= w["scale_hi"] and k["ef"] in w["efs"] and k["prob"] in w["probs"]
        assert w["samples_lo"] <= k["samples"] <= w["samples_hi"]


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
