"""Pins of the oracle's random-number layer against sources that are not the oracle.

* Philox4x32-10 block function: compared with PyTorch ATen's and rocRAND's
  engines (both *called*, host builds), and with the pure-Python twin.
* Coin word and start-vertex layouts: recomputed from those external Philox
  blocks.
* Threshold rule: exact rational arithmetic on the fp32 value.
"""

import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import pytwin

HERE = os.path.dirname(os.path.abspath(__file__))
TORCH_INC = None


def _torch_include():
    import torch.utils.cpp_extension as ext
    return ext.include_paths()[0]


@pytest.fixture(scope="module")
def ref_programs(tmp_path_factory):
    d = tmp_path_factory.mktemp("philox_ref")
    progs = {}
    aten = d / "aten_philox"
    subprocess.check_call(["g++", "-O1", "-std=c++17", f"-I{_torch_include()}",
                           os.path.join(HERE, "philox_ref", "aten_philox.cpp"), "-o", str(aten)])
    progs["aten"] = str(aten)
    if shutil.which("hipcc"):
        roc = d / "rocrand_philox"
        subprocess.check_call(["hipcc", "-O1", "-std=c++17",
                               os.path.join(HERE, "philox_ref", "rocrand_philox.cpp"), "-o", str(roc)])
        progs["rocrand"] = str(roc)
    return progs


def _run(prog, rows):
    text = "\n".join(" ".join(str(int(x)) for x in r) for r in rows) + "\n"
    out = subprocess.run([prog], input=text, capture_output=True, text=True, check=True).stdout
    return [tuple(int(x) for x in line.split()) for line in out.strip().splitlines()]


def _cases():
    rng = np.random.Generator(np.random.PCG64(2311))
    rows = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 0, 0, 0, 0, 0), (0, 0, 0, 1, 0, 0),
            (0, 0, 0, 0, 0, 1), (0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0)]
    for _ in range(300):
        rows.append(tuple(int(x) for x in rng.integers(0, 2**32, size=6, dtype=np.uint64)))
    return rows


def test_philox_block_matches_aten_rocrand_and_twin(ref_programs):
    rows = _cases()
    ours = [oracle.philox4x32_10(r[:4], r[4:]) for r in rows]
    twin = [pytwin.philox4x32_10(r[:4], r[4:]) for r in rows]
    assert ours == twin
    aten = _run(ref_programs["aten"], rows)
    assert ours == aten
    if "rocrand" in ref_programs:
        assert ours == _run(ref_programs["rocrand"], rows)


def test_coin_and_start_layout_from_external_blocks(ref_programs):
    """coin(s,e) = word e&3 of block (e>>2, s lo, s hi, 0); start(s) = word s&3 of
    block ((s>>2) lo, s>>34, 0, 1) scaled by n with a 64-bit multiply-shift."""
    rng = np.random.Generator(np.random.PCG64(7))
    seeds = [0, 42, 2**32 + 17, 2**64 - 1]
    rows, expect_coin = [], []
    for seed in seeds:
        for _ in range(40):
            s = int(rng.integers(0, 2**40))
            e = int(rng.integers(0, 2**34))
            rows.append((e >> 2, s & 0xFFFFFFFF, s >> 32, 0, seed & 0xFFFFFFFF, seed >> 32))
            expect_coin.append((seed, s, e))
    blocks = _run(ref_programs["aten"], rows)
    for (seed, s, e), blk in zip(expect_coin, blocks):
        assert oracle.coin_word(seed, s, e) == blk[e & 3]
        assert pytwin.coin_word(seed, s, e) == blk[e & 3]
    rows, expect_start = [], []
    for seed in seeds:
        for _ in range(40):
            s = int(rng.integers(0, 2**36))
            n = int(rng.integers(1, 2**32))
            rows.append(((s >> 2) & 0xFFFFFFFF, s >> 34, 0, 1, seed & 0xFFFFFFFF, seed >> 32))
            expect_start.append((seed, s, n))
    blocks = _run(ref_programs["aten"], rows)
    for (seed, s, n), blk in zip(expect_start, blocks):
        want = (blk[s & 3] * n) >> 32
        assert oracle.start_vertex(seed, s, n) == want
        assert pytwin.start_vertex(seed, s, n) == want
        assert 0 <= want < n


def test_high_sample_word_is_used():
    # samples that differ only above bit 31 must draw different coins
    diffs = sum(oracle.coin_word(42, s, 1000) != oracle.coin_word(42, s + 2**32, 1000)
                for s in range(64))
    assert diffs >= 60


WORKED = {  # fp32 probability -> threshold, from floor(p * 2^32) in exact arithmetic
    0.01: 0x028F5C28, 0.05: 0x0CCCCCD0, 0.1: 0x199999A0, 0.5: 0x80000000,
    1.0 / 3.0: 0x55555580, 1.0 / 7.0: 0x24924940, 1.0 / 16.0: 0x10000000,
    1.0: 0xFFFFFFFF, 0.0: 0,
}


def _exact_thr(p32):
    p = Fraction(float(np.float32(p32)))
    if p >= 1:
        return 0xFFFFFFFF
    return int(p * 2**32)  # floor for non-negative rationals


def test_thr32_worked_values():
    for p, t in WORKED.items():
        assert oracle.thr32(p) == t, p
        assert pytwin.thr32(p) == t, p
        assert _exact_thr(p) == t, p
    largest_below_one = float(np.nextafter(np.float32(1.0), np.float32(0.0)))
    assert oracle.thr32(largest_below_one) == 0xFFFFFF00


def test_thr32_exact_rational_and_probability():
    """floor(p 2^32) for random fp32 p; and P(r < thr) = thr / 2^32 equals p
    exactly whenever p >= 2^-9 (so the coin keeps an edge with probability p)."""
    rng = np.random.Generator(np.random.PCG64(99))
    ps = np.concatenate([rng.random(2000, dtype=np.float32),
                         (rng.random(500, dtype=np.float32) * np.float32(2**-9)),
                         np.array([2**-9, 2**-24, 2**-149], dtype=np.float32)])
    for p in ps.tolist():
        t = oracle.thr32(p)
        assert t == _exact_thr(p) == pytwin.thr32(p)
        if p >= 2**-9:
            assert Fraction(t, 2**32) == Fraction(float(np.float32(p)))
        else:
            assert Fraction(t, 2**32) <= Fraction(float(np.float32(p))) < Fraction(t + 1, 2**32)


def test_coin_frequency_matches_threshold():
    """Empirical keep-rate over many (s, e) pairs is within 5 sigma of thr/2^32."""
    seed = 5
    thr = oracle.thr32(0.3)
    N = 200_000
    rng = np.random.Generator(np.random.PCG64(3))
    ss = rng.integers(0, 2**33, size=N)
    es = rng.integers(0, 2**32, size=N)
    kept = sum(oracle.edge_live(seed, int(s), int(e), thr) for s, e in zip(ss, es))
    p = thr / 2**32
    assert abs(kept - N * p) < 5 * (N * p * (1 - p)) ** 0.5
    assert oracle.edge_live(seed, 1, 2, 0xFFFFFFFF)
    assert not any(oracle.edge_live(seed, s, 7, 0) for s in range(1000))


def test_start_vertices_uniform():
    n = 13
    N = 130_000
    counts = np.bincount([oracle.start_vertex(42, s, n) for s in range(N)], minlength=n)
    from scipy.stats import chisquare
    assert chisquare(counts).pvalue > 1e-6
