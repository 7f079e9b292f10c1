#!/usr/bin/env python3
"""RRR-set sampling throughput on one MI355X: fused BPTs vs the unfused traversal.

    python bench.py [--steps K] [--warmup W] [--workload rmat22-p0.01] [--gpus 1]

One "step" samples the whole workload once (all its RRR sets) with the fused
traversal at the chosen colour count; inputs are resident in HBM and the sets
are written to device memory.  The default workload is the largest one that
fits one GPU: R-MAT scale 22, uniform p = 0.01, 1,000,000 samples.  Prints one
JSON line: samples/s (the value), traversed edges/s, the unfused and other
colour-count rates on the same GPU (timed with --variant-steps steps each),
the traversal kernel's roofline, and the CPU oracle timed on the host cores
on a fixed subset of sample ids (whose sets are also compared with the GPU's,
set by set).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("RRR samples/sec and traversed edges/sec (fused vs unfused, bit-exact); % HBM peak")

WORKLOADS = {
    # R-MAT scale 20, edge factor 16, weighted cascade, 100,000 samples
    "rmat20-wc": dict(kind="rmat", scale=20, ef=16, a=0.57, b=0.19, c=0.19, graph_seed=20, prob="wc",
                      samples=100_000, seed=42, colors=(64, 256), cpu_stride=1, listing_stride=1),
    # R-MAT scale 22, edge factor 16, uniform p = 0.01, 1,000,000 samples
    # (the CPU oracle runs on the sample ids that are multiples of 97: 10,310 sets)
    "rmat22-p0.01": dict(kind="rmat", scale=22, ef=16, a=0.57, b=0.19, c=0.19, graph_seed=22, prob=0.01,
                         samples=1_000_000, seed=42, colors=(64, 128, 256), cpu_stride=97, listing_stride=20),
    # 32 uneven R-MAT instances (scale 12-21, edge factor 8/16/32, uniform p 0.01/0.05/0.1 or weighted
    # cascade, 1k-200k samples, log-uniform), all sampled by one bpt_sample_rrr_jobs call; each
    # instance's sample count is capped so its sets hold at most 2^27 vertex ids
    "rmat-mix32": dict(kind="mix", instances=32, draw_seed=2311, scale_lo=12, scale_hi=21, efs=(8, 16, 32),
                       probs=(0.01, 0.05, 0.1, "wc"), samples_lo=1_000, samples_hi=200_000, out_budget=1 << 27,
                       check_per_instance=16),
    # serving: 8 resident weighted-cascade R-MAT graphs (scale 16-22, edge factor 16), Poisson arrivals of
    # requests for 10k-1M samples (log-uniform), a quarter of them for k = 50 influence-maximization seeds
    "serve8": dict(kind="serve", scales=(16, 17, 18, 19, 20, 20, 21, 22), ef=16, requests=2000, draw_seed=2023,
                   samples_lo=10_000, samples_hi=1_000_000, seeds_fraction=0.25, k=50, load=0.8,
                   check_every=100),
    # Erdos-Renyi n = 1,000, m = 10,000, p = 0.1, 64 samples
    "er1000-p0.1": dict(kind="er", n=1000, m=10_000, graph_seed=42, prob=0.1, samples=64, seed=42, colors=(64,),
                        cpu_stride=1, listing_stride=1),
}

# ALU roofline of one Philox4x32-10 block on gfx950: per round two
# v_mad_u64_u32 (each gives both halves of a 32x32 product) and two three-way
# xors (one v_bitop3_b32 each), all at the full vector issue rate.  In the
# first round only counter word 0 (the quad) differs between the quads of one
# sample, so that round costs one multiply and one xor per block: 2 + 9 x 4 =
# 38 for the rounds, plus ~8 compare/select for the four coins, against
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9
SLOTS_PER_BLOCK = 38 + 8
PEAK_PHILOX_BLOCKS = LANE_SLOTS_PER_S / SLOTS_PER_BLOCK

KERNEL_SOURCES = ["paper_2311_10201_amd/csrc/bpt_fused.hip", "paper_2311_10201_amd/csrc/bpt_rng.hpp",
                  "paper_2311_10201_amd/csrc/bpt_internal.hpp"]


def kernel_digest() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_graph(w):
    import graphgen
    import numpy as np
    if w["kind"] == "rmat":
        src, dst = graphgen.rmat_graph(w["scale"], w["ef"], w["a"], w["b"], w["c"], seed=w["graph_seed"])
        n = 1 << w["scale"]
    else:
        n = w["n"]
        src, dst = graphgen.er_graph(n, w["m"], seed=w["graph_seed"])
    if w["prob"] == "wc":
        prob = graphgen.wc_prob(n, dst)
    else:
        prob = graphgen.uniform_prob(len(src), w["prob"])
    return n, src, dst, prob.astype(np.float32)


def measured_traffic(workload: str, colors: int, workgroup_size: int):
    """HBM bytes per traversal launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel sources and launch shape; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    e = rec.get(f"{workload}/C{colors}")
    if not e or e.get("kernel_digest") != kernel_digest() or e.get("workgroup_size") != workgroup_size:
        return None
    return e.get("bytes_per_launch")


def fusion_study(out_path: str) -> int:
    """Work saved by fusing and colour occupancy (the paper's synthetic analysis
    of Section 3.2 with its LFR figure, and Theorem 1 of Section 3.1) measured
    on the fused kernel's own counters: LFR graphs with 10,000 vertices and average degree 4, 11, 16
    (three graph seeds each), uniform traversal probability 0.01 ... 0.5,
    10,240 random-start samples under three sample seeds, colours 8 ... 1024.

      work ratio  = EA(C) / TE: edges the fused traversal scans over the edges
                    C separate traversals scan (EA(1) = TE; Theorem 1: <= 1).
      occupancy   = members / (C * frontier entries): the mean fraction of the
                    batch's colours present in a frontier entry.
    Both counters are checked against the oracle's level-synchronous
    accounting by the GPU parity tests."""
    import numpy as np
    import torch

    import graphgen
    import paper_2311_10201_amd as bpt

    n, S = 10_000, 10_240
    degrees, graph_seeds = (4, 11, 16), (2, 3, 4)
    probs, sample_seeds, colours = (0.01, 0.1, 0.2, 0.3, 0.4, 0.5), (1, 2, 3), (8, 16, 32, 64, 128, 256, 512, 1024)
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    cap = n * S
    vert = torch.empty(cap, dtype=torch.int32, device="cuda")
    rows, tuned = [], []
    for deg in degrees:
        for gs in graph_seeds:
            src, dst = graphgen.lfr_graph(n, deg, gs)
            for p in probs:
                g = bpt.bpt_create_graph(n, src, dst, graphgen.uniform_prob(len(src), p))
                for ss in sample_seeds:
                    te = None
                    for c in colours:
                        st, total, cnt = bpt.bpt_sample_rrr_device(g, 0, S, c, ss, 0, stream, off, vert, cap)
                        assert st == bpt.BPT_OK, st
                        assert te is None or cnt.sample_edges == te  # TE does not depend on C
                        te = cnt.sample_edges
                        rows.append(dict(degree=deg, graph_seed=gs, m=len(src), p=p, seed=ss, colors=c,
                                         sample_edges=cnt.sample_edges, edge_accesses=cnt.edge_accesses,
                                         frontier_entries=cnt.frontier_entries, members=cnt.members,
                                         traversal_ms=cnt.traversal_ns / 1e6))
                tuned.append(dict(degree=deg, graph_seed=gs, p=p, colors=bpt.bpt_tune_colors(g, S, 1)))
                bpt.bpt_free(g)
            log(f"fusion study: degree {deg} graph seed {gs} done")
    with open(out_path, "w") as f:
        json.dump(dict(n=n, samples=S, rows=rows, tuned=tuned), f)

    def mean(deg, p, c, fn):
        xs = [fn(r) for r in rows if r["degree"] == deg and r["p"] == p and r["colors"] == c]
        return sum(xs) / len(xs)

    for title, fn in (("work ratio EA(C)/TE (%)", lambda r: 100 * r["edge_accesses"] / max(1, r["sample_edges"])),
                      ("colour occupancy (%)", lambda r: 100 * r["members"] / max(1, r["colors"] * r["frontier_entries"]))):
        print(f"\n{title}, mean over 3 graph seeds x 3 sample seeds\n")
        print("| degree | p | " + " | ".join(f"C={c}" for c in colours) + " |")
        print("|---|---|" + "---|" * len(colours))
        for deg in degrees:
            for p in probs:
                print(f"| {deg} | {p} | " + " | ".join(f"{mean(deg, p, c, fn):.2f}" for c in colours) + " |")
    print("\nfused traversal time (ms per launch of 10,240 samples), mean over the 9 runs; "
          "autotuner's pick (bpt_tune_colors, sample seed 1) per graph seed\n")
    print("| degree | p | " + " | ".join(f"C={c}" for c in colours) + " | fastest | tuner |")
    print("|---|---|" + "---|" * (len(colours) + 2))
    for deg in degrees:
        for p in probs:
            t = [mean(deg, p, c, lambda r: r["traversal_ms"]) for c in colours]
            fastest = colours[min(range(len(t)), key=lambda i: t[i])]
            picks = ",".join(str(x["colors"]) for x in tuned if x["degree"] == deg and x["p"] == p)
            print(f"| {deg} | {p} | " + " | ".join(f"{x:.3f}" for x in t) + f" | {fastest} | {picks} |")
    return 0


def order_study(out_path: str) -> int:
    """Batch composition (the paper's heuristics of Section 5): samples in id
    order, sorted by start vertex, and sorted by the start's rank in a reverse
    Cuthill-McKee order of the graph.  Edge accesses, colour occupancy and
    traversal time of the same sets under each."""
    import numpy as np
    import scipy.sparse as sp
    import torch
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    import graphgen
    import paper_2311_10201_amd as bpt

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cases = []
    src, dst = graphgen.rmat_graph(20, 16, 0.57, 0.19, 0.19, seed=20)
    cases.append(("R-MAT 20 WC", 1 << 20, src, dst, graphgen.wc_prob(1 << 20, dst), 100_000, 42))
    src, dst = graphgen.rmat_graph(22, 16, 0.57, 0.19, 0.19, seed=22)
    cases.append(("R-MAT 22 p=0.01", 1 << 22, src, dst, graphgen.uniform_prob(len(src), 0.01), 100_000, 42))
    for deg, p in ((16, 0.1), (16, 0.2), (4, 0.4)):
        src, dst = graphgen.lfr_graph(10_000, deg, 2)
        cases.append((f"LFR n=10k degree {deg} p={p}", 10_000, src, dst, graphgen.uniform_prob(len(src), p), 10_240, 1))
    rows = []
    for name, n, src, dst, prob, S, seed in cases:
        a = sp.csr_matrix((np.ones(len(src), dtype=np.float32), (src, dst)), shape=(n, n))
        t = time.perf_counter()
        perm = reverse_cuthill_mckee((a + a.T).tocsr(), symmetric_mode=True)
        rank = np.empty(n, dtype=np.uint32)
        rank[perm] = np.arange(n, dtype=np.uint32)
        log(f"order study: {name}: RCM in {time.perf_counter() - t:.1f}s")
        g = bpt.bpt_create_graph(n, src, dst, prob)
        off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
        cap = 1 << 22
        vert = torch.empty(cap, dtype=torch.int32, device="cuda")
        for C in (64, 256):
            for label, flags, rk in (("sample ids", 0, None), ("sorted starts", bpt.BPT_FLAG_SORTED_STARTS, None),
                                     ("sorted RCM ranks", bpt.BPT_FLAG_SORTED_STARTS, rank)):
                bpt.bpt_graph_set_vertex_order(g, rk)
                times = []
                for rep in range(4):
                    st, total, cnt = bpt.bpt_sample_rrr_device(g, 0, S, C, seed, flags, stream, off, vert, cap)
                    if st == bpt.BPT_ERANGE:
                        cap = total + total // 8
                        vert = torch.empty(cap, dtype=torch.int32, device="cuda")
                        st, total, cnt = bpt.bpt_sample_rrr_device(g, 0, S, C, seed, flags, stream, off, vert, cap)
                    assert st == bpt.BPT_OK
                    if rep:
                        times.append(cnt.traversal_ns / 1e6)
                rows.append(dict(case=name, colors=C, order=label, ea=cnt.edge_accesses, te=cnt.sample_edges,
                                 entries=cnt.frontier_entries, members=cnt.members,
                                 traversal_ms=float(np.median(times))))
                log(f"order study: {name} C={C} {label}: EA/TE {cnt.edge_accesses / max(1, cnt.sample_edges):.4f} "
                    f"{np.median(times):.3f} ms")
        bpt.bpt_free(g)
        del vert, off
        torch.cuda.empty_cache()
    with open(out_path, "w") as f:
        json.dump(rows, f)
    print("| graph | C | batch order | EA / TE | colour occupancy | traversal ms |")
    print("|---|---|---|---|---|---|")
    for r in rows:
        occ = r["members"] / max(1, r["colors"] * r["entries"])
        print(f"| {r['case']} | {r['colors']} | {r['order']} | {r['ea'] / max(1, r['te']):.4f} | {100 * occ:.2f}% | "
              f"{r['traversal_ms']:.3f} |")
    return 0


def plan_study(out_path: str) -> int:
    """Per-call cost of the host-synchronous call (bpt_sample_rrr_device)
    against a plan (bpt_plan_enqueue) run eagerly and as a captured hipGraph,
    for a one-batch call (64 samples) and the R-MAT 20 workload.  Every path's
    sets are compared with the host-synchronous call's."""
    import numpy as np
    import torch

    import graphgen
    import paper_2311_10201_amd as bpt

    torch.cuda.set_device(0)
    cases = []
    src, dst = graphgen.er_graph(1000, 10_000, seed=42)
    cases.append(("ER n=1,000 m=10,000 p=0.1", 1000, src, dst, graphgen.uniform_prob(len(src), 0.1), 64, 64, 400))
    src, dst = graphgen.rmat_graph(20, 16, 0.57, 0.19, 0.19, seed=20)
    cases.append(("R-MAT 20 WC", 1 << 20, src, dst, graphgen.wc_prob(1 << 20, dst), 100_000, 64, 20))
    rows = []
    for name, n, src, dst, prob, S, C, reps in cases:
        g = bpt.bpt_create_graph(n, src, dst, prob)
        stream = torch.cuda.Stream()
        off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
        cap = max(1024, 64 * S)
        vert = torch.empty(cap, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(stream):
            st, total, _ = bpt.bpt_sample_rrr_device(g, 0, S, C, 42, 0, stream, off, vert, cap)
        assert st == bpt.BPT_OK
        ref_off, ref_vert = off.cpu().clone(), vert[:total].cpu().clone()

        def timed(fn, sync_each):
            for _ in range(3):
                fn()
            stream.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
                if sync_each:
                    stream.synchronize()
            stream.synchronize()
            return (time.perf_counter() - t) / reps * 1e6

        def device_call():
            st_, _, _ = bpt.bpt_sample_rrr_device(g, 0, S, C, 42, 0, stream, off, vert, cap)
            assert st_ == bpt.BPT_OK

        plan = bpt.bpt_plan_create(g, S, C, 0)
        res = torch.zeros(2, dtype=torch.int64, device="cuda")
        params = torch.tensor([0, 42], dtype=torch.int64, device="cuda")

        def plan_call():
            bpt.bpt_plan_enqueue(plan, 0, S, 42, params, stream, off, vert, cap, res)

        def check(what):
            stream.synchronize()
            status, members = res.cpu().tolist()
            assert status == bpt.BPT_OK and members == total, (what, status, members, total)
            assert torch.equal(off.cpu(), ref_off) and torch.equal(vert[:total].cpu(), ref_vert), what

        row = dict(case=name, samples=S, colors=C, reps=reps)
        row["device_call_us"] = timed(device_call, True)
        with torch.cuda.stream(stream):
            row["plan_eager_us"] = timed(plan_call, True)
            check("plan eager")
            row["plan_eager_pipelined_us"] = timed(plan_call, False)
            check("plan eager, pipelined")
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream, capture_error_mode="thread_local"):
            plan_call()
        with torch.cuda.stream(stream):
            res.zero_()
            row["graph_replay_us"] = timed(graph.replay, True)
            check("graph replay")
            row["graph_replay_pipelined_us"] = timed(graph.replay, False)
            check("graph replay, pipelined")
        log(f"plan study: {name}: " + ", ".join(f"{k} {v:.1f}" for k, v in row.items() if k.endswith("_us")))
        rows.append(row)
        del graph
        plan.close()
        bpt.bpt_free(g)
        del vert, off
        torch.cuda.empty_cache()
    with open(out_path, "w") as f:
        json.dump(rows, f)
    print("| call | samples | host-synchronous call | plan, eager | plan, eager, pipelined | graph replay | "
          "graph replay, pipelined |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['case']} | {r['samples']} | {r['device_call_us']:.1f} us | {r['plan_eager_us']:.1f} us | "
              f"{r['plan_eager_pipelined_us']:.1f} us | {r['graph_replay_us']:.1f} us | "
              f"{r['graph_replay_pipelined_us']:.1f} us |")
    return 0


def mix_instances(w):
    """The seeded draw of the mix's instances (shapes only; graphs come later)."""
    import math

    import numpy as np
    rng = np.random.Generator(np.random.PCG64(w["draw_seed"]))
    out = []
    for i in range(w["instances"]):
        scale = int(rng.integers(w["scale_lo"], w["scale_hi"] + 1))
        ef = int(rng.choice(np.array(w["efs"])))
        prob = w["probs"][int(rng.integers(len(w["probs"])))]
        samples = int(round(math.exp(rng.uniform(math.log(w["samples_lo"]), math.log(w["samples_hi"])))))
        out.append(dict(scale=scale, ef=ef, prob=prob, samples=samples, graph_seed=1000 + i, seed=42 + i))
    return out


def bench_mix(args, w) -> int:
    """Many uneven sampling jobs: one bpt_sample_rrr_jobs call (one persistent
    fused launch per mask width) against one bpt_sample_rrr_device call per
    instance, on the same GPU and buffers."""
    import numpy as np
    import torch

    import graphgen
    import paper_2311_10201_amd as bpt

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    insts = mix_instances(w)
    t0 = time.perf_counter()
    for k in insts:
        src, dst = graphgen.rmat_graph(k["scale"], k["ef"], 0.57, 0.19, 0.19, seed=k["graph_seed"])
        n = 1 << k["scale"]
        prob = graphgen.wc_prob(n, dst) if k["prob"] == "wc" else graphgen.uniform_prob(len(src), k["prob"])
        k.update(n=n, m=len(src), src=src, dst=dst, p=prob, g=bpt.bpt_create_graph(n, src, dst, prob))
    log(f"mix: {len(insts)} graphs generated and built in {time.perf_counter() - t0:.1f}s")

    def device_run(k, S, cap):
        off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
        vert = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
        st, total, cnt = bpt.bpt_sample_rrr_device(k["g"], 0, S, k.get("colors", 0), k["seed"], 0, stream, off,
                                                   vert, cap)
        return st, total, cnt, off, vert

    # output budget from a 256-sample pilot (the sets' mean size)
    for k in insts:
        cap = 1 << 20
        st, total, _, _, _ = device_run(k, 256, cap)
        if st == bpt.BPT_ERANGE:
            st, total, _, _, _ = device_run(k, 256, total)
        mean = max(1.0, total / 256)
        k["samples"] = int(max(64, min(k["samples"], w["out_budget"] // int(np.ceil(mean)))))
        # colours when sampled alone: measured by the autotuner, or the library's rule
        k["colors"] = (bpt.bpt_tune_colors(k["g"], k["samples"], k["seed"]) if args.tune
                       else bpt.bpt_default_colors(k["g"], k["samples"]))
    S_all = sum(k["samples"] for k in insts)
    log(f"mix: {S_all} samples in all; colours {[k['colors'] for k in insts]}")

    # reference outputs: one call per instance (exact buffer sizes)
    for k in insts:
        st, total, cnt, off, vert = device_run(k, k["samples"], 1 << 20)
        if st == bpt.BPT_ERANGE:
            st, total, cnt, off, vert = device_run(k, k["samples"], total)
        assert st == bpt.BPT_OK
        k.update(total=total, off_ref=off, vert_ref=vert)
    jobs = [bpt.Job(k["g"], 0, k["samples"], k["seed"], torch.empty(k["samples"] + 1, dtype=torch.int64, device="cuda"),
                    torch.empty(max(k["total"], 1), dtype=torch.int32, device="cuda"), k["total"], k["colors"])
            for k in insts]
    st, cnt = bpt.bpt_sample_rrr_jobs(jobs, stream)
    assert st == bpt.BPT_OK
    same = all(j.total == k["total"] and torch.equal(j.d_offsets, k["off_ref"]) and
               torch.equal(j.d_vertices[:j.total], k["vert_ref"][:k["total"]]) for j, k in zip(jobs, insts))
    log(f"mix: one launch == per-instance calls on all {S_all} sets: {same}")

    def time_batched():
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, c = bpt.bpt_sample_rrr_jobs(jobs, stream)
        torch.cuda.synchronize()
        assert st == bpt.BPT_OK
        return time.perf_counter() - t, c

    def time_sequential():
        torch.cuda.synchronize()
        t = time.perf_counter()
        for k, j in zip(insts, jobs):
            st, _, _ = bpt.bpt_sample_rrr_device(k["g"], 0, k["samples"], k["colors"], k["seed"], 0, stream,
                                                 j.d_offsets, j.d_vertices, j.capacity)
            assert st == bpt.BPT_OK
        torch.cuda.synchronize()
        return time.perf_counter() - t

    for _ in range(max(1, args.warmup)):
        time_batched()
        time_sequential()
    bt, cnts = zip(*[time_batched() for _ in range(args.steps)])
    sq = [time_sequential() for _ in range(args.steps)]
    sec, sec_seq = sum(bt) / len(bt), sum(sq) / len(sq)
    cnt = cnts[-1]
    trav_s = sum(c.traversal_ns for c in cnts) / len(cnts) / 1e9
    achieved = cnt.philox_blocks / trav_s
    result = {
        "metric": "RRR samples/sec over a 32-instance R-MAT mix: one multi-job fused launch vs one call per "
                  "instance (bit-exact)",
        "value": S_all / sec, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "instances": len(insts), "samples": S_all,
                   "members": int(cnt.members),
                   "mix": [dict(scale=k["scale"], ef=k["ef"], prob=k["prob"], m=k["m"], samples=k["samples"],
                                colors=k["colors"]) for k in insts],
                   "colors": "bpt_tune_colors per instance" if args.tune else "the library's rule per instance"},
        "edges_per_s": cnt.sample_edges / sec,
        "sequential": {"samples_per_s": S_all / sec_seq, "ms_per_step": sec_seq * 1e3},
        "speedup_vs_sequential": sec_seq / sec,
        "roofline": {"bound": "alu", "kernel": "fused_bpt_kernel (all mask widths of the mix)",
                     "achieved": achieved / 1e9, "peak": PEAK_PHILOX_BLOCKS / 1e9,
                     "unit": "G Philox4x32-10 blocks/s", "frac": achieved / PEAK_PHILOX_BLOCKS, "traffic": None,
                     "per_launch": {"philox_blocks": cnt.philox_blocks, "traversal_ms": trav_s * 1e3}},
        "parity": None,
    }
    log(f"mix: batched {sec * 1e3:.2f} ms, sequential {sec_seq * 1e3:.2f} ms")

    ok = same
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or min(16, len(os.sched_getaffinity(0)))
        cpu_s, n_cpu, te = 0.0, 0, 0
        for k, j in zip(insts, jobs):
            ids = np.unique(np.linspace(0, k["samples"] - 1, w["check_per_instance"]).astype(np.uint64))
            og = oracle.Graph(k["n"], k["src"], k["dst"], k["p"])
            t = time.perf_counter()
            ref = og.sample_ids(k["seed"], ids, nthreads=threads)
            cpu_s += time.perf_counter() - t
            n_cpu += len(ids)
            te += int(ref.te.sum())
            off = j.d_offsets.cpu().numpy().view(np.uint64)
            for i, s_id in enumerate(ids.tolist()):
                got = j.d_vertices[int(off[s_id]):int(off[s_id + 1])].cpu().numpy().view(np.uint32)
                ok = ok and np.array_equal(got, ref.set_of(i))
        result["cpu_baseline"] = {"value": n_cpu / cpu_s, "unit": "samples/s", "cores": threads, "kind": "oracle",
                                  "sample": f"{n_cpu} sample ids spread over the {len(insts)} instances "
                                            "(oracle time only, graph builds excluded)",
                                  "edges_per_s": te / cpu_s}
        result["parity"] = (f"one launch == per-instance calls on all {S_all} sets; bit-exact vs oracle on "
                            f"{n_cpu} sampled sets" if ok else "MISMATCH")
        log(f"mix: oracle parity {'ok' if ok else 'FAILED'}")
    print(json.dumps(result), flush=True)
    return 0 if ok else 1


def bench_serve(args, w) -> int:
    """The serving loop against one-request-at-a-time service of the same
    Poisson request stream.  One-at-a-time service times are measured request
    by request (alone on the GPU); its latencies are those of a FIFO queue fed
    with them.  The server run submits every request at its arrival time and
    takes latencies from the server's completion stamps."""
    import math
    import threading

    import numpy as np
    import torch

    import graphgen
    import paper_2311_10201_amd as bpt

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    graphs = []
    for i, sc in enumerate(w["scales"]):
        src, dst = graphgen.rmat_graph(sc, w["ef"], 0.57, 0.19, 0.19, seed=500 + i)
        n = 1 << sc
        graphs.append(dict(n=n, g=bpt.bpt_create_graph(n, src, dst, graphgen.wc_prob(n, dst))))
    log(f"serve: {len(graphs)} graphs built in {time.perf_counter() - t0:.1f}s")
    rng = np.random.Generator(np.random.PCG64(w["draw_seed"]))
    N = args.requests or w["requests"]
    reqs = []
    for i in range(N):
        gi = int(rng.integers(len(graphs)))
        S = int(round(math.exp(rng.uniform(math.log(w["samples_lo"]), math.log(w["samples_hi"])))))
        frac = w["seeds_fraction"] if args.seeds_fraction < 0 else args.seeds_fraction
        kind = bpt.BPT_REQ_SEEDS if rng.random() < frac else bpt.BPT_REQ_SAMPLE
        reqs.append(dict(gi=gi, S=S, kind=kind, seed=10_000 + i, first=0))
    # set-size means per graph (for caller buffers of sample requests)
    for gr in graphs:
        off = torch.empty(4097, dtype=torch.int64, device="cuda")
        cap = 1 << 24
        st, total, _ = bpt.bpt_sample_rrr_device(gr["g"], 0, 4096, 0, 1, 0, stream, off,
                                                 torch.empty(cap, dtype=torch.int32, device="cuda"), cap)
        assert st in (bpt.BPT_OK, bpt.BPT_ERANGE)
        gr["mean"] = max(1.0, total / 4096)

    def buffers(r):
        cap = int(r["S"] * graphs[r["gi"]]["mean"] * 2.0) + 65536
        return (torch.empty(r["S"] + 1, dtype=torch.int64, device="cuda"),
                torch.empty(cap, dtype=torch.int32, device="cuda"), cap)

    def alone(r):
        """One request by itself: sets into buffers, plus the seeds for a seed request."""
        off, vert, cap = buffers(r)
        g = graphs[r["gi"]]
        st, total, _ = bpt.bpt_sample_rrr_device(g["g"], r["first"], r["S"], 0, r["seed"], 0, stream, off, vert, cap)
        assert st == bpt.BPT_OK, st
        seeds = None
        if r["kind"] == bpt.BPT_REQ_SEEDS:
            seeds = bpt.bpt_max_cover(off, vert, r["S"], g["n"], w["k"], stream)[0]
        return off, vert, total, seeds

    # a single large request alone: through the server (chunked launches on two
    # streams) and as one library call, to show what chunking costs
    chunk_check = None
    big = dict(gi=4, S=1_000_000, kind=bpt.BPT_REQ_SAMPLE, seed=7, first=0)
    alone(big)
    torch.cuda.synchronize()
    t = time.perf_counter()
    alone(big)
    torch.cuda.synchronize()
    t_alone = time.perf_counter() - t
    srv0 = bpt.Server()
    off0, vert0, cap0 = buffers(big)
    for rep in range(2):
        q0 = bpt.Request(big["kind"], graphs[big["gi"]]["g"], 0, big["S"], big["seed"], d_offsets=off0,
                         d_vertices=vert0, capacity=cap0, tag=rep)
        t = time.perf_counter()
        srv0.submit(q0)
        q0 = srv0.wait(60.0)
        t_srv = time.perf_counter() - t
    launches0 = srv0.stats()["launches"] / 2
    srv0.close()
    chunk_check = {"samples": big["S"], "graph": f"R-MAT {w['scales'][big['gi']]} WC", "alone_ms": t_alone * 1e3,
                   "server_ms": t_srv * 1e3, "server_launches": launches0}
    log(f"serve: one 1M-sample request alone {t_alone * 1e3:.1f} ms, through the server {t_srv * 1e3:.1f} ms "
        f"({launches0:.0f} launches)")
    del off0, vert0

    # one at a time: service time of each request alone, after two requests on
    # every graph (the library sizes a graph's workspace from its set-size history)
    for gi in range(len(graphs)):
        first = next((r for r in reqs if r["gi"] == gi), None)
        for _ in range(2 if first else 0):
            alone(first)
    torch.cuda.synchronize()
    service = np.zeros(N)
    for i, r in enumerate(reqs):
        t = time.perf_counter()
        alone(r)
        torch.cuda.synchronize()
        service[i] = time.perf_counter() - t
    for i in range(0, N, max(1, N // 20)):
        log(f"serve: request {i}: graph {reqs[i]['gi']} samples {reqs[i]['S']} kind {reqs[i]['kind']} "
            f"alone {service[i] * 1e3:.2f} ms")
    serial_s = float(service.sum())
    capacity = N / serial_s
    load = args.load or w["load"]
    rate = load * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / rate, N))
    fin = np.zeros(N)
    clock = 0.0
    for i in range(N):  # FIFO single server
        clock = max(clock, arrivals[i]) + service[i]
        fin[i] = clock
    lat_serial = fin - arrivals
    samples = sum(r["S"] for r in reqs)
    log(f"serve: one at a time {serial_s:.1f}s of service, capacity {capacity:.1f} req/s; arrivals at {rate:.1f}/s")

    # the server, same arrival times; every request and its output buffers are
    # made before the clock starts, so the submitting thread only waits and submits.
    # The graphs' cached workspaces from the one-at-a-time pass are released first
    # (the server sizes its own traversal slots from the memory left).
    for gr in graphs:
        bpt.bpt_graph_release_cache(gr["g"])
    torch.cuda.empty_cache()
    srv = bpt.Server()
    done = {}
    prepared = []
    for i, r in enumerate(reqs):
        g = graphs[r["gi"]]["g"]
        if r["kind"] == bpt.BPT_REQ_SAMPLE:
            off, vert, cap = buffers(r)
            q = bpt.Request(r["kind"], g, r["first"], r["S"], r["seed"], d_offsets=off, d_vertices=vert,
                            capacity=cap, tag=i)
        else:
            q = bpt.Request(r["kind"], g, r["first"], r["S"], r["seed"], k=w["k"], tag=i)
        prepared.append(q)
    torch.cuda.synchronize()
    # warm-up before the clock, as at a service's start: the largest graph's
    # request on both lanes sizes their traversal workspaces and pools
    t = time.perf_counter()
    gbig = max(range(len(graphs)), key=lambda i: graphs[i]["n"])
    warm_req = dict(gi=gbig, S=w["samples_hi"], kind=bpt.BPT_REQ_SAMPLE, seed=7, first=0)
    off_w, vert_w, cap_w = buffers(warm_req)
    for rep in range(2):
        srv.submit(bpt.Request(bpt.BPT_REQ_SAMPLE, graphs[gbig]["g"], 0, w["samples_hi"], 7, d_offsets=off_w,
                               d_vertices=vert_w, capacity=cap_w, tag=-1))
        assert srv.wait(120.0) is not None
        log(f"serve: warm-up request {rep} done after {time.perf_counter() - t:.2f} s")
    del off_w, vert_w
    warm = srv.stats()
    lag = np.zeros(N)

    def submitter():
        base = srv.now()
        for i, q in enumerate(prepared):
            delay = base + arrivals[i] - srv.now()
            if delay > 0:
                time.sleep(delay)
            q.arrival = base + arrivals[i]
            srv.submit(q)
            lag[i] = q.t_submit - q.arrival

    th = threading.Thread(target=submitter)
    t_run = time.perf_counter()
    th.start()
    while len(done) < N:
        q = srv.wait(30.0)
        if q is None:
            log("serve: no completion for 30 s")
            break
        done[q.tag] = q
        if len(done) % 250 == 0:
            log(f"serve: {len(done)} of {N} completed")
    th.join()
    run_s = time.perf_counter() - t_run
    info = srv.stats()
    for key in ("launches", "served", "busy_s", "sample_s", "cover_s", "alloc_s", "resampled"):
        info[key] -= warm[key]
    launches, served = info["launches"], info["served"]
    srv.close()
    ok = len(done) == N and all(q.status == bpt.BPT_OK for q in done.values())
    lat_srv = np.array([done[i].t_done - done[i].arrival for i in range(N)]) if ok else np.zeros(1)

    # results identical alone and in the mix (every check_every-th request)
    same = ok
    for i in range(0, N, w["check_every"]):
        if not same:
            break
        q, r = done[i], reqs[i]
        off, vert, total, seeds = alone(r)
        torch.cuda.synchronize()
        if r["kind"] == bpt.BPT_REQ_SAMPLE:
            same = q.total == total and torch.equal(q.d_offsets, off) and torch.equal(q.d_vertices[:total],
                                                                                    vert[:total])
        else:
            same = q.total == total and np.array_equal(q.seeds[:w["k"]], seeds)

    def pct(x, p):
        return float(np.percentile(x, p)) * 1e3 if len(x) else None

    breakdown = None
    if ok:
        kinds = np.array([r["kind"] for r in reqs])
        sizes = np.array([r["S"] for r in reqs])
        start = np.array([done[i].t_start - done[i].arrival for i in range(N)])
        third = np.percentile(sizes, [100 / 3, 200 / 3])
        groups = {"sample_requests": kinds == bpt.BPT_REQ_SAMPLE, "seed_requests": kinds == bpt.BPT_REQ_SEEDS,
                  "smallest_third": sizes <= third[0], "largest_third": sizes > third[1]}
        breakdown = {name: {"server_p50_ms": pct(lat_srv[m], 50), "server_p99_ms": pct(lat_srv[m], 99),
                            "one_at_a_time_p50_ms": pct(lat_serial[m], 50),
                            "one_at_a_time_p99_ms": pct(lat_serial[m], 99)} for name, m in groups.items()}
        breakdown["server_wait_to_first_launch_p50_ms"] = pct(start, 50)
        breakdown["server_wait_to_first_launch_p99_ms"] = pct(start, 99)
        early = arrivals < 1.0
        breakdown["server_wait_to_first_launch_first_second_p99_ms"] = pct(start[early], 99)
        breakdown["server_wait_to_first_launch_after_first_second_p99_ms"] = pct(start[~early], 99)
        breakdown["submit_lag_p50_ms"] = pct(lag, 50)
        breakdown["submit_lag_p99_ms"] = pct(lag, 99)

    result = {
        "metric": "RRR requests served (sets or k = 50 influence-maximization seeds): samples/s and p50/p99 "
                  "latency, serving loop vs one request at a time",
        "value": samples / run_s, "unit": "samples/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": run_s * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": args.workload, "graphs": [f"R-MAT {sc} EF {w['ef']} WC" for sc in w["scales"]],
                   "requests": N, "samples": samples, "seeds_requests": sum(r["kind"] for r in reqs),
                   "k": w["k"], "arrival_rate_per_s": rate, "load_vs_one_at_a_time": load},
        "server": {"p50_ms": pct(lat_srv, 50), "p99_ms": pct(lat_srv, 99), "launches": launches,
                   "requests_per_launch": served / max(1, launches), "wall_s": run_s,
                   "worker_s": {k: info[k] for k in ("busy_s", "sample_s", "cover_s", "alloc_s")},
                   "resampled": info["resampled"], "batch_us_estimate": info["batch_s"] * 1e6},
        "one_at_a_time": {"p50_ms": pct(lat_serial, 50), "p99_ms": pct(lat_serial, 99), "service_s": serial_s,
                          "capacity_req_per_s": capacity, "samples_per_s_at_capacity": samples / serial_s},
        "chunking_check": chunk_check,
        "latency_breakdown": breakdown,
        "parity": (f"server results == the same requests alone on {len(range(0, N, w['check_every']))} checked "
                   "requests" if same else "MISMATCH or failed requests"),
    }
    print(json.dumps(result), flush=True)
    return 0 if same else 1


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22-p0.01", choices=sorted(WORKLOADS))
    ap.add_argument("--variant-steps", type=int, default=1,
                    help="timed steps of each comparison variant (unfused, other colour counts)")
    ap.add_argument("--colors", type=int, default=0, help="0: pick the fastest listed colour count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the library's launch-shape tuner")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 1 GiB device-to-device copy (known bytes, for counter scaling)")
    ap.add_argument("--only", default="", help="time only this variant (fused64, fused256, unfused, ...)")
    ap.add_argument("--requests", type=int, default=0, help="serve8: number of requests (default 2000)")
    ap.add_argument("--seeds-fraction", type=float, default=-1.0,
                    help="serve8: share of influence-maximization requests (default 0.25)")
    ap.add_argument("--load", type=float, default=0.0,
                    help="serve8: arrival rate as a multiple of one-at-a-time capacity (default 0.8)")
    ap.add_argument("--tune", action="store_true",
                    help="rmat-mix32: choose each instance's colours with bpt_tune_colors (untimed)")
    ap.add_argument("--order-study", default="", metavar="OUT.json",
                    help="instead of the benchmark: id-order vs sorted-start vs RCM-sorted batches")
    ap.add_argument("--plan-study", default="", metavar="OUT.json",
                    help="instead of the benchmark: per-call cost of the host-synchronous call vs a plan, eager "
                         "and captured into a hipGraph")
    ap.add_argument("--fusion-study", default="", metavar="OUT.json",
                    help="instead of the benchmark: edge accesses and colour occupancy of the fused traversal "
                         "vs colour count and probability on LFR graphs; writes the records to OUT.json")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this library has no multi-GPU path "
              "(sampling shards by sample-id range; see the design notes)", file=sys.stderr)
        return 2

    if args.fusion_study:
        return fusion_study(args.fusion_study)
    if args.order_study:
        return order_study(args.order_study)
    if args.plan_study:
        return plan_study(args.plan_study)

    import numpy as np
    import torch

    import paper_2311_10201_amd as bpt

    w = WORKLOADS[args.workload]
    if w["kind"] == "mix":
        return bench_mix(args, w)
    if w["kind"] == "serve":
        return bench_serve(args, w)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.int32, device="cuda")
        b = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        a.copy_(b)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy: 1 GiB read + 1 GiB written")
    log(f"workload {args.workload}: generating graph")
    n, src, dst, prob = make_graph(w)
    m = len(src)
    S, seed = w["samples"], w["seed"]
    t0 = time.perf_counter()
    g = bpt.bpt_create_graph(n, src, dst, prob)
    log(f"graph n={n} m={m} layout={bpt.bpt_graph_info(g)[2]} built in {time.perf_counter() - t0:.2f}s")
    stream = torch.cuda.current_stream()
    tuner = None
    if not args.no_tune and not args.only:
        # the library's launch-shape tuner on its capped trial (8 .. 1024 colours, then the colour
        # schedule); untimed, reported beside the full-size variants
        t0 = time.perf_counter()
        tc = bpt.bpt_tune_colors(g, S, seed)
        tuner = {"colors": tc, "seconds": time.perf_counter() - t0,
                 "note": "bpt_tune_colors on its trial of min(S, 16 x 64 x resident workgroups) samples"}
        log(f"tuner: {tc} colours in {tuner['seconds']:.1f}s")
    off = torch.empty(S + 1, dtype=torch.int64, device="cuda")
    cap = max(1 << 20, 48 * S)
    vert = torch.empty(cap, dtype=torch.int32, device="cuda")

    def step(colors, flags=0):
        nonlocal vert, cap
        st, total, cnt = bpt.bpt_sample_rrr_device(g, 0, S, colors, seed, flags, stream, off, vert, cap)
        if st == bpt.BPT_ERANGE:  # grow the buffer; the library only re-assembles the CSR
            del vert
            cap = total + total // 16
            vert = torch.empty(cap, dtype=torch.int32, device="cuda")
            st, total, cnt = bpt.bpt_sample_rrr_device(g, 0, S, colors, seed, flags, stream, off, vert, cap)
        assert st == bpt.BPT_OK
        return total, cnt

    def timed_one(colors, flags):
        torch.cuda.synchronize()
        t = time.perf_counter()
        cnt = step(colors, flags)[1]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        if dt > 1.0:
            log(f"  call took {dt:.2f}s (traversal {cnt.traversal_ns / 1e9:.2f}s)")
        return dt, cnt

    def timed(colors, flags, steps):
        total_s, cnts = 0.0, []
        for _ in range(steps):
            dt, cnt = timed_one(colors, flags)
            total_s += dt
            cnts.append(cnt)
        return total_s / steps, cnts

    big = m > (1 << 25)  # per-variant workspaces and output pools take tens of GB

    def between_variants():
        if big:
            bpt.bpt_graph_release_cache(g)

    variants = [(c, 0) for c in w["colors"]] + [(0, bpt.BPT_FLAG_UNFUSED)]
    if args.only:
        variants = [v for v in variants if ("unfused" if v[1] else f"fused{v[0]}") == args.only]
        if not variants:
            print(f"unknown variant {args.only}", file=sys.stderr)
            return 2
    # every variant: one untimed call (it builds the variant's workspace and
    # sizes the output buffer), then --variant-steps timed calls; the fastest
    # listed colour count on those warm calls becomes the headline unless
    # --colors names one
    others = {}
    for c, fl in variants:
        name = "unfused" if fl else f"fused{c}"
        between_variants()
        dt0, cnt0 = timed_one(c, fl)
        log(f"first call {name}: {dt0 * 1e3:.2f} ms, members={cnt0.members}")
        s2, c2 = timed(c, fl, max(1, args.variant_steps))
        others[name] = dict(samples_per_s=S / s2, ms_per_step=s2 * 1e3, steps=max(1, args.variant_steps),
                            traversal_ms=sum(x.traversal_ns for x in c2) / len(c2) / 1e6,
                            edge_accesses=c2[-1].edge_accesses, philox_blocks=c2[-1].philox_blocks,
                            workgroups=c2[-1].workgroups)
        log(f"{name}: {s2 * 1e3:.2f} ms/step")

    fused_done = [c for c in w["colors"] if f"fused{c}" in others]
    if not fused_done:
        print("--only must name a fused variant (the headline is the fused traversal)", file=sys.stderr)
        return 2
    colors = args.colors or min(fused_done, key=lambda c: others[f"fused{c}"]["ms_per_step"])
    between_variants()
    for _ in range(max(1, args.warmup)):
        timed_one(colors, 0)
    log(f"timing fused C={colors}: {args.steps} steps after {max(1, args.warmup)} warmup calls")
    sec, cnts = timed(colors, 0, args.steps)
    cnt = cnts[-1]
    value = S / sec
    te_per_s = cnt.sample_edges / sec
    trav_s = sum(c.traversal_ns for c in cnts) / len(cnts) / 1e9
    blocks = cnt.philox_blocks
    others[f"fused{colors}"] = dict(samples_per_s=value, ms_per_step=sec * 1e3, steps=args.steps,
                                    traversal_ms=trav_s * 1e3, edge_accesses=cnt.edge_accesses,
                                    philox_blocks=blocks, workgroups=cnt.workgroups)
    # keep the headline output's sets that the oracle will recompute (every
    # cpu_stride-th sample id) for the parity check
    total = int(off[-1].item())
    gpu_off = off.cpu().numpy().view(np.uint64).copy()
    check_ids = np.arange(0, S, w["cpu_stride"], dtype=np.uint64)
    if w["cpu_stride"] == 1:
        gpu_sets = vert[:total].cpu().numpy().view(np.uint32).copy()
    else:
        idx = torch.as_tensor(check_ids.astype(np.int64), device="cuda")
        lo, hi = off[idx], off[idx + 1]
        lens = hi - lo
        pos = torch.repeat_interleave(lo - (torch.cumsum(lens, 0) - lens), lens)
        pos += torch.arange(int(lens.sum().item()), device="cuda")
        gpu_sets = vert[pos].cpu().numpy().view(np.uint32).copy()
        del idx, lo, hi, lens, pos

    # host-resident result (adds the device-to-host copy of the CSR over PCIe);
    # skipped when the result is too large to copy around in a benchmark
    host_api = None
    if total * 4 <= (2 << 30):
        bpt.bpt_sample_rrr(g, S, colors, seed)
        t = time.perf_counter()
        host_res = bpt.bpt_sample_rrr(g, S, colors, seed)
        host_s = time.perf_counter() - t
        host_same = bool(np.array_equal(host_res.offsets, gpu_off) and
                         np.array_equal(host_res.vertices, vert[:total].cpu().numpy().view(np.uint32)))
        host_api = {"samples_per_s": S / host_s, "ms": host_s * 1e3, "same_as_device": host_same,
                    "note": "bpt_sample_rrr: device sampling plus the device-to-host copy of the CSR"}
        del host_res

    achieved = blocks / trav_s
    traffic = measured_traffic(args.workload, colors, cnt.workgroup_size)
    # algorithmic bytes of the launch from the per-unit figures (W = C / 8 bytes
    # per mask): per frontier entry the row bounds (8 B), its mask (W) and the
    # row's threshold (4 B, per-row layout; per-edge thresholds 4 B per edge
    # access); per live coin the source id (4 B), the fetch-ors on visited and
    # next frontier (2W) and a queue entry (4 B); per member its touched entry,
    # its output id (4 B each) and the clearing of its visited mask (W)
    W = colors // 8
    layout = bpt.bpt_graph_info(g)[2]
    thr_bytes = {0: 0, 1: 4 * cnt.frontier_entries, 2: 4 * cnt.edge_accesses}.get(layout, 0)
    algo_bytes = (cnt.frontier_entries * (8 + W) + thr_bytes + cnt.live_coins * (8 + 2 * W) +
                  cnt.members * (8 + W))
    # the library's rule for the instantiation with tail helping (one-word masks,
    # sets of 1,024+ members on average, unless BPT_HELP forces it)
    forced = os.environ.get("BPT_HELP")
    helping = colors <= 64 and (forced == "1" if forced in ("0", "1") else cnt.members >= 1024 * S)
    roofline = {
        "bound": "alu",
        "kernel": f"fused_bpt_kernel<{max(1, colors // 64)}, {cnt.workgroup_size}, {'true' if helping else 'false'}>",
        "achieved": achieved / 1e9,
        "peak": PEAK_PHILOX_BLOCKS / 1e9,
        "unit": "G Philox4x32-10 blocks/s",
        "frac": achieved / PEAK_PHILOX_BLOCKS,
        "traffic": traffic,
        "per_launch": {"philox_blocks": blocks, "traversal_ms": trav_s * 1e3,
                       "workgroup_size": cnt.workgroup_size, "workgroups": cnt.workgroups,
                       "frontier_entries": cnt.frontier_entries, "live_coins": cnt.live_coins,
                       "members": cnt.members, "algorithmic_bytes": algo_bytes,
                       "kernel_digest": kernel_digest()},
    }
    hbm_bytes = None
    if traffic:
        hbm_bytes = traffic / trav_s
        roofline["hbm_GBps"] = hbm_bytes / 1e9
        roofline["hbm_frac_of_8TBps"] = hbm_bytes / 8e12
        roofline["traffic_over_algorithmic"] = traffic / max(1, algo_bytes)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "graph": (f"R-MAT scale {w['scale']}, edge factor {w['ef']}, a={w['a']} b={w['b']} c={w['c']}, "
                      "self-loops and duplicates dropped" if w["kind"] == "rmat"
                      else f"Erdos-Renyi n={w['n']} m={w['m']}"),
            "prob": "weighted cascade 1/indeg(v)" if w["prob"] == "wc" else f"uniform {w['prob']}",
            "n": n, "m": m, "samples": S, "colors": colors, "seed": seed,
        },
        "edges_per_s": te_per_s,
        "sample_edges": cnt.sample_edges,
        "edge_accesses": cnt.edge_accesses,
        "fusion_ratio_te_over_ea": cnt.sample_edges / max(1, cnt.edge_accesses),
        "members": cnt.members,
        "max_levels": cnt.max_levels,
        "fused_vs_unfused": (value / others["unfused"]["samples_per_s"]) if "unfused" in others else None,
        "host_api": host_api,
        "variants": others,
        "tuner": tuner,
        "roofline": roofline,
    }

    if not args.no_cpu_baseline:
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        affinity = len(os.sched_getaffinity(0))
        # the host's CPU share per GPU is 16 cores; use every core of it the process may run on
        threads = args.cpu_threads or min(16, affinity)
        cpu_model = ""
        try:
            with open("/proc/cpuinfo") as f:
                cpu_model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
        except OSError:
            pass
        log(f"host: nproc {os.cpu_count()}, affinity {affinity} cores, {cpu_model}; oracle on {threads} threads")
        og = oracle.Graph(n, src, dst, prob)
        t = time.perf_counter()
        ref = og.sample_ids(seed, check_ids, nthreads=threads)
        cpu_s = time.perf_counter() - t
        sizes = (gpu_off[check_ids.astype(np.int64) + 1] - gpu_off[check_ids.astype(np.int64)]).astype(np.uint64)
        same = bool(np.array_equal(np.diff(ref.offsets), sizes) and np.array_equal(ref.members, gpu_sets))
        n_cpu = len(check_ids)
        result["cpu_baseline"] = {
            "value": n_cpu / cpu_s, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": (f"all {S} samples of the workload" if n_cpu == S else
                       f"{n_cpu} of the {S} samples (the ids that are multiples of {w['cpu_stride']})") +
                      f", one reverse BFS per sample, {cpu_model}",
            "edges_per_s": float(ref.te.sum()) / cpu_s,
            "seconds": cpu_s,
            "host": {"nproc": os.cpu_count(), "affinity_cores": affinity, "cpu_model": cpu_model},
        }
        result["parity"] = (f"bit-exact vs oracle on {n_cpu} of {S} sets" if same else "MISMATCH vs oracle")
        log(f"cpu oracle: {cpu_s:.2f}s on {threads} threads; parity {'ok' if same else 'FAILED'}")
        if not same:
            print(json.dumps(result), flush=True)
            return 1
        # Philox blocks Listing 1 would still need (its visited mask skips the coins
        # of sources already reached at the member's depth or less), as a share of
        # the blocks this kernel evaluates, from the oracle's sets of a subset of ids
        sub = np.arange(0, len(ref), w["listing_stride"])
        lens = (ref.offsets[sub + 1] - ref.offsets[sub]).astype(np.int64)
        pos = np.repeat(ref.offsets[sub].astype(np.int64) - (np.cumsum(lens) - lens), lens) + np.arange(lens.sum())
        part_off = np.zeros(len(sub) + 1, np.uint64)
        part_off[1:] = np.cumsum(lens)
        part_mem, part_dist = ref.members[pos], ref.dist[pos]
        chunks = [c for c in np.array_split(np.arange(len(sub)), threads) if len(c)]

        def blocks_of(ch):
            lo, hi = int(part_off[ch[0]]), int(part_off[ch[-1] + 1])
            piece = oracle.RRRSets(ref.sample_ids[sub[ch]], part_off[ch[0]:ch[-1] + 2] - part_off[ch[0]],
                                   part_mem[lo:hi], part_dist[lo:hi], ref.te[sub[ch]])
            a, l = oracle.coin_blocks(og, piece)
            return int(a.sum()), int(l.sum())

        with ThreadPoolExecutor(threads) as ex:
            sums = list(ex.map(blocks_of, chunks))
        b_all, b_listing = sum(x[0] for x in sums), sum(x[1] for x in sums)
        ratio = b_listing / max(1, b_all)
        roofline["listing_blocks_ratio"] = ratio
        roofline["frac_of_listing_coins"] = roofline["frac"] * ratio
        roofline["listing_note"] = (f"Philox blocks Listing 1's visited mask leaves needed / blocks evaluated = "
                                    f"{b_listing}/{b_all} on the oracle's sets of {len(sub)} sample ids "
                                    f"(multiples of {w['cpu_stride'] * w['listing_stride']}); frac_of_listing_coins "
                                    "counts only those blocks as useful work")
        if w["cpu_stride"] * w["listing_stride"] == 1 and b_all != blocks:
            log(f"Philox blocks: kernel {blocks}, oracle {b_all}")
            result["parity"] = "MISMATCH: Philox-block counter differs from the oracle's count"
            print(json.dumps(result), flush=True)
            return 1

    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
