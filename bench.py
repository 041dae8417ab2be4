"""Benchmark of the spliced protein-to-genome DP on one MI355X.

Default run (``--config all``): every workload of the metric in one process.

* Headline (``value``, ``roofline``, ``cpu_baseline``): the batch of 10,000
  planted-gene pairs (protein lengths log-normal around 400 aa, 1.2x-padded
  regions up to 40 kb, score-only, LOCAL, int32), inputs resident in HBM
  before the timed region.  One step = one ``mpg_align_batch_dev`` call over
  the whole batch (plan upload, prepass, DP, end-cell reduction),
  synchronised.  ``cpu_baseline`` times the oracle on a bounded sample of the
  same pairs and compares its results with the GPU's (``mismatches``).
* ``legs.traceback``: the same 10,000 pairs with full traceback.
* ``legs.longtail`` (run last): 200 pairs of 3-8k aa x 100-300 kb plus 2,000 short ones,
  traceback, in one call under a 240 GiB direction-bit budget (its ~250 GB
  of direction bits then fit one wave).
* ``legs.serving``: 200,000 jobs submitted one by one at Poisson arrival
  times through ``mpg_submit``/``mpg_poll``: p50/p99 latency from the
  scheduled arrival to the result (overall and per class), served GCUPS, the
  same jobs run one pair per launch, and every served result compared with a
  batched run of the same jobs.

Each workload can also run alone (``--config``): ``batch``, ``batch16``,
``traceback``, ``single``, ``longtail``, ``serving``, and the next rows'
``profile``, ``chain``, ``chaining``, ``rescore``.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X integer issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_INT_OPS = 256 * 4 * 16 * 2.4e9
# VALU instructions one cell of Eq. (full) needs (LOCAL, score-only):
# I 3, D 3, A 2, B 2, C 2, M 1, frameshifts 3, acceptors 3, H max3 x3, floor 1.
# The pseudogene guard's second pass (GLOBAL, no intron states): I 3, D 3,
# M 1, frameshifts 3, H max3 x2 over M, I, D and the two frameshift terms.
OPS_PER_CELL = {"score": 23, "traceback": 23, "global_no_intron": 12}
METRIC = "GCUPS batched spliced DP (bit-exact) + p50/p99 latency at fixed arrival rate"

# Copy-calibrated HBM traffic of the dominant DP kernel, per workload, as
# recorded by rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs in profiles/.  The
# figure is reported only while the kernel sources still hash to the value
# recorded beside it (otherwise the counters describe an older kernel).
TRAFFIC_PROFILE = {"batch": "dp_kernel_k2_local_score__batch10k.md",
                   "traceback": "dp_kernel_local_traceback__traceback10k.md",
                   "batch16": "dp16_kernel_k2_local_score__batch10k.md"}
DP_SOURCES = ["paper_2210_08052_amd/csrc/" + f for f in
              ("mpg_dp.h", "mpg_internal.h", "mpg_walk.h", "mpg_dp_k1.hip", "mpg_dp_k2.hip",
               "mpg_dp_k4.hip", "mpg_dp16.hip")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(config: str):
    from paper_2210_08052_amd import workloads as W
    if config == "batch":
        pairs = W.batch_pairs(10000, seed=2)
        tb = False
        desc = "planted-gene batch: 10,000 pairs, score-only, LOCAL"
    elif config == "batch16":
        pairs = W.batch_pairs(10000, seed=2)
        tb = False
        desc = "planted-gene batch: 10,000 pairs, score-only, LOCAL, int16 lanes"
    elif config == "traceback":
        pairs = W.batch_pairs(10000, seed=2)
        tb = True
        desc = "planted-gene batch: 10,000 pairs, full traceback, LOCAL"
    elif config == "single":
        pairs = [W.single_pair(1)]
        tb = True
        desc = "single planted pair: 100 aa x 3,000 nt, full traceback, LOCAL"
    elif config == "longtail":
        pairs = W.long_tail(200, 2000, seed=4)
        tb = True
        desc = "long-tail batch: 200 pairs 3-8k aa x 100-300 kb + 2,000 short, traceback, LOCAL"
    else:
        raise SystemExit("unknown --config %s" % config)
    return pairs, tb, desc


def recorded_traffic(config: str):
    import hashlib
    name = TRAFFIC_PROFILE.get(config)
    if not name:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", name)).read()
        h = hashlib.sha256()
        for f in DP_SOURCES:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except OSError:
        return None
    fields = dict(ln.split(":", 1) for ln in text.splitlines()
                  if ln.startswith(("traffic_bytes_per_launch:", "dp_source_sha256:")))
    if fields.get("dp_source_sha256", "").strip() != h.hexdigest():
        return None
    return int(fields["traffic_bytes_per_launch"])


def _res_key(r, tb):
    """Comparable fields of a result: status, score and end cell, plus begin
    cell and op string with traceback (a dict from the GPU, or an oracle
    Result)."""
    if isinstance(r, dict):
        st, sc, gb, ge, pb, pe, ops = (r["status"], r["score"], r["g_beg"], r["g_end"],
                                       r["p_beg"], r["p_end"], r.get("ops"))
    else:
        st, sc, gb, ge, pb, pe, ops = r.status, r.score, r.g_beg, r.g_end, r.p_beg, r.p_end, r.ops
    if st != 0:
        return (st,)
    return (st, sc, ge, pe, gb, pb, ops) if tb else (st, sc, ge, pe)


def cpu_baseline(pairs, tb: bool, budget_s: float, gpu=None):
    """The oracle, as it stands, on all host cores, on a bounded sample: pairs
    in a seeded random order, fed to the pool in chunks until the wall time
    reaches the budget.  With `gpu` (the GPU's result for every pair, from the
    timed run) each sampled pair's oracle result is compared with the GPU's:
    status, score and end cell, and with traceback the begin cell and op
    string; `mismatches` counts the pairs that differ."""
    import oracle
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(pairs))
    chunk = threads * 4
    k, cells, mism = 0, 0, 0
    t0 = time.perf_counter()
    while k < len(order) and time.perf_counter() - t0 < budget_s:
        idx = order[k:k + chunk]
        part = [pairs[i] for i in idx]
        res = oracle.align_many([(p.prot, p.dna) for p in part], None, tb, threads)
        if gpu is not None:
            mism += sum(1 for i, r in zip(idx, res) if _res_key(gpu[i], tb) != _res_key(r, tb))
        cells += sum(len(p.prot) * len(p.dna) for p in part)
        k += len(part)
    dt = time.perf_counter() - t0
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    out = {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
           "kind": "oracle",
           "sample": "%d of %d pairs (seeded random order), %.3g cells, %.1f s wall, %s" % (
               k, len(pairs), cells, dt, model)}
    if gpu is not None:
        out["checked"] = int(k)
        out["mismatches"] = int(mism)
    return out


def cpu_baseline_chains(chains, budget_s: float):
    """The oracle's anchor-driven alignment, as it stands, on all host cores
    (one chain per task) over a bounded sample; the rate counts the DP cells
    of the pieces, as the GPU figure does."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import chain as ochain
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(12345)
    order = rng.permutation(len(chains))

    def piece_cells(c):
        prot, dna, anchors, k = c[0], c[1], c[2], c[3]
        runs = ochain.anchor_runs(anchors, k, len(dna), len(prot))
        x1, y1, _ = runs[0]
        xr, yr, lr = runs[-1]
        tot = x1 * y1 + (len(dna) - xr - 3 * lr) * (len(prot) - yr - lr)
        for (xa, ya, la), (xb, yb, _) in zip(runs, runs[1:]):
            tot += (xb - xa - 3 * la) * (yb - ya - la)
        return tot

    def one(c):
        ochain.align_chain(c[0].decode(), c[1].decode(), c[2], c[3], sc, want_tb=True)
        return piece_cells(c)

    import oracle
    sc = oracle.default_scoring()
    k, cells = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        while k < len(order) and time.perf_counter() - t0 < budget_s:
            part = [chains[i] for i in order[k:k + threads * 4]]
            cells += sum(ex.map(one, part))
            k += len(part)
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d chains (seeded random order), %.3g piece cells, %.1f s wall" % (
                k, len(chains), cells, dt)}


def bench_chains(args):
    """Anchor-driven alignment of 10,000 planted genes with chains of true
    seed hits (6 residues each), full traceback: one step is one
    mpg_align_chains_dev over all chains (pieces in one batch, then the
    stitch kernel).  GCUPS count the DP cells of the pieces."""
    import torch
    from paper_2210_08052_amd import mpg
    from paper_2210_08052_amd import workloads as W
    t0 = time.time()
    jobs = W.chain_jobs(10000, seed=6)
    chains = [(p.prot, p.dna, a, 6, True) for p, a in jobs]
    region_cells = int(sum(len(c[0]) * len(c[1]) for c in chains))
    log("workload chain: %d chains, %d anchors, generated in %.1f s" % (
        len(chains), sum(len(c[2]) for c in chains), time.time() - t0))
    pb, db, cs = mpg.pack_chains(chains)
    dev = torch.device("cuda:0")
    d_prot = torch.frombuffer(bytearray(pb), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db), dtype=torch.uint8).to(dev)
    p = mpg.params()
    cap = cs.ops_capacity(p)
    d_ops = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    d_out = torch.empty(len(chains) * mpg.DEV_RESULT_DTYPE.itemsize, dtype=torch.uint8,
                        device=dev)
    ctx = mpg.Context(0)
    stream = torch.cuda.Stream(device=dev)
    ctx.set_stream(stream.cuda_stream)

    enqueue_s = [0.0]

    def step():
        t = time.perf_counter()
        ctx.align_chains_dev(p, d_prot.data_ptr(), d_dna.data_ptr(), cs, d_out.data_ptr(),
                             d_ops.data_ptr(), cap)
        enqueue_s[0] += time.perf_counter() - t

    for w in range(args.warmup):
        step()
        ctx.sync()
        log("warmup %d done" % w)
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)
    log("warmup results: %d/%d ok, score sum %d" % (int((out["status"] == 0).sum()), len(out),
                                                   int(out["score"].sum())))
    ctx.enable_timing(True)
    ctx.timing(reset=True)
    torch.cuda.synchronize()
    ctx.sync()
    enqueue_s[0] = 0.0
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        ctx.sync()
        log("step %d done" % k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.timing(reset=True)
    cells = tim["cells"] // max(1, args.steps)
    ms_step = dt * 1e3 / args.steps
    gcups = cells / (dt / args.steps) / 1e9
    dp_ms = tim["dp_ms"] / max(1, args.steps)
    ops = OPS_PER_CELL["traceback"]
    peak = PEAK_INT_OPS / 1e12
    achieved = cells * ops / (dp_ms * 1e-3) / 1e12
    log("step %.3f ms, GCUPS %.1f (%d piece cells, %.1f%% of the regions' %d); DP kernels "
        "%.3f ms/step, prepass %.3f ms, walk %.3f ms, host %.3f ms (whole call on the host "
        "%.3f ms)" % (
            ms_step, gcups, cells, 100.0 * cells / region_cells, region_cells, dp_ms,
            tim["prepass_ms"] / args.steps, tim["walk_ms"] / args.steps,
            tim["host_ms"] / args.steps, enqueue_s[0] * 1e3 / args.steps))
    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline_chains([c[:4] for c in chains], args.cpu_budget)
        log("cpu baseline: %s" % json.dumps(cpu))
    line = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded planted genes, chains of true seed hits)",
        "config": {"workload": "anchor-driven alignment: 10,000 planted genes, chains of "
                               "6-residue seed hits, traceback; EXTEND_LEFT/GLOBAL/EXTEND pieces",
                   "chains": len(chains), "cells": cells, "region_cells": region_cells,
                   "traceback": True, "chains_per_s": round(len(chains) / (dt / args.steps), 1)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": "Tops/s (int32 lane-ops)", "frac": round(achieved / peak, 4),
                     "traffic": recorded_traffic("chain"),
                     "kernel_gcups": round(cells / (dp_ms * 1e-3) / 1e9, 2), "ops_per_cell": ops,
                     "dp_ms_per_step": round(dp_ms, 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def cpu_baseline_profiles(jobs, budget_s: float):
    """The oracle on position-specific queries, on all host cores, over a
    bounded sample (score only, as the GPU run)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    sc = oracle.default_scoring()
    threads = len(os.sched_getaffinity(0))
    order = np.random.default_rng(12345).permutation(len(jobs))
    oracle._load()

    def one(k):
        p, S, G = jobs[k]
        oracle.align_profile(S, G, p.dna, sc, want_tb=False)
        return len(p.prot) * len(p.dna)

    k, cells = 0, 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(threads) as ex:
        while k < len(order) and time.perf_counter() - t0 < budget_s:
            part = order[k:k + threads * 4]
            cells += sum(ex.map(one, part))
            k += len(part)
    dt = time.perf_counter() - t0
    return {"value": round(cells / dt / 1e9, 4), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": "%d of %d profile queries (seeded random order), %.3g cells, %.1f s wall" % (
                k, len(jobs), cells, dt)}


def bench_profiles(args):
    """Position-specific queries: the 10,000-pair batch with every query
    protein replaced by a family profile (per-column scores and gap costs),
    score-only, LOCAL; one step is one mpg_align_profiles_dev."""
    import torch
    from paper_2210_08052_amd import mpg
    from paper_2210_08052_amd import workloads as W
    t0 = time.time()
    jobs = W.profile_jobs(10000, seed=2, profile_seed=7)
    cells = int(sum(len(p.prot) * len(p.dna) for p, _, _ in jobs))
    log("workload profile: %d queries, generated in %.1f s" % (len(jobs), time.time() - t0))
    fb, db, segs, cap = mpg.pack_profiles([(S, G, p.dna, False) for p, S, G in jobs])
    dev = torch.device("cuda:0")
    d_prof = torch.frombuffer(bytearray(fb), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db), dtype=torch.uint8).to(dev)
    d_ops = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    d_out = torch.empty(len(jobs) * mpg.DEV_RESULT_DTYPE.itemsize, dtype=torch.uint8,
                        device=dev)
    ctx = mpg.Context(0)
    stream = torch.cuda.Stream(device=dev)
    ctx.set_stream(stream.cuda_stream)
    p = mpg.params()

    def step():
        ctx.align_profiles_dev(p, d_prof.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(),
                               d_ops.data_ptr(), cap)

    for w in range(args.warmup):
        step()
        ctx.sync()
        log("warmup %d done" % w)
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)
    log("warmup results: %d/%d ok, score sum %d" % (int((out["status"] == 0).sum()), len(out),
                                                   int(out["score"].sum())))
    ctx.enable_timing(True)
    ctx.timing(reset=True)
    torch.cuda.synchronize()
    ctx.sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        ctx.sync()
        log("step %d done" % k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.timing(reset=True)
    ms_step = dt * 1e3 / args.steps
    gcups = cells / (dt / args.steps) / 1e9
    dp_ms = tim["dp_ms"] / max(1, args.steps)
    ops = OPS_PER_CELL["score"]
    peak = PEAK_INT_OPS / 1e12
    achieved = cells * ops / (dp_ms * 1e-3) / 1e12
    log("step %.3f ms, GCUPS %.1f; DP kernels %.3f ms/step (%.1f GCUPS), prepass %.3f ms, "
        "host %.3f ms" % (ms_step, gcups, dp_ms, cells / (dp_ms * 1e-3) / 1e9,
                          tim["prepass_ms"] / args.steps, tim["host_ms"] / args.steps))
    cpu = None
    if args.cpu_budget > 0:
        cpu = cpu_baseline_profiles(jobs, args.cpu_budget)
        log("cpu baseline: %s" % json.dumps(cpu))
    line = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded planted genes, family profiles)",
        "config": {"workload": "position-specific queries: 10,000 planted-gene regions, family "
                               "profiles (per-column scores and gap costs), score-only, LOCAL",
                   "pairs": len(jobs), "cells": cells, "traceback": False, "mode": "LOCAL"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": "Tops/s (int32 lane-ops)", "frac": round(achieved / peak, 4),
                     "traffic": recorded_traffic("profile"),
                     "kernel_gcups": round(cells / (dp_ms * 1e-3) / 1e9, 2), "ops_per_cell": ops,
                     "dp_ms_per_step": round(dp_ms, 3)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_chaining(args):
    """Chaining (first round, binned genome) of 10,000 anchor sets: the true
    seed hits of planted genes plus spurious hits; one step is one
    mpg_chain_anchors_dev.  The rate counts candidate pairs (i < j) of the
    O(n^2) recurrence."""
    import torch
    from paper_2210_08052_amd import mpg
    from paper_2210_08052_amd import workloads as W
    t0 = time.time()
    sets = W.chaining_sets(10000, seed=8, binned=True)
    ns = np.array([len(a) for a in sets], dtype=np.int64)
    pairs = int((ns * (ns - 1) // 2).sum())
    off = np.zeros(len(sets) + 1, dtype=np.int64)
    off[1:] = np.cumsum(ns)
    log("workload chaining: %d sets, %d anchors, %d candidate pairs, generated in %.1f s" % (
        len(sets), int(off[-1]), pairs, time.time() - t0))
    dev = torch.device("cuda:0")
    allv = np.ascontiguousarray(np.concatenate(sets))
    d_a = torch.from_numpy(allv).to(dev)
    tot = int(off[-1])
    cp = mpg.chaining_params()
    d_f = torch.empty(tot, dtype=torch.float64, device=dev)
    d_p = torch.empty(tot, dtype=torch.int32, device=dev)
    d_i = torch.empty(tot, dtype=torch.int32, device=dev)
    d_t = torch.empty(len(sets) * cp.max_chains * 16, dtype=torch.uint8, device=dev)
    d_n = torch.empty(len(sets), dtype=torch.int32, device=dev)
    ctx = mpg.Context(0)
    stream = torch.cuda.Stream(device=dev)
    ctx.set_stream(stream.cuda_stream)

    def step():
        ctx.chain_anchors_dev(cp, d_a.data_ptr(), off, d_f.data_ptr(), d_p.data_ptr(),
                              d_i.data_ptr(), d_t.data_ptr(), d_n.data_ptr())

    for w in range(args.warmup):
        step()
        ctx.sync()
        log("warmup %d done" % w)
    log("warmup: %d sets chained, best chain mean %.1f" % (
        int((d_n.cpu().numpy() > 0).sum()),
        float(np.frombuffer(d_t.cpu().numpy().tobytes(), dtype=mpg.CHAIN_OUT_DTYPE)["score"]
              .reshape(len(sets), cp.max_chains)[:, 0].mean())))
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev0.record(stream)
    for k in range(args.steps):
        step()
        log("step %d enqueued" % k)
    with torch.cuda.stream(stream):
        ev1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1) / args.steps
    ms_step = dt * 1e3 / args.steps
    rate = pairs / (dt / args.steps) / 1e9
    log("step %.3f ms (stream %.3f ms), %.2f G candidate pairs/s" % (ms_step, gpu_ms, rate))
    cpu = None
    if args.cpu_budget > 0:
        from oracle import chaining as C
        order = np.random.default_rng(12345).permutation(len(sets))
        k, done = 0, 0
        t1 = time.perf_counter()
        while k < len(order) and time.perf_counter() - t1 < args.cpu_budget:
            a = sets[order[k]]
            C.chain(a)
            done += len(a) * (len(a) - 1) // 2
            k += 1
        dt1 = time.perf_counter() - t1
        cpu = {"value": round(done / dt1 / 1e9, 5), "unit": "G candidate pairs/s", "cores": 1,
               "kind": "oracle",
               "sample": "%d of %d sets (seeded random order), %d pairs, %.1f s wall" % (
                   k, len(sets), done, dt1)}
        log("cpu baseline: %s" % json.dumps(cpu))
    line = {
        "metric": "chaining candidate pairs per second (fp64, Eq. gap / gap-pen)",
        "value": round(rate, 3), "unit": "G candidate pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (planted-gene seed hits plus spurious hits)",
        "config": {"workload": "chaining: 10,000 anchor sets, binned genome, k 6, G 200 kb, "
                               "beta 0.75, 30 chains", "sets": len(sets), "anchors": tot,
                   "candidate_pairs": pairs, "stream_ms_per_step": round(gpu_ms, 3)},
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_rescore(args):
    """Pseudogene guard on the traced 10,000-pair batch: the traced pass runs
    once before the timed region; one step is one mpg_rescore_spliced_dev
    (coding sequences cut on the GPU, the end-to-end second alignment, the
    final scores).  GCUPS count the second alignment's cells."""
    import torch
    from paper_2210_08052_amd import mpg
    from paper_2210_08052_amd import workloads as W
    t0 = time.time()
    pairs = W.batch_pairs(10000, seed=2)
    pb, db, segs = mpg.pack_pairs([(p.prot, p.dna, True) for p in pairs])
    log("workload rescore: %d pairs, generated in %.1f s" % (len(pairs), time.time() - t0))
    dev = torch.device("cuda:0")
    d_prot = torch.frombuffer(bytearray(pb), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db), dtype=torch.uint8).to(dev)
    cap = int(mpg.lib().mpg_ops_capacity(segs.ctypes.data, len(segs)))
    d_ops = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    d_out = torch.empty(len(pairs) * mpg.DEV_RESULT_DTYPE.itemsize, dtype=torch.uint8,
                        device=dev)
    n = len(pairs)
    fin = torch.empty(3 * n, dtype=torch.int32, device=dev)
    ctx = mpg.Context(0)
    stream = torch.cuda.Stream(device=dev)
    ctx.set_stream(stream.cuda_stream)
    p = mpg.params()
    ctx.align_batch_dev(p, d_prot.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(),
                        d_ops.data_ptr(), cap)
    ctx.sync()
    log("traced pass done")

    def step():
        ctx.rescore_spliced_dev(p, d_prot.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(),
                                d_ops.data_ptr(), fin.data_ptr(), fin.data_ptr() + 4 * n,
                                fin.data_ptr() + 8 * n)

    for w in range(args.warmup):
        step()
        ctx.sync()
        log("warmup %d done" % w)
    f = fin.cpu().numpy()
    ex = f[n:2 * n]
    log("warmup results: %d/%d ok, single-exon %d, mean exons %.2f" % (
        int((f[2 * n:] == 0).sum()), n, int((ex == 1).sum()), float(ex.mean())))
    ctx.enable_timing(True)
    ctx.timing(reset=True)
    torch.cuda.synchronize()
    ctx.sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step()
        ctx.sync()
        log("step %d done" % k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.timing(reset=True)
    cells = tim["cells"] // max(1, args.steps)
    ms_step = dt * 1e3 / args.steps
    gcups = cells / (dt / args.steps) / 1e9
    dp_ms = tim["dp_ms"] / max(1, args.steps)
    ops = OPS_PER_CELL["global_no_intron"]
    peak = PEAK_INT_OPS / 1e12
    achieved = cells * ops / (dp_ms * 1e-3) / 1e12
    log("step %.3f ms, GCUPS %.1f (%d cells); DP kernels %.3f ms/step, prepass %.3f ms, "
        "host %.3f ms" % (ms_step, gcups, cells, dp_ms, tim["prepass_ms"] / args.steps,
                          tim["host_ms"] / args.steps))
    line = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded planted genes)",
        "config": {"workload": "pseudogene guard on the traced 10,000-pair batch: coding-sequence "
                               "cut and end-to-end rescoring without introns",
                   "pairs": n, "cells": cells, "mode": "GLOBAL, no intron states"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": "Tops/s (int32 lane-ops)", "frac": round(achieved / peak, 4),
                     "traffic": None, "kernel_gcups": round(cells / (dp_ms * 1e-3) / 1e9, 2),
                     "ops_per_cell": ops, "dp_ms_per_step": round(dp_ms, 3)},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


# Arrival rate of the serving workload (jobs/s): 0.7 x the batched capacity
# (one mpg_align_batch call over the first 20,000 jobs of the same stream,
# measured by ``--config serving --calibrate``), rounded to two significant
# digits and frozen here.
SERVING_RATE = 24000.0  # 0.7 x 34,233 jobs/s: batched capacity of the first 20,000 jobs on MI355X
LONG_REGION = 50000  # regions above this length come from the long-tail mixture
SERVING_TB_BUDGET = 96 << 30  # device bytes for traceback direction bits while serving


def end_to_end_ms(mpg, ctx, pairs, tb, p, reps=2):
    """Best of `reps` wall times of one mpg_align_batch over host buffers:
    sequences copied to the device, records and op strings copied back (the
    PCIe-inclusive time; never the headline value)."""
    import ctypes
    n = len(pairs)
    arr = (mpg.mpg_pair * n)()
    for k, q in enumerate(pairs):
        arr[k].prot, arr[k].plen = q.prot, len(q.prot)
        arr[k].dna, arr[k].dlen = q.dna, len(q.dna)
        arr[k].flags = mpg.MPG_WANT_TB if tb else 0
    out = (mpg.mpg_result * n)()
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        mpg.check(mpg.lib().mpg_align_batch(ctx.ptr, ctypes.byref(p), arr, n, out),
                  "mpg_align_batch")
        best = min(best, time.perf_counter() - t)
        mpg.lib().mpg_result_release(ctx.ptr, out, n)
    return best * 1e3


def _percentiles(x):
    if len(x) == 0:
        return None
    q = np.percentile(np.asarray(x, dtype=np.float64), [50, 99])
    return {"p50_ms": round(float(q[0]), 3), "p99_ms": round(float(q[1]), 3), "n": int(len(x))}


def run_served(mpg, p, jobs, arrivals_s, keep=(), log_every=20000):
    """Open-loop submission of jobs at their arrival times (seconds from t0)
    into a serving context.  Returns (t0_ns, due_ns, done_ns, submit_ns,
    status, kept results, stats); kept results are the full results of the
    job indices in `keep`."""
    import threading
    srv = mpg.Context(0, tb_budget_bytes=SERVING_TB_BUDGET)
    # warm-up: a few short jobs through the same context
    nw = min(64, len(jobs))
    for q in jobs[:nw]:
        srv.submit(p, q.prot, q.dna, want_tb=q.want_tb)
    got = 0
    while got < nw:
        got += len(srv.poll(256, 100000))
    base = nw + 1  # job ids are consecutive from 1 in a fresh context
    n = len(jobs)
    done_ns = np.zeros(n, dtype=np.int64)
    sub_ns = np.zeros(n, dtype=np.int64)
    status = np.zeros(n, dtype=np.int32)
    kept = {}
    keep_ids = set(int(k) + base for k in keep)
    t0 = time.monotonic_ns() + 20_000_000
    due = t0 + np.round(np.asarray(arrivals_s) * 1e9).astype(np.int64)
    finished = threading.Event()

    def poller():
        cnt = 0
        while cnt < n:
            res, full = srv.poll_raw(4096, 20000, keep_ids)
            for jid, ta, td, st in res:
                k = jid - base
                done_ns[k] = td
                sub_ns[k] = ta
                status[k] = st
                cnt += 1
                if cnt % log_every == 0:
                    log("served %d/%d" % (cnt, n))
            for jid, r in full.items():
                kept[jid - base] = r
        finished.set()

    th = threading.Thread(target=poller, daemon=True)
    th.start()
    for k, q in enumerate(jobs):
        wait = int(due[k]) - time.monotonic_ns()
        if wait > 300_000:
            time.sleep((wait - 200_000) / 1e9)
        while time.monotonic_ns() < due[k]:
            pass
        while True:
            jid = srv.submit(p, q.prot, q.dna, want_tb=q.want_tb)
            if jid >= 0:
                if jid != base + k:
                    raise RuntimeError("unexpected job id %d for job %d" % (jid, k))
                break
            if jid != mpg.MPG_E_AGAIN:
                raise RuntimeError("mpg_submit failed: %d" % jid)
            time.sleep(1e-4)
    finished.wait()
    stats = srv.stats()
    srv.close()
    return t0, due, done_ns, sub_ns, status, kept, stats


def bench_serving(args):
    import torch  # noqa: F401  (one HIP runtime for torch and the library)
    from paper_2210_08052_amd import mpg
    from paper_2210_08052_amd import workloads as W
    n = args.jobs
    t_gen = time.time()
    jobs, arr1 = W.serving_jobs(n, rate_per_s=1.0, seed=5,
                                progress=lambda k: log("generated %d jobs" % k),
                                workers=min(16, len(os.sched_getaffinity(0))))
    log("serving workload: %d jobs generated in %.1f s" % (n, time.time() - t_gen))
    cells = np.array([len(q.prot) * len(q.dna) for q in jobs], dtype=np.float64)
    is_long = np.array([len(q.dna) > LONG_REGION for q in jobs])
    is_tb = np.array([q.want_tb for q in jobs])
    p = mpg.params()
    if args.calibrate:
        # batched capacity: the first 20,000 jobs as one mpg_align_batch call
        m = min(20000, n)
        sample = [(q.prot, q.dna, q.want_tb) for q in jobs[:m]]
        with mpg.Context(0) as ctx:
            ctx.align_batch(sample[:200], p)
            tc = time.perf_counter()
            ctx.align_batch(sample, p)
            span_b = time.perf_counter() - tc
        cap = m / span_b
        rate = float("%.2g" % (0.7 * cap))
        log("batched capacity %.1f jobs/s (%.1f GCUPS) on %d jobs; 0.7x = %.4g jobs/s" % (
            cap, cells[:m].sum() / span_b / 1e9, m, rate))
        # for comparison: the same jobs submitted at once through the serving path
        t0, due, done, _, _, _, st = run_served(mpg, p, jobs[:m], np.zeros(m))
        span_s = (done.max() - t0) / 1e9
        log("serving drain %.1f jobs/s (%.1f GCUPS)" % (m / span_s, cells[:m].sum() / span_s / 1e9))
        print(json.dumps({"calibration": {"jobs": m, "batched_s": round(span_b, 3),
                                          "batched_jobs_per_s": round(cap, 1),
                                          "serving_drain_s": round(span_s, 3),
                                          "rate_jobs_per_s": rate}}), flush=True)
        return
    rate = args.rate or SERVING_RATE
    if not rate:
        raise SystemExit("no arrival rate: run --config serving --calibrate first or pass --rate")
    arrivals = arr1 / rate
    rng = np.random.default_rng(7)
    if args.check <= 0 or args.check >= n:
        sample = np.arange(n)
    else:
        sample = np.sort(rng.choice(n, size=args.check, replace=False))
    t0, due, done, subm, status, kept, st = run_served(mpg, p, jobs, arrivals, keep=sample)
    lat = (done - due) / 1e6
    lag = (subm - due) / 1e6
    bad = int((status != 0).sum())
    keep = np.arange(n) >= int(0.05 * n)  # drop the first 5% (warm-up)
    span = (done.max() - t0) / 1e9
    served = {
        "all": _percentiles(lat[keep]),
        "short": _percentiles(lat[keep & ~is_long]),
        "long": _percentiles(lat[keep & is_long]),
        "traceback": _percentiles(lat[keep & is_tb]),
        "score_only": _percentiles(lat[keep & ~is_tb]),
    }
    gcups = cells.sum() / span / 1e9
    log("served %d jobs in %.2f s: %.1f GCUPS, latency %s" % (n, span, gcups, served["all"]))

    # the same jobs, one pair per launch, first come first served, on the
    # same GPU and arrival times, for a bounded time
    base = mpg.Context(0)
    bl, bcells, bk = [], 0.0, 0
    bt0 = time.monotonic_ns()
    bdue = bt0 + np.round(arrivals * 1e9).astype(np.int64)
    busy = 0.0
    while bk < n and (time.monotonic_ns() - bt0) / 1e9 < args.baseline_budget:
        now = time.monotonic_ns()
        if now < bdue[bk]:
            time.sleep((bdue[bk] - now) / 1e9)
        q = jobs[bk]
        ts = time.monotonic_ns()
        r = base.align_batch([(q.prot, q.dna, q.want_tb)], p)[0]
        te = time.monotonic_ns()
        busy += (te - ts) / 1e9
        if r["status"] != 0:
            bad += 1
        bl.append((te - bdue[bk]) / 1e6)
        bcells += cells[bk]
        bk += 1
    base.close()
    baseline = {"jobs": bk, "latency": _percentiles(bl),
                "sustained_jobs_per_s": round(bk / busy, 1) if busy else None,
                "sustained_gcups": round(bcells / busy / 1e9, 2) if busy else None,
                "saturated": bool(bk < n and bdue[bk] < time.monotonic_ns())}
    log("one-pair-per-launch: %s" % json.dumps(baseline))

    # served results equal batched results for the same jobs (every job, or a
    # seeded sample)
    tcheck = time.perf_counter()
    with mpg.Context(0) as ctx:
        ref = ctx.align_batch([(jobs[k].prot, jobs[k].dna, jobs[k].want_tb) for k in sample], p)
    keys = ("status", "score", "g_beg", "g_end", "p_beg", "p_end", "ops")
    mism = sum(1 for k, r in zip(sample, ref)
               if k not in kept or any(kept[k][f] != r[f] for f in keys))
    log("served vs batched: %d of %d jobs differ (%.1f s)" % (mism, len(sample),
                                                         time.perf_counter() - tcheck))
    line = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(span * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded planted genes)",
        "config": {"workload": "serving: %d jobs, Poisson arrivals at %.4g jobs/s, 90/10 batch/"
                               "long-tail mixture, 50%% traceback, LOCAL" % (n, rate),
                   "jobs": n, "cells": float(cells.sum()), "rate_jobs_per_s": rate,
                   "tb_budget_bytes": SERVING_TB_BUDGET},
        "latency": served,
        "submit_lag_ms": _percentiles(lag[keep]),
        "failed_jobs": bad,
        "served_vs_batched_mismatches": {"checked": int(len(sample)), "mismatches": mism},
        "one_pair_per_launch": baseline,
        "serving_stats": st,
        "gpu_max_hw_queues": os.environ.get("GPU_MAX_HW_QUEUES"),
    }
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="all",
                    help="all (default: batch as the headline, then traceback, longtail and "
                         "serving legs), batch, batch16, traceback, single, longtail, serving, "
                         "profile, chain, chaining, rescore")
    ap.add_argument("--tb-budget-gib", type=float, default=None,
                    help="traceback budget of the context in GiB (default: 240 for longtail, "
                         "whose direction bits total ~250 GB, so they fit one wave; else "
                         "the library's 64)")
    ap.add_argument("--cpu-budget", type=float, default=15.0,
                    help="seconds of oracle work for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibrate", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--jobs", type=int, default=200000, help="serving: number of jobs")
    ap.add_argument("--rate", type=float, default=0.0, help="serving: arrival rate override")
    ap.add_argument("--calibrate", action="store_true",
                    help="serving: measure the batched capacity on the first 20,000 jobs")
    ap.add_argument("--baseline-budget", type=float, default=20.0,
                    help="serving: seconds of one-pair-per-launch baseline")
    ap.add_argument("--check", type=int, default=0,
                    help="serving: jobs re-run as a batch and compared (0 = all)")
    args = ap.parse_args()
    if args.copy_calibrate:
        import torch
        src = torch.ones(1 << 30, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied 3 x 1 GiB")
        return
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: pairs are independent, so a batch shards "
              "across GPUs with no exchange, and the figure here is one GPU's share.",
              file=sys.stderr)
        sys.exit(2)

    if args.config == "chain":
        bench_chains(args)
        return
    if args.config == "profile":
        bench_profiles(args)
        return
    if args.config == "chaining":
        bench_chaining(args)
        return
    if args.config == "rescore":
        bench_rescore(args)
        return

    if args.config in ("serving", "all"):
        # the serving scheduler runs several streams at once; give them
        # hardware queues of their own (read when the HIP runtime starts,
        # which is after this point: torch is imported later).  The record
        # states the value in effect.
        os.environ["GPU_MAX_HW_QUEUES"] = "16"
    if args.config == "serving":
        line = bench_serving(args)
        if line is not None:
            print(json.dumps(line), flush=True)
        return

    import torch
    from paper_2210_08052_amd import mpg

    if args.config != "all":
        leg = run_batch_leg(mpg, torch, args.config, args.steps, args.warmup, args.cpu_budget,
                            args.tb_budget_gib)
        print(json.dumps(leg), flush=True)
        return

    # every workload of the metric: the 10,000-pair batch (the headline), the
    # same pairs with traceback, the serving stream and the long-tail batch.
    # Serving runs before the long-tail leg: right after the long-tail's ~250 GB
    # of direction bits are freed, the device is slow to serve new work for
    # about a second (serving p99 973 ms against 6.9 ms when run alone).
    t_all = time.time()
    line = run_batch_leg(mpg, torch, "batch", args.steps, args.warmup, args.cpu_budget, None)
    legs = {}

    def batch_leg(name, steps):
        leg = run_batch_leg(mpg, torch, name, steps, 1, 0.0, None, e2e=False)
        legs[name] = leg_summary(leg)
        log("%s leg: %s" % (name, json.dumps(legs[name])))

    batch_leg("traceback", min(args.steps, 10))
    args.baseline_budget = min(args.baseline_budget, 10.0)
    legs["serving"] = bench_serving(args)
    batch_leg("longtail", min(args.steps, 3))
    line["legs"] = legs
    line["wall_s_all_legs"] = round(time.time() - t_all, 1)
    print(json.dumps(line), flush=True)


def leg_summary(leg):
    """The fields of a batch leg that the combined line carries."""
    r = leg["roofline"]
    return {"workload": leg["config"]["workload"], "pairs": leg["config"]["pairs"],
            "cells": leg["config"]["cells"], "steps": leg["steps"], "warmup": leg["warmup"],
            "ms_per_step": leg["ms_per_step"], "gcups": leg["value"],
            "kernel_gcups": r["kernel_gcups"], "dp_ms_per_step": r["dp_ms_per_step"],
            "roofline_frac": r["frac"], "ops_per_cell": r["ops_per_cell"],
            "traffic": r["traffic"], "autotune": leg["autotune"],
            "tb_budget_gib": leg["config"].get("tb_budget_gib")}


def dev_results(mpg, d_out, d_ops, n, tb):
    """Result dicts of a device-resident call (records and op strings)."""
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)[:n]
    ops = d_ops.cpu().numpy().tobytes() if tb else b""
    res = []
    for k in range(n):
        r = {f: int(out[f][k]) for f in ("status", "score", "g_beg", "g_end", "p_beg", "p_end")}
        r["ops"] = None
        if tb and r["status"] == 0:
            o0, ln = int(out["ops_off"][k]), int(out["ops_len"][k])
            r["ops"] = ops[o0:o0 + ln].decode()
        res.append(r)
    return res


def run_batch_leg(mpg, torch, config, steps, warmup, cpu_budget, tb_budget_gib, e2e=True):
    """One batch workload: sequences resident in HBM, the strip width tuned on
    the workload itself, `warmup` untimed and `steps` timed calls of
    mpg_align_batch_dev, each synchronised.  Returns its JSON line."""
    t0 = time.time()
    pairs, tb, desc = build_workload(config)
    log("workload %s: %d pairs, generated in %.1f s" % (config, len(pairs), time.time() - t0))
    cells = int(sum(len(p.prot) * len(p.dna) for p in pairs))
    pb, db, segs = mpg.pack_pairs([(p.prot, p.dna, tb) for p in pairs])

    dev = torch.device("cuda:0")
    d_prot = torch.frombuffer(bytearray(pb), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db), dtype=torch.uint8).to(dev)
    cap = int(mpg.lib().mpg_ops_capacity(segs.ctypes.data, len(segs)))
    d_ops = torch.empty(max(cap, 1), dtype=torch.uint8, device=dev)
    d_out = torch.empty(len(pairs) * mpg.DEV_RESULT_DTYPE.itemsize, dtype=torch.uint8,
                        device=dev)
    budget_gib = tb_budget_gib
    if budget_gib is None:
        budget_gib = 240.0 if config == "longtail" else 0.0
    ctx = mpg.Context(0, tb_budget_bytes=int(budget_gib * (1 << 30)))
    stream = torch.cuda.Stream(device=dev)
    ctx.set_stream(stream.cuda_stream)
    i16 = config == "batch16"
    p = mpg.params(flags=mpg.MPG_ALLOW_I16) if i16 else mpg.params()
    # kernel width from timed runs of this very workload
    tuning = ctx.autotune(p, d_prot.data_ptr(), d_dna.data_ptr(), segs)
    log("autotune: %s" % json.dumps(tuning))

    def step():
        ctx.align_batch_dev(p, d_prot.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(),
                            d_ops.data_ptr(), cap)

    for w in range(warmup):
        step()
        ctx.sync()
        log("warmup %d done" % w)
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)
    n_ok = int((out["status"] == 0).sum())
    log("warmup results: %d/%d ok, score sum %d" % (n_ok, len(out), int(out["score"].sum())))

    ctx.enable_timing(True)
    ctx.timing(reset=True)
    torch.cuda.synchronize()
    ctx.sync()
    t0 = time.perf_counter()
    for k in range(steps):
        step()
        ctx.sync()
        log("step %d done" % k)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    tim = ctx.timing(reset=True)
    ms_step = dt * 1e3 / steps
    gcups = cells / (dt / steps) / 1e9
    dp_ms = tim["dp_ms"] / max(1, steps)
    if i16:
        # 27 packed int16 operations advance two cells: 27 int16 lane-ops per
        # cell against twice the int32 lane rate
        ops = 27
        peak = 2 * PEAK_INT_OPS / 1e12
        runit = "Tops/s (int16 lane-ops)"
        if tim["i16_pairs"] != len(pairs) * steps:
            raise SystemExit("int16 kernel ran %d pairs, expected %d" % (
                tim["i16_pairs"], len(pairs) * steps))
    else:
        ops = OPS_PER_CELL["traceback" if tb else "score"]
        peak = PEAK_INT_OPS / 1e12
        runit = "Tops/s (int32 lane-ops)"
    achieved = cells * ops / (dp_ms * 1e-3) / 1e12
    kernel_gcups = cells / (dp_ms * 1e-3) / 1e9
    log("step %.3f ms, GCUPS %.1f; DP kernels %.3f ms/step (%.1f GCUPS), prepass %.3f ms, "
        "walk %.3f ms, host %.3f ms" % (ms_step, gcups, dp_ms, kernel_gcups,
                                        tim["prepass_ms"] / steps, tim["walk_ms"] / steps,
                                        tim["host_ms"] / steps))
    # the last timed step's results, for the oracle comparison
    gpu_res = dev_results(mpg, d_out, d_ops, len(pairs), tb) if cpu_budget > 0 else None

    e2e_ms = None
    if e2e:
        e2e_ms = end_to_end_ms(mpg, ctx, pairs, tb, p)
        log("end to end over host buffers: %.3f ms (%.1f GCUPS)" % (
            e2e_ms, cells / (e2e_ms * 1e-3) / 1e9))
    ctx.close()
    del d_prot, d_dna, d_ops, d_out
    torch.cuda.empty_cache()

    cpu = None
    if cpu_budget > 0:
        cpu = cpu_baseline(pairs, tb, cpu_budget, gpu=gpu_res)
        log("cpu baseline: %s" % json.dumps(cpu))

    line = {
        "metric": METRIC, "value": round(gcups, 2), "unit": "GCUPS", "n_gpus": 1,
        "steps": steps, "warmup": warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int16" if i16 else "int32",
        "data": "synthetic (seeded planted genes)",
        "config": {"workload": desc, "pairs": len(pairs), "cells": cells,
                   "traceback": tb, "mode": "LOCAL"},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                     "unit": runit, "frac": round(achieved / peak, 4),
                     "traffic": recorded_traffic(config), "kernel_gcups": round(kernel_gcups, 2),
                     "ops_per_cell": ops,
                     "dp_ms_per_step": round(dp_ms, 3)},
        "cpu_baseline": cpu,
        "autotune": tuning,
    }
    if budget_gib:
        line["config"]["tb_budget_gib"] = budget_gib
    if e2e_ms is not None:
        line["end_to_end"] = {"ms": round(e2e_ms, 3),
                              "gcups": round(cells / (e2e_ms * 1e-3) / 1e9, 2),
                              "what": "one mpg_align_batch over host buffers (sequences in, "
                                      "records and op strings out over PCIe)"}
    return line


if __name__ == "__main__":
    main()
