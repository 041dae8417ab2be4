"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times (sequences resident in HBM, one mpg_align_batch_dev call over
the whole batch, the strip width autotuned on the batch itself), compared
with the oracle element by element: status, score, begin and end cells, and
the op string for traced pairs.

* The 10,000-pair planted batch: every pair, score-only and with traceback.
* The long-tail batch: 200 pairs of 3,000-8,000 residues x 100-300 kb plus
  2,000 short ones in one call under a 240 GiB direction-bit budget (one
  wave, as bench.py runs it).  The
  oracle traces every short pair and a seeded sample of 20 long pairs (it
  stores two bytes per cell, so its concurrency is capped by host memory);
  every long pair's traced path is rescored by the oracle's rescorer, and the
  score-only run must agree with the traced one on all 2,200 pairs."""
import os
import time

import numpy as np
import pytest

import oracle
from oracle.rescore import rescore
from paper_2210_08052_amd import mpg
from paper_2210_08052_amd import workloads as W

from _cases import key_gpu, key_orc

pytestmark = pytest.mark.gpu


def _run_dev(ctx, pairs, tb, p, tune=True):
    """One device-resident call over all pairs, as bench.py runs it."""
    import torch
    dev = torch.device("cuda:0")
    pb, db, segs = mpg.pack_pairs([(q.prot, q.dna, tb) for q in pairs])
    d_prot = torch.frombuffer(bytearray(pb), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db), dtype=torch.uint8).to(dev)
    cap = int(mpg.lib().mpg_ops_capacity(segs.ctypes.data, len(segs)))
    d_ops = torch.zeros(max(cap, 1), dtype=torch.uint8, device=dev)
    d_out = torch.zeros(len(pairs) * mpg.DEV_RESULT_DTYPE.itemsize, dtype=torch.uint8,
                        device=dev)
    if tune:
        ctx.autotune(p, d_prot.data_ptr(), d_dna.data_ptr(), segs)
    ctx.align_batch_dev(p, d_prot.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(),
                        d_ops.data_ptr(), cap)
    ctx.sync()
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)
    ops = d_ops.cpu().numpy().tobytes() if tb else b""
    res = []
    for k in range(len(pairs)):
        r = {f: int(out[f][k]) for f in ("status", "score", "g_beg", "g_end", "p_beg", "p_end")}
        r["ops"] = None
        if tb and r["status"] == 0:
            o0, ln = int(out["ops_off"][k]), int(out["ops_len"][k])
            r["ops"] = ops[o0:o0 + ln].decode()
        res.append(r)
    return res


def _mem_available():
    try:
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemAvailable:"):
                return int(ln.split()[1]) * 1024
    except OSError:
        pass
    return 16 << 30


def _oracle_threads(max_cells):
    """Threads for oracle traceback runs: all cores, capped so that every
    thread's two bytes per cell fit half the available host memory."""
    cores = len(os.sched_getaffinity(0))
    per = 2 * max_cells + (64 << 20)
    return max(1, min(cores, int(0.5 * _mem_available() // per)))


def _mismatches(got, exp, tb, idx=None):
    idx = range(len(exp)) if idx is None else idx
    bad = []
    for k, e in zip(idx, exp):
        if key_gpu(got[k], tb) != key_orc(e, tb):
            bad.append((int(k), key_gpu(got[k], tb)[:5], key_orc(e, tb)[:5]))
    return bad


@pytest.mark.timeout(900)
def test_batch_10k_every_pair():
    """All 10,000 planted pairs: GPU score-only and traceback against the
    oracle's traceback run (which also fixes score and end cell)."""
    pairs = W.batch_pairs(10000, seed=2)
    p = mpg.params()
    with mpg.Context(0) as ctx:
        so = _run_dev(ctx, pairs, False, p)
        tb = _run_dev(ctx, pairs, True, p)
    t0 = time.time()
    exp = oracle.align_many([(q.prot, q.dna) for q in pairs], oracle.default_scoring(),
                            want_tb=True,
                            threads=_oracle_threads(max(q.cells for q in pairs)))
    print("oracle traced 10,000 pairs in %.1f s" % (time.time() - t0), flush=True)
    bad_so = _mismatches(so, exp, False)
    bad_tb = _mismatches(tb, exp, True)
    assert not bad_so, "score-only: %d of 10000 differ, first %s" % (len(bad_so), bad_so[:3])
    assert not bad_tb, "traceback: %d of 10000 differ, first %s" % (len(bad_tb), bad_tb[:3])


@pytest.mark.timeout(900)
def test_long_tail_full_size_against_oracle():
    pairs = W.long_tail(200, 2000, seed=4)
    p = mpg.params()
    with mpg.Context(0, tb_budget_bytes=240 << 30) as ctx:
        tb = _run_dev(ctx, pairs, True, p)
        so = _run_dev(ctx, pairs, False, p, tune=False)
    is_long = np.array([len(q.prot) >= 3000 for q in pairs])
    assert is_long.sum() == 200
    for k, (a, b) in enumerate(zip(tb, so)):
        assert a["status"] == b["status"] == 0, k
        assert (a["score"], a["g_end"], a["p_end"]) == (b["score"], b["g_end"], b["p_end"]), k
    # every long pair's path: valid, ends at the reported cell, scores the
    # reported score
    sc = oracle.default_scoring()
    for k in np.flatnonzero(is_long):
        q, r = pairs[k], tb[k]
        s, ge, pe = rescore(q.prot.decode(), q.dna.decode(), sc, r["g_beg"], r["p_beg"], r["ops"])
        assert (s, ge, pe) == (r["score"], r["g_end"], r["p_end"]), int(k)
    # the oracle traces a seeded sample of 20 long pairs and every short pair
    rng = np.random.default_rng(2024)
    longs = np.sort(rng.choice(np.flatnonzero(is_long), size=20, replace=False))
    shorts = np.flatnonzero(~is_long)
    t0 = time.time()
    th = _oracle_threads(max(pairs[k].cells for k in longs))
    exp_long = oracle.align_many([(pairs[k].prot, pairs[k].dna) for k in longs], sc,
                                 want_tb=True, threads=th)
    print("oracle traced 20 long pairs (%.3g cells) in %.1f s on %d threads" % (
        sum(pairs[k].cells for k in longs), time.time() - t0, th), flush=True)
    exp_short = oracle.align_many([(pairs[k].prot, pairs[k].dna) for k in shorts], sc,
                                  want_tb=True)
    bad = _mismatches(tb, exp_long, True, longs) + _mismatches(tb, exp_short, True, shorts)
    assert not bad, "%d of %d differ, first %s" % (len(bad), len(longs) + len(shorts), bad[:3])
