"""Shared helpers for the GPU parity tests: run the same inputs through the
HIP library (C ABI) and the CPU oracle and compare element by element.

Scoring inputs never flow from one side to the other: default parameters come
from each side's own defaults (their equality is a CPU test), random ones from
the neutral input generator."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import params as oparams
from paper_2210_08052_amd import mpg
from paper_2210_08052_amd import workloads as W


def scorings(mode=0, flags=0, rand_seed=None):
    """(gpu params, oracle Scoring) for the same scoring inputs."""
    oflags = flags & 3  # the oracle knows only NO_INTRON and NO_FRAMESHIFT
    if rand_seed is None:
        return (mpg.params(mode=mode, flags=flags),
                oparams.default_scoring(mode=mode, flags=oflags))
    r = W.random_scoring(rand_seed)
    g = mpg.params(mode=mode, flags=flags, q=r["q"], e=r["e"], f=r["f"], r=r["r"],
                   mat=r["mat"], donor=r["donor"], acceptor=r["acceptor"])
    o = oparams.default_scoring(mode=mode, flags=oflags, q=r["q"], e=r["e"], f=r["f"],
                                r=r["r"], mat=r["mat"], donor=r["donor"],
                                acceptor=r["acceptor"])
    return g, o


def key_gpu(r, tb):
    if r["status"] == mpg.MPG_E_NOALN:
        return ("noaln",)
    assert r["status"] == 0, r
    if tb:
        return (r["score"], r["g_beg"], r["g_end"], r["p_beg"], r["p_end"], r["ops"])
    return (r["score"], r["g_end"], r["p_end"])


def key_orc(r, tb):
    if r.status == oracle.E_NOALN:
        return ("noaln",)
    if tb:
        return (r.score, r.g_beg, r.g_end, r.p_beg, r.p_end, r.ops)
    return (r.score, r.g_end, r.p_end)


def compare(ctx, pairs, gpar, opar, tb, threads=0, label=""):
    """Align pairs [(prot, dna), ...] on both sides; assert equality."""
    got = ctx.align_batch([(p, d, tb) for p, d in pairs], gpar)
    exp = oracle.align_many(pairs, opar, want_tb=tb, threads=threads)
    bad = []
    for k, (g, e) in enumerate(zip(got, exp)):
        if key_gpu(g, tb) != key_orc(e, tb):
            bad.append((k, key_gpu(g, tb), key_orc(e, tb), len(pairs[k][0]), len(pairs[k][1])))
    assert not bad, "%s: %d/%d mismatches, first: %s" % (label, len(bad), len(pairs), bad[:3])
    return got
