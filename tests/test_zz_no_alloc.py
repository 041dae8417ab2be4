"""The allocation-free batch entry point (mpg_align_batch_dev_noalloc) against
mpg_align_batch_dev on the same device-resident inputs: identical records and
op strings on two calls in a row, the second with a smaller input (the fixed
scratch array then still holds the first call's leftovers), and a clear
MPG_E_RANGE, with nothing written, for a call beyond the array's size."""
import numpy as np
import pytest

from paper_2210_08052_amd import mpg
from paper_2210_08052_amd import workloads as W

pytestmark = pytest.mark.gpu


def _upload(jobs):
    import torch
    dev = torch.device("cuda:0")
    pb, db, segs = mpg.pack_pairs(jobs)
    d_prot = torch.frombuffer(bytearray(pb + b"\0"), dtype=torch.uint8).to(dev)
    d_dna = torch.frombuffer(bytearray(db + b"\0"), dtype=torch.uint8).to(dev)
    cap = int(mpg.lib().mpg_ops_capacity(segs.ctypes.data, len(segs)))
    return d_prot, d_dna, segs, cap


def _run(ctx, entry, g, d_prot, d_dna, segs, cap, fill):
    """Records and op strings of one call; the output buffers start filled
    with `fill` so that untouched bytes show."""
    import torch
    dev = torch.device("cuda:0")
    n = len(segs)
    d_out = torch.full((n * mpg.DEV_RESULT_DTYPE.itemsize,), fill, dtype=torch.uint8, device=dev)
    d_ops = torch.full((max(cap, 1),), fill, dtype=torch.uint8, device=dev)
    rc = entry(g, d_prot.data_ptr(), d_dna.data_ptr(), segs, d_out.data_ptr(), d_ops.data_ptr(),
               cap)
    ctx.sync()
    out = np.frombuffer(d_out.cpu().numpy().tobytes(), dtype=mpg.DEV_RESULT_DTYPE)
    return rc, out, d_ops.cpu().numpy().tobytes()


def _results(out, ops, segs, p):
    res = []
    for k in range(len(out)):
        tb = bool((int(segs["flags"][k]) | p.flags) & mpg.MPG_WANT_TB)
        r = tuple(int(out[f][k]) for f in ("status", "score", "g_beg", "g_end", "p_beg", "p_end"))
        if tb and r[0] == 0:
            o0, ln = int(out["ops_off"][k]), int(out["ops_len"][k])
            r += (ops[o0:o0 + ln], ops[o0 + ln])
        res.append(r)
    return res


def _entry_ref(ctx):
    def call(*a):
        ctx.align_batch_dev(*a)
        return 0
    return call


@pytest.mark.parametrize("flags", [0, mpg.MPG_ALLOW_I16])
def test_noalloc_equals_batch_dev_twice(flags):
    big = [(p.prot, p.dna, k % 4 == 0) for k, p in enumerate(W.batch_pairs(40, seed=31))]
    small = [(p, d, k % 3 == 0) for k, (p, d) in enumerate(
        (q.prot, q.dna) for q in W.random_pairs(12, 32, max_prot=300, max_dna=1500))]
    g = mpg.params(flags=flags)
    with mpg.Context(0) as ctx:
        for label, jobs in (("first, larger", big), ("second, smaller", small)):
            print("case noalloc flags=%d %s: %d pairs" % (flags, label, len(jobs)), flush=True)
            d_prot, d_dna, segs, cap = _upload(jobs)
            rc0, ref, ops0 = _run(ctx, _entry_ref(ctx), g, d_prot, d_dna, segs, cap, 0xA5)
            rc1, got, ops1 = _run(ctx, ctx.align_batch_dev_noalloc, g, d_prot, d_dna, segs, cap,
                                  0x5A)
            assert rc0 == 0 and rc1 == 0, (rc0, rc1)
            a, b = _results(ref, ops0, segs, g), _results(got, ops1, segs, g)
            assert all(r[0] == 0 for r in a), label
            diff = [k for k in range(len(a)) if a[k] != b[k]]
            assert not diff, "%s: %d of %d differ, first %s vs %s" % (
                label, len(diff), len(a), a[diff[0]], b[diff[0]])


def test_noalloc_rejects_beyond_scratch():
    """A traceback pair whose direction bits alone exceed the scratch array:
    MPG_E_RANGE before anything is enqueued; the next call still works."""
    rng = np.random.default_rng(33)
    prot = "".join(rng.choice(list("ACDEFGHIKLMNPQRSTVWY"), size=3000)).encode()
    dna = "".join(rng.choice(list("ACGT"), size=30000)).encode()
    assert 3000 * 30000 * 9 // 8 > mpg.MPG_NOALLOC_SCRATCH_BYTES
    g = mpg.params()
    with mpg.Context(0) as ctx:
        d_prot, d_dna, segs, cap = _upload([(prot, dna, True)])
        rc, out, ops = _run(ctx, ctx.align_batch_dev_noalloc, g, d_prot, d_dna, segs, cap, 0x77)
        assert rc == mpg.MPG_E_RANGE
        assert set(out.tobytes()) == {0x77} and set(ops) == {0x77}
        assert "range" in mpg.strerror(rc).lower() or "limit" in mpg.strerror(rc).lower()
        jobs = [(q.prot, q.dna, True) for q in W.random_pairs(5, 34, max_prot=200, max_dna=900)]
        d_prot, d_dna, segs, cap = _upload(jobs)
        _, ref, ops0 = _run(ctx, _entry_ref(ctx), g, d_prot, d_dna, segs, cap, 0)
        rc1, got, ops1 = _run(ctx, ctx.align_batch_dev_noalloc, g, d_prot, d_dna, segs, cap, 1)
        assert rc1 == 0
        assert _results(ref, ops0, segs, g) == _results(got, ops1, segs, g)
