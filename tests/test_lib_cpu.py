"""CPU-side checks of the C-ABI library: it loads, exports every declared
symbol, its host-only calls behave, and its default scoring inputs equal the
oracle's independently written ones.  No GPU is touched here."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import params as oparams
from paper_2210_08052_amd import mpg
from paper_2210_08052_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "mpg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpg_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = mpg.lib()
    names = declared_functions()
    assert len(names) >= 15
    for nm in names:
        assert hasattr(L, nm), nm
    assert sorted(mpg.EXPORTS) == names


def test_struct_layouts(tmp_path):
    """ctypes mirrors match the C compiler's layout of include/mpg.h."""
    import subprocess
    structs = {"mpg_params": mpg.mpg_params, "mpg_pair": mpg.mpg_pair,
               "mpg_result": mpg.mpg_result, "mpg_seg": mpg.mpg_seg,
               "mpg_dev_result": mpg.mpg_dev_result, "mpg_stats": mpg.mpg_stats,
               "mpg_timing": mpg.mpg_timing, "mpg_tuning": mpg.mpg_tuning,
               "mpg_chain": mpg.mpg_chain, "mpg_chain_seg": mpg.mpg_chain_seg,
               "mpg_profile_pair": mpg.mpg_profile_pair,
               "mpg_profile_seg": mpg.mpg_profile_seg,
               "mpg_chaining_params": mpg.mpg_chaining_params,
               "mpg_chain_out": mpg.mpg_chain_out}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mpg.h"', 'int main(void){']
    for nm, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (nm, nm))
        for f, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (nm, f, nm, f))
    lines.append("return 0;}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = dict(ln.split() for ln in subprocess.check_output([str(exe)]).decode().splitlines())
    for nm, cls in structs.items():
        assert int(got[nm]) == ctypes.sizeof(cls), nm
        for f, _ in cls._fields_:
            assert int(got[nm + "." + f]) == getattr(cls, f).offset, (nm, f)
    assert mpg.SEG_DTYPE.itemsize == ctypes.sizeof(mpg.mpg_seg)
    assert mpg.DEV_RESULT_DTYPE.itemsize == ctypes.sizeof(mpg.mpg_dev_result)
    for f, _ in mpg.mpg_seg._fields_:
        assert mpg.SEG_DTYPE.fields[f][1] == getattr(mpg.mpg_seg, f).offset
    for f, _ in mpg.mpg_dev_result._fields_:
        assert mpg.DEV_RESULT_DTYPE.fields[f][1] == getattr(mpg.mpg_dev_result, f).offset


def test_default_params_equal_oracle_defaults():
    g = mpg.params_arrays(mpg.params())
    o = oparams.default_scoring()
    assert (g["q"], g["e"], g["f"], g["r"], g["mode"], g["flags"]) == (o.q, o.e, o.f, o.r, 0, 0)
    assert (g["mat"] == o.mat).all()
    assert (g["gcode"] == o.gcode).all()
    assert (g["donor"] == o.donor).all()
    assert (g["acceptor"] == o.acceptor).all()


def test_generator_tables_agree_with_library():
    """The generator's BLOSUM62 copy (20 standard residues) equals the
    library's matrix."""
    g = mpg.params_arrays(mpg.params())["mat"]
    b20 = W._b62_20()
    assert (g[:20, :20] == b20).all()


def test_params_check():
    L = mpg.lib()
    p = mpg.params()
    assert L.mpg_params_check(ctypes.byref(p), 8000, 300000) == mpg.MPG_OK
    assert L.mpg_params_check(ctypes.byref(p), 40000, 1000) == mpg.MPG_E_RANGE
    assert L.mpg_params_check(ctypes.byref(p), 100, 2000000) == mpg.MPG_E_RANGE
    bad = mpg.params(q=-1)
    assert L.mpg_params_check(ctypes.byref(bad), 10, 10) == mpg.MPG_E_INVAL
    bad = mpg.params(q=0, e=0)
    assert L.mpg_params_check(ctypes.byref(bad), 10, 10) == mpg.MPG_E_INVAL
    bad = mpg.params(mode=4)
    assert L.mpg_params_check(ctypes.byref(bad), 10, 10) == mpg.MPG_E_INVAL
    bad = mpg.params(mode=-1)
    assert L.mpg_params_check(ctypes.byref(bad), 10, 10) == mpg.MPG_E_INVAL
    left = mpg.params(mode=mpg.MPG_EXTEND_LEFT)
    # a 0 floor, like LOCAL: only the best score bounds the values
    assert L.mpg_params_check(ctypes.byref(left), 1000, 1000000) == mpg.MPG_OK
    bad = mpg.params(flags=64)
    assert L.mpg_params_check(ctypes.byref(bad), 10, 10) == mpg.MPG_E_INVAL
    g = mpg.params(mode=mpg.MPG_GLOBAL)
    # EXTEND/GLOBAL bound: (n + m) * max penalty must stay below 2^24
    assert L.mpg_params_check(ctypes.byref(g), 1000, 100000) == mpg.MPG_OK
    assert L.mpg_params_check(ctypes.byref(g), 1000, 1000000) == mpg.MPG_E_RANGE


def test_strerror_and_capacity():
    for st in range(0, -8, -1):
        assert mpg.strerror(st)
    segs = np.zeros(3, dtype=mpg.SEG_DTYPE)
    segs["plen"] = [10, 0, 5]
    segs["dlen"] = [30, 7, 0]
    segs["flags"] = [mpg.MPG_WANT_TB, 0, mpg.MPG_WANT_TB]
    cap = mpg.lib().mpg_ops_capacity(segs.ctypes.data, 3)
    assert cap == (2 * 40 + 1) + 1 + (2 * 5 + 1)


def test_null_arguments_are_rejected():
    L = mpg.lib()
    assert L.mpg_align_batch(None, None, None, 0, None) == mpg.MPG_E_INVAL
    assert L.mpg_ctx_create(None, 0, 0, 0) == mpg.MPG_E_INVAL
    assert L.mpg_poll(None, None, 0, 0) == mpg.MPG_E_INVAL
    assert L.mpg_cancel(None, 1) == mpg.MPG_E_INVAL
    p = mpg.params()
    assert L.mpg_align_batch_dev_noalloc(None, ctypes.byref(p), None, None, None, 0, None, None,
                                         0) == mpg.MPG_E_INVAL
    assert L.mpg_set_allocator(None, mpg.ALLOC_FN(), mpg.RELEASE_FN(), None) == mpg.MPG_E_INVAL


def test_chaining_defaults_are_the_papers():
    """Methods, "Chaining": k-mers of 6 residues, G = 200 kb, beta = 0.75,
    binned first round, top 30 chains."""
    cp = mpg.chaining_params()
    assert (cp.k, cp.G, cp.beta, cp.binned, cp.max_chains) == (6, 200000, 0.75, 1, 30)
