"""CPU oracle for the spliced protein-to-genome DP -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of ``bench.py`` may
import this package.  It never touches the GPU library and the GPU library
never touches it.

* ``mpg_oracle.c``: full-matrix int64 DP of Eq. (full) with the readings
  listed in its header, plus traceback and op-string emission.
* ``params``: the oracle's own scoring constants.
* ``brute``: exhaustive maximisation over the segment grammar (tiny inputs).
* ``rescore``: recomputes a score from (begin, op string).
* ``gotoh``: textbook three-state affine-gap alignment on translated frames.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass

import numpy as np

from . import params
from .params import Scoring, default_scoring

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

LOCAL, EXTEND, GLOBAL, EXTEND_LEFT = 0, 1, 2, 3
NO_INTRON, NO_FS = 1, 2
OK, E_NOALN = 0, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no intrinsics, no vector pragmas)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_align.restype = ctypes.c_int
        lib.orc_align.argtypes = [
            ctypes.c_char_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
            ctypes.c_int32, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p,
            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_align_profile.restype = ctypes.c_int
        lib.orc_align_profile.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
            ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_char_p,
            ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        lib.orc_dna_code.restype = ctypes.c_int
        lib.orc_aa_code.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Result:
    status: int
    score: int
    g_beg: int
    g_end: int
    p_beg: int
    p_end: int
    ops: str | None

    def key(self):
        return (self.status, self.score, self.g_beg, self.g_end, self.p_beg, self.p_end,
                self.ops)


def _b(x) -> bytes:
    return x.encode() if isinstance(x, str) else bytes(x)


def align(prot, dna, sc: Scoring | None = None, want_tb: bool = True) -> Result:
    """Align one protein to one genomic region (both ASCII)."""
    lib = _load()
    sc = sc or default_scoring()
    p, d = _b(prot), _b(dna)
    out = (ctypes.c_int64 * 5)()
    cap = 2 * (len(p) + len(d)) + 64 if want_tb else 1
    buf = ctypes.create_string_buffer(cap)
    olen = ctypes.c_int64(0)
    st = lib.orc_align(p, len(p), d, len(d), sc.q, sc.e, sc.f, sc.r, sc.flags, sc.mode,
                       sc.mat.ctypes.data, sc.gcode.ctypes.data, sc.donor.ctypes.data,
                       sc.acceptor.ctypes.data, 1 if want_tb else 0, out, buf, cap,
                       ctypes.byref(olen))
    if st == E_NOALN:
        return Result(st, 0, -1, -1, -1, -1, None)
    if st != OK:
        raise RuntimeError("oracle failed with status %d" % st)
    ops = buf.raw[: olen.value].decode() if want_tb else None
    return Result(OK, int(out[0]), int(out[1]), int(out[2]), int(out[3]), int(out[4]), ops)


def align_profile(S, gap, dna, sc: Scoring | None = None, want_tb: bool = True) -> Result:
    """Align a position-specific query to one genomic region.

    S: (m, 24) int8, the score of each translated amino acid at each column;
    gap: (m + 1, 4) int16, per column the I open/extend costs (columns 1..m)
    and the D open/extend costs (columns 0..m).  sc supplies f, r, the flags,
    the mode, the genetic code and the splice tables (its q, e and matrix are
    not used)."""
    lib = _load()
    sc = sc or default_scoring()
    S = np.ascontiguousarray(S, dtype=np.int8)
    gap = np.ascontiguousarray(gap, dtype=np.int16)
    m = S.shape[0]
    if S.shape != (m, 24) or gap.shape != (m + 1, 4):
        raise ValueError("profile shapes")
    d = _b(dna)
    out = (ctypes.c_int64 * 5)()
    cap = 2 * (m + len(d)) + 64 if want_tb else 1
    buf = ctypes.create_string_buffer(cap)
    olen = ctypes.c_int64(0)
    st = lib.orc_align_profile(S.ctypes.data, gap.ctypes.data, m, d, len(d), sc.f, sc.r,
                               sc.flags, sc.mode, sc.gcode.ctypes.data, sc.donor.ctypes.data,
                               sc.acceptor.ctypes.data, 1 if want_tb else 0, out, buf, cap,
                               ctypes.byref(olen))
    if st == E_NOALN:
        return Result(st, 0, -1, -1, -1, -1, None)
    if st != OK:
        raise RuntimeError("oracle failed with status %d" % st)
    ops = buf.raw[: olen.value].decode() if want_tb else None
    return Result(OK, int(out[0]), int(out[1]), int(out[2]), int(out[3]), int(out[4]), ops)


def align_many(pairs, sc: Scoring | None = None, want_tb: bool = True, threads: int = 0):
    """Align a list of (prot, dna) pairs on a thread pool (one pair per task).

    The C call releases the interpreter lock, so the pool runs on all cores."""
    sc = sc or default_scoring()
    if threads <= 0:
        threads = len(os.sched_getaffinity(0))
    _load()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda pr: align(pr[0], pr[1], sc, want_tb), pairs))


def dna_code(ch: str) -> int:
    return _load().orc_dna_code(ord(ch))


def aa_code(ch: str) -> int:
    return _load().orc_aa_code(ord(ch))
