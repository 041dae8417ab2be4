"""Thin ctypes binding of ``libmpg.so`` (the C ABI declared in include/mpg.h).

Only argument marshalling happens here: every step of the alignment runs in
the library's HIP kernels.  If the library is not built this module raises on
import of the library (``lib()``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# The in-tree build; MPG_LIBRARY may name another build of the same sources
# (tuning variants).
LIB_PATH = os.environ.get("MPG_LIBRARY") or os.path.join(HERE, "libmpg.so")

MPG_OK, MPG_E_INVAL, MPG_E_RANGE, MPG_E_NOMEM = 0, -1, -2, -3
MPG_E_AGAIN, MPG_E_DEVICE, MPG_E_NOALN, MPG_E_CANCELLED = -4, -5, -6, -7
MPG_LOCAL, MPG_EXTEND, MPG_GLOBAL, MPG_EXTEND_LEFT = 0, 1, 2, 3
MPG_NO_INTRON, MPG_NO_FRAMESHIFT, MPG_WANT_TB, MPG_ALLOW_I16 = 1, 2, 4, 8
MPG_MAX_DNA, MPG_MAX_PROT = 1040000, 32000
MPG_NOALLOC_SCRATCH_BYTES = 64 << 20


class mpg_params(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int32), ("e", ctypes.c_int32), ("f", ctypes.c_int32),
                ("r", ctypes.c_int32), ("flags", ctypes.c_uint32), ("mode", ctypes.c_int32),
                ("mat", (ctypes.c_int8 * 24) * 24), ("gcode", ctypes.c_uint8 * 64),
                ("donor", ctypes.c_uint8 * 125), ("acceptor", ctypes.c_uint8 * 125),
                ("_pad", ctypes.c_uint8 * 2)]


class mpg_pair(ctypes.Structure):
    _fields_ = [("prot", ctypes.c_char_p), ("plen", ctypes.c_int32),
                ("dna", ctypes.c_char_p), ("dlen", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class mpg_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("score", ctypes.c_int32),
                ("g_beg", ctypes.c_int32), ("g_end", ctypes.c_int32),
                ("p_beg", ctypes.c_int32), ("p_end", ctypes.c_int32),
                ("ops", ctypes.c_void_p), ("ops_len", ctypes.c_int32), ("_pad", ctypes.c_int32),
                ("job_id", ctypes.c_uint64), ("t_arrive_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


class mpg_chain(ctypes.Structure):
    _fields_ = [("prot", ctypes.c_char_p), ("plen", ctypes.c_int32),
                ("dna", ctypes.c_char_p), ("dlen", ctypes.c_int32),
                ("anchors", ctypes.c_void_p), ("nanchors", ctypes.c_int32),
                ("k", ctypes.c_int32), ("flags", ctypes.c_uint32), ("_pad", ctypes.c_int32)]


class mpg_chain_seg(ctypes.Structure):
    _fields_ = [("prot_off", ctypes.c_int64), ("dna_off", ctypes.c_int64),
                ("plen", ctypes.c_int32), ("dlen", ctypes.c_int32),
                ("anchors", ctypes.c_void_p), ("nanchors", ctypes.c_int32),
                ("k", ctypes.c_int32), ("flags", ctypes.c_uint32), ("_pad", ctypes.c_int32)]


class mpg_profile_pair(ctypes.Structure):
    _fields_ = [("score", ctypes.c_void_p), ("gap", ctypes.c_void_p), ("m", ctypes.c_int32),
                ("dna", ctypes.c_char_p), ("dlen", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class mpg_profile_seg(ctypes.Structure):
    _fields_ = [("prof_off", ctypes.c_int64), ("dna_off", ctypes.c_int64),
                ("m", ctypes.c_int32), ("dlen", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("smax", ctypes.c_int32), ("pmax", ctypes.c_int32), ("_pad", ctypes.c_int32)]


class mpg_chaining_params(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("G", ctypes.c_int32), ("beta", ctypes.c_double),
                ("binned", ctypes.c_int32), ("max_chains", ctypes.c_int32)]


class mpg_chain_out(ctypes.Structure):
    _fields_ = [("score", ctypes.c_double), ("first", ctypes.c_int32), ("len", ctypes.c_int32)]


CHAIN_OUT_DTYPE = np.dtype([("score", "<f8"), ("first", "<i4"), ("len", "<i4")])


class mpg_seg(ctypes.Structure):
    _fields_ = [("prot_off", ctypes.c_int64), ("dna_off", ctypes.c_int64),
                ("plen", ctypes.c_int32), ("dlen", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("_pad", ctypes.c_int32)]


class mpg_dev_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("score", ctypes.c_int32),
                ("g_beg", ctypes.c_int32), ("g_end", ctypes.c_int32),
                ("p_beg", ctypes.c_int32), ("p_end", ctypes.c_int32),
                ("ops_off", ctypes.c_int64), ("ops_len", ctypes.c_int32),
                ("_pad", ctypes.c_int32)]


class mpg_stats(ctypes.Structure):
    _fields_ = [(nm, ctypes.c_uint64) for nm in (
        "submitted", "completed", "cancelled", "rejected_again", "rejected_range", "batches",
        "cells", "queue_depth", "in_flight", "tb_bytes_in_use", "tb_bytes_peak", "tb_budget",
        "short_streams", "long_streams")]


class mpg_timing(ctypes.Structure):
    _fields_ = [("prepass_ms", ctypes.c_double), ("dp_ms", ctypes.c_double),
                ("walk_ms", ctypes.c_double), ("dp_spans", ctypes.c_uint64),
                ("calls", ctypes.c_uint64), ("host_ms", ctypes.c_double),
                ("i16_pairs", ctypes.c_uint64), ("cells", ctypes.c_uint64),
                ("seg_packs", ctypes.c_uint64)]


class mpg_tuning(ctypes.Structure):
    _fields_ = [("gcups", ctypes.c_double * 3), ("i16_gcups", ctypes.c_double * 2),
                ("K", ctypes.c_int32), ("K16", ctypes.c_int32), ("narrow_cols", ctypes.c_int32),
                ("seg_packs", ctypes.c_int32), ("narrow_gcups", ctypes.c_double * 4),
                ("seg_gcups", ctypes.c_double * 2)]


SEG_DTYPE = np.dtype([("prot_off", "<i8"), ("dna_off", "<i8"), ("plen", "<i4"),
                      ("dlen", "<i4"), ("flags", "<u4"), ("_pad", "<i4")])
DEV_RESULT_DTYPE = np.dtype([("status", "<i4"), ("score", "<i4"), ("g_beg", "<i4"),
                             ("g_end", "<i4"), ("p_beg", "<i4"), ("p_end", "<i4"),
                             ("ops_off", "<i8"), ("ops_len", "<i4"), ("_pad", "<i4")])

EXPORTS = ["mpg_ctx_create", "mpg_ctx_destroy", "mpg_set_stream", "mpg_params_default",
           "mpg_params_check", "mpg_align_batch", "mpg_ops_capacity", "mpg_align_batch_dev",
           "mpg_sync", "mpg_submit", "mpg_poll", "mpg_cancel", "mpg_get_stats",
           "mpg_result_release", "mpg_strerror", "mpg_enable_timing", "mpg_get_timing",
           "mpg_autotune", "mpg_plan_create", "mpg_plan_launch", "mpg_plan_graph",
           "mpg_plan_destroy", "mpg_rescore_spliced", "mpg_align_chains",
           "mpg_chain_ops_capacity", "mpg_align_chains_dev", "mpg_align_profiles",
           "mpg_profile_bytes", "mpg_align_profiles_dev", "mpg_chaining_params_default",
           "mpg_chain_anchors", "mpg_chain_anchors_dev", "mpg_rescore_spliced_dev",
           "mpg_align_batch_dev_noalloc", "mpg_set_allocator"]

# mpg_set_allocator callbacks: alloc(bytes, user) -> device pointer or NULL;
# release(ptr, user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def lib():
    """Load the in-tree library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname; loading torch
        # first makes this library bind to that copy, so one process never
        # holds two HIP runtimes (the second would find no GPU).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmpg.so is not built; run python -m paper_2210_08052_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.mpg_ctx_create.argtypes = [P(ctypes.c_void_p), ctypes.c_int, ctypes.c_uint64,
                                     ctypes.c_uint32]
        L.mpg_ctx_destroy.argtypes = [ctypes.c_void_p]
        L.mpg_ctx_destroy.restype = None
        L.mpg_set_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.mpg_params_default.argtypes = [P(mpg_params)]
        L.mpg_params_default.restype = None
        L.mpg_params_check.argtypes = [P(mpg_params), ctypes.c_int32, ctypes.c_int32]
        L.mpg_align_batch.argtypes = [ctypes.c_void_p, P(mpg_params), P(mpg_pair),
                                      ctypes.c_int32, P(mpg_result)]
        L.mpg_ops_capacity.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.mpg_ops_capacity.restype = ctypes.c_int64
        L.mpg_align_batch_dev.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.mpg_align_batch_dev_noalloc.argtypes = L.mpg_align_batch_dev.argtypes
        L.mpg_set_allocator.argtypes = [ctypes.c_void_p, ALLOC_FN, RELEASE_FN, ctypes.c_void_p]
        L.mpg_sync.argtypes = [ctypes.c_void_p]
        L.mpg_submit.argtypes = [ctypes.c_void_p, P(mpg_params), P(mpg_pair),
                                 P(ctypes.c_uint64)]
        L.mpg_poll.argtypes = [ctypes.c_void_p, P(mpg_result), ctypes.c_int32, ctypes.c_int32]
        L.mpg_cancel.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.mpg_get_stats.argtypes = [ctypes.c_void_p, P(mpg_stats)]
        L.mpg_result_release.argtypes = [ctypes.c_void_p, P(mpg_result), ctypes.c_int32]
        L.mpg_result_release.restype = None
        L.mpg_enable_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.mpg_get_timing.argtypes = [ctypes.c_void_p, P(mpg_timing), ctypes.c_int]
        L.mpg_autotune.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                   P(mpg_tuning)]
        L.mpg_plan_create.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      P(ctypes.c_void_p)]
        L.mpg_plan_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.mpg_plan_graph.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.mpg_plan_destroy.argtypes = [ctypes.c_void_p]
        L.mpg_plan_destroy.restype = None
        L.mpg_rescore_spliced.argtypes = [ctypes.c_void_p, P(mpg_params), P(mpg_pair),
                                          P(mpg_result), ctypes.c_int32, P(ctypes.c_int32),
                                          P(ctypes.c_int32), P(ctypes.c_int32)]
        L.mpg_align_chains.argtypes = [ctypes.c_void_p, P(mpg_params), P(mpg_chain),
                                       ctypes.c_int32, P(mpg_result)]
        L.mpg_chain_ops_capacity.argtypes = [P(mpg_params), P(mpg_chain_seg), ctypes.c_int32]
        L.mpg_chain_ops_capacity.restype = ctypes.c_int64
        L.mpg_align_chains_dev.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                           ctypes.c_void_p, P(mpg_chain_seg), ctypes.c_int32,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.mpg_align_profiles.argtypes = [ctypes.c_void_p, P(mpg_params), P(mpg_profile_pair),
                                         ctypes.c_int32, P(mpg_result)]
        L.mpg_profile_bytes.argtypes = [ctypes.c_int32]
        L.mpg_profile_bytes.restype = ctypes.c_int64
        L.mpg_align_profiles_dev.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                             ctypes.c_void_p, P(mpg_profile_seg),
                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int64]
        L.mpg_chaining_params_default.argtypes = [P(mpg_chaining_params)]
        L.mpg_chaining_params_default.restype = None
        L.mpg_chain_anchors.argtypes = [ctypes.c_void_p, P(mpg_chaining_params), ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        L.mpg_chain_anchors_dev.argtypes = L.mpg_chain_anchors.argtypes
        L.mpg_rescore_spliced_dev.argtypes = [ctypes.c_void_p, P(mpg_params), ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]
        L.mpg_strerror.argtypes = [ctypes.c_int]
        L.mpg_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(st: int) -> str:
    return lib().mpg_strerror(st).decode()


def check(st: int, what: str = "mpg call"):
    if st < 0:
        raise RuntimeError("%s failed: %s (%d)" % (what, strerror(st), st))
    return st


def params(**kw) -> mpg_params:
    """Library defaults (mpg_params_default) with fields overridden by kw:
    q, e, f, r, flags, mode (ints) and mat (24x24), gcode (64), donor and
    acceptor (125) arrays."""
    p = mpg_params()
    lib().mpg_params_default(ctypes.byref(p))
    for k in ("q", "e", "f", "r", "flags", "mode"):
        if k in kw and kw[k] is not None:
            setattr(p, k, int(kw[k]))
    if kw.get("mat") is not None:
        m = np.ascontiguousarray(kw["mat"], dtype=np.int8).reshape(24, 24)
        ctypes.memmove(ctypes.addressof(p.mat), m.ctypes.data, 576)
    for k, n in (("gcode", 64), ("donor", 125), ("acceptor", 125)):
        if kw.get(k) is not None:
            a = np.ascontiguousarray(kw[k], dtype=np.uint8).reshape(n)
            ctypes.memmove(ctypes.addressof(getattr(p, k)), a.ctypes.data, n)
    return p


def params_arrays(p: mpg_params) -> dict:
    """The arrays of a params struct (for comparisons in tests)."""
    return {"q": p.q, "e": p.e, "f": p.f, "r": p.r, "flags": p.flags, "mode": p.mode,
            "mat": np.ctypeslib.as_array(p.mat).copy(),
            "gcode": np.ctypeslib.as_array(p.gcode).copy(),
            "donor": np.ctypeslib.as_array(p.donor).copy(),
            "acceptor": np.ctypeslib.as_array(p.acceptor).copy()}


class Context:
    """Owns one mpg_ctx on a HIP device."""

    def __init__(self, device: int = 0, tb_budget_bytes: int = 0):
        self.ptr = ctypes.c_void_p()
        check(lib().mpg_ctx_create(ctypes.byref(self.ptr), device, tb_budget_bytes, 0),
              "mpg_ctx_create")

    def close(self):
        if self.ptr:
            lib().mpg_ctx_destroy(self.ptr)
            self.ptr = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_allocator(self, alloc=None, release=None):
        """Device memory of the context's workspaces from Python callables:
        alloc(nbytes) -> device pointer (int, 0 on failure), release(ptr).
        Both None: back to hipMalloc/hipFree.  The callables are kept alive
        with the context."""
        if alloc is None and release is None:
            cbs = (ALLOC_FN(), RELEASE_FN())
        else:
            cbs = (ALLOC_FN(lambda n, _u: alloc(n) or None),
                   RELEASE_FN(lambda q, _u: release(q)))
        check(lib().mpg_set_allocator(self.ptr, cbs[0], cbs[1], None), "mpg_set_allocator")
        self._alloc_cbs = getattr(self, "_alloc_cbs", []) + [cbs]

    def set_stream(self, stream_handle: int):
        check(lib().mpg_set_stream(self.ptr, ctypes.c_void_p(stream_handle)), "mpg_set_stream")

    # ---- host-memory batch
    def align_batch(self, pairs, p: mpg_params, want_tb=None):
        """pairs: list of (prot, dna[, want_tb]) bytes; returns a list of dicts."""
        n = len(pairs)
        arr = (mpg_pair * max(n, 1))()
        keep = []
        for k, pr in enumerate(pairs):
            prot, dna = pr[0], pr[1]
            tb = pr[2] if len(pr) > 2 else want_tb
            prot = prot.encode() if isinstance(prot, str) else bytes(prot)
            dna = dna.encode() if isinstance(dna, str) else bytes(dna)
            keep.append((prot, dna))
            arr[k].prot = prot
            arr[k].plen = len(prot)
            arr[k].dna = dna
            arr[k].dlen = len(dna)
            arr[k].flags = MPG_WANT_TB if tb else 0
        out = (mpg_result * max(n, 1))()
        check(lib().mpg_align_batch(self.ptr, ctypes.byref(p), arr, n, out), "mpg_align_batch")
        res = [_result_dict(out[k]) for k in range(n)]
        lib().mpg_result_release(self.ptr, out, n)
        return res

    def align_chains(self, chains, p: mpg_params, want_tb=None):
        """chains: list of (prot, dna, anchors [(x, y), ...], k[, want_tb]);
        returns a list of result dicts."""
        n = len(chains)
        arr = (mpg_chain * max(n, 1))()
        keep = []
        for c, ch in enumerate(chains):
            prot = ch[0].encode() if isinstance(ch[0], str) else bytes(ch[0])
            dna = ch[1].encode() if isinstance(ch[1], str) else bytes(ch[1])
            anc = np.ascontiguousarray(np.asarray(ch[2], dtype=np.int32).reshape(-1))
            tb = ch[4] if len(ch) > 4 else want_tb
            keep.append((prot, dna, anc))
            arr[c].prot, arr[c].plen, arr[c].dna, arr[c].dlen = prot, len(prot), dna, len(dna)
            arr[c].anchors = anc.ctypes.data if anc.size else None
            arr[c].nanchors = anc.size // 2
            arr[c].k = int(ch[3])
            arr[c].flags = MPG_WANT_TB if tb else 0
        out = (mpg_result * max(n, 1))()
        check(lib().mpg_align_chains(self.ptr, ctypes.byref(p), arr, n, out), "mpg_align_chains")
        res = [_result_dict(out[k]) for k in range(n)]
        lib().mpg_result_release(self.ptr, out, n)
        return res

    def align_chains_dev(self, p: mpg_params, d_prot, d_dna, chains, d_out, d_ops,
                         ops_cap: int):
        """Enqueue on the context's stream; chains is a ChainSegs (pack_chains)."""
        check(lib().mpg_align_chains_dev(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                         ctypes.c_void_p(d_dna), chains.arr, chains.n,
                                         ctypes.c_void_p(d_out), ctypes.c_void_p(d_ops),
                                         ops_cap), "mpg_align_chains_dev")

    def align_profiles(self, pairs, p: mpg_params, want_tb=None):
        """pairs: list of (score (m, 24) int8, gap (m + 1, 4) int16, dna[, want_tb]);
        returns a list of result dicts."""
        n = len(pairs)
        arr = (mpg_profile_pair * max(n, 1))()
        keep = []
        for k, pr in enumerate(pairs):
            S = np.ascontiguousarray(pr[0], dtype=np.int8)
            G = np.ascontiguousarray(pr[1], dtype=np.int16)
            dna = pr[2].encode() if isinstance(pr[2], str) else bytes(pr[2])
            tb = pr[3] if len(pr) > 3 else want_tb
            keep.append((S, G, dna))
            arr[k].score = S.ctypes.data if S.size else None
            arr[k].gap = G.ctypes.data
            arr[k].m = S.shape[0]
            arr[k].dna, arr[k].dlen = dna, len(dna)
            arr[k].flags = MPG_WANT_TB if tb else 0
        out = (mpg_result * max(n, 1))()
        check(lib().mpg_align_profiles(self.ptr, ctypes.byref(p), arr, n, out),
              "mpg_align_profiles")
        res = [_result_dict(out[k]) for k in range(n)]
        lib().mpg_result_release(self.ptr, out, n)
        return res

    def align_profiles_dev(self, p: mpg_params, d_prof, d_dna, segs, d_out, d_ops,
                           ops_cap: int):
        """Enqueue on the context's stream; segs from pack_profiles."""
        check(lib().mpg_align_profiles_dev(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prof),
                                           ctypes.c_void_p(d_dna), segs.arr, segs.n,
                                           ctypes.c_void_p(d_out), ctypes.c_void_p(d_ops),
                                           ops_cap), "mpg_align_profiles_dev")

    def chain_anchors(self, sets, cp=None):
        """sets: list of anchor lists [(x, y), ...] sorted by (x, y).  Returns per
        set a dict: f, pred (numpy arrays), chains [(score, [indices])] best
        first, and status (0, or a negative code for the set)."""
        cp = cp or chaining_params()
        arrs = [np.asarray(a, dtype=np.int32).reshape(-1, 2) for a in sets]
        off = np.zeros(len(sets) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(a) for a in arrs])
        allv = np.ascontiguousarray(np.concatenate(arrs) if arrs else np.zeros((0, 2), np.int32))
        tot = int(off[-1])
        f = np.zeros(max(tot, 1), np.float64)
        pred = np.zeros(max(tot, 1), np.int32)
        idx = np.zeros(max(tot, 1), np.int32)
        top = np.zeros(max(len(sets) * cp.max_chains, 1), dtype=CHAIN_OUT_DTYPE)
        ntop = np.zeros(max(len(sets), 1), np.int32)
        check(lib().mpg_chain_anchors(self.ptr, ctypes.byref(cp), allv.ctypes.data,
                                      off.ctypes.data, len(sets), f.ctypes.data,
                                      pred.ctypes.data, idx.ctypes.data, top.ctypes.data,
                                      ntop.ctypes.data), "mpg_chain_anchors")
        out = []
        for s_, a in enumerate(arrs):
            lo, hi = int(off[s_]), int(off[s_ + 1])
            nt = int(ntop[s_])
            chains = []
            for r in range(max(nt, 0)):
                t = top[s_ * cp.max_chains + r]
                first, ln = int(t["first"]), int(t["len"])
                chains.append((float(t["score"]), [int(v) for v in idx[lo + first:lo + first + ln]]))
            out.append({"f": f[lo:hi].copy(), "pred": pred[lo:hi].astype(np.int64),
                        "chains": chains, "status": min(nt, 0)})
        return out

    def chain_anchors_dev(self, cp, d_anchors, set_off: np.ndarray, d_f, d_pred, d_idx, d_top,
                          d_ntop):
        """Enqueue on the context's stream (set_off: int64 host array)."""
        check(lib().mpg_chain_anchors_dev(self.ptr, ctypes.byref(cp), ctypes.c_void_p(d_anchors),
                                          set_off.ctypes.data, len(set_off) - 1,
                                          ctypes.c_void_p(d_f), ctypes.c_void_p(d_pred),
                                          ctypes.c_void_p(d_idx), ctypes.c_void_p(d_top),
                                          ctypes.c_void_p(d_ntop)), "mpg_chain_anchors_dev")

    def rescore_spliced_dev(self, p: mpg_params, d_prot, d_dna, segs: np.ndarray, d_res, d_ops,
                            d_score, d_exons, d_status):
        """Pseudogene guard on a traced device batch (see mpg_rescore_spliced_dev)."""
        check(lib().mpg_rescore_spliced_dev(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                            ctypes.c_void_p(d_dna), segs.ctypes.data, len(segs),
                                            ctypes.c_void_p(d_res), ctypes.c_void_p(d_ops),
                                            ctypes.c_void_p(d_score), ctypes.c_void_p(d_exons),
                                            ctypes.c_void_p(d_status)), "mpg_rescore_spliced_dev")

    def rescore_spliced(self, pairs, results, p: mpg_params):
        """Pseudogene guard for traced results of align_batch on the same
        pairs: a list of (status, score, exons) per pair."""
        n = len(pairs)
        arr = (mpg_pair * max(n, 1))()
        res = (mpg_result * max(n, 1))()
        keep = []
        for k, (pr, r) in enumerate(zip(pairs, results)):
            prot = pr[0].encode() if isinstance(pr[0], str) else bytes(pr[0])
            dna = pr[1].encode() if isinstance(pr[1], str) else bytes(pr[1])
            ops = r["ops"].encode() if r.get("ops") is not None else None
            keep.append((prot, dna, ops))
            arr[k].prot, arr[k].plen, arr[k].dna, arr[k].dlen = prot, len(prot), dna, len(dna)
            res[k].status, res[k].score = r["status"], r["score"]
            res[k].g_beg, res[k].g_end = r["g_beg"], r["g_end"]
            res[k].p_beg, res[k].p_end = r["p_beg"], r["p_end"]
            if ops is not None:
                res[k].ops = ctypes.cast(ctypes.c_char_p(ops), ctypes.c_void_p).value
                res[k].ops_len = len(ops)
        sc = (ctypes.c_int32 * max(n, 1))()
        ex = (ctypes.c_int32 * max(n, 1))()
        st = (ctypes.c_int32 * max(n, 1))()
        check(lib().mpg_rescore_spliced(self.ptr, ctypes.byref(p), arr, res, n, sc, ex, st),
              "mpg_rescore_spliced")
        return [(st[k], sc[k], ex[k]) for k in range(n)]

    # ---- device-resident batch (torch tensors for memory only)
    def align_batch_dev(self, p: mpg_params, d_prot, d_dna, segs: np.ndarray, d_out, d_ops,
                        ops_cap: int):
        """Enqueue on the context's stream.  d_prot/d_dna/d_out/d_ops are
        device pointers (ints); segs a SEG_DTYPE numpy array."""
        segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
        check(lib().mpg_align_batch_dev(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                        ctypes.c_void_p(d_dna), segs.ctypes.data, len(segs),
                                        ctypes.c_void_p(d_out), ctypes.c_void_p(d_ops),
                                        int(ops_cap)), "mpg_align_batch_dev")

    def align_batch_dev_noalloc(self, p: mpg_params, d_prot, d_dna, segs: np.ndarray, d_out,
                                d_ops, ops_cap: int) -> int:
        """As align_batch_dev through the allocation-free entry point; returns
        its status (MPG_E_RANGE when the call exceeds the fixed scratch)."""
        segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
        return lib().mpg_align_batch_dev_noalloc(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                                 ctypes.c_void_p(d_dna), segs.ctypes.data,
                                                 len(segs), ctypes.c_void_p(d_out),
                                                 ctypes.c_void_p(d_ops), int(ops_cap))

    def sync(self):
        check(lib().mpg_sync(self.ptr), "mpg_sync")

    def enable_timing(self, on: bool = True):
        check(lib().mpg_enable_timing(self.ptr, 1 if on else 0), "mpg_enable_timing")

    def timing(self, reset: bool = True) -> dict:
        t = mpg_timing()
        check(lib().mpg_get_timing(self.ptr, ctypes.byref(t), 1 if reset else 0),
              "mpg_get_timing")
        return {k: getattr(t, k) for k, _ in mpg_timing._fields_}

    # ---- serving
    def submit(self, p: mpg_params, prot: bytes, dna: bytes, want_tb: bool = False) -> int:
        pr = mpg_pair(prot, len(prot), dna, len(dna), MPG_WANT_TB if want_tb else 0)
        jid = ctypes.c_uint64(0)
        st = lib().mpg_submit(self.ptr, ctypes.byref(p), ctypes.byref(pr), ctypes.byref(jid))
        if st < 0:
            return st
        return int(jid.value)

    def poll(self, max_results: int = 256, timeout_us: int = 0):
        out = (mpg_result * max_results)()
        k = check(lib().mpg_poll(self.ptr, out, max_results, timeout_us), "mpg_poll")
        res = [_result_dict(out[i]) for i in range(k)]
        lib().mpg_result_release(self.ptr, out, k)
        return res

    def poll_raw(self, max_results: int = 4096, timeout_us: int = 0, keep=None):
        """Like poll, but returns (job_id, t_arrive_ns, t_done_ns, status)
        tuples, plus the full result dicts of the job ids in `keep` (fast path
        for latency measurements)."""
        out = (mpg_result * max_results)()
        k = check(lib().mpg_poll(self.ptr, out, max_results, timeout_us), "mpg_poll")
        res, full = [], {}
        for i in range(k):
            jid = int(out[i].job_id)
            res.append((jid, int(out[i].t_arrive_ns), int(out[i].t_done_ns), out[i].status))
            if keep is not None and jid in keep:
                full[jid] = _result_dict(out[i])
        lib().mpg_result_release(self.ptr, out, k)
        return res, full

    def autotune(self, p: mpg_params = None, d_prot=0, d_dna=0, segs=None) -> dict:
        """mpg_autotune on a device-resident sample (segs: SEG_DTYPE array) or,
        without one, on the built-in sample; returns rates and chosen widths."""
        t = mpg_tuning()
        if segs is None:
            st = lib().mpg_autotune(self.ptr, None, None, None, None, 0, ctypes.byref(t))
        else:
            segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
            st = lib().mpg_autotune(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                    ctypes.c_void_p(d_dna), segs.ctypes.data_as(ctypes.c_void_p),
                                    len(segs), ctypes.byref(t))
        check(st, "mpg_autotune")
        return {"gcups": list(t.gcups), "i16_gcups": list(t.i16_gcups), "K": t.K, "K16": t.K16,
                "narrow_cols": t.narrow_cols, "seg_packs": t.seg_packs,
                "narrow_gcups": list(t.narrow_gcups), "seg_gcups": list(t.seg_gcups)}

    def plan(self, p: mpg_params, d_prot, d_dna, segs: np.ndarray, d_out, d_ops, ops_cap: int):
        """mpg_plan_create: a Plan bound to these device buffers."""
        segs = np.ascontiguousarray(segs, dtype=SEG_DTYPE)
        h = ctypes.c_void_p()
        check(lib().mpg_plan_create(self.ptr, ctypes.byref(p), ctypes.c_void_p(d_prot),
                                    ctypes.c_void_p(d_dna), segs.ctypes.data_as(ctypes.c_void_p),
                                    len(segs), ctypes.c_void_p(d_out), ctypes.c_void_p(d_ops),
                                    int(ops_cap), ctypes.byref(h)), "mpg_plan_create")
        return Plan(h)

    def cancel(self, job_id: int) -> int:
        return lib().mpg_cancel(self.ptr, ctypes.c_uint64(job_id))

    def stats(self) -> dict:
        s = mpg_stats()
        check(lib().mpg_get_stats(self.ptr, ctypes.byref(s)), "mpg_get_stats")
        return {k: int(getattr(s, k)) for k, _ in mpg_stats._fields_}


class Plan:
    """A planned batch (mpg_plan_*): launch, capture into a graph, replay."""

    def __init__(self, handle):
        self.h = handle

    def launch(self, stream_handle: int = 0):
        check(lib().mpg_plan_launch(self.h, ctypes.c_void_p(stream_handle or None)),
              "mpg_plan_launch")

    def graph(self, stream_handle: int):
        check(lib().mpg_plan_graph(self.h, ctypes.c_void_p(stream_handle)), "mpg_plan_graph")

    def close(self):
        if self.h:
            lib().mpg_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_dict(r: mpg_result) -> dict:
    ops = ctypes.string_at(r.ops, r.ops_len).decode() if r.ops else None
    return {"status": r.status, "score": r.score, "g_beg": r.g_beg, "g_end": r.g_end,
            "p_beg": r.p_beg, "p_end": r.p_end, "ops": ops, "job_id": int(r.job_id),
            "t_arrive_ns": int(r.t_arrive_ns), "t_done_ns": int(r.t_done_ns)}


class ChainSegs:
    """Device-resident chains: the mpg_chain_seg array and the anchors it
    points to (kept alive here)."""

    def __init__(self, arr, n, keep):
        self.arr, self.n, self._keep = arr, n, keep

    def ops_capacity(self, p: mpg_params) -> int:
        return int(lib().mpg_chain_ops_capacity(ctypes.byref(p), self.arr, self.n))


def pack_chains(chains):
    """chains: list of (prot, dna, anchors, k[, want_tb]); returns
    (prot_bytes, dna_bytes, ChainSegs) for align_chains_dev."""
    n = len(chains)
    arr = (mpg_chain_seg * max(n, 1))()
    keep, pb, db = [], [], []
    po = do = 0
    for c, ch in enumerate(chains):
        prot, dna = bytes(ch[0]), bytes(ch[1])
        anc = np.ascontiguousarray(np.asarray(ch[2], dtype=np.int32).reshape(-1))
        keep.append(anc)
        arr[c].prot_off, arr[c].dna_off = po, do
        arr[c].plen, arr[c].dlen = len(prot), len(dna)
        arr[c].anchors = anc.ctypes.data if anc.size else None
        arr[c].nanchors = anc.size // 2
        arr[c].k = int(ch[3])
        arr[c].flags = MPG_WANT_TB if (len(ch) > 4 and ch[4]) else 0
        pb.append(prot)
        db.append(dna)
        po += len(prot)
        do += len(dna)
    return b"".join(pb), b"".join(db), ChainSegs(arr, n, keep)


class ProfileSegs:
    """The mpg_profile_seg array for align_profiles_dev."""

    def __init__(self, arr, n):
        self.arr, self.n = arr, n


def pack_profiles(pairs):
    """pairs: list of (score, gap, dna[, want_tb]); returns (profile bytes in the
    device layout, dna bytes, ProfileSegs, ops capacity with want_tb flags)."""
    n = len(pairs)
    arr = (mpg_profile_seg * max(n, 1))()
    blocks, dbs = [], []
    fo = do = 0
    cap = 0
    for k, pr in enumerate(pairs):
        S = np.ascontiguousarray(pr[0], dtype=np.int8)
        G = np.ascontiguousarray(pr[1], dtype=np.int16)
        m = S.shape[0]
        dna = bytes(pr[2])
        tb = len(pr) > 3 and pr[3]
        nb = int(lib().mpg_profile_bytes(m))
        blk = bytearray(nb)
        blk[:24 * m] = S.tobytes()
        go = nb - 8 * (m + 1)
        blk[go:] = G.tobytes()
        used = G[1:, :2].sum(axis=1) if m else np.zeros(0, np.int64)
        pmax = max([int(-S.min()) if S.size else 0, int(G[:, 2:].sum(axis=1).max())] +
                   ([int(used.max())] if m else []))
        arr[k].prof_off, arr[k].dna_off = fo, do
        arr[k].m, arr[k].dlen = m, len(dna)
        arr[k].flags = MPG_WANT_TB if tb else 0
        arr[k].smax = max(0, int(S.max()) if S.size else 0)
        arr[k].pmax = pmax
        blocks.append(bytes(blk))
        dbs.append(dna)
        fo += nb
        do += len(dna)
        cap += 2 * (m + len(dna)) + 1 if tb else 1
    return b"".join(blocks), b"".join(dbs), ProfileSegs(arr, n), cap


def chaining_params(**kw) -> mpg_chaining_params:
    """The library's chaining defaults (k 6, G 200,000, beta 0.75, binned,
    30 chains), with keyword overrides."""
    cp = mpg_chaining_params()
    lib().mpg_chaining_params_default(ctypes.byref(cp))
    for k2, v in kw.items():
        setattr(cp, k2, v)
    return cp


def pack_pairs(pairs):
    """Concatenate proteins and regions; returns (prot_bytes, dna_bytes, segs)."""
    segs = np.zeros(len(pairs), dtype=SEG_DTYPE)
    pb, db = [], []
    po = do = 0
    for k, pr in enumerate(pairs):
        prot, dna = pr[0], pr[1]
        tb = pr[2] if len(pr) > 2 else False
        segs[k] = (po, do, len(prot), len(dna), MPG_WANT_TB if tb else 0, 0)
        pb.append(prot)
        db.append(dna)
        po += len(prot)
        do += len(dna)
    return b"".join(pb), b"".join(db), segs
