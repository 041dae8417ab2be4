"""Pins of the CPU oracle against things the paper and mathematics fix.

None of these compare the oracle with itself: they use exhaustive search over
an independent segment grammar, a textbook affine-gap aligner, a path
rescorer, the paper's worked alignment and splice-model case lists, and
structural invariants.
"""
import json
import math
import os
import random

import numpy as np
import pytest

import oracle
from oracle import brute, gotoh, params, rescore

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NEG = float("-inf")


def _rand_case(rng, max_n=10, max_m=3, dna_alpha="ACGTGTAG", prot_alpha="ARNDCW*X"):
    n = rng.randint(0, max_n)
    m = rng.randint(0, max_m)
    dna = "".join(rng.choice(dna_alpha) for _ in range(n))
    prot = "".join(rng.choice(prot_alpha) for _ in range(m))
    return prot, dna


def _rand_scoring(rng, mode=None, flags=None, tables=False):
    kw = dict(q=rng.randint(0, 6), e=rng.randint(1, 3), f=rng.randint(0, 8),
              r=rng.randint(0, 10),
              mode=rng.randint(0, 3) if mode is None else mode,
              flags=rng.randint(0, 3) if flags is None else flags)
    if tables:
        m = np.array([[rng.randint(-5, 8) for _ in range(24)] for _ in range(24)])
        m = np.triu(m) + np.triu(m, 1).T
        kw["mat"] = m.astype(np.int8)
        kw["donor"] = np.array([rng.randint(0, 9) for _ in range(125)], np.uint8)
        kw["acceptor"] = np.array([rng.randint(0, 9) for _ in range(125)], np.uint8)
    return params.default_scoring(**kw)


# --------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(6))
def test_brute_force_matches_oracle(seed):
    """Exhaustive optimum over the segment grammar == oracle score, in every
    mode and flag combination, with tie-prone small penalties; the oracle's
    own path rescored == its score and ends at its end cell."""
    rng = random.Random(1000 + seed)
    for _ in range(120):
        prot, dna = _rand_case(rng)
        sc = _rand_scoring(rng, tables=(seed % 2 == 1))
        res = oracle.align(prot, dna, sc, want_tb=True)
        best = brute.best_score(prot, dna, sc)
        if res.status == oracle.E_NOALN:
            assert best == NEG, (prot, dna, sc.mode)
            continue
        assert res.score == best, (prot, dna, sc.mode, sc.flags)
        s, ge, pe = rescore.rescore(prot, dna, sc, res.g_beg, res.p_beg, res.ops)
        assert (s, ge, pe) == (res.score, res.g_end, res.p_end), (prot, dna, res)


def test_brute_force_degenerate_penalties():
    """All penalties zero (maximal ties, degenerate introns)."""
    rng = random.Random(7)
    for _ in range(60):
        prot, dna = _rand_case(rng, max_n=9, max_m=3)
        for mode in (0, 1, 2, 3):
            sc = params.default_scoring(q=0, e=1, f=0, r=0, mode=mode,
                                        donor=np.zeros(125, np.uint8),
                                        acceptor=np.zeros(125, np.uint8))
            res = oracle.align(prot, dna, sc)
            best = brute.best_score(prot, dna, sc)
            if res.status == oracle.E_NOALN:
                assert best == NEG
                continue
            assert res.score == best
            assert rescore.rescore(prot, dna, sc, res.g_beg, res.p_beg, res.ops)[0] == best


def test_score_only_equals_traceback_run():
    rng = random.Random(11)
    for _ in range(100):
        prot, dna = _rand_case(rng, max_n=60, max_m=12, dna_alpha="ACGTN")
        sc = _rand_scoring(rng)
        a = oracle.align(prot, dna, sc, want_tb=True)
        b = oracle.align(prot, dna, sc, want_tb=False)
        assert (a.status, a.score, a.g_end, a.p_end) == (b.status, b.score, b.g_end, b.p_end)


# ------------------------------------------------------- Gotoh reduction
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_reduces_to_gotoh_without_introns_and_frameshifts(mode):
    """With introns and frameshifts removed, Eq. (full) is affine-gap
    alignment on a translated frame (LOCAL: best of 3 frames)."""
    rng = random.Random(20 + mode)
    ct = params.codon_table()
    for _ in range(150):
        prot, dna = _rand_case(rng, max_n=45, max_m=12, dna_alpha="ACGTN",
                               prot_alpha=params.AA)
        sc = params.default_scoring(q=rng.randint(0, 12), e=rng.randint(1, 3), mode=mode,
                                    flags=oracle.NO_INTRON | oracle.NO_FS)
        res = oracle.align(prot, dna, sc)
        exp = gotoh.spliced_reduction(prot, dna, sc, ct)
        got = NEG if res.status == oracle.E_NOALN else res.score
        assert got == exp, (prot, dna, mode)


# -------------------------------------------------------- worked example
def test_worked_example_alignment():
    """The paper's worked alignment is reproduced exactly (op string and
    score) once mismatches and long gaps are made expensive."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    intr = g["intron"]
    geno = ("GAGGCC" + "CGC" + "TCA" + "CC" + intr + "C" + "ACA" + "AG" + "CGC" + "TAT"
            + "A" + "GCC" + "TAC")
    # the genome row of the paper with the intron interior filled in
    shown = g["paper_rows"]["Geno"].replace("-", "")
    assert geno.startswith(shown.split("gt")[0])
    assert geno.endswith(shown.split("ag")[-1])
    mat = np.full((24, 24), g["diag_matrix"]["off"], np.int8)
    np.fill_diagonal(mat, g["diag_matrix"]["diag"])
    exp_ops = g["ops_by_hand"].replace("{L}", str(len(intr) + 3))
    for q, e, f, r in g["param_sets"]:
        sc = params.default_scoring(q=q, e=e, f=f, r=r, mode=oracle.GLOBAL, mat=mat)
        res = oracle.align(g["protein"], geno, sc)
        hand = 8 * g["diag_matrix"]["diag"] - 2 * (q + e) - r - 2 * f
        assert res.ops == exp_ops
        assert res.score == hand
        assert (res.g_beg, res.g_end, res.p_beg, res.p_end) == (0, len(geno), 0, 11)


def test_worked_example_blosum_bound():
    """Under BLOSUM62 and the default penalties the optimum is at least the
    hand-summed score of the paper's path (8 matrix terms, 2 gaps, 1 intron,
    2 frameshifts)."""
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    intr = g["intron"]
    geno = ("GAGGCC" + "CGC" + "TCA" + "CC" + intr + "C" + "ACA" + "AG" + "CGC" + "TAT"
            + "A" + "GCC" + "TAC")
    sc = params.default_scoring(mode=oracle.GLOBAL)
    b = params.blosum62()
    ix = params.AA.index
    diag = sum(int(b[ix(a)][ix(a)]) for a in "EARTRYAY")
    hand = diag - 2 * (sc.q + sc.e) - sc.r - 2 * sc.f
    path = g["ops_by_hand"].replace("{L}", str(len(intr) + 3))
    assert rescore.rescore(g["protein"], geno, sc, 0, 0, path)[0] == hand
    assert oracle.align(g["protein"], geno, sc).score >= hand


def test_worked_example_translations():
    g = json.load(open(os.path.join(GOLDEN, "worked_example.json")))
    ct = params.codon_table()
    for cod, aa in g["codons_by_hand"].items():
        assert ct[cod] == aa
    gc = params.gcode()
    for cod, aa in g["codons_by_hand"].items():
        k = 16 * "ACGT".index(cod[0]) + 4 * "ACGT".index(cod[1]) + "ACGT".index(cod[2])
        assert params.AA[gc[k]] == aa


# --------------------------------------------------------------- splice
# Cases exactly as listed in "Splice models" (final model) and at the end of
# "DP for protein-to-genome alignment" (simple model).
DONOR_CASES = [(("GTA", "GTG"), 0), (("GTC", "GTT"), 8), (("GC",), 15), (("AT",), 21)]
ACCEPTOR_CASES = [(("CAG", "TAG"), 0), (("AAG", "GAG"), 8), (("AC",), 21)]


def _paper_donor(tri):
    for pats, v in DONOR_CASES:
        for p in pats:
            if tri.startswith(p):
                return v
    return 30


def _paper_acceptor(tri):
    for pats, v in ACCEPTOR_CASES:
        for p in pats:
            if tri.endswith(p):
                return v
    return 30


def test_splice_final_model_all_3mers():
    d, a = params.splice_tables("final")
    n = 0
    for b1 in "ACGTN":
        for b2 in "ACGTN":
            for b3 in "ACGTN":
                k = 25 * "ACGTN".index(b1) + 5 * "ACGTN".index(b2) + "ACGTN".index(b3)
                tri = b1 + b2 + b3
                assert d[k] == _paper_donor(tri), tri
                assert a[k] == _paper_acceptor(tri), tri
                n += 1
    assert n == 125
    # spot values of the readings: GTN falls through to 30, NAC is an AC acceptor
    assert d[25 * 2 + 5 * 3 + 4] == 30 and a[25 * 4 + 5 * 0 + 1] == 21


def test_splice_simple_model():
    d, a = params.splice_tables("simple", p=17)
    for k in range(125):
        tri = "ACGTN"[k // 25] + "ACGTN"[(k // 5) % 5] + "ACGTN"[k % 5]
        assert d[k] == (0 if tri[:2] == "GT" else 17)
        assert a[k] == (0 if tri[1:] == "AG" else 17)


def test_splice_closed_form_ac_acceptor():
    """2*log2(99.81/0.10) ~= 20 (the paper rounds; its table then uses 21)."""
    v = 2 * math.log2(99.81 / 0.10)
    assert abs(v - 19.93) < 0.01 and round(v) == 20


def test_donor_acceptor_index_semantics():
    """d(x) reads T[x+1..x+3] and a(x) reads T[x-2..x]: an N-intron with a
    GTA...CAG boundary costs exactly r; shifting the intron by one base makes
    the boundary non-canonical, which the oracle must pay for."""
    ex1 = "ATGGCTTGGAAA"      # M A W K
    ex2 = "TTTCCCGGG"         # F P G
    intr = "GTA" + "C" * 30 + "CAG"
    prot = "MAWKFPG"
    mat = np.full((24, 24), -20, np.int8)
    np.fill_diagonal(mat, 10)
    sc = params.default_scoring(q=20, e=20, f=50, r=7, mode=oracle.GLOBAL, mat=mat)
    res = oracle.align(prot, ex1 + intr + ex2, sc)
    assert res.ops == "4M%dN3M" % len(intr)
    assert res.score == 70 - 7


# --------------------------------------------------------------- tables
def test_blosum62_symmetric_and_known_entries():
    b = params.blosum62()
    assert (b == b.T).all()
    ix = params.AA.index
    assert b[ix("W")][ix("W")] == 11 and b[ix("C")][ix("C")] == 9
    assert b[ix("*")][ix("*")] == 1 and b[ix("A")][ix("*")] == -4


def test_standard_code_structure():
    ct = params.codon_table()
    assert len(ct) == 64
    assert sorted(k for k, v in ct.items() if v == "*") == ["TAA", "TAG", "TGA"]
    assert ct["ATG"] == "M" and ct["TGG"] == "W"
    counts = {}
    for v in ct.values():
        counts[v] = counts.get(v, 0) + 1
    assert counts["L"] == 6 and counts["R"] == 6 and counts["S"] == 6 and counts["I"] == 3


def test_encodings():
    assert [oracle.dna_code(c) for c in "ACGTacgtNnRX-"] == [0, 1, 2, 3, 0, 1, 2, 3, 4, 4, 4, 4, 4]
    assert [oracle.aa_code(c) for c in "ARNDCQEGHILKMFPSTWYVBZX*"] == list(range(24))
    assert oracle.aa_code("a") == 0 and oracle.aa_code("J") == 22 and oracle.aa_code("?") == 22


# ------------------------------------------------------------ invariants
def test_mode_nesting_and_monotonicity():
    """LOCAL >= EXTEND >= GLOBAL (source and sink sets nest), and no score
    increases when a penalty increases."""
    rng = random.Random(31)
    for _ in range(80):
        prot, dna = _rand_case(rng, max_n=60, max_m=15, dna_alpha="ACGTGTAG",
                               prot_alpha=params.AA)
        base = _rand_scoring(rng, mode=0, flags=0)
        sl = oracle.align(prot, dna, base, False).score
        se = oracle.align(prot, dna, base.replace(mode=1), False).score
        sx = oracle.align(prot, dna, base.replace(mode=3), False).score
        g = oracle.align(prot, dna, base.replace(mode=2), False)
        assert sl >= se and sl >= sx >= 0
        if g.status == 0:
            assert se >= g.score and sx >= g.score
        for field in ("q", "e", "f", "r"):
            bigger = base.replace(**{field: getattr(base, field) + rng.randint(1, 5)})
            assert oracle.align(prot, dna, bigger, False).score <= sl
        d2 = np.minimum(base.donor.astype(int) + 3, 255).astype(np.uint8)
        assert oracle.align(prot, dna, base.replace(donor=d2), False).score <= sl


def test_all_trp_reaches_the_score_bound():
    """Each protein residue adds at most the matrix's largest entry (W:W = 11
    under BLOSUM62) and every other term is a penalty, so a score is at most
    11 m.  W^m against (TGG)^m in random flanks attains it on an ungapped path
    of m codon:residue steps; at m = 2,955 and 2,956 the scores straddle the
    int16 lanes' admission bound (32,511)."""
    from paper_2210_08052_amd import workloads as W
    sc = params.default_scoring()
    for pr in W.near_bound_pairs(9)[:2]:
        m = len(pr.prot)
        r = oracle.align(pr.prot, pr.dna, sc, want_tb=True)
        assert r.score == 11 * m
        assert r.ops == "%dM" % m and (r.p_beg, r.p_end) == (0, m)
        assert r.g_end - r.g_beg == 3 * m
        assert pr.dna[r.g_beg:r.g_end] == b"TGG" * m


def test_empty_inputs():
    sc = params.default_scoring()
    for mode in (0, 1):
        r = oracle.align("", "", sc.replace(mode=mode))
        assert (r.score, r.g_beg, r.g_end, r.p_beg, r.p_end, r.ops) == (0, 0, 0, 0, 0, "")
        r = oracle.align("MKV", "", sc.replace(mode=mode))
        assert r.score == 0 and r.ops == ""
    r = oracle.align("", "", sc.replace(mode=2))
    assert r.status == 0 and r.score == 0
    r = oracle.align("MK", "", sc.replace(mode=2))
    assert r.status == 0 and r.score == -(sc.q + 2 * sc.e) and r.ops == "2I"
    r = oracle.align("", "ACGTA", sc.replace(mode=2, flags=3))
    assert r.status == oracle.E_NOALN
    for prot, dna in (("", ""), ("MK", ""), ("", "ACGTA")):
        r = oracle.align(prot, dna, sc.replace(mode=3))
        assert (r.status, r.score, r.g_beg, r.g_end, r.p_beg, r.p_end, r.ops) == \
            (0, 0, len(dna), len(dna), len(prot), len(prot), "")


def test_left_extension_is_reversed_extension():
    """Without introns, every path step (codon:residue, gap, frameshift) is
    symmetric under reversal once codons are read backwards, so the best
    alignment that starts anywhere and ends at (n, m) equals the best
    extension from the origin of the reversed sequences with a reversed
    genetic code."""
    rng = random.Random(41)
    for _ in range(60):
        prot, dna = _rand_case(rng, max_n=90, max_m=25, dna_alpha="ACGTN",
                               prot_alpha=params.AA)
        sc = _rand_scoring(rng, mode=3, flags=rng.choice([1, 3]), tables=True)
        gc = np.array([sc.gcode[16 * (k % 4) + 4 * ((k // 4) % 4) + k // 16]
                       for k in range(64)], np.uint8)
        rev = sc.replace(mode=1, gcode_tab=gc)
        a = oracle.align(prot, dna, sc, True)
        b = oracle.align(prot[::-1], dna[::-1], rev, False)
        assert a.score == b.score, (prot, dna)
        assert (a.g_end, a.p_end) == (len(dna), len(prot))
        s, ge, pe = rescore.rescore(prot, dna, sc, a.g_beg, a.p_beg, a.ops)
        assert (s, ge, pe) == (a.score, a.g_end, a.p_end)


# ------------------------------------------------- planted mistakes are caught
MUTANTS = [
    # the printed match term H(i-3,j)+s consumes no residue
    ("addsc(getH(&rw, i - 3, j - 1), S ? S[24 * (j - 1) + tri] : mat[tri * 24 + P[j]])",
     "addsc(getH(&rw, i - 3, j), S ? S[24 * (j - 1) + tri] : mat[tri * 24 + P[j]])"),
    # phase-1 donor read one base late
    ("int64_t op = pen(getH(&rw, i - 1, j - 1), r + d0);",
     "int64_t op = pen(getH(&rw, i - 1, j - 1), r + dp1);"),
    # phase-1 acceptor read at a(i-1) instead of a(i-2)
    ("cand[C_B] = pen(Bv, am2);", "cand[C_B] = pen(Bv, am1);"),
    # frameshift insertion that also consumes a residue
    ("cand[C_G2] = pen(getH(&rw, i - 2, j), f);",
     "cand[C_G2] = pen(getH(&rw, i - 2, j - 1), f);"),
    # gap extension cost dropped
    ("Dv = pen(Dv, gap ? gap[4 * j + 3] : e);", "Dv = pen(Dv, gap ? gap[4 * j + 3] : 0);"),
    # wrong codon index order
    ("return c->gcode[16 * b1 + 4 * b2 + b3];", "return c->gcode[16 * b3 + 4 * b2 + b1];"),
    # left extension read at its best cell instead of at (n, m)
    ("const int fixed_end = mode == ORC_GLOBAL || mode == ORC_EXTEND_LEFT;",
     "const int fixed_end = mode == ORC_GLOBAL;"),
    # left extension started only at the origin
    ("const int floor0 = mode == ORC_LOCAL || mode == ORC_EXTEND_LEFT;",
     "const int floor0 = mode == ORC_LOCAL;"),
]


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_planted_mistake_is_detected(k, tmp_path):
    """Each plausible slip in the oracle's arithmetic makes a pin fail."""
    import ctypes
    import subprocess
    src = open(os.path.join(os.path.dirname(oracle.__file__), "mpg_oracle.c")).read()
    old, new = MUTANTS[k]
    assert old in src
    so = tmp_path / "mut.so"
    cfile = tmp_path / "mut.c"
    cfile.write_text(src.replace(old, new))
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", str(so),
                           str(cfile)])
    lib = ctypes.CDLL(str(so))
    lib.orc_align.restype = ctypes.c_int
    lib.orc_align.argtypes = oracle._load().orc_align.argtypes
    ct = params.codon_table()
    rng = random.Random(500 + k)
    caught = False
    for _ in range(2000):
        prot, dna = _rand_case(rng, max_n=12, max_m=3, prot_alpha=params.AA)
        sc = _rand_scoring(rng, tables=True)
        out = (ctypes.c_int64 * 5)()
        buf = ctypes.create_string_buffer(256)
        olen = ctypes.c_int64(0)
        st = lib.orc_align(prot.encode(), len(prot), dna.encode(), len(dna), sc.q, sc.e, sc.f,
                           sc.r, sc.flags, sc.mode, sc.mat.ctypes.data, sc.gcode.ctypes.data,
                           sc.donor.ctypes.data, sc.acceptor.ctypes.data, 1, out, buf, 256,
                           ctypes.byref(olen))
        best = brute.best_score(prot, dna, sc)
        if st != 0:
            caught |= best != NEG
        else:
            caught |= out[0] != best
        if not caught and sc.flags == 3:
            caught |= out[0] != gotoh.spliced_reduction(prot, dna, sc, ct) if st == 0 else False
        if caught:
            break
    assert caught, MUTANTS[k]
