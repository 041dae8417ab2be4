"""Pins of the position-specific (profile) query in the oracle (Discussion:
position-specific substitution and gap costs for profile queries): reduction
to the protein DP, brute force, a textbook Gotoh with position-specific
costs, monotonicity, and planted mistakes."""
import os
import random

import numpy as np
import pytest

import oracle
from oracle import brute, gotoh, params
from oracle.rescore import parse

NEG = float("-inf")


def _profile_of(prot, sc):
    """The profile that a protein and one matrix with uniform gaps make."""
    S = np.array([[sc.mat[a][oracle.aa_code(c)] for a in range(24)] for c in prot], np.int8)
    S = S.reshape(len(prot), 24)
    gap = np.tile(np.array([sc.q, sc.e, sc.q, sc.e], np.int16), (len(prot) + 1, 1))
    return S, gap


def _rand_profile(rng, m, lo=-6, hi=9, gmax=9):
    S = np.array([[rng.randint(lo, hi) for _ in range(24)] for _ in range(m)], np.int8)
    S = S.reshape(m, 24)
    gap = np.array([[rng.randint(0, gmax), rng.randint(1, 4), rng.randint(0, gmax),
                     rng.randint(1, 4)] for _ in range(m + 1)], np.int16)
    return S, gap


def _rand_dna(rng, n, alpha="ACGTGTAGN"):
    return "".join(rng.choice(alpha) for _ in range(n))


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_profile_of_a_protein_is_the_protein_dp(mode):
    """Rows of the matrix picked by the residues, uniform q and e: every
    field of the result equals the protein DP's, traceback included."""
    rng = random.Random(70 + mode)
    for _ in range(40):
        prot = "".join(rng.choice(params.AA) for _ in range(rng.randint(0, 30)))
        dna = _rand_dna(rng, rng.randint(0, 200))
        sc = params.default_scoring(q=rng.randint(0, 12), e=rng.randint(1, 3),
                                    f=rng.randint(5, 30), r=rng.randint(5, 40), mode=mode,
                                    flags=rng.randint(0, 3))
        S, gap = _profile_of(prot, sc)
        a = oracle.align(prot, dna, sc, True)
        b = oracle.align_profile(S, gap, dna, sc, True)
        assert a.key() == b.key(), (prot, dna, mode)


@pytest.mark.parametrize("seed", range(4))
def test_profile_brute_force(seed):
    """Exhaustive optimum with position-specific costs equals the oracle."""
    rng = random.Random(900 + seed)
    for _ in range(80):
        m = rng.randint(0, 3)
        dna = _rand_dna(rng, rng.randint(0, 11))
        S, gap = _rand_profile(rng, m)
        sc = params.default_scoring(f=rng.randint(0, 8), r=rng.randint(0, 10),
                                    mode=rng.randint(0, 3), flags=rng.randint(0, 3))
        res = oracle.align_profile(S, gap, dna, sc, True)
        best = brute.best_score("", dna, sc, S=S, gap=gap)
        if res.status == oracle.E_NOALN:
            assert best == NEG
            continue
        assert res.score == best, (dna, S.tolist(), gap.tolist(), sc.mode, sc.flags)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_profile_reduces_to_position_specific_gotoh(mode):
    """No introns, no frameshifts: affine alignment of the translated frame
    against the profile with each column's own costs."""
    rng = random.Random(950 + mode)
    ct = params.codon_table()
    for _ in range(60):
        m = rng.randint(0, 14)
        dna = _rand_dna(rng, rng.randint(0, 48), "ACGTN")
        S, gap = _rand_profile(rng, m, gmax=12)
        sc = params.default_scoring(mode=mode, flags=oracle.NO_INTRON | oracle.NO_FS)
        res = oracle.align_profile(S, gap, dna, sc, False)
        exp = gotoh.spliced_reduction("", dna, sc, ct, S=S, gap=gap)
        got = NEG if res.status == oracle.E_NOALN else res.score
        assert got == exp, (dna, mode)


def test_profile_monotone_in_its_costs():
    rng = random.Random(99)
    for _ in range(40):
        m = rng.randint(1, 20)
        dna = _rand_dna(rng, rng.randint(10, 150))
        S, gap = _rand_profile(rng, m)
        sc = params.default_scoring(mode=0)
        base = oracle.align_profile(S, gap, dna, sc, False).score
        col = rng.randint(0, m)
        g2 = gap.copy()
        g2[col] += np.array([rng.randint(0, 5), rng.randint(0, 3), rng.randint(0, 5),
                             rng.randint(0, 3)], np.int16)
        assert oracle.align_profile(S, g2, dna, sc, False).score <= base
        S2 = S.copy()
        S2[rng.randint(0, m - 1)] += 1
        assert oracle.align_profile(S2, gap, dna, sc, False).score >= base


def test_profile_path_rescores():
    """The traced path scored by hand with the per-column costs."""
    rng = random.Random(5)
    ct = params.codon_table()
    for _ in range(60):
        m = rng.randint(1, 12)
        dna = _rand_dna(rng, rng.randint(6, 80), "ACGT")
        S, gap = _rand_profile(rng, m)
        sc = params.default_scoring(mode=rng.randint(0, 3), flags=oracle.NO_INTRON)
        res = oracle.align_profile(S, gap, dna, sc, True)
        if res.status != oracle.OK:
            continue
        g, j, tot = res.g_beg, res.p_beg, 0
        for L, op in parse(res.ops):
            if op == "M":
                for _ in range(L):
                    tot += int(S[j][params.AA.index(ct[dna[g:g + 3]])])
                    g, j = g + 3, j + 1
            elif op == "I":
                tot -= int(gap[j + 1][0]) + sum(int(gap[u][1]) for u in range(j + 1, j + L + 1))
                j += L
            elif op == "D":
                tot -= int(gap[j][2]) + L * int(gap[j][3])
                g += 3 * L
            elif op == "F":
                tot -= sc.f
                g, j = g + L, j + 1
            else:  # G
                tot -= sc.f
                g += L
        assert (tot, g, j) == (res.score, res.g_end, res.p_end), res


MUTANTS = [
    # I costs read at the previous column
    ("int64_t op = pen(getH(&rw, i, j - 1), gap ? gap[4 * j] : q);",
     "int64_t op = pen(getH(&rw, i, j - 1), gap ? gap[4 * (j - 1)] : q);"),
    # D extension cost taken from the I slot
    ("Dv = pen(Dv, gap ? gap[4 * j + 3] : e);", "Dv = pen(Dv, gap ? gap[4 * j + 1] : e);"),
    # profile row of the next column
    ("S ? S[24 * (j - 1) + tri]", "S ? S[24 * (j < m ? j : j - 1) + tri]"),
]


@pytest.mark.parametrize("k", range(len(MUTANTS)))
def test_profile_planted_mistake_is_detected(k, tmp_path):
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
    lib.orc_align_profile.restype = ctypes.c_int
    lib.orc_align_profile.argtypes = oracle._load().orc_align_profile.argtypes
    rng = random.Random(700 + k)
    caught = False
    for _ in range(2000):
        m = rng.randint(1, 3)
        dna = _rand_dna(rng, rng.randint(3, 11))
        S, gap = _rand_profile(rng, m)
        sc = params.default_scoring(f=rng.randint(0, 8), r=rng.randint(0, 10),
                                    mode=rng.randint(0, 3), flags=rng.randint(0, 3))
        out = (ctypes.c_int64 * 5)()
        buf = ctypes.create_string_buffer(256)
        olen = ctypes.c_int64(0)
        st = lib.orc_align_profile(S.ctypes.data, gap.ctypes.data, m, dna.encode(), len(dna),
                                   sc.f, sc.r, sc.flags, sc.mode, sc.gcode.ctypes.data,
                                   sc.donor.ctypes.data, sc.acceptor.ctypes.data, 1, out, buf,
                                   256, ctypes.byref(olen))
        best = brute.best_score("", dna, sc, S=S, gap=gap)
        caught |= (best != NEG) if st != 0 else (out[0] != best)
        if caught:
            break
    assert caught, MUTANTS[k]
