"""Exhaustive optimum over the segment grammar -- TEST INFRASTRUCTURE ONLY.

An alignment of Eq. (full) is a chain of segments, each leaving state H at a
cell and entering state H at a later cell (Methods, "DP for protein-to-genome
alignment"; symbols of the worked alignment in "Residue alignment with dynamic
programming"):

====  ===========================  ==========================================
seg   consumes (nt : residues)      cost
====  ===========================  ==========================================
M     3 : 1                          + s(i,j)   (codon ending at i vs P[j])
I^L   0 : L   (L >= 1)               - (q + e L)
D^L   3L : 0  (L >= 1)               - (q + e L)
F1/F2 1 or 2 : 1                     - f        (frameshift substitution, "$")
G1/G2 1 or 2 : 0                     - f        (frameshift insertion, "+")
N     rows i0..k : 0                 - (r + d(i0-1) + a(k))     phase-0 intron
U     rows i0..k : 1                 - (r + d(i0)   + a(k-2))   phase-1
V     rows i0..k : 1                 - (r + d(i0+1) + a(k-1))   phase-2
====  ===========================  ==========================================

The recursion below maximises the summed cost over every chain of segments
ending at each cell.  It has no per-state open/extend bookkeeping, so it does
not share the structure of the cell recurrence it checks.  Pure Python: only
for tiny inputs (n <= ~12, m <= ~4).
"""
from __future__ import annotations

from functools import lru_cache

NEG = float("-inf")

_DNA = {"A": 0, "C": 1, "G": 2, "T": 3}
_AA = "ARNDCQEGHILKMFPSTWYVBZX*"


def _enc_dna(s: str):
    return [_DNA.get(ch.upper(), 4) for ch in s]


def _enc_aa(s: str):
    out = []
    for ch in s:
        c = ch.upper()
        out.append(_AA.index(c) if c in _AA else 22)
    return out


def best_score(prot: str, dna: str, sc, S=None, gap=None) -> float:
    """Maximum path score for ``sc.mode`` (LOCAL=0, EXTEND=1, GLOBAL=2,
    EXTEND_LEFT=3: start anywhere, end at (n, m)); -inf when GLOBAL has no
    path.

    With a position-specific query (S: m rows of 24 scores, gap: m+1 rows of
    I open, I extend, D open, D extend) prot is ignored: a codon at column j
    scores S[j-1][codon's amino acid], a run of residues j0..j1 against no
    genome costs I-open(j0) + the I-extend costs of j0..j1, and a run of L
    codons against no residue after column j costs D-open(j) + L D-extend(j)."""
    T = [4] + _enc_dna(dna)   # 1-based
    P = [22] + (_enc_aa(prot) if S is None else [0] * len(S))
    n, m = len(T) - 1, len(P) - 1
    q, e, f, r = sc.q, sc.e, sc.f, sc.r

    def subst(i, j):
        if S is None:
            return int(sc.mat[tr(i)][P[j]])
        return int(S[j - 1][tr(i)])

    def ins_cost(j0, j1):
        if gap is None:
            return q + e * (j1 - j0 + 1)
        return int(gap[j0][0]) + sum(int(gap[u][1]) for u in range(j0, j1 + 1))

    def del_cost(j, L):
        if gap is None:
            return q + e * L
        return int(gap[j][2]) + L * int(gap[j][3])
    no_intron = bool(sc.flags & 1)
    no_fs = bool(sc.flags & 2)
    local = sc.mode in (0, 3)

    def base(x):
        return T[x] if 1 <= x <= n else 4

    def tr(i):
        b = (base(i - 2), base(i - 1), base(i))
        if 4 in b:
            return 22
        return int(sc.gcode[16 * b[0] + 4 * b[1] + b[2]])

    def d(x):
        return int(sc.donor[25 * base(x + 1) + 5 * base(x + 2) + base(x + 3)])

    def a(x):
        return int(sc.acceptor[25 * base(x - 2) + 5 * base(x - 1) + base(x)])

    @lru_cache(maxsize=None)
    def best_to(i, j):
        if i < 0 or j < 0:
            return NEG
        v = 0 if (local or (i == 0 and j == 0)) else NEG
        if i >= 3 and j >= 1:
            v = max(v, best_to(i - 3, j - 1) + subst(i, j))
        for L in range(1, j + 1):
            v = max(v, best_to(i, j - L) - ins_cost(j - L + 1, j))
        for L in range(1, i // 3 + 1):
            v = max(v, best_to(i - 3 * L, j) - del_cost(j, L))
        if not no_fs:
            for k in (1, 2):
                v = max(v, best_to(i - k, j - 1) - f)
                v = max(v, best_to(i - k, j) - f)
        if not no_intron:
            for i0 in range(1, i + 1):
                v = max(v, best_to(i0 - 1, j) - (r + d(i0 - 1) + a(i)))
                v = max(v, best_to(i0 - 1, j - 1) - (r + d(i0) + a(i - 2)))
                v = max(v, best_to(i0 - 1, j - 1) - (r + d(i0 + 1) + a(i - 1)))
        return v

    if sc.mode in (2, 3):
        return best_to(n, m)
    return max(best_to(i, j) for i in range(n + 1) for j in range(m + 1))
