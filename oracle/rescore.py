"""Op-string rescorer -- TEST INFRASTRUCTURE ONLY.

Recomputes the score of an alignment from its begin cell and its run-length
op string, segment by segment (segment costs as in ``brute``), and returns
the cell where it ends.  Op letters: ``M`` codon:residue, ``I`` residues with
no genome, ``D`` deleted codons, ``F`` frameshift substitution (1 or 2 nt, one
residue; the "$" of the paper's worked alignment), ``G`` frameshift insertion
(1 or 2 nt; the "+"), ``N``/``U``/``V`` phase-0/1/2 intron with the total
nucleotides consumed (for U and V this includes the split codon's bases).
"""
from __future__ import annotations

import re

_TOK = re.compile(r"(\d+)([MIDFGNUV])")
_DNA = {"A": 0, "C": 1, "G": 2, "T": 3}
_AA = "ARNDCQEGHILKMFPSTWYVBZX*"


class BadPath(ValueError):
    pass


def parse(ops: str):
    toks = _TOK.findall(ops)
    if "".join(a + b for a, b in toks) != ops:
        raise BadPath("malformed op string %r" % ops)
    return [(int(a), b) for a, b in toks]


def rescore(prot: str, dna: str, sc, g_beg: int, p_beg: int, ops: str):
    """Return (score, g_end, p_end) of the path; raise BadPath if it leaves the
    matrix or uses a transition that the flags remove."""
    T = [4] + [_DNA.get(ch.upper(), 4) for ch in dna]
    P = [22] + [(_AA.index(ch.upper()) if ch.upper() in _AA else 22) for ch in prot]
    n, m = len(T) - 1, len(P) - 1

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

    i, j, s = g_beg, p_beg, 0
    for L, op in parse(ops):
        if L < 1:
            raise BadPath("zero-length token")
        if op == "M":
            for _ in range(L):
                i += 3
                j += 1
                if i > n or j > m:
                    raise BadPath("M leaves the matrix")
                s += int(sc.mat[tr(i)][P[j]])
        elif op == "I":
            s -= sc.q + sc.e * L
            j += L
        elif op == "D":
            s -= sc.q + sc.e * L
            i += 3 * L
        elif op in "FG":
            if sc.flags & 2:
                raise BadPath("frameshift with frameshifts disabled")
            if L not in (1, 2):
                raise BadPath("frameshift length %d" % L)
            s -= sc.f
            i += L
            if op == "F":
                j += 1
        else:
            if sc.flags & 1:
                raise BadPath("intron with introns disabled")
            i0, k = i + 1, i + L
            if op == "N":
                s -= sc.r + d(i0 - 1) + a(k)
            elif op == "U":
                s -= sc.r + d(i0) + a(k - 2)
                j += 1
            else:
                s -= sc.r + d(i0 + 1) + a(k - 1)
                j += 1
            i = k
        if i > n or j > m:
            raise BadPath("path leaves the matrix at %s" % op)
    return s, i, j
