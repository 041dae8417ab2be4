"""Textbook affine-gap alignment of a protein against translated DNA frames --
TEST INFRASTRUCTURE ONLY.

Three separate states in the style of Eq. (durbin) (Methods, "DP with affine
gap cost"), with its printed typo corrected: the deletion state opens from
M(i-1,j) or I(i-1,j) and extends from D(i-1,j).  A gap of g residues costs
q + e*g.  With introns and frameshifts disabled, Eq. (full) must reduce to
this on each reading frame (the reduction chain Eq. (full) -> Eq. (fs) ->
Eq. (ae86) == Eq. (durbin) of the same subsection).

Written independently of the oracle's cell recurrence: its own translation,
its own loops, rows over translated codons instead of nucleotides.
"""
from __future__ import annotations

NEG = float("-inf")
_AA = "ARNDCQEGHILKMFPSTWYVBZX*"


def translate(dna: str, frame: int, codon_table: dict) -> str:
    """Translate complete codons of dna[frame:], any non-ACGT base gives X."""
    out = []
    s = dna.upper()
    for k in range(frame, len(s) - 2, 3):
        cod = s[k:k + 3]
        if all(ch in "ACGT" for ch in cod):
            out.append(codon_table[cod])
        else:
            out.append("X")
    return "".join(out)


def gotoh(prot: str, xlat: str, mat, q: int, e: int, kind: str, S=None, gap=None) -> float:
    """kind: 'local' (Smith-Waterman-Gotoh), 'extend' (start at (0,0), free
    end), 'global' (Needleman-Wunsch-Gotoh) or 'end' (start anywhere, end at
    the last codon and the last residue).  With a position-specific query (S,
    gap as in brute.best_score) prot and mat are not used: residue b scores
    S[b-1][codon], and the gap costs of the affine recurrences are the ones of
    the column the gap is at."""
    if S is None:
        P = [(_AA.index(c.upper()) if c.upper() in _AA else 22) for c in prot]
    else:
        P = [0] * len(S)
    X = [(_AA.index(c) if c in _AA else 22) for c in xlat]
    L, m = len(X), len(P)

    def sub(a, b):  # codon a (1-based) against residue b (1-based)
        return int(mat[X[a - 1]][P[b - 1]]) if S is None else int(S[b - 1][X[a - 1]])

    def oi(b):  # open + first extension of a residue gap at column b
        return q + e if gap is None else int(gap[b][0]) + int(gap[b][1])

    def ei(b):
        return e if gap is None else int(gap[b][1])

    def od(b):
        return q + e if gap is None else int(gap[b][2]) + int(gap[b][3])

    def ed(b):
        return e if gap is None else int(gap[b][3])

    def start(a, b):
        if kind in ("local", "end"):
            return 0
        return 0 if (a == 0 and b == 0) else NEG

    M = [[NEG] * (m + 1) for _ in range(L + 1)]
    Ix = [[NEG] * (m + 1) for _ in range(L + 1)]  # protein residue unmatched
    Dy = [[NEG] * (m + 1) for _ in range(L + 1)]  # codon unmatched
    best = 0 if kind != "global" else NEG
    for a in range(L + 1):
        for b in range(m + 1):
            if a >= 1 and b >= 1:
                M[a][b] = sub(a, b) + max(
                    M[a - 1][b - 1], Ix[a - 1][b - 1], Dy[a - 1][b - 1], start(a - 1, b - 1))
            if b >= 1:
                Ix[a][b] = max(M[a][b - 1] - oi(b), Ix[a][b - 1] - ei(b),
                               Dy[a][b - 1] - oi(b), start(a, b - 1) - oi(b))
            if a >= 1:
                Dy[a][b] = max(M[a - 1][b] - od(b), Dy[a - 1][b] - ed(b),
                               Ix[a - 1][b] - od(b), start(a - 1, b) - od(b))
            if kind in ("local", "extend"):
                best = max(best, M[a][b], Ix[a][b], Dy[a][b])
    if kind == "global":
        if L == 0 and m == 0:
            return 0
        return max(M[L][m], Ix[L][m], Dy[L][m])
    if kind == "end":
        return max(M[L][m], Ix[L][m], Dy[L][m], 0)
    return best


def spliced_reduction(prot: str, dna: str, sc, codon_table: dict, S=None, gap=None) -> float:
    """Expected Eq. (full) score with introns and frameshifts disabled.

    LOCAL: best Smith-Waterman-Gotoh over the three forward frames.
    EXTEND: frame 0 from the origin.  GLOBAL: frame 0, defined only when the
    region is a whole number of codons (else -inf = no alignment).
    EXTEND_LEFT: the frame whose last codon ends at the region's end, free
    start, fixed end."""
    if sc.mode == 0:
        return max(gotoh(prot, translate(dna, ph, codon_table), sc.mat, sc.q, sc.e, "local", S, gap)
                   for ph in range(3))
    if sc.mode == 1:
        return gotoh(prot, translate(dna, 0, codon_table), sc.mat, sc.q, sc.e, "extend", S, gap)
    if sc.mode == 3:
        return gotoh(prot, translate(dna, len(dna) % 3, codon_table), sc.mat, sc.q, sc.e, "end", S, gap)
    if len(dna) % 3 != 0:
        return NEG
    return gotoh(prot, translate(dna, 0, codon_table), sc.mat, sc.q, sc.e, "global", S, gap)
