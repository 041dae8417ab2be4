"""Pseudogene guard -- TEST INFRASTRUCTURE ONLY.

Methods, "Avoiding pseudogenes": an unspliced pseudogene of a spliced gene
can outscore the gene because it pays no intron penalties.  So, after the
spliced alignment, the protein is aligned again to the translated coding
region with the introns removed, and an alignment with a single exon is
further charged the intron open score r of Eq. (full).

Readings taken here (the paper states the idea in two sentences):
  * the coding sequence is the genome bases the op string consumes, in
    order, without each intron's interior: an N token (phase 0) drops all its
    bases; a U token (phase 1) keeps its first base and its last two, a V
    token (phase 2) its first two and its last one -- the bases of the codon
    the intron splits (a U/V token shorter than 3 keeps all its bases);
  * the new score is the end-to-end (GLOBAL) optimum of Eq. (fs), i.e.
    Eq. (full) without intron states, between the aligned protein segment
    P[p_beg..p_end) and that coding sequence, with the same scoring;
  * exons = number of N/U/V tokens + 1; a single exon subtracts r.

Parity unpinned for these readings (the mode of the second DP and the
split-codon handling); the pins in the tests are the lower bound that the
original path itself provides, closed forms on hand-made cases, and the
oracle DP (itself pinned) for the second alignment.
"""
from __future__ import annotations

from . import GLOBAL, NO_INTRON, OK, align
from .rescore import parse


def coding_sequence(dna: str, g_beg: int, ops: str):
    """(coding sequence, intron count) of the alignment starting at genome
    offset g_beg (0-based: the first consumed base is dna[g_beg])."""
    out = []
    i = g_beg  # bases consumed so far = index of the next base
    introns = 0
    for L, op in parse(ops):
        if op == "M" or op == "D":
            out.append(dna[i:i + 3 * L])
            i += 3 * L
        elif op == "I":
            pass
        elif op in "FG":
            out.append(dna[i:i + L])
            i += L
        else:
            introns += 1
            seg = dna[i:i + L]
            if op == "N":
                pass
            elif L < 3:
                out.append(seg)
            elif op == "U":
                out.append(seg[:1] + seg[L - 2:])
            else:
                out.append(seg[:2] + seg[L - 1:])
            i += L
    return "".join(out), introns


def pseudo_rescore(prot: str, dna: str, res, sc):
    """(status, adjusted score, exon count) for one traced oracle result."""
    cds, introns = coding_sequence(dna, res.g_beg, res.ops)
    seg = prot[res.p_beg:res.p_end]
    r2 = align(seg, cds, sc.replace(mode=GLOBAL, flags=sc.flags | NO_INTRON), want_tb=False)
    exons = introns + 1
    if r2.status != OK:
        return r2.status, 0, exons
    return OK, r2.score - (sc.r if exons == 1 else 0), exons
