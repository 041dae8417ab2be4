"""Pins of the pseudogene guard (Methods, "Avoiding pseudogenes") in the
oracle: the coding sequence cut out of an op string, and the rescored value
bounded below by the original path itself."""
import numpy as np
import pytest

import oracle
from oracle import pseudo
from oracle.rescore import parse, rescore
from paper_2210_08052_amd import workloads as W


def test_coding_sequence_hand_cases():
    intron = "GT" + "A" * 20 + "AG"
    # phase 0: the whole token is intron
    cds, k = pseudo.coding_sequence("ATG" + intron + "TGG", 0, "1M%dN1M" % len(intron))
    assert (cds, k) == ("ATGTGG", 1)
    # phase 1: codon base, intron, two codon bases
    dna = "ATG" + "T" + intron + "GG" + "AAA"
    cds, k = pseudo.coding_sequence(dna, 0, "1M%dU1M" % (len(intron) + 3))
    assert (cds, k) == ("ATGTGGAAA", 1)
    # phase 2: two codon bases, intron, one codon base
    dna = "ATG" + "TG" + intron + "G" + "AAA"
    cds, k = pseudo.coding_sequence(dna, 0, "1M%dV1M" % (len(intron) + 3))
    assert (cds, k) == ("ATGTGGAAA", 1)
    # a start inside the region, gaps and frameshifts
    cds, k = pseudo.coding_sequence("CCCC" + "ATGAAA" + "T" + "GGG", 4, "2M1I1G1D")
    assert (cds, k) == ("ATGAAATGGG", 0)
    # a degenerate short U keeps its bases
    cds, k = pseudo.coding_sequence("ATGCC", 0, "1M2U")
    assert (cds, k) == ("ATGCC", 1)


def _projected_ops(ops):
    """The original path on the coding sequence: N tokens vanish, every U/V
    token becomes the codon it splits (1M)."""
    out = []
    for L, op in parse(ops):
        if op == "N":
            continue
        if op in "UV":
            assert L >= 3
            out.append("1M")
        else:
            out.append("%d%s" % (L, op))
    return "".join(out)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_rescore_bounded_by_projected_path(seed):
    """The original path with its introns cut out is an end-to-end path of
    the second DP; the second DP's optimum is at least its score."""
    sc = oracle.default_scoring()
    pairs = W.batch_pairs(12, seed=seed)
    seen_introns = 0
    for p in pairs:
        prot, dna = p.prot.decode(), p.dna.decode()
        res = oracle.align(prot, dna, sc, want_tb=True)
        if any(op in "UV" and L < 3 for L, op in parse(res.ops)):
            continue
        st, adj, exons = pseudo.pseudo_rescore(prot, dna, res, sc)
        assert st == oracle.OK
        cds, introns = pseudo.coding_sequence(dna, res.g_beg, res.ops)
        seen_introns += introns
        seg = prot[res.p_beg:res.p_end]
        proj = _projected_ops(res.ops)
        s_proj, ge, pe = rescore(seg, cds, sc.replace(mode=oracle.GLOBAL), 0, 0, proj)
        assert (ge, pe) == (len(cds), len(seg))
        raw = adj + (sc.r if exons == 1 else 0)
        assert raw >= s_proj
        # the projected path gains every intron's penalty back
        assert s_proj >= res.score
    assert seen_introns > 0


def test_single_exon_pays_r():
    """A gene without introns: the second DP is the end-to-end optimum on
    the aligned genome span itself, minus r."""
    sc = oracle.default_scoring()
    rng = np.random.default_rng(9)
    prot, gene, _ = W.planted_gene(rng, 60, 0.1, 0, [], [])
    dna = "ACGTTGCA" + gene.tobytes().decode() + "TTGACCA"
    prot = prot.decode()
    res = oracle.align(prot, dna, sc, want_tb=True)
    st, adj, exons = pseudo.pseudo_rescore(prot, dna, res, sc)
    assert exons == 1 and "N" not in res.ops and "U" not in res.ops and "V" not in res.ops
    direct = oracle.align(prot[res.p_beg:res.p_end], dna[res.g_beg:res.g_end],
                          sc.replace(mode=oracle.GLOBAL, flags=oracle.NO_INTRON), want_tb=False)
    assert adj == direct.score - sc.r
