"""The seeded input generator: determinism and the stated workload shapes."""
import numpy as np

from paper_2210_08052_amd import workloads as W


def test_single_pair_shape():
    p = W.single_pair(1)
    assert len(p.prot) == 100 and len(p.dna) == 3000 and p.want_tb
    assert len(p.truth["exons"]) == 3 and all(p.truth["canonical"])
    assert all(80 <= L <= 400 for L in p.truth["intron_lens"])
    assert p.truth["n_subst"] == 20 and len(p.truth["frameshifts"]) == 1
    for (a, b), (c, d) in zip(p.truth["exons"][:-1], p.truth["exons"][1:]):
        assert p.dna[b:b + 2] == b"GT" and p.dna[c - 2:c] == b"AG"


def test_determinism():
    assert W.digest(W.batch_pairs(50, seed=2)) == W.digest(W.batch_pairs(50, seed=2))
    assert W.digest(W.batch_pairs(50, seed=2)) != W.digest(W.batch_pairs(50, seed=3))
    assert W.digest([W.single_pair(1)]) == W.digest([W.single_pair(1)])


def test_batch_distribution():
    ps = W.batch_pairs(400, seed=2)
    m = np.array([len(p.prot) for p in ps])
    n = np.array([len(p.dna) for p in ps])
    assert m.min() >= 50 and m.max() <= 2000 and 300 < np.median(m) < 500
    assert n.max() <= 40000
    assert set(b"".join(p.dna for p in ps)) <= set(b"ACGT")
    assert set(b"".join(p.prot for p in ps)) <= set(W.STD20.encode())


def test_long_tail_shape():
    ps = W.long_tail(3, 10, seed=4)
    longs = [p for p in ps if len(p.prot) >= 3000]
    assert len(longs) == 3 and len(ps) == 13
    for p in longs:
        assert 100000 <= len(p.dna) <= 300000 and len(p.truth["exons"]) >= 5
    assert all(p.want_tb for p in ps)


def test_reverse_translation_codes_the_mutated_protein():
    """Every synonymous codon table entry of the generator translates back to
    its residue under the standard code (cross-check of the generator's copy
    of the code against the oracle's)."""
    from oracle import params
    ct = params.codon_table()
    for aa, cods in W._SYN.items():
        for c in cods.split():
            assert ct[c] == aa
    assert sum(len(c.split()) for c in W._SYN.values()) == 61
