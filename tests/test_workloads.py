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


def _sha(*objs):
    """SHA-256 over workload objects: pairs (letters and traceback flag),
    arrays (dtype and bytes), ints, floats and nested lists/tuples."""
    import hashlib
    h = hashlib.sha256()

    def add(o):
        if isinstance(o, (bytes, bytearray)):
            h.update(o)
        elif isinstance(o, np.ndarray):
            h.update(str(o.dtype).encode())
            h.update(np.ascontiguousarray(o).tobytes())
        elif isinstance(o, (list, tuple)):
            h.update(b"[%d" % len(o))
            for x in o:
                add(x)
        elif isinstance(o, W.Pair):
            add(o.prot)
            add(o.dna)
            h.update(bytes([int(o.want_tb)]))
        elif isinstance(o, (int, np.integer)):
            h.update(int(o).to_bytes(8, "little", signed=True))
        elif isinstance(o, float):
            h.update(np.float64(o).tobytes())
        else:
            raise TypeError(type(o))

    for o in objs:
        add(o)
    return h.hexdigest()


# Pinned digests of the workloads the benchmark and the parity tests run: a
# change of numpy's generators or of the recipe changes every workload, and
# must show here rather than silently.
DIGESTS = {
    "single": "6da4e5ecea1f8c17a8d58eee21b856e32e563a4569e348eb0c47c84235518de4",
    "batch": "d932ddfa876680e68dbc94cfe7332021af2fe9661c55b08894176621a848f00c",
    "longtail": "558176c14225c17fc4a9750d7a4d55bcf22ba2622b279e78545284d5e66ab73f",
    "serving_first_5000": "7f65181921e965b1e639ff030abd136670e867b636abd5bf36641b5280efa65c",
    "chain_1000": "15615f3cfd122d22659be7e7ba8f1236c2ece52bd64d76d8c7af3cd0d727dacc",
    "profile_1000": "162e04091b90ab8e075687cfe0f513635ee5b5e8f4babe7277c04ba337720ce5",
    "chaining_1000": "57adacdaf4de5080f70dce910a1801c692566457903da1264972a36d343ae88a",
    "near_bound": "46d07401a56adec4ee83b457c64303f7c82e34505bf75b5a07385b4ea796dd22",
    "self_pairs_11": "0ff4873f34b0be62e0b238f3cfee2fb39e2399b99377f604a5530d088608db07",
    "near_bound_scoring": "1d7334d9c9cb67bafa3f1843c99299ff163fc4e7ab6fe4a2d209f258b0ff8444",
}


def _nb_scoring(seed, big, maxpos):
    r = W.near_bound_scoring(seed, maxpos=maxpos, big_penalties=big)
    return [r["q"], r["e"], r["f"], r["r"], r["mat"], r["donor"], r["acceptor"]]


def test_dataset_digests_pinned():
    got = {
        "single": _sha([W.single_pair(1)]),
        "batch": _sha(W.batch_pairs(10000, seed=2)),
        "longtail": _sha(W.long_tail(200, 2000, seed=4)),
        "serving_first_5000": _sha(*W.serving_jobs(5000, rate_per_s=1.0, seed=5)),
        "chain_1000": _sha(W.chain_jobs(1000, seed=6)),
        "profile_1000": _sha(W.profile_jobs(1000, seed=2, profile_seed=7)),
        "chaining_1000": _sha(W.chaining_sets(1000, seed=8)),
        "near_bound": _sha(W.near_bound_pairs(9)),
        "self_pairs_11": _sha(W.self_pairs(11, [270, 271, 269, 255, 200, 150, 90])),
        "near_bound_scoring": _sha([_nb_scoring(1, False, 120), _nb_scoring(2, True, 120),
                                    _nb_scoring(3, False, 127)]),
    }
    assert got == DIGESTS


def test_serving_stream_is_the_same_in_parallel_and_by_prefix():
    a, ta = W.serving_jobs(2500, seed=5)
    b, tb = W.serving_jobs(2500, seed=5, workers=3)
    c, tc = W.serving_jobs(1200, seed=5)
    assert _sha(a, ta) == _sha(b, tb)
    assert _sha(a[:1200], ta[:1200]) == _sha(c, tc)
