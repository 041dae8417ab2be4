"""Seeded synthetic planted-gene workloads.

This module only makes inputs: proteins, genomic regions and (for parity
tests) random scoring tables.  It holds none of the DP's arithmetic and is the
one module that both the GPU path and the CPU oracle consume.

The paper measures on real proteomes and genomes (Results, "Evaluation
datasets"); those are not available here, so seeded planted genes with the
same kind of structure stand in for them:

1. draw a query protein of L residues uniformly over the 20 standard amino
   acids;
2. mutate round(rho*L) distinct positions, replacing a by b != a with
   probability proportional to 2**(S(a,b)/2) under BLOSUM62 (no stops);
3. reverse-translate the mutated protein with uniformly chosen synonymous
   codons (standard genetic code, no start or stop codon added);
4. plant frameshifts: each inserts one random base or deletes one base
   (50/50) at a uniform coding position;
5. split the coding sequence into E exons (every exon >= 10 nt, cut points
   >= 3 nt away from frameshifts) joined by introns made of a donor
   dinucleotide, a uniform random interior and an acceptor dinucleotide;
   canonical introns are GT..AG, non-canonical ones are uniform over
   GC..AG, AT..AC and a random dinucleotide pair other than (GT, AG);
6. pad both flanks with uniform random DNA.

All draws use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

STD20 = "ARNDCQEGHILKMFPSTWYV"
BASES = np.frombuffer(b"ACGT", dtype=np.uint8)

# BLOSUM62 restricted to the 20 standard residues, rows/cols in STD20 order;
# used only for the substitution likelihood of step 2.
_B62_20 = """
 4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0
-1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3
-2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3
-2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3
 0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1
-1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2
-1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2
 0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3
-2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3
-1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3
-1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1
-1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2
-1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1
-2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1
-1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2
 1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2
 0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0
-3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3
-2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1
 0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4
"""

# Synonymous codons of the standard code, per residue.
_SYN = {
    "A": "GCT GCC GCA GCG", "R": "CGT CGC CGA CGG AGA AGG", "N": "AAT AAC",
    "D": "GAT GAC", "C": "TGT TGC", "Q": "CAA CAG", "E": "GAA GAG",
    "G": "GGT GGC GGA GGG", "H": "CAT CAC", "I": "ATT ATC ATA",
    "L": "TTA TTG CTT CTC CTA CTG", "K": "AAA AAG", "M": "ATG", "F": "TTT TTC",
    "P": "CCT CCC CCA CCG", "S": "TCT TCC TCA TCG AGT AGC",
    "T": "ACT ACC ACA ACG", "W": "TGG", "Y": "TAT TAC",
    "V": "GTT GTC GTA GTG",
}


def _b62_20() -> np.ndarray:
    rows = [ln.split() for ln in _B62_20.strip().splitlines()]
    return np.array(rows, dtype=np.int64)


def _subst_cdf() -> np.ndarray:
    s = _b62_20().astype(np.float64)
    w = np.power(2.0, s / 2.0)
    np.fill_diagonal(w, 0.0)
    w /= w.sum(axis=1, keepdims=True)
    return np.cumsum(w, axis=1)


def _syn_table():
    tab = np.zeros((20, 6, 3), dtype=np.uint8)
    cnt = np.zeros(20, dtype=np.int64)
    for k, aa in enumerate(STD20):
        cods = _SYN[aa].split()
        cnt[k] = len(cods)
        for c, cod in enumerate(cods):
            tab[k, c] = np.frombuffer(cod.encode(), dtype=np.uint8)
    return tab, cnt


_CDF = _subst_cdf()
_SYNTAB, _SYNCNT = _syn_table()
_STD = np.frombuffer(STD20.encode(), dtype=np.uint8)


@dataclass
class Pair:
    """One synthetic job: query protein and genomic region (ASCII bytes)."""
    prot: bytes
    dna: bytes
    want_tb: bool = False
    truth: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return len(self.prot) * len(self.dna)


def _rand_dna(rng, k: int) -> np.ndarray:
    return BASES[rng.integers(0, 4, size=k)]


def _intron(rng, length: int, canonical: bool) -> np.ndarray:
    interior = _rand_dna(rng, max(0, length - 4))
    if canonical:
        d, a = b"GT", b"AG"
    else:
        kind = rng.integers(0, 3)
        if kind == 0:
            d, a = b"GC", b"AG"
        elif kind == 1:
            d, a = b"AT", b"AC"
        else:
            while True:
                d = bytes(BASES[rng.integers(0, 4, size=2)])
                a = bytes(BASES[rng.integers(0, 4, size=2)])
                if (d, a) != (b"GT", b"AG"):
                    break
    return np.concatenate([np.frombuffer(d, np.uint8), interior, np.frombuffer(a, np.uint8)])


def _cuts(rng, cds_len: int, n_cuts: int, avoid: list) -> list | None:
    """n_cuts distinct cut points, every piece >= 10 nt, >= 3 nt from avoid."""
    if n_cuts == 0:
        return []
    lo, hi = 10, cds_len - 10
    if hi - lo + 1 < n_cuts:
        return None
    for _ in range(100):
        c = np.sort(rng.choice(np.arange(lo, hi + 1), size=n_cuts, replace=False))
        if n_cuts > 1 and np.min(np.diff(c)) < 10:
            continue
        if any(abs(int(x) - a) < 3 for x in c for a in avoid):
            continue
        return [int(x) for x in c]
    return None


def planted_gene(rng, L: int, rho: float, n_fs: int, intron_lens: list,
                 canonical: list, residues=None):
    """Steps 1-5: returns (query protein bytes, gene bytes, truth dict).
    ``residues`` (indices into STD20) replaces the draw of step 1."""
    prot = rng.integers(0, 20, size=L) if residues is None else np.asarray(residues, np.int64)
    mut = prot.copy()
    k = int(round(rho * L))
    if k:
        pos = rng.choice(L, size=k, replace=False)
        u = rng.random(k)
        for p, uu in zip(pos, u):
            b = int(np.searchsorted(_CDF[mut[p]], uu, side="right"))
            mut[p] = min(b, 19)
    idx = np.floor(rng.random(L) * _SYNCNT[mut]).astype(np.int64)
    cds = _SYNTAB[mut, idx].reshape(-1).copy()
    # where each residue's codon starts in the coding sequence, -1 once a
    # frameshift has broken it (bookkeeping only: no draws)
    cpos = np.arange(L, dtype=np.int64) * 3
    fs = []
    for _ in range(n_fs):
        if len(cds) < 8:
            break
        p = int(rng.integers(3, len(cds) - 3))
        if rng.random() < 0.5:
            cds = np.insert(cds, p, BASES[rng.integers(0, 4)])
            fs.append(("ins", p))
            ok = cpos >= 0
            cpos[ok & (cpos < p) & (cpos + 3 > p)] = -1
            cpos[(cpos >= 0) & (cpos >= p)] += 1
        else:
            cds = np.delete(cds, p)
            fs.append(("del", p))
            ok = cpos >= 0
            cpos[ok & (cpos <= p) & (cpos + 3 > p)] = -1
            cpos[(cpos >= 0) & (cpos > p)] -= 1
    cuts = None
    n_introns = len(intron_lens)
    while n_introns > 0:
        cuts = _cuts(rng, len(cds), n_introns, [p for _, p in fs])
        if cuts is not None:
            break
        n_introns -= 1
    cuts = cuts or []
    pieces, introns = [], []
    prev = 0
    for c in range(len(cuts)):
        pieces.append(cds[prev:cuts[c]])
        introns.append(_intron(rng, int(intron_lens[c]), bool(canonical[c])))
        prev = cuts[c]
    pieces.append(cds[prev:])
    parts = []
    exons = []
    off = 0
    for e, piece in enumerate(pieces):
        exons.append((off, off + len(piece)))
        parts.append(piece)
        off += len(piece)
        if e < len(introns):
            parts.append(introns[e])
            off += len(introns[e])
    gene = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    # codon positions in the gene; a codon split by an intron gets -1
    codon_at = np.full(L, -1, dtype=np.int64)
    shift = 0
    bounds = list(cuts) + [len(cds)]
    lo = 0
    for e, hi in enumerate(bounds):
        sel = (cpos >= lo) & (cpos + 3 <= hi)
        codon_at[sel] = cpos[sel] + shift
        if e < len(introns):
            shift += len(introns[e])
        lo = hi
    truth = {"exons": exons, "cuts": cuts, "frameshifts": fs, "n_subst": k,
             "intron_lens": [len(x) for x in introns],
             "canonical": [bool(x) for x in canonical[:len(introns)]],
             "codon_at": codon_at, "kept": mut == prot}
    return _STD[prot].tobytes(), gene, truth


def _finish(rng, prot, gene, truth, region: int, left: int) -> Pair:
    right = region - len(gene) - left
    dna = np.concatenate([_rand_dna(rng, left), gene, _rand_dna(rng, right)])
    truth = dict(truth)
    truth["gene_start"] = left
    truth["exons"] = [(a + left, b + left) for a, b in truth["exons"]]
    if "codon_at" in truth:
        ca = truth["codon_at"].copy()
        ca[ca >= 0] += left
        truth["codon_at"] = ca
    return Pair(prot, dna.tobytes(), False, truth)


def single_pair(seed: int = 1) -> Pair:
    """One pair: 100 aa, 20 substitutions, one 1-nt frameshift, 3 exons split
    by 2 GT..AG introns of 80-400 nt, region exactly 3,000 nt; traceback on."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ilens = [int(x) for x in rng.integers(80, 401, size=2)]
    prot, gene, truth = planted_gene(rng, 100, 0.20, 1, ilens, [True, True])
    region = 3000
    left = int(rng.integers(0, region - len(gene) + 1))
    p = _finish(rng, prot, gene, truth, region, left)
    p.want_tb = True
    return p


def _short_pair(rng, L: int) -> Pair | None:
    n_ex = int(rng.geometric(0.2))
    ilens = [int(np.clip(round(rng.lognormal(math.log(300), 1.0)), 60, 10000))
             for _ in range(n_ex - 1)]
    canon = [bool(rng.random() < 0.8) for _ in range(n_ex - 1)]
    rho = float(rng.uniform(0.10, 0.40))
    n_fs = int(rng.integers(0, 3))
    prot, gene, truth = planted_gene(rng, L, rho, n_fs, ilens, canon)
    region = int(round(1.2 * len(gene)))
    if region > 40000:
        return None
    left = int(rng.integers(0, region - len(gene) + 1))
    return _finish(rng, prot, gene, truth, region, left)


def batch_pairs(n_pairs: int = 10000, seed: int = 2) -> list:
    """Planted-gene pairs: L = clip(round(LogNormal(ln 400, 0.5)), 50, 2000),
    exon count Geometric(0.2) (mean 5), intron length
    clip(round(LogNormal(ln 300, 1.0)), 60, 10000), substitution rate
    U(0.1, 0.4), 0-2 frameshifts, 80% canonical introns, region round(1.2 x
    span) (pairs above 40,000 nt are redrawn)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    while len(out) < n_pairs:
        L = int(np.clip(round(rng.lognormal(math.log(400), 0.5)), 50, 2000))
        p = _short_pair(rng, L)
        if p is not None:
            out.append(p)
    return out


def _long_pair(rng) -> Pair:
    R = int(rng.integers(100000, 300001))
    L = int(rng.integers(3000, 8001))
    n_int = max(4, int(round((R / 1.2 - 3 * L) / 3300.0)))
    while True:
        ilens = None
        for _ in range(100):
            cand = [int(np.clip(round(rng.lognormal(math.log(2000), 1.0)), 60, 50000))
                    for _ in range(n_int)]
            if 3 * L + 2 + sum(cand) <= 0.9 * R:
                ilens = cand
                break
        if ilens is not None or n_int == 0:
            break
        n_int -= 1
    ilens = ilens or []
    canon = [bool(rng.random() < 0.8) for _ in ilens]
    rho = float(rng.uniform(0.10, 0.40))
    n_fs = int(rng.integers(0, 3))
    prot, gene, truth = planted_gene(rng, L, rho, n_fs, ilens, canon)
    lo = int(math.ceil(0.05 * R))
    hi = R - len(gene) - lo
    left = int(rng.integers(lo, max(lo, hi) + 1))
    left = min(left, R - len(gene))
    return _finish(rng, prot, gene, truth, R, left)


def long_tail(n_long: int = 200, n_short: int = 2000, seed: int = 4) -> list:
    """200 long pairs (L ~ U{3000..8000}, region ~ U[100k, 300k], intron
    clip(round(LogNormal(ln 2000, 1.0)), 60, 50000)) mixed with 2,000 short
    pairs (L ~ U{100..300}, otherwise the batch rules); traceback on."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = [_long_pair(rng) for _ in range(n_long)]
    while len(out) < n_long + n_short:
        p = _short_pair(rng, int(rng.integers(100, 301)))
        if p is not None:
            out.append(p)
    order = rng.permutation(len(out))
    out = [out[i] for i in order]
    for p in out:
        p.want_tb = True
    return out


SERVING_CHUNK = 1000  # jobs per independently seeded chunk of the serving stream


def _serving_chunk(args) -> list:
    """Jobs [c * SERVING_CHUNK, ...) of the serving stream: chunk c draws from
    its own generator PCG64(SeedSequence([seed, 1, c])), so the stream is the
    same whichever process draws which chunk.  The serving jobs keep no
    ground truth (only the letters and the traceback flag are used)."""
    seed, c, count, p_long_mix, p_tb = args
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1, c])))
    out = []
    for _ in range(count):
        if rng.random() >= p_long_mix:
            p = None
            while p is None:
                L = int(np.clip(round(rng.lognormal(math.log(400), 0.5)), 50, 2000))
                p = _short_pair(rng, L)
        elif rng.random() < 200.0 / 2200.0:
            p = _long_pair(rng)
        else:
            p = None
            while p is None:
                p = _short_pair(rng, int(rng.integers(100, 301)))
        p.want_tb = bool(rng.random() < p_tb)
        p.truth = {}
        out.append(p)
    return out


def serving_jobs(n_jobs: int = 200000, rate_per_s: float = 1000.0, seed: int = 5,
                 p_long_mix: float = 0.1, p_tb: float = 0.5, progress=None, workers: int = 1):
    """Poisson job stream: each job is a batch-distribution pair w.p. 0.9, else
    a long-tail-mixture pair (long w.p. 200/2200); traceback w.p. 0.5.
    Returns (pairs, arrival_times_s).  Jobs come in chunks of SERVING_CHUNK,
    each drawn from its own seeded generator (so the first k jobs of a longer
    stream are the stream of k jobs, and `workers` processes draw the chunks
    in parallel with the same result); the exponential inter-arrival gaps
    come from PCG64(SeedSequence([seed, 2])) and scale exactly as 1/rate_per_s.
    ``progress(k)`` is called every 10,000 jobs if given."""
    tasks = [(seed, c, min(SERVING_CHUNK, n_jobs - c * SERVING_CHUNK), p_long_mix, p_tb)
             for c in range((n_jobs + SERVING_CHUNK - 1) // SERVING_CHUNK)]
    jobs = []

    def take(part):
        before = len(jobs)
        jobs.extend(part)
        if progress is not None and len(jobs) // 10000 > before // 10000:
            progress(len(jobs) // 10000 * 10000)

    if workers > 1 and len(tasks) > 1:
        import multiprocessing
        from concurrent.futures import ProcessPoolExecutor
        # fresh interpreters: the parent may already hold a GPU runtime
        ctx = multiprocessing.get_context("spawn")
        with ProcessPoolExecutor(max_workers=min(workers, len(tasks)), mp_context=ctx) as ex:
            for part in ex.map(_serving_chunk, tasks):
                take(part)
    else:
        for t in tasks:
            take(_serving_chunk(t))
    grng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    gaps = grng.exponential(1.0 / rate_per_s, size=n_jobs)
    return jobs, np.cumsum(gaps)


def random_pairs(n: int, seed: int, max_prot: int = 40, max_dna: int = 400,
                 alphabet_dna: str = "ACGT", alphabet_prot: str = STD20,
                 min_prot: int = 0, min_dna: int = 0) -> list:
    """Unstructured random pairs (uniform lengths and letters)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    da = np.frombuffer(alphabet_dna.encode(), np.uint8)
    pa = np.frombuffer(alphabet_prot.encode(), np.uint8)
    out = []
    for _ in range(n):
        m = int(rng.integers(min_prot, max_prot + 1))
        L = int(rng.integers(min_dna, max_dna + 1))
        out.append(Pair(pa[rng.integers(0, len(pa), m)].tobytes(),
                        da[rng.integers(0, len(da), L)].tobytes()))
    return out


def random_scoring(seed: int, with_tables: bool = True) -> dict:
    """Random scoring inputs (penalties, symmetric 24x24 matrix, splice tables)
    for parity tests; zeros and equal values are drawn on purpose to force
    ties."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {"q": int(rng.integers(0, 13)), "e": int(rng.integers(1, 4)),
           "f": int(rng.integers(0, 30)), "r": int(rng.integers(0, 40))}
    if with_tables:
        m = rng.integers(-6, 12, size=(24, 24))
        m = np.triu(m) + np.triu(m, 1).T
        out["mat"] = m.astype(np.int8)
        out["donor"] = rng.integers(0, 31, size=125).astype(np.uint8)
        out["acceptor"] = rng.integers(0, 31, size=125).astype(np.uint8)
    return out


def near_bound_pairs(seed: int = 9) -> list:
    """Pairs whose best LOCAL score under BLOSUM62 lies just under the int16
    lanes' admission bound (m * 11 <= 32,511 for a protein of m residues, W:W
    = 11 being the matrix's largest entry): Trp-rich proteins of 2,940-2,956
    residues against their own planted genes.

    * pair 0: W^2955 against (TGG)^2955 in random flanks (best score exactly
      11 * 2955 = 32,505);
    * pair 1: W^2956 against (TGG)^2956 (bound 32,516: beyond it);
    * pairs 2-9: 97-99.9 % W (the rest uniform over the 20 residues),
      0-0.5 % substitutions, 0-1 frameshift, 1-2 canonical introns of 60-300 nt,
      300-700 nt flanks."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = STD20.index("W")
    out = []
    for L in (2955, 2956):
        left, right = int(rng.integers(300, 701)), int(rng.integers(300, 701))
        gene = np.frombuffer(b"TGG" * L, np.uint8)
        dna = np.concatenate([_rand_dna(rng, left), gene, _rand_dna(rng, right)])
        out.append(Pair(b"W" * L, dna.tobytes(), False, {"gene_start": left}))
    for _ in range(8):
        L = int(rng.integers(2940, 2956))
        frac_w = float(rng.uniform(0.97, 0.999))
        res = np.where(rng.random(L) < frac_w, w, rng.integers(0, 20, size=L))
        n_in = int(rng.integers(1, 3))
        ilens = [int(x) for x in rng.integers(60, 301, size=n_in)]
        prot, gene, truth = planted_gene(rng, L, float(rng.uniform(0.0, 0.005)),
                                         int(rng.integers(0, 2)), ilens, [True] * n_in,
                                         residues=res)
        left, right = int(rng.integers(300, 701)), int(rng.integers(300, 701))
        out.append(_finish(rng, prot, gene, truth, len(gene) + left + right, left))
    return out


def near_bound_scoring(seed: int, maxpos: int = 120, big_penalties: bool = False) -> dict:
    """Random scoring inputs with large entries for int16-bound tests: a
    symmetric 24x24 matrix drawn in [-128, maxpos - 1] whose 20 standard
    diagonal entries are maxpos (so a protein against its own reverse
    translation scores maxpos per residue), and penalties either moderate
    (gap open 0-40, extend 1-10, frameshift 0-60, intron 0-80, splice tables
    0-30) or near the int16 lanes' penalty limit of 8,192 (gap open
    1,000-5,000, extend 500-3,000, frameshift 4,000-8,000, intron
    5,000-7,600, splice tables 0-255)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.integers(-128, maxpos, size=(24, 24))
    m = np.triu(m) + np.triu(m, 1).T
    m[np.arange(20), np.arange(20)] = maxpos
    if big_penalties:
        q, e = int(rng.integers(1000, 5001)), int(rng.integers(500, 3001))
        out = {"q": q, "e": min(e, 8192 - q), "f": int(rng.integers(4000, 8001)),
               "r": int(rng.integers(5000, 7601))}
        hi = 256
    else:
        out = {"q": int(rng.integers(0, 41)), "e": int(rng.integers(1, 11)),
               "f": int(rng.integers(0, 61)), "r": int(rng.integers(0, 81))}
        hi = 31
    out["mat"] = m.astype(np.int8)
    out["donor"] = rng.integers(0, hi, size=125).astype(np.uint8)
    out["acceptor"] = rng.integers(0, hi, size=125).astype(np.uint8)
    return out


def self_pairs(seed: int, lengths, rho: float = 0.01) -> list:
    """One planted gene per protein length (uniform residues, rho
    substitutions, 0-1 frameshift, 0-2 canonical introns of 60-300 nt,
    100-400 nt flanks): against a matrix whose diagonal is its largest entry
    the best score is close to length * that entry."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for L in lengths:
        n_in = int(rng.integers(0, 3))
        ilens = [int(x) for x in rng.integers(60, 301, size=n_in)]
        prot, gene, truth = planted_gene(rng, int(L), rho, int(rng.integers(0, 2)), ilens,
                                         [True] * n_in)
        left, right = int(rng.integers(100, 401)), int(rng.integers(100, 401))
        out.append(_finish(rng, prot, gene, truth, len(gene) + left + right, left))
    return out


def true_anchors(pair: Pair, k: int = 6) -> list:
    """Every exact seed hit of k residues on the planted path: (x, y) with
    residues y..y+k-1 unchanged by the substitutions and their codons
    consecutive and whole in the region at x, x+3, ... (0-based)."""
    ca, kept = pair.truth["codon_at"], pair.truth["kept"]
    L = len(ca)
    good = (ca >= 0) & kept
    out = []
    for y in range(0, L - k + 1):
        w = ca[y:y + k]
        if good[y:y + k].all() and (np.diff(w) == 3).all():
            out.append((int(w[0]), y))
    return out


def chain_jobs(n_chains: int = 10000, seed: int = 6, k: int = 6, keep: float = 0.25) -> list:
    """Planted-gene pairs of the batch distribution with a chain of anchors
    each: the true seed hits of k residues (see true_anchors), each kept with
    probability `keep` (so kept hits often overlap on one diagonal), in
    genome order.  Pairs without a kept hit are redrawn.  Returns a list of
    (Pair, anchors)."""
    pairs = batch_pairs(int(n_chains * 1.3) + 16, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    out = []
    for p in pairs:
        hits = true_anchors(p, k)
        sel = [h for h, u in zip(hits, rng.random(len(hits))) if u < keep]
        if not sel:
            continue
        out.append((p, sorted(sel)))
        if len(out) == n_chains:
            break
    if len(out) < n_chains:
        raise RuntimeError("not enough chains drawn")
    return out


_B62_20_ARR = None


def family_profile(prot: bytes, rng, members: int = 3, loop_rate: float = 0.02,
                   loop_len: int = 6) -> tuple:
    """A position-specific query standing in for a gene-family profile: column
    j averages (rounded half to even) the BLOSUM62 rows of the query residue
    and of `members` family members' residues, each the query residue with
    probability 0.7, else drawn from it with the substitution law of step 2;
    amino acids B, Z and X score -1 and the stop -4.  Gap costs are 11 to
    open and 1 to extend, except in loops: runs of loop_len columns starting
    with probability loop_rate per column, where opening costs 5.  Returns
    (score (m, 24) int8, gap (m + 1, 4) int16)."""
    global _B62_20_ARR
    if _B62_20_ARR is None:
        _B62_20_ARR = _b62_20().astype(np.float64)
    idx = np.array([STD20.index(chr(c)) for c in prot], dtype=np.int64)
    m = len(idx)
    S = np.zeros((m, 24), dtype=np.int8)
    if m:
        keep = rng.random((m, members)) < 0.7
        draws = rng.random((m, members))
        rows = np.empty((m, members + 1), dtype=np.int64)
        rows[:, 0] = idx
        for t in range(members):
            for j in range(m):
                rows[j, t + 1] = idx[j] if keep[j, t] else min(
                    int(np.searchsorted(_CDF[idx[j]], draws[j, t], side="right")), 19)
        S[:, :20] = np.rint(_B62_20_ARR[rows].mean(axis=1)).astype(np.int8)
        S[:, 20:23] = -1
        S[:, 23] = -4
    gap = np.tile(np.array([11, 1, 11, 1], dtype=np.int16), (m + 1, 1))
    starts = np.nonzero(rng.random(m + 1) < loop_rate)[0]
    for st in starts:
        gap[st:st + loop_len, 0] = 5
        gap[st:st + loop_len, 2] = 5
    return S, gap


def profile_jobs(n: int = 10000, seed: int = 2, profile_seed: int = 7) -> list:
    """The planted-gene batch (batch_pairs(n, seed)) with each query protein
    replaced by its family profile (family_profile, its own generator seeded
    with profile_seed).  Returns a list of (Pair, score, gap)."""
    pairs = batch_pairs(n, seed=seed)
    rng = np.random.Generator(np.random.PCG64(profile_seed))
    return [(p,) + family_profile(p.prot, rng) for p in pairs]


def chaining_sets(n_sets: int = 10000, seed: int = 8, k: int = 6, keep: float = 0.5,
                  noise: float = 1.0, spread: int = 2_000_000, binned: bool = True) -> list:
    """Anchor sets for chaining, one per planted gene of the batch recipe
    (seed `seed`): the true seed hits (true_anchors) kept with probability
    `keep`, placed at a random locus of a 100-Mb genome, plus Poisson(noise x
    hits + 5) spurious hits uniform within `spread` bases of the locus and
    uniform in the protein.  x is the genome base, or its 256-bp bin when
    binned.  Each set is sorted by (x, y).  Returns a list of int32 arrays of
    shape (n, 2)."""
    pairs = batch_pairs(n_sets, seed=seed)
    rng = np.random.Generator(np.random.PCG64(seed + 2000))
    out = []
    for p in pairs:
        hits = true_anchors(p, k)
        L = len(p.prot)
        sel = [h for h, u in zip(hits, rng.random(len(hits))) if u < keep]
        base = int(rng.integers(spread, 100_000_000 - spread))
        nn = int(rng.poisson(noise * len(sel) + 5))
        xs = [base + x for x, _ in sel] + [int(v) for v in
                                           rng.integers(base - spread, base + spread, nn)]
        ys = [y for _, y in sel] + [int(v) for v in rng.integers(0, max(1, L - k + 1), nn)]
        a = np.array(list(zip(xs, ys)), dtype=np.int64).reshape(-1, 2)
        if binned:
            a[:, 0] //= 256
        a = a[np.lexsort((a[:, 1], a[:, 0]))]
        out.append(a.astype(np.int32))
    return out


def digest(pairs) -> str:
    """SHA-256 over the concatenated pairs (determinism checks)."""
    h = hashlib.sha256()
    for p in pairs:
        h.update(len(p.prot).to_bytes(4, "little"))
        h.update(p.prot)
        h.update(len(p.dna).to_bytes(4, "little"))
        h.update(p.dna)
    return h.hexdigest()
