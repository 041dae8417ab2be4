"""Scoring inputs for the oracle -- TEST INFRASTRUCTURE ONLY.

The oracle keeps its own copy of every constant it uses (substitution matrix,
genetic code, splice tables); nothing here is shared with the GPU library.

* Amino-acid alphabet, 24 letters in the order of the NCBI BLOSUM files:
  ``ARNDCQEGHILKMFPSTWYVBZX*``.
* BLOSUM62 (Henikoff & Henikoff 1992; the paper scores in "BLOSUM scaling",
  Splice models subsection).  The paper does not name its matrix; BLOSUM62 is
  the default reading.  The matrix is an input of the DP, so parity does not
  depend on this choice.
* The standard genetic code (NCBI translation table 1), written here in the
  classic T,C,A,G nesting order.
* Splice models, "Splice models" subsection: the final model gives the donor
  penalty d(i) from T[i+1..i+3] and the acceptor penalty a(i) from T[i-2..i];
  the simple model (end of "DP for protein-to-genome alignment") charges p for
  a donor not starting GT and an acceptor not ending AG.
"""
from __future__ import annotations

import numpy as np

AA = "ARNDCQEGHILKMFPSTWYVBZX*"
DNA = "ACGTN"

_BLOSUM62_TEXT = """
   A  R  N  D  C  Q  E  G  H  I  L  K  M  F  P  S  T  W  Y  V  B  Z  X  *
A  4 -1 -2 -2  0 -1 -1  0 -2 -1 -1 -1 -1 -2 -1  1  0 -3 -2  0 -2 -1  0 -4
R -1  5  0 -2 -3  1  0 -2  0 -3 -2  2 -1 -3 -2 -1 -1 -3 -2 -3 -1  0 -1 -4
N -2  0  6  1 -3  0  0  0  1 -3 -3  0 -2 -3 -2  1  0 -4 -2 -3  3  0 -1 -4
D -2 -2  1  6 -3  0  2 -1 -1 -3 -4 -1 -3 -3 -1  0 -1 -4 -3 -3  4  1 -1 -4
C  0 -3 -3 -3  9 -3 -4 -3 -3 -1 -1 -3 -1 -2 -3 -1 -1 -2 -2 -1 -3 -3 -2 -4
Q -1  1  0  0 -3  5  2 -2  0 -3 -2  1  0 -3 -1  0 -1 -2 -1 -2  0  3 -1 -4
E -1  0  0  2 -4  2  5 -2  0 -3 -3  1 -2 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
G  0 -2  0 -1 -3 -2 -2  6 -2 -4 -4 -2 -3 -3 -2  0 -2 -2 -3 -3 -1 -2 -1 -4
H -2  0  1 -1 -3  0  0 -2  8 -3 -3 -1 -2 -1 -2 -1 -2 -2  2 -3  0  0 -1 -4
I -1 -3 -3 -3 -1 -3 -3 -4 -3  4  2 -3  1  0 -3 -2 -1 -3 -1  3 -3 -3 -1 -4
L -1 -2 -3 -4 -1 -2 -3 -4 -3  2  4 -2  2  0 -3 -2 -1 -2 -1  1 -4 -3 -1 -4
K -1  2  0 -1 -3  1  1 -2 -1 -3 -2  5 -1 -3 -1  0 -1 -3 -2 -2  0  1 -1 -4
M -1 -1 -2 -3 -1  0 -2 -3 -2  1  2 -1  5  0 -2 -1 -1 -1 -1  1 -3 -1 -1 -4
F -2 -3 -3 -3 -2 -3 -3 -3 -1  0  0 -3  0  6 -4 -2 -2  1  3 -1 -3 -3 -1 -4
P -1 -2 -2 -1 -3 -1 -1 -2 -2 -3 -3 -1 -2 -4  7 -1 -1 -4 -3 -2 -2 -1 -2 -4
S  1 -1  1  0 -1  0  0  0 -1 -2 -2  0 -1 -2 -1  4  1 -3 -2 -2  0  0  0 -4
T  0 -1  0 -1 -1 -1 -1 -2 -2 -1 -1 -1 -1 -2 -1  1  5 -2 -2  0 -1 -1  0 -4
W -3 -3 -4 -4 -2 -2 -3 -2 -2 -3 -2 -3 -1  1 -4 -3 -2 11  2 -3 -4 -3 -2 -4
Y -2 -2 -2 -3 -2 -1 -2 -3  2 -1 -1 -2 -1  3 -3 -2 -2  2  7 -1 -3 -2 -1 -4
V  0 -3 -3 -3 -1 -2 -2 -3 -3  3  1 -2  1 -1 -2 -2  0 -3 -1  4 -3 -2 -1 -4
B -2 -1  3  4 -3  0  1 -1  0 -3 -4  0 -3 -3 -2  0 -1 -4 -3 -3  4  1 -1 -4
Z -1  0  0  1 -3  3  4 -2  0 -3 -3  1 -1 -3 -1  0 -1 -3 -2 -2  1  4 -1 -4
X  0 -1 -1 -1 -2 -1 -1 -1 -1 -1 -1 -1 -1 -1 -2  0  0 -2 -1 -1 -1 -1 -1 -4
* -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4 -4  1
"""

# NCBI translation table 1, first/second/third base each running T, C, A, G.
_TCAG = "TCAG"
_CODE_TCAG = "FFLLSSSSYY**CC*WLLLLPPPPHHQQRRRRIIIMTTTTNNKKSSRRVVVVAAAADDEEGGGG"


def blosum62() -> np.ndarray:
    """24x24 int8 BLOSUM62 in the order of ``AA``."""
    lines = [ln for ln in _BLOSUM62_TEXT.strip("\n").splitlines() if ln.strip()]
    header = lines[0].split()
    assert "".join(header) == AA
    mat = np.zeros((24, 24), dtype=np.int8)
    for r, ln in enumerate(lines[1:]):
        parts = ln.split()
        assert parts[0] == AA[r]
        mat[r, :] = [int(x) for x in parts[1:]]
    return mat


def codon_table() -> dict:
    """Codon (upper-case string) -> one-letter amino acid, standard code."""
    out = {}
    k = 0
    for b1 in _TCAG:
        for b2 in _TCAG:
            for b3 in _TCAG:
                out[b1 + b2 + b3] = _CODE_TCAG[k]
                k += 1
    return out


def gcode() -> np.ndarray:
    """uint8[64]: index 16*b1+4*b2+b3 with A,C,G,T = 0..3 -> amino-acid code."""
    tab = codon_table()
    g = np.zeros(64, dtype=np.uint8)
    for b1 in range(4):
        for b2 in range(4):
            for b3 in range(4):
                cod = "ACGT"[b1] + "ACGT"[b2] + "ACGT"[b3]
                g[16 * b1 + 4 * b2 + b3] = AA.index(tab[cod])
    return g


def donor_final(tri: str) -> int:
    """Final-model donor penalty for the intron's first three bases."""
    if tri in ("GTA", "GTG"):
        return 0
    if tri in ("GTC", "GTT"):
        return 8
    if tri[:2] == "GC":
        return 15
    if tri[:2] == "AT":
        return 21
    return 30


def acceptor_final(tri: str) -> int:
    """Final-model acceptor penalty for the intron's last three bases."""
    if tri in ("CAG", "TAG"):
        return 0
    if tri in ("AAG", "GAG"):
        return 8
    if tri[1:] == "AC":
        return 21
    return 30


def _table(fn) -> np.ndarray:
    t = np.zeros(125, dtype=np.uint8)
    for b1 in range(5):
        for b2 in range(5):
            for b3 in range(5):
                t[25 * b1 + 5 * b2 + b3] = fn(DNA[b1] + DNA[b2] + DNA[b3])
    return t


def splice_tables(model: str = "final", p: int = 20):
    """(donor[125], acceptor[125]) uint8 tables over ACGTN 3-mers."""
    if model == "final":
        return _table(donor_final), _table(acceptor_final)
    if model == "simple":
        return (_table(lambda t: 0 if t[:2] == "GT" else p),
                _table(lambda t: 0 if t[1:] == "AG" else p))
    if model == "none":
        return np.zeros(125, np.uint8), np.zeros(125, np.uint8)
    raise ValueError(model)


class Scoring:
    """All scoring inputs of one DP call (oracle side)."""

    def __init__(self, q=11, e=1, f=23, r=29, flags=0, mode=0, mat=None,
                 gcode_tab=None, donor=None, acceptor=None):
        self.q, self.e, self.f, self.r = int(q), int(e), int(f), int(r)
        self.flags, self.mode = int(flags), int(mode)
        self.mat = np.ascontiguousarray(blosum62() if mat is None else mat, dtype=np.int8)
        self.gcode = np.ascontiguousarray(gcode() if gcode_tab is None else gcode_tab,
                                          dtype=np.uint8)
        if donor is None or acceptor is None:
            d, a = splice_tables("final")
            donor = d if donor is None else donor
            acceptor = a if acceptor is None else acceptor
        self.donor = np.ascontiguousarray(donor, dtype=np.uint8)
        self.acceptor = np.ascontiguousarray(acceptor, dtype=np.uint8)

    def replace(self, **kw):
        d = dict(q=self.q, e=self.e, f=self.f, r=self.r, flags=self.flags, mode=self.mode,
                 mat=self.mat, gcode_tab=self.gcode, donor=self.donor,
                 acceptor=self.acceptor)
        d.update(kw)
        return Scoring(**d)


def default_scoring(**kw) -> Scoring:
    """Defaults: q=11, e=1, f=23, r=29 (half-bit units), BLOSUM62, final splice
    model, LOCAL mode.  The paper gives no values for q, e, f or r."""
    return Scoring(**kw)
