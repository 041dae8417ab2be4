"""Anchor-driven alignment of one protein to one region -- TEST INFRASTRUCTURE
ONLY.

Methods, opening paragraph and "Residue alignment with dynamic programming":
after chaining, the DP closes the unaligned regions between consecutive
anchors of a chain and extends outwards from the two terminal anchors.  This
module writes that orchestration out on top of the oracle DP.

Readings taken here (the paper describes the orchestration in two sentences):
  * an anchor (x, y) of k residues is a seed hit: the k codons of the region
    starting at base x (0-based) align one to one, without gaps, to the
    residues y .. y+k-1 (M steps scored by s);
  * anchors come in genome order; an anchor on the same diagonal as the
    current run (x - x0 == 3 (y - y0)) that overlaps or abuts it extends the
    run; an anchor that starts at or after the run's end in both sequences
    starts a new run; any other anchor (overlapping off the diagonal, or
    going backwards) is dropped.  An anchor outside the sequences is an
    error;
  * the pieces, for runs (x_1, y_1, l_1) .. (x_R, y_R, l_R):
      left   P[0, y_1)              vs T[0, x_1)              EXTEND_LEFT
      gap t  P[y_t + l_t, y_{t+1})  vs T[x_t + 3 l_t, x_{t+1})  GLOBAL
      right  P[y_R + l_R, m)        vs T[x_R + 3 l_R, n)        EXTEND
    each is a DP call of its own (bases outside a piece count as N, as for
    any call);
  * the score is the sum of the pieces' optima and the runs' M scores; the
    path is their concatenation (adjacent M runs merged); a piece that fails
    (no end-to-end path of a gap, or out of range) fails the chain with its
    status.

Because a piece starts and ends in state H next to an M step of a run, the
optimum over paths forced through the runs is the sum of the pieces' optima;
the pins in the tests check this against the unconstrained LOCAL optimum
when the runs lie on an optimal path.
"""
from __future__ import annotations

from . import E_NOALN, EXTEND, EXTEND_LEFT, GLOBAL, OK, Result, aa_code, align, dna_code
from .rescore import parse


def anchor_runs(anchors, k: int, n: int, m: int):
    """Runs (x, y, l) from anchors [(x, y), ...] in genome order."""
    if k <= 0:
        raise ValueError("anchor length must be positive")
    runs = []
    for x, y in anchors:
        if x < 0 or y < 0 or x + 3 * k > n or y + k > m:
            raise ValueError("anchor (%d, %d) outside the sequences" % (x, y))
        if runs:
            x0, y0, l0 = runs[-1]
            if x - x0 == 3 * (y - y0) and y0 <= y <= y0 + l0:
                runs[-1] = (x0, y0, max(l0, y + k - y0))
                continue
            if not (x >= x0 + 3 * l0 and y >= y0 + l0):
                continue
        runs.append((x, y, k))
    return runs


def _run_score(prot: str, dna: str, x: int, y: int, l: int, sc) -> int:
    """Sum of s over the run's codons: codon T[x+3u .. x+3u+2] against P[y+u]."""
    tot = 0
    for u in range(l):
        b = [dna_code(c) for c in dna[x + 3 * u: x + 3 * u + 3]]
        tr = 22 if 4 in b else int(sc.gcode[16 * b[0] + 4 * b[1] + b[2]])
        tot += int(sc.mat[tr][aa_code(prot[y + u])])
    return tot


def _join(parts):
    """Concatenate op strings and M runs, merging adjacent tokens of M."""
    toks = []
    for part in parts:
        for L, op in (parse(part) if isinstance(part, str) else [part]):
            if L == 0:
                continue
            if toks and op == "M" and toks[-1][1] == "M":
                toks[-1] = (toks[-1][0] + L, "M")
            else:
                toks.append((L, op))
    return "".join("%d%s" % t for t in toks)


def align_chain(prot: str, dna: str, anchors, k: int, sc, want_tb: bool = True) -> Result:
    """Align along a chain of anchors; sc's own mode is not used."""
    n, m = len(dna), len(prot)
    runs = anchor_runs(anchors, k, n, m)
    if not runs:
        raise ValueError("a chain needs at least one anchor")
    x1, y1, _ = runs[0]
    xr, yr, lr = runs[-1]
    left = align(prot[:y1], dna[:x1], sc.replace(mode=EXTEND_LEFT), want_tb)
    gaps = []
    for (xa, ya, la), (xb, yb, _) in zip(runs, runs[1:]):
        gaps.append(align(prot[ya + la:yb], dna[xa + 3 * la:xb], sc.replace(mode=GLOBAL), want_tb))
    right = align(prot[yr + lr:], dna[xr + 3 * lr:], sc.replace(mode=EXTEND), want_tb)
    for r in [left] + gaps + [right]:
        if r.status != OK:
            return Result(r.status, 0, -1, -1, -1, -1, None)
    score = left.score + sum(g.score for g in gaps) + right.score
    score += sum(_run_score(prot, dna, x, y, l, sc) for x, y, l in runs)
    g_end = xr + 3 * lr + right.g_end
    p_end = yr + lr + right.p_end
    if not want_tb:
        return Result(OK, score, -1, g_end, -1, p_end, None)
    parts = [left.ops]
    for t, (x, y, l) in enumerate(runs):
        parts.append((l, "M"))
        parts.append(gaps[t].ops if t < len(gaps) else right.ops)
    return Result(OK, score, left.g_beg, g_end, left.p_beg, p_end, _join(parts))


__all__ = ["anchor_runs", "align_chain", "E_NOALN"]
