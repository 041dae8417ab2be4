"""Pins of the chaining oracle (Methods, "Chaining"): closed forms of
Eq. (gap) and Eq. (gap-pen), brute force over all chains, hand examples of
chain extraction."""
import itertools
import math
import random

import numpy as np
import pytest

from oracle import chaining as C

TOL = 1e-9


def test_gap_closed_forms():
    # binned: 3dy against 256(dx - 1) and 256(dx + 1)
    assert C.gap(1, 170, True) == 0
    assert C.gap(1, 171, True) == 3 * 171 - 512
    assert C.gap(0, 1, True) == 0  # same bin: no definite gap
    assert C.gap(0, 86, True) == 258 - 256
    assert C.gap(5, 1, True) == 3 - 1024
    assert C.gap(5, 341, True) == 1023 - 1024 and C.gap(5, 342, True) == 0
    assert C.gap(5, 512, True) == 0 and C.gap(5, 513, True) == 1539 - 1536
    assert C.gap(4, 256, True) == 0  # 768 inside [768, 1280]
    assert C.gap(4, 255, True) == 765 - 768
    # second round: base resolution
    assert C.gap(30, 10, False) == 0 and C.gap(31, 10, False) == -1
    assert C.gap(100, 40, False) == 20


def test_gap_penalty_closed_forms():
    b, G = 0.75, 200000
    assert C.gamma(0, b, G) == 0.0
    assert C.gamma(3, b, G) == pytest.approx(1 + 0.75 * 2)
    assert C.gamma(-3, b, G) == pytest.approx(1.0)               # min(1, 1.5)
    assert C.gamma(-7, b, G) == pytest.approx(2.25)              # min(7/3, 2.25)
    assert C.gamma(-6, b, G) == pytest.approx(2.0)               # min(2, 2.10)
    assert C.gamma(G - 1, b, G) == pytest.approx((G - 1) / 3 + 0.75 * math.log2(G))
    assert C.gamma(G, b, G) == math.inf and C.gamma(-G, b, G) == math.inf


def _brute_f(x, y, k, beta, G, binned):
    """f(j) as the best chain ending at j over every increasing sequence of
    anchors: k plus, per consecutive pair, min(dy, k) - gamma(gap)."""
    n = len(x)
    f = []
    for j in range(n):
        best = float(k)
        for r in range(1, n):
            for sub in itertools.combinations(range(j), r):
                seq = list(sub) + [j]
                s = float(k)
                ok = True
                for a, b2 in zip(seq, seq[1:]):
                    dx, dy = x[b2] - x[a], y[b2] - y[a]
                    if dx < 0 or dy <= 0:
                        ok = False
                        break
                    gm = float(C.gamma(C.gap(dx, dy, binned), beta, G))
                    if gm == math.inf:
                        ok = False
                        break
                    s += min(dy, k) - gm
                if ok:
                    best = max(best, s)
        f.append(best)
    return np.array(f)


@pytest.mark.parametrize("binned", [True, False])
def test_chain_dp_equals_brute_force(binned):
    rng = random.Random(3 + binned)
    for _ in range(40):
        n = rng.randint(1, 7)
        pts = sorted((rng.randint(0, 12 if binned else 300), rng.randint(0, 60))
                     for _ in range(n))
        x = [p[0] for p in pts]
        y = [p[1] for p in pts]
        k = rng.randint(2, 7)
        beta = rng.choice([0.5, 0.75, 1.0])
        G = rng.choice([50, 200, 200000])
        f, pred = C.chain_dp(x, y, k, beta, G, binned)
        assert np.allclose(f, _brute_f(x, y, k, beta, G, binned), atol=TOL, rtol=0)
        for j in range(n):  # pred reaches f(j), and is the first such i
            if pred[j] >= 0:
                i = pred[j]
                dx, dy = x[j] - x[i], y[j] - y[i]
                v = f[i] + min(dy, k) - C.gamma(C.gap(dx, dy, binned), beta, G)
                assert abs(v - f[j]) <= TOL and v > k
            else:
                assert f[j] == k


def test_one_diagonal_is_one_chain():
    """Anchors every k residues on one diagonal at base resolution: no gap,
    each link adds k."""
    k = 6
    anchors = [(100 + 3 * y, y) for y in range(0, 60, k)]
    f, pred, chains = C.chain(anchors, k=k, binned=False)
    assert list(f) == [k * (t + 1) for t in range(len(anchors))]
    assert chains == [(float(k * len(anchors)), list(range(len(anchors))))]


def test_far_copies_are_separate_chains():
    """Two copies of a diagonal more than G apart in the genome: two chains,
    ranked by length; the start value k beats any link over |g| >= G."""
    k = 6
    a = [(3 * y, y) for y in range(0, 30, k)]
    b = [(500000 + 3 * y, y) for y in range(0, 48, k)]
    f, pred, chains = C.chain(sorted(a + b), k=k, binned=False)
    assert [round(s) for s, _ in chains] == [k * len(b), k * len(a)]
    assert chains[0][1] == list(range(len(a), len(a) + len(b)))


def test_extraction_invariants():
    rng = random.Random(17)
    for _ in range(30):
        n = rng.randint(1, 200)
        pts = sorted((rng.randint(0, 4000), rng.randint(0, 500)) for _ in range(n))
        f, pred, chains = C.chain(pts, binned=bool(rng.random() < 0.5), max_chains=30)
        seen = set()
        scores = [s for s, _ in chains]
        assert scores == sorted(scores, reverse=True)
        for s, idx in chains:
            assert not seen & set(idx)
            seen |= set(idx)
            assert idx == sorted(idx)
            for a, b in zip(idx, idx[1:]):
                assert pred[b] == a
            stop = pred[idx[0]]
            assert abs(s - (f[idx[-1]] - (f[stop] if stop >= 0 else 0.0))) <= TOL
