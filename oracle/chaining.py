"""Chaining of seed anchors -- TEST INFRASTRUCTURE ONLY.

Methods, "Chaining": a 1-D max-plus DP over the anchors of one protein,
Eq. (gap) for the minimum gap between two anchors on a binned genome (bins
of 256 bp), the chaining recurrence f(j) and the gap penalty Eq. (gap-pen);
the second round works at base resolution with the gap 3*dy - dx.

Readings taken here:
  * anchors come sorted by genome position x, then residue position y; i can
    precede j only when x_i <= x_j and y_i < y_j (the premise of Eq. (gap));
  * f(j) = max(k, max over valid i < j of f(i) + min(y_j - y_i, k) - gamma(g));
    gamma is infinite (i cannot precede j) when |g| >= G; pred(j) is the
    first i reaching the maximum, or -1 when the start value k is not beaten;
  * log2 and the divisions are fp64 (the paper fixes no precision); values
    are compared with a tolerance derived from fp64 rounding (see the tests);
  * chains: anchors are taken in descending f (ties: smaller index first);
    each not yet used anchor starts a chain that follows pred until it meets
    -1 or a used anchor; its score is f(end) minus f(that used anchor) (or
    minus 0).  Chains are ranked by score (ties: the chain extracted first)
    and the first max_chains are kept ("top 30 chains").

Parity unpinned for the extraction and ranking rules above; the DP itself is
pinned by brute force over all chains on small inputs and by closed forms.
"""
from __future__ import annotations

import numpy as np

BIN = 256


def gap(dx, dy, binned: bool):
    """Eq. (gap) (binned) or the second round's 3*dy - dx, elementwise."""
    dx = np.asarray(dx, dtype=np.int64)
    dy = np.asarray(dy, dtype=np.int64)
    if not binned:
        return 3 * dy - dx
    lo = BIN * (dx - 1)
    hi = BIN * (dx + 1)
    return np.where(3 * dy < lo, 3 * dy - lo, np.where(3 * dy > hi, 3 * dy - hi, 0))


def gamma(g, beta: float, G: int):
    """Eq. (gap-pen), elementwise, +inf where |g| >= G."""
    g = np.asarray(g, dtype=np.int64)
    a = np.abs(g).astype(np.float64)
    lg = beta * np.log2(a + 1.0)
    out = np.where(g > 0, a / 3.0 + lg, np.minimum(a / 3.0, lg))
    out = np.where(g == 0, 0.0, out)
    return np.where(np.abs(g) >= G, np.inf, out)


def chain_dp(x, y, k: int = 6, beta: float = 0.75, G: int = 200000, binned: bool = True):
    """(f, pred) for anchors sorted by (x, y)."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    n = len(x)
    f = np.zeros(n, dtype=np.float64)
    pred = np.full(n, -1, dtype=np.int64)
    for j in range(n):
        best, bi = float(k), -1
        if j:
            dx = x[j] - x[:j]
            dy = y[j] - y[:j]
            v = f[:j] + np.minimum(dy, k) - gamma(gap(dx, dy, binned), beta, G)
            v = np.where((dx >= 0) & (dy > 0), v, -np.inf)
            i = int(np.argmax(v))  # first maximum
            if v[i] > best:
                best, bi = float(v[i]), i
        f[j], pred[j] = best, bi
    return f, pred


def extract(f, pred, max_chains: int = 30):
    """Chains as [(score, [anchor indices ascending]), ...], best first."""
    n = len(f)
    order = sorted(range(n), key=lambda j: (-f[j], j))
    used = np.zeros(n, dtype=bool)
    chains = []
    for j in order:
        if used[j]:
            continue
        idx = []
        t = j
        while t != -1 and not used[t]:
            idx.append(t)
            used[t] = True
            t = int(pred[t])
        score = f[j] - (f[t] if t != -1 else 0.0)
        chains.append((float(score), idx[::-1]))
    ranked = sorted(range(len(chains)), key=lambda c: (-chains[c][0], c))
    return [chains[c] for c in ranked[:max_chains]]


def chain(anchors, k: int = 6, beta: float = 0.75, G: int = 200000, binned: bool = True,
          max_chains: int = 30):
    """anchors: [(x, y), ...] sorted by (x, y).  Returns (f, pred, chains)."""
    a = np.asarray(anchors, dtype=np.int64).reshape(-1, 2)
    f, pred = chain_dp(a[:, 0], a[:, 1], k, beta, G, binned)
    return f, pred, extract(f, pred, max_chains)
