"""Pure-Python brute force for tiny inputs, written from the paper's literal
definitions (not from the oracle): min-max scaled features, threshold sets
B_p of Section 3.1 as exact rational midpoints, decoding by eq. benc into a
threshold *value*, and routing by value comparison x_scaled < b_t (Section 2).
Used only to pin the oracle."""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def threshold_sets(X):
    """Per feature: (sorted unique values, scaled values, B_p as Fractions)."""
    X = np.asarray(X, dtype=np.float32)
    out = []
    for f in range(X.shape[1]):
        u = sorted({Fraction(float(v)) for v in X[:, f]})
        lo, hi = u[0], u[-1]
        span = hi - lo
        scaled = [(v - lo) / span if span != 0 else Fraction(0) for v in u]
        B = [Fraction(0)] + [(scaled[i] + scaled[i + 1]) / 2 for i in range(len(u) - 1)] + [Fraction(1)]
        out.append((u, scaled, B))
    return out


def scaled_value(ts, f, x):
    u, scaled, _ = ts[f]
    return scaled[u.index(Fraction(float(x)))]


def route_value(X, ts, i, feat, thr_index, D):
    """Leaf (0-based) of sample i; feat is 1-based (0 = no split), thr_index is
    the 1-based index i of eq. benc into B_p."""
    t = 1
    SB = (1 << D) - 1
    while t <= SB:
        a = feat[t - 1]
        if a == 0:
            left = False
        else:
            b = ts[a - 1][2][thr_index[t - 1] - 1]
            left = scaled_value(ts, a - 1, X[i][a - 1]) < b
        t = 2 * t if left else 2 * t + 1
    return t - (1 << D)


def counts_value(X, y, K, feat, thr_index, D, idx=None):
    SL = 1 << D
    c = [[0] * K for _ in range(SL)]
    ts = threshold_sets(X)
    rows = range(len(y)) if idx is None else idx
    for i in rows:
        c[route_value(X, ts, i, feat, thr_index, D)][int(y[i])] += 1
    return c


def correct_of(counts):
    return sum(max(row) for row in counts)


def rank_route(ranks, i, feat, tau, D):
    """Routing with integer ranks, written independently of the oracle."""
    t = 1
    SB = (1 << D) - 1
    while t <= SB:
        a = int(feat[t - 1])
        left = a != 0 and int(ranks[a - 1][i]) < int(tau[t - 1])
        t = 2 * t if left else 2 * t + 1
    return t - (1 << D)


def rank_counts(ranks, y, K, feat, tau, D, idx=None):
    SL = 1 << D
    c = [[0] * K for _ in range(SL)]
    rows = range(len(y)) if idx is None else idx
    for i in rows:
        c[rank_route(ranks, i, feat, tau, D)][int(y[i])] += 1
    return c


def all_nodes(n_unique):
    """Every (feat, tau) a node can take: (0, 0) and (f, tau) for tau in
    [0, n_f]."""
    out = [(0, 0)]
    for f, nf in enumerate(n_unique, start=1):
        out += [(f, t) for t in range(int(nf) + 1)]
    return out


def best_depth1(ranks, n_unique, y, K, idx):
    best = -1
    for f, t in all_nodes(n_unique):
        c = rank_counts(ranks, y, K, [f], [t], 1, idx)
        best = max(best, correct_of(c))
    return best


def best_depth2(ranks, n_unique, y, K):
    """Brute force over every 3-node tree."""
    nodes = all_nodes(n_unique)
    best = -1
    for a in nodes:
        for b in nodes:
            for c in nodes:
                feat = [a[0], b[0], c[0]]
                tau = [a[1], b[1], c[1]]
                best = max(best, correct_of(rank_counts(ranks, y, K, feat, tau, 2)))
    return best
