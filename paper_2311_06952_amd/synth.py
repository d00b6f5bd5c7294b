"""Seeded synthetic inputs shaped like the paper's workloads.

This module only produces input data (float32 feature matrices, uint8 class
labels, request descriptions).  It holds none of the method's arithmetic: no
threshold sets, no decoding, no rank routing, no counting.  Both the HIP path
(through the tests and the benchmark) and the CPU oracle consume its output.

The paper trains on UCI datasets (47 to 11M samples, 3 to 73 continuous
features, 2 to 29 classes; Section 5).  None of them is available here, so
seeded stand-ins with comparable shapes are generated:

* planted trees: labels from a random axis-aligned tree with float
  thresholds placed between the 20th and 80th percentile of the samples that
  reach each node, plus independent label flips;
* Gaussian mixtures: K class means drawn from N(0, 2 I), samples from
  N(mu_y, I), y uniform.

Randomness comes from numpy's PCG64 generator keyed by the given seed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def planted_tree(rng: np.random.Generator, X: np.ndarray, feats: int, K: int,
                 depth: int, noise: float):
    """A random depth-`depth` planted tree over features [0, feats) of X and
    the labels it assigns, each flipped to a different class with prob
    `noise`.  Node t (heap order, 1-based) sends a sample left iff
    X[:, feat[t-1]] < thr[t-1].  Returns (y, feat, thr, leaf_class)."""
    n = X.shape[0]
    SB = (1 << depth) - 1
    feat = np.zeros(SB, dtype=np.int64)
    thr = np.zeros(SB, dtype=np.float32)
    node = np.ones(n, dtype=np.int64)
    for level in range(depth):
        for t in range(1 << level, 2 << level):
            members = np.nonzero(node == t)[0]
            f = int(rng.integers(feats))
            feat[t - 1] = f
            if members.size == 0:
                thr[t - 1] = np.inf
                continue
            vals = np.sort(X[members, f])
            q = rng.uniform(0.2, 0.8)
            thr[t - 1] = vals[int(q * (vals.size - 1))]
            go_left = X[members, f] < thr[t - 1]
            node[members] = np.where(go_left, 2 * t, 2 * t + 1)
    n_leaves = 1 << depth
    while True:
        leaf_class = rng.integers(K, size=n_leaves)
        if np.unique(leaf_class).size >= min(2, K):
            break
    y = leaf_class[node - n_leaves].astype(np.int64)
    if noise > 0.0 and K > 1:
        flip = rng.random(n) < noise
        shift = 1 + rng.integers(K - 1, size=n)
        y = np.where(flip, (y + shift) % K, y)
    return y.astype(np.uint8), feat, thr, leaf_class


def planted_tree_labels(rng: np.random.Generator, X: np.ndarray, feats: int, K: int,
                        depth: int, noise: float) -> np.ndarray:
    """Labels of a random planted tree (see planted_tree)."""
    return planted_tree(rng, X, feats, K, depth, noise)[0]


def gaussian_mixture(rng: np.random.Generator, n: int, F: int, K: int,
                     mean_var: float = 2.0):
    mu = rng.normal(0.0, np.sqrt(mean_var), size=(K, F))
    y = rng.integers(K, size=n)
    X = (mu[y] + rng.normal(0.0, 1.0, size=(n, F))).astype(np.float32)
    return X, y.astype(np.uint8)


@dataclass
class Workload:
    name: str
    X: np.ndarray          # float32 [n][F], row-major
    y: np.ndarray          # uint8 [n]
    K: int
    D: int                 # tree depth
    P: int                 # population size
    G: int                 # generations
    M: float = 0.5         # mutation factor
    CR: float = 0.9        # crossover probability
    D_MH: int = 0          # moving-horizon depth (0: plain DEOCT)

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def F(self) -> int:
        return self.X.shape[1]


def plain_small(seed: int = 1, n: int = 1000) -> Workload:
    """n = 1000, F = 4 features U[0,1), K = 2, labels from a planted depth-2
    tree over all four features with 10% flips; depth-2 trees, P = 32,
    50 generations, M = 0.5, CR = 0.9."""
    rng = _rng(seed)
    X = rng.random((n, 4), dtype=np.float32)
    y = planted_tree_labels(rng, X, 4, 2, 2, 0.10)
    return Workload("plain_small_n1000_F4_K2_D2_P32_G50", X, y, 2, 2, 32, 50)


def plain_scale(seed: int = 1, n: int = 100_000) -> Workload:
    """n = 100,000, F = 16 Gaussian-mixture features, K = 3; depth-3 trees,
    P = 256, 200 generations."""
    rng = _rng(seed)
    X, y = gaussian_mixture(rng, n, 16, 3)
    return Workload("plain_scale_n100k_F16_K3_D3_P256_G200", X, y, 3, 3, 256, 200)


def plain_scale_heldout(seed: int = 1, n: int = 1_000_000, draw_seed: int = 2):
    """Rows from the same mixture as plain_scale(seed) (its component means),
    with draws of their own: a held-out set for the trained tree."""
    mu = _rng(seed).normal(0.0, np.sqrt(2.0), size=(3, 16))
    rng = _rng(draw_seed)
    y = rng.integers(3, size=n)
    X = (mu[y] + rng.normal(0.0, 1.0, size=(n, 16))).astype(np.float32)
    return X, y.astype(np.uint8)


def plain_large(seed: int = 1, n: int = 1_000_000) -> Workload:
    """n = 1,000,000, F = 32: features 0-15 from a 4-component Gaussian
    mixture, 16-31 U[0,1) noise; K = 4 labels from a planted depth-5 tree
    over features 0-15 with 5% flips; depth-4 trees, P = 512, 100
    generations."""
    rng = _rng(seed)
    Xg, _ = gaussian_mixture(rng, n, 16, 4)
    Xu = rng.random((n, 16), dtype=np.float32)
    X = np.ascontiguousarray(np.concatenate([Xg, Xu], axis=1))
    y = planted_tree_labels(rng, X, 16, 4, 5, 0.05)
    return Workload("plain_large_n1M_F32_K4_D4_P512_G100", X, y, 4, 4, 512, 100)


def batched_mh(seed: int = 1, n: int = 1_000_000) -> Workload:
    """n = 1,000,000, F = 20 Gaussian-mixture features, K = 3; final depth 8,
    horizon 3, P = 128 per subproblem, 100 generations."""
    rng = _rng(seed)
    X, y = gaussian_mixture(rng, n, 20, 3)
    return Workload("batched_mh_n1M_F20_K3_D8_H3_P128_G100", X, y, 3, 8, 128, 100, D_MH=3)


def served_mh(seed: int = 1, n: int = 10_000_000) -> Workload:
    """The served configuration's moving-horizon run: n = 10,000,000, F = 8
    Gaussian-mixture features, K = 2; final depth 8, horizon 3, P = 128, 100
    generations."""
    rng = _rng(seed)
    X, y = gaussian_mixture(rng, n, 8, 2)
    return Workload("served_mh_n10M_F8_K2_D8_H3_P128_G100", X, y, 2, 8, 128, 100, D_MH=3)


def random_small(seed: int, n: int, F: int, K: int, levels: int | None = None,
                 dtype=np.float32) -> tuple[np.ndarray, np.ndarray]:
    """Small test data.  With `levels`, feature values are drawn from
    `levels` distinct values so that ties are common."""
    rng = _rng(seed)
    if levels is None:
        X = rng.random((n, F), dtype=np.float32)
    else:
        X = (rng.integers(levels, size=(n, F)) / max(levels - 1, 1)).astype(np.float32)
    y = rng.integers(K, size=n).astype(np.uint8)
    return X.astype(dtype), y


@dataclass
class Request:
    rid: int
    arrival: float   # seconds after stream start
    n: int
    F: int
    K: int
    D: int
    P: int = 128
    G: int = 100
    seed: int = 0

    def data(self) -> tuple[np.ndarray, np.ndarray]:
        rng = _rng(self.seed)
        return gaussian_mixture(rng, self.n, self.F, self.K)


def request_stream(seed: int, count: int, rate: float, n_lo: float = 1e3,
                   n_hi: float = 1e7) -> list[Request]:
    """Subtree-solve requests with Poisson arrivals at `rate` per second:
    n = round(10^U(log10 n_lo, log10 n_hi)), F ~ U{4..32}, K ~ U{2..10},
    D ~ U{2..4}, P = 128, G = 100; request j's data seed is seed * 1000003 + j."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps)
    out = []
    for j in range(count):
        n = int(round(10 ** rng.uniform(np.log10(n_lo), np.log10(n_hi))))
        F = int(rng.integers(4, 33))
        K = int(rng.integers(2, 11))
        D = int(rng.integers(2, 5))
        out.append(Request(j, float(t[j]), n, F, K, D, seed=seed * 1000003 + j))
    return out
