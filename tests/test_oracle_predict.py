"""Pins of the oracle's tree application to new samples (Section 2 routing
with the Section 3.1 threshold sets; the test accuracy of Section 4; readings
R2 and R13): against the paper's literal scaled midpoint sets in exact
rationals, and against rank routing on the training rows.  Also the encoding
of a tree into genes (reading R14), pinned by the decode of eqs. aenc and
benc."""
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2311_06952_amd import synth


def _literal_left(ts, f, tau, x):
    """x goes left at a split (feature f, 0-based; rank threshold tau) under
    the paper's rule: min-max scale x with the training range and compare it
    with the (tau+1)-th element of B_p.  tau = n_p is reading R2 (all left)."""
    u, _, B = ts[f]
    if tau >= len(u):
        return True
    lo, hi = u[0], u[-1]
    span = hi - lo
    xs = (Fraction(float(x)) - lo) / span if span != 0 else Fraction(float(x)) - lo
    return xs < B[tau]


@pytest.mark.parametrize("seed,n,levels", [(1, 30, 6), (2, 50, None), (3, 12, 2), (4, 40, 1)])
def test_depth1_decisions_equal_literal_midpoints(seed, n, levels):
    X, y = synth.random_small(seed, n, 3, 2, levels)
    ts = brute.threshold_sets(X)
    ranks, nu = oracle.rank_encode(X)
    rng = np.random.default_rng(seed)
    # held-out values: the training values, exact midpoints, values outside
    # the training range and random values in between
    for f in range(3):
        u = np.unique(X[:, f])
        mids = ((u[:-1].astype(np.float64) + u[1:]) / 2).astype(np.float32)
        span = float(u[-1] - u[0]) + 1.0
        extra = np.array([u[0] - span, u[-1] + span, np.nextafter(u[0], -np.inf),
                          np.nextafter(u[-1], np.inf)], dtype=np.float32)
        vals = np.concatenate([u, mids, extra,
                               rng.uniform(u[0] - 1, u[-1] + 1, 40).astype(np.float32)])
        T = np.zeros((len(vals), 3), dtype=np.float32)
        T[:, f] = vals
        for tau in range(int(nu[f]) + 1):
            feat = np.array([f + 1], dtype=np.uint8)
            thr = oracle.tree_thresholds(X, feat, np.array([tau], dtype=np.uint32), 1)
            pred, _ = oracle.predict(T, feat, thr, np.array([0, 1], dtype=np.uint8), 1)
            want = [0 if _literal_left(ts, f, tau, v) else 1 for v in vals]
            assert list(pred) == want, (f, tau)


def test_hand_worked_thresholds():
    # feature 1 has training values {-2, 1, 1, 4}, feature 2 is constant 7
    X = np.array([[1, 7], [-2, 7], [4, 7], [1, 7]], dtype=np.float32)
    feat = np.array([1, 1, 2], dtype=np.uint8)
    for tau, beta in ((0, -2.0), (1, -0.5), (2, 2.5), (3, np.inf)):
        thr = oracle.tree_thresholds(X, feat, np.array([tau, 1, 0], dtype=np.uint32), 2)
        assert thr[0] == beta
        assert thr[1] == -0.5 and thr[2] == 7.0
    # constant feature: tau = 1 = n_p sends everything left
    thr = oracle.tree_thresholds(X, np.array([2], dtype=np.uint8), np.array([1], dtype=np.uint32),
                                 1)
    assert thr[0] == np.inf
    # no split (and a feature past F) sends every sample right
    thr = oracle.tree_thresholds(X, np.array([0, 3, 1], dtype=np.uint8),
                                 np.array([2, 1, 1], dtype=np.uint32), 2)
    assert list(thr) == [0.0, 0.0, -0.5]
    T = np.array([[-100, 0], [100, 0]], dtype=np.float32)
    label = np.array([1, 2, 3, 4], dtype=np.uint8)
    pred, correct = oracle.predict(T, np.array([0, 3, 1], dtype=np.uint8), thr, label, 2,
                                   y=np.array([3, 3], dtype=np.uint8))
    # root has no split: right child (node 3, feature 1 at -0.5) decides
    assert list(pred) == [3, 4] and correct == 1


def test_negative_zero_is_one_value():
    X = np.array([[-0.0], [0.0], [1.0], [-1.0]], dtype=np.float32)
    thr = oracle.tree_thresholds(X, np.array([1], dtype=np.uint8), np.array([2], dtype=np.uint32),
                                 1)
    assert thr[0] == 0.5  # unique values -1, 0, 1
    thr = oracle.tree_thresholds(X, np.array([1], dtype=np.uint8), np.array([3], dtype=np.uint32),
                                 1)
    assert thr[0] == np.inf


@pytest.mark.parametrize("seed,n,F,K,D,levels", [(5, 300, 4, 3, 3, 12), (6, 500, 6, 2, 4, None),
                                                 (7, 200, 3, 5, 2, 3)])
def test_training_rows_follow_rank_routing(seed, n, F, K, D, levels):
    """On the rows a tree was trained on, value routing with the thresholds
    equals rank routing, and the correct count equals the fitness count."""
    X, y = synth.random_small(seed, n, F, K, levels)
    ds = oracle.dataset_from_X(X, y, K)
    rng = np.random.default_rng(seed)
    SB = (1 << D) - 1
    for _ in range(5):
        feat = rng.integers(0, F + 1, size=SB).astype(np.uint8)
        tau = np.array([rng.integers(0, ds.n_unique[f - 1] + 1) if f else 0 for f in feat],
                       dtype=np.uint32)
        _, correct, label, _ = oracle.fitness(ds, feat[None], tau[None], D)
        thr = oracle.tree_thresholds(X, feat, tau, D)
        pred, got = oracle.predict(X, feat, thr, label[0], D, y=y)
        leaves = [brute.rank_route(ds.ranks, i, feat, tau, D) for i in range(n)]
        np.testing.assert_array_equal(pred, label[0][leaves])
        assert got == correct[0]


def test_nan_in_training_column_is_rejected():
    X = np.array([[1.0], [np.nan]], dtype=np.float32)
    with pytest.raises(Exception):
        oracle.tree_thresholds(X, np.array([1], dtype=np.uint8), np.array([1], dtype=np.uint32), 1)


# --------------------------------------------------------------------------
# encoding a tree into genes (inverse of eq. aenc / eq. benc; reading R14)
# --------------------------------------------------------------------------
def test_encode_hand_worked():
    nu = np.array([3, 9], dtype=np.uint32)
    g = oracle.tree_encode(np.array([1, 0, 2], np.uint8), np.array([2, 5, 9], np.uint32), 2, 2, nu)
    # a^ = feat + 0.5; b^ = (tau + 0.5) / (n_f + 1); no split: (0.5, 0)
    assert list(g[0]) == [1.5, 0.5, 2.5, 2.5 / 4, 0.0, 9.5 / 10]


@pytest.mark.parametrize("D,F,nu_hi", [(1, 3, 5), (3, 16, 100_000), (5, 7, 2), (2, 200, 1 << 24),
                                       (4, 1, 1)])
def test_decode_of_encode_is_identity(D, F, nu_hi):
    """Every (feature, tau) pair, tau from 0 to n_f, survives the round trip
    through the decode of eqs. aenc and benc."""
    rng = np.random.default_rng(D * 1000 + F)
    nu = rng.integers(1, nu_hi + 1, size=F).astype(np.uint32)
    nu[0] = nu_hi
    SB = (1 << D) - 1
    P = 64
    feat = rng.integers(0, F + 1, size=(P, SB)).astype(np.uint8)
    tau = np.array([[[0, nu[f - 1], rng.integers(0, nu[f - 1] + 1)][rng.integers(0, 3)] if f else 0
                     for f in row] for row in feat], dtype=np.uint32)
    genes = oracle.tree_encode(feat, tau, D, F, nu)
    f2, t2 = oracle.decode(genes, D, F, nu)
    np.testing.assert_array_equal(f2, feat)
    np.testing.assert_array_equal(t2, tau)
