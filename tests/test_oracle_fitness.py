"""Pins of the oracle's routing, counting and epilogue (Section 2 tree
semantics, Algorithm 1 walk, eq. opt_c, eq. opt_all, Section 3.2 fitness;
readings R2, R5, R6, R7)."""
import json
import os

import numpy as np
import pytest

import brute
import oracle
from paper_2311_06952_amd import synth


def _golden(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "hand_worked_depth2.json")))
    X = np.array(g["X"], dtype=np.float32)
    ds = oracle.dataset_from_X(X, np.array(g["y"], dtype=np.uint8), g["K"])
    return g, X, ds


def test_golden_hand_worked_fitness(golden_dir):
    g, X, ds = _golden(golden_dir)
    D = g["D"]
    for tr in g["trees"]:
        feat = np.array([tr["feat"]], dtype=np.uint8)
        tau = np.array([tr["tau"]], dtype=np.uint32)
        for i, leaf in enumerate(tr["leaf_of_sample"]):
            assert oracle.route(ds, i, feat[0], tau[0], D) == leaf
        counts, correct, label, cost = oracle.fitness(ds, feat, tau, D)
        np.testing.assert_array_equal(counts[0], np.array(tr["counts"]))
        assert list(label[0]) == tr["label"]
        assert correct[0] == tr["correct"]
        assert cost[0] == tr["cost_alpha0_nmin1"]
        _, _, _, cost2 = oracle.fitness(ds, feat, tau, D, n_min=2, alpha=0.5)
        assert cost2[0] == tr["cost_alpha0.5_nmin2"]


def test_golden_matches_literal_threshold_values(golden_dir):
    # the same trees routed with the literal float thresholds of B_p
    g, X, ds = _golden(golden_dir)
    ts = brute.threshold_sets(X)
    for f, key in enumerate(("B_1", "B_2")):
        # the fixture's values are the decimal ones; X is float32
        assert [float(b) for b in ts[f][2]] == pytest.approx(g["thresholds_scaled"][key],
                                                              abs=1e-6)
    for tr in g["trees"]:
        thr_index = [t + 1 for t in tr["tau"]]
        c = brute.counts_value(X, g["y"], g["K"], tr["feat"], thr_index, g["D"])
        assert c == tr["counts"]


@pytest.mark.parametrize("seed,n,F,K,D,levels", [(1, 40, 2, 2, 1, None), (2, 60, 3, 3, 2, 5),
                                                 (3, 50, 2, 4, 3, None), (4, 30, 4, 2, 4, 3)])
def test_rank_routing_equals_midpoint_value_routing(seed, n, F, K, D, levels):
    # reading R2: for threshold index i <= n_p, "rank < i - 1" is the same
    # partition as "x_scaled < beta_i" with exact midpoints.
    X, y = synth.random_small(seed, n, F, K, levels)
    ds = oracle.dataset_from_X(X, y, K)
    rng = np.random.default_rng(seed)
    SB = (1 << D) - 1
    for _ in range(6):
        feat = rng.integers(0, F + 1, size=SB).astype(np.uint8)
        tau = np.array([rng.integers(0, ds.n_unique[f - 1]) if f else 0 for f in feat],
                       dtype=np.uint32)
        counts, correct, _, _ = oracle.fitness(ds, feat[None], tau[None], D)
        want = brute.counts_value(X, y, K, list(feat), [t + 1 for t in tau], D)
        np.testing.assert_array_equal(counts[0], np.array(want))
        assert correct[0] == brute.correct_of(want)


def test_top_threshold_sends_everything_left():
    # reading R2: tau = n_p (index n_p + 1) sends every sample left
    X, y = synth.random_small(5, 40, 2, 2)
    ds = oracle.dataset_from_X(X, y, 2)
    feat = np.array([[1]], dtype=np.uint8)
    tau = np.array([[ds.n_unique[0]]], dtype=np.uint32)
    counts, _, _, _ = oracle.fitness(ds, feat, tau, 1)
    assert counts[0, 0].sum() == 40 and counts[0, 1].sum() == 0


def _random_trees(rng, P, D, ds):
    SB = (1 << D) - 1
    feat = rng.integers(0, ds.F + 1, size=(P, SB)).astype(np.uint8)
    tau = np.zeros((P, SB), dtype=np.uint32)
    for r in range(P):
        for t in range(SB):
            f = feat[r, t]
            tau[r, t] = rng.integers(0, ds.n_unique[f - 1] + 1) if f else 0
    return feat, tau


@pytest.mark.parametrize("D", [1, 2, 3, 5])
def test_count_invariants(D):
    X, y = synth.random_small(7, 500, 4, 3, levels=20)
    ds = oracle.dataset_from_X(X, y, 3)
    rng = np.random.default_rng(D)
    feat, tau = _random_trees(rng, 16, D, ds)
    counts, correct, label, cost = oracle.fitness(ds, feat, tau, D)
    nk = np.bincount(y, minlength=3)
    assert (counts.sum(axis=(1, 2)) == 500).all()
    assert (counts.sum(axis=1) == nk[None, :]).all()
    assert (correct >= nk.max()).all() and (correct <= 500).all()
    assert (correct == counts.max(axis=2).sum(axis=1)).all()
    assert (label == np.argmax(counts, axis=2)).all()     # first maximum
    assert (cost == 500 - correct).all()
    # permutation of the sample order leaves counts unchanged
    perm = rng.permutation(500)
    c2, _, _, _ = oracle.fitness(ds, feat, tau, D, idx=perm)
    np.testing.assert_array_equal(c2, counts)
    # shards sum to the whole
    parts = np.array_split(np.arange(500), 3)
    acc = sum(oracle.fitness(ds, feat, tau, D, idx=p)[0] for p in parts)
    np.testing.assert_array_equal(acc, counts)


def test_all_no_split_tree_puts_everything_in_last_leaf():
    X, y = synth.random_small(8, 200, 3, 4)
    ds = oracle.dataset_from_X(X, y, 4)
    for D in (1, 2, 4):
        SB = (1 << D) - 1
        counts, correct, _, _ = oracle.fitness(ds, np.zeros((1, SB), np.uint8),
                                               np.zeros((1, SB), np.uint32), D)
        np.testing.assert_array_equal(counts[0, -1], np.bincount(y, minlength=4))
        assert counts[0, :-1].sum() == 0
        assert correct[0] == np.bincount(y).max()


def test_fitness_matches_rank_brute_force_on_subsets():
    X, y = synth.random_small(9, 120, 3, 3, levels=6)
    ds = oracle.dataset_from_X(X, y, 3)
    rng = np.random.default_rng(1)
    feat, tau = _random_trees(rng, 8, 3, ds)
    idx = rng.choice(120, size=47, replace=False).astype(np.uint32)
    counts, correct, _, _ = oracle.fitness(ds, feat, tau, 3, idx=idx)
    for r in range(8):
        want = brute.rank_counts(ds.ranks, y, 3, feat[r], tau[r], 3, idx=list(idx))
        np.testing.assert_array_equal(counts[r], np.array(want))


def test_penalties():
    # Section 3.2: alpha * #splits + #{leaves with 0 < n_l < n_min}
    X, y = synth.random_small(10, 30, 2, 2)
    ds = oracle.dataset_from_X(X, y, 2)
    rng = np.random.default_rng(3)
    feat, tau = _random_trees(rng, 10, 2, ds)
    counts, correct, _, cost = oracle.fitness(ds, feat, tau, 2, n_min=5, alpha=0.25)
    for r in range(10):
        nl = counts[r].sum(axis=1)
        viol = int(((nl > 0) & (nl < 5)).sum())
        want = (30 - int(correct[r])) + 0.25 * int((feat[r] != 0).sum()) + viol
        assert cost[r] == want


def test_planted_tree_is_representable():
    # reading R12: a planted tree without label noise is matched exactly by a
    # tree in rank space: tau = number of unique values below the threshold.
    rng = np.random.Generator(np.random.PCG64(21))
    X = rng.random((2000, 6), dtype=np.float32)
    y, pf, thr, leaf_class = synth.planted_tree(rng, X, 6, 3, 3, 0.0)
    ds = oracle.dataset_from_X(X, y, 3)
    feat = (pf + 1).astype(np.uint8)
    tau = np.array([np.searchsorted(np.unique(X[:, f]), t, side="left")
                    for f, t in zip(pf, thr)], dtype=np.uint32)
    counts, correct, label, _ = oracle.fitness(ds, feat[None], tau[None], 3)
    assert correct[0] == 2000
