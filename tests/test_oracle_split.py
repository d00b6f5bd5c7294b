"""Pins of the oracle's exact depth-1 split (Algorithm 2 horizon-1 branch,
reading R10), exhaustive depth-2 optimum (reading R11) and greedy tree."""
import numpy as np
import pytest

import brute
import oracle
from paper_2311_06952_amd import synth


@pytest.mark.parametrize("seed,n,F,K,levels", [(1, 30, 2, 2, None), (2, 45, 3, 3, 4),
                                               (3, 25, 3, 4, 3), (4, 12, 1, 2, None),
                                               (5, 1, 2, 2, None)])
def test_split1_equals_brute_force(seed, n, F, K, levels):
    X, y = synth.random_small(seed, n, F, K, levels)
    ds = oracle.dataset_from_X(X, y, K)
    f, t, c = oracle.split1(ds)
    assert c == brute.best_depth1(ds.ranks, ds.n_unique, y, K, None)
    # the returned split attains it, and no earlier candidate does (R10 order)
    got = brute.correct_of(brute.rank_counts(ds.ranks, y, K, [f], [t], 1))
    assert got == c
    nk_max = np.bincount(y, minlength=K).max()
    if c == nk_max:
        assert (f, t) == (0, 0)
    else:
        for f2 in range(1, F + 1):
            for t2 in range(1, int(ds.n_unique[f2 - 1])):
                if (f2, t2) == (f, t):
                    break
                assert brute.correct_of(brute.rank_counts(ds.ranks, y, K, [f2], [t2], 1)) < c
            else:
                continue
            break
    # degenerate thresholds never beat no split
    assert 0 < t < ds.n_unique[f - 1] if f else t == 0


def test_split1_on_subsets():
    X, y = synth.random_small(6, 60, 3, 3, levels=5)
    ds = oracle.dataset_from_X(X, y, 3)
    rng = np.random.default_rng(0)
    for _ in range(5):
        idx = np.sort(rng.choice(60, size=rng.integers(1, 60), replace=False))
        f, t, c = oracle.split1(ds, idx=idx)
        assert c == brute.best_depth1(ds.ranks, ds.n_unique, y, 3, list(idx))


@pytest.mark.parametrize("seed,n,F,K,levels", [(1, 10, 2, 2, None), (2, 12, 2, 3, 4),
                                               (3, 9, 1, 2, None), (4, 12, 2, 2, 3)])
def test_opt2_equals_brute_force_over_all_3_node_trees(seed, n, F, K, levels):
    X, y = synth.random_small(seed, n, F, K, levels)
    ds = oracle.dataset_from_X(X, y, K)
    c, feat, tau = oracle.opt2(ds)
    assert c == brute.best_depth2(ds.ranks, ds.n_unique, y, K)
    _, correct, _, _ = oracle.fitness(ds, feat[None], tau[None], 2)
    assert correct[0] == c


def test_greedy_tree_depth1_is_split1():
    X, y = synth.random_small(11, 80, 3, 3, levels=8)
    ds = oracle.dataset_from_X(X, y, 3)
    f, t, _ = oracle.split1(ds)
    feat, tau = oracle.greedy_tree(ds, 1)
    assert (feat[0], tau[0]) == (f, t)


def test_greedy_tree_children_are_split1_of_their_subsets():
    X, y = synth.random_small(12, 200, 4, 3, levels=10)
    ds = oracle.dataset_from_X(X, y, 3)
    feat, tau = oracle.greedy_tree(ds, 2)
    root_left = np.nonzero((feat[0] != 0) & (ds.ranks[max(feat[0], 1) - 1] < tau[0]))[0]
    root_right = np.setdiff1d(np.arange(200), root_left)
    for node, idx in ((1, root_left), (2, root_right)):
        if len(idx) > 1 and len(np.unique(y[idx])) > 1:
            f, t, _ = oracle.split1(ds, idx=idx)
            assert (feat[node], tau[node]) == (f, t)
        else:
            assert (feat[node], tau[node]) == (0, 0)
