"""Pins of the oracle's CART (Gini; reading R15), the warm start of
Algorithm 2 and of the plain DEOCT runs of Section 4, and of the moving
horizon's warm-start variants (Algorithm 2's warm-start branch; the ablation
rows of Table 2).  CART is pinned against exact rational arithmetic on small
data and against scikit-learn's Gini tree (the library routine the reading
stands in for) on continuous data."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth


def _gini_score(ranks_f, y, K, idx, th):
    """sum_k L_k^2 / |L| + sum_k R_k^2 / |R| as an exact rational, None when
    a side is empty."""
    left = ranks_f[idx] < th
    nL, nR = int(left.sum()), int((~left).sum())
    if nL == 0 or nR == 0:
        return None
    L = np.bincount(y[idx][left], minlength=K).astype(object)
    R = np.bincount(y[idx][~left], minlength=K).astype(object)
    return Fraction(int(sum(v * v for v in L)), nL) + Fraction(int(sum(v * v for v in R)), nR)


def _check_node(ds, y, K, idx, f, t):
    """(f, t) is a best Gini split of the subset idx, or (0, 0) when the
    subset is pure or no threshold sends samples both ways; with a unique
    best, it is that one."""
    scores = {}
    if len(np.unique(y[idx])) > 1:
        for f2 in range(1, ds.F + 1):
            for t2 in range(1, int(ds.n_unique[f2 - 1])):
                s = _gini_score(ds.ranks[f2 - 1], y, K, idx, t2)
                if s is not None:
                    scores[(f2, t2)] = s
    if not scores:
        assert (f, t) == (0, 0)
        return
    best = max(scores.values())
    assert scores.get((f, t)) == best
    tied = [k for k, v in scores.items() if v == best]
    if len(tied) == 1:
        assert (f, t) == tied[0]


def _subset(ds, feat, tau, node, n):
    """Samples reaching heap node `node` (1-based)."""
    path = []
    u = node
    while u > 1:
        path.append(u)
        u //= 2
    idx = np.arange(n)
    u = 1
    for v in reversed(path):
        f = feat[u - 1]
        left = (f != 0) & (ds.ranks[max(f, 1) - 1][idx] < tau[u - 1])
        idx = idx[left] if v == 2 * u else idx[~left]
        u = v
    return idx


@pytest.mark.parametrize("seed,n,F,K,levels,D", [(1, 30, 2, 2, None, 1), (2, 40, 3, 3, 4, 2),
                                                 (3, 25, 3, 4, 3, 3), (4, 12, 1, 2, None, 2),
                                                 (5, 1, 2, 2, None, 2), (6, 36, 4, 2, 2, 3)])
def test_cart_nodes_are_exact_gini_optima(seed, n, F, K, levels, D):
    X, y = synth.random_small(seed, n, F, K, levels)
    ds = oracle.dataset_from_X(X, y, K)
    feat, tau = oracle.cart(ds, D)
    for node in range(1, (1 << D)):
        _check_node(ds, y, K, _subset(ds, feat, tau, node, n), int(feat[node - 1]),
                    int(tau[node - 1]))


def test_cart_pure_and_constant_subsets_do_not_split():
    X, y = synth.random_small(7, 50, 3, 3, levels=6)
    ds = oracle.dataset_from_X(X, y, 3)
    pure = np.nonzero(y == 2)[0]
    feat, tau = oracle.cart(ds, 2, idx=pure)
    assert not feat.any() and not tau.any()
    # samples that agree on every feature cannot be separated
    Xc = np.repeat(X[:1], 20, axis=0)
    yc = (np.arange(20) % 3).astype(np.uint8)
    dc = oracle.dataset_from_X(Xc, yc, 3)
    feat, tau = oracle.cart(dc, 3)
    assert not feat.any() and not tau.any()


@pytest.mark.parametrize("seed,n,F,K,D", [(1, 400, 5, 3, 3), (2, 700, 8, 4, 4),
                                          (3, 300, 3, 2, 5)])
def test_cart_partitions_equal_sklearn_gini_tree(seed, n, F, K, D):
    """On continuous data (no tied values, so no two thresholds give the same
    partition) the oracle's CART and scikit-learn's Gini tree of the same
    depth split the samples into the same leaves."""
    sk = pytest.importorskip("sklearn.tree")
    rng = np.random.default_rng(seed)
    X = rng.random((n, F)).astype(np.float32)
    # labels with structure, so that splits are decisive
    y = ((X[:, 0] > 0.4).astype(int) + (X[:, 1 % F] > 0.7) + (X[:, 2 % F] > 0.5)) % K
    y = np.where(rng.random(n) < 0.1, rng.integers(K, size=n), y).astype(np.uint8)
    ds = oracle.dataset_from_X(X, y, K)
    feat, tau = oracle.cart(ds, D)
    leaf = np.empty(n, dtype=np.int64)
    for i in range(n):
        u = 1
        for _ in range(D):
            f = feat[u - 1]
            u = 2 * u if (f != 0 and ds.ranks[f - 1][i] < tau[u - 1]) else 2 * u + 1
        leaf[i] = u
    clf = sk.DecisionTreeClassifier(criterion="gini", max_depth=D, random_state=0)
    clf.fit(X.astype(np.float64), y)
    ref = clf.apply(X.astype(np.float64))

    def blocks(a):
        return sorted(tuple(np.nonzero(a == v)[0]) for v in np.unique(a))
    assert blocks(leaf) == blocks(ref)


def _planted(seed, n=600, F=12, K=3):
    """Labels from a depth-3 axis-aligned tree on features 1..3; features
    4..F are noise."""
    rng = np.random.default_rng(seed)
    X = rng.random((n, F)).astype(np.float32)
    y = np.where(X[:, 0] < 0.5, np.where(X[:, 1] < 0.3, 0, 1), np.where(X[:, 2] < 0.6, 2, 0))
    return X, y.astype(np.uint8)


@pytest.mark.parametrize("flags", [oracle.MH_WS_CART, oracle.MH_WS_DEOCT | oracle.MH_WS_DEOCT_CART])
def test_mh_warm_start_reaches_the_cart_tree(flags):
    """With no DE generations and three individuals per subproblem, each
    node's DE returns the best of its warm start and two random trees.  On
    planted noise-free data the CART warm start is far better than random
    trees over twelve features, so every DE-solved node (depth <= D - 2)
    commits the root of its warm start: the CART split of its subset (CART
    flag), or the whole-tree CART's split at the same location (whole-tree
    DEOCT warm-started by CART; here the node subsets are CART's own, so the
    two agree).  Nodes at depth D - 1 take the exact depth-1 split."""
    X, y = _planted(3)
    ds = oracle.dataset_from_X(X, y, 3)
    D = 4
    prm = oracle.de_params(3, 0, 0.5, 0.9, 11)
    got = oracle.mh_train(ds, D, D, prm, flags=flags)
    cf, ct = oracle.cart(ds, D)
    for node in range(1, 1 << (D - 1)):
        assert (got["feat"][node - 1], got["tau"][node - 1]) == (cf[node - 1], ct[node - 1])
    for node in range(1 << (D - 1), 1 << D):
        idx = _subset(ds, got["feat"], got["tau"], node, ds.n)
        if len(idx) > 1 and len(np.unique(y[idx])) > 1:
            f, t, _ = oracle.split1(ds, idx=idx)
            assert (got["feat"][node - 1], got["tau"][node - 1]) == (f, t)


def _tree_cost(ds, feat, tau, D):
    _, correct, _, cost = oracle.fitness(ds, feat[None], tau[None], D)
    return cost[0]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mh_warm_starts_never_lose_to_their_source(seed):
    """Depth 2, horizon 2: the root's DE is warm-started with a depth-2 tree
    and keeps the best individual it has seen, and the two children then take
    exact depth-1 splits of their subsets, so the moving-horizon tree costs no
    more than that warm start: CART's depth-2 tree (CART flag), the whole-tree
    DEOCT (DEOCT flag), or CART's tree via the whole-tree DEOCT warm-started
    with it (both DEOCT flags)."""
    X, y = synth.random_small(seed, 500, 5, 3, levels=12)
    ds = oracle.dataset_from_X(X, y, 3)
    prm = oracle.de_params(8, 4, 0.5, 0.9, 40 + seed)
    cf, ct = oracle.cart(ds, 2)
    c_cart = _tree_cost(ds, cf, ct, 2)
    d = oracle.deoct(ds, 2, prm)
    c_deoct = d["cost"]
    assert oracle.mh_train(ds, 2, 2, prm, flags=oracle.MH_WS_CART)["cost"] <= c_cart
    assert oracle.mh_train(ds, 2, 2, prm, flags=oracle.MH_WS_DEOCT)["cost"] <= c_deoct
    both = oracle.MH_WS_DEOCT | oracle.MH_WS_DEOCT_CART
    assert oracle.mh_train(ds, 2, 2, prm, flags=both)["cost"] <= c_cart
    # no flags: the plain moving horizon is unchanged by the new argument
    plain = oracle.mh_train(ds, 2, 2, prm)
    assert plain["cost"] == oracle.mh_train(ds, 2, 2, prm, flags=0)["cost"]


def test_subtree_follows_the_paths_from_its_root():
    """Node u of the subtree at t is the node reached from t by following u's
    binary digits after the leading one (0 = left child, 1 = right child);
    nodes past the tree's depth carry no split."""
    D = 5
    rng = np.random.default_rng(4)
    feat = rng.integers(1, 200, size=(1 << D) - 1).astype(np.uint8)
    tau = np.arange(1, 1 << D, dtype=np.uint32) * 7
    for t in range(1, 1 << D):
        for De in (1, 2, 3, 4):
            sf, st = oracle.subtree(feat, tau, D, t, De)
            for u in range(1, 1 << De):
                v = t
                for bit in bin(u)[3:]:
                    v = 2 * v + int(bit)
                if v < (1 << D):
                    assert (sf[u - 1], st[u - 1]) == (feat[v - 1], tau[v - 1])
                else:
                    assert (sf[u - 1], st[u - 1]) == (0, 0)
