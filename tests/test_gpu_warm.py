"""GPU parity of tree encoding and warm starts (the inverse of eq. aenc / eq.
benc, reading R14; the warm-started DEOCT variants of Section 4): genes
bit-equal to the oracle's, decode(encode) the identity, and warm-started
runs equal to the oracle's and never worse than the tree they start from."""
import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


@pytest.mark.parametrize("D,F,P", [(1, 3, 5), (3, 16, 256), (6, 9, 40), (10, 4, 3)])
def test_encode_matches_oracle_and_decodes_back(mh, D, F, P):
    X, y = synth.random_small(300 + D, 4000, F, 3, levels=None if D % 2 else 25)
    ds = mh.dataset(X, y, 3)
    nu = ds.n_unique.cpu().numpy().astype(np.uint32)
    rng = np.random.default_rng(D)
    SB = (1 << D) - 1
    feat = rng.integers(0, F + 2, size=(P, SB)).astype(np.uint8)  # F + 1: not a feature
    tau = np.array([[[0, nu[f - 1], rng.integers(0, nu[f - 1] + 1)][rng.integers(0, 3)]
                     if 0 < f <= F else rng.integers(0, 9) for f in row] for row in feat],
                   dtype=np.uint32)
    genes = mh.tree_encode(feat, tau, D, F, ds.n_unique)
    want = oracle.tree_encode(feat, tau, D, F, nu)
    np.testing.assert_array_equal(genes.cpu().numpy(), want)
    f2, t2 = mh.tree_decode(genes, D, F, ds.n_unique)
    keep = feat <= F
    np.testing.assert_array_equal(f2.cpu().numpy(), np.where(keep, feat, 0))
    np.testing.assert_array_equal(t2.cpu().numpy().view(np.uint32), np.where(keep & (feat > 0),
                                                                              tau, 0))


@pytest.mark.parametrize("seed,D", [(1, 3), (2, 4)])
def test_warm_start_from_greedy_tree(mh, seed, D):
    """The greedy tree (moving horizon with horizon 1: exact depth-1 splits)
    encoded into one warm individual: the warm-started DEOCT equals the
    oracle's and is at least as good as the greedy tree."""
    X, y = synth.random_small(seed, 6000, 7, 3, levels=30)
    ds = mh.dataset(X, y, 3)
    prm = mh.de_params(16, 3, 0.5, 0.9, seed)
    greedy = mh.mh_train(ds, D, 1, prm)
    warm = mh.tree_encode(greedy["feat"], greedy["tau"], D, 7, ds.n_unique).cpu().numpy()
    got = mh.subtree_solve(ds, D, mh.de_params(64, 25, 0.5, 0.9, 50 + seed), warm=warm,
                           with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, 3), D,
                        oracle.de_params(64, 25, 0.5, 0.9, 50 + seed), warm=warm, with_pop=True)
    for k in ("feat", "tau", "label"):
        np.testing.assert_array_equal(got[k], want[k])
    for k in ("pop", "pop_cost"):
        np.testing.assert_array_equal(got[k].view(np.uint64), want[k].view(np.uint64))
    assert got["correct"] == want["correct"] and got["cost"] == want["cost"]
    assert got["correct"] >= greedy["correct"]


def test_warm_start_from_earlier_run(mh, monkeypatch):
    """A DEOCT run continued from its own best tree (the full-tree warm start)
    on the persistent and per-generation kernels."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(77, 9000, 8, 4)
    first = None
    for persist in ("0", "1"):
        monkeypatch.setenv("MHDEOCT_PERSIST", persist)
        ctx = capi.Context(0)
        ds = mh.dataset(X, y, 4, ctx=ctx)
        t1 = mh.subtree_solve(ds, 3, mh.de_params(128, 15, 0.5, 0.9, 1), ctx=ctx)
        warm = mh.tree_encode(t1["feat"], t1["tau"], 3, 8, ds.n_unique, ctx=ctx).cpu().numpy()
        t2 = mh.subtree_solve(ds, 3, mh.de_params(128, 15, 0.5, 0.9, 2), warm=warm, ctx=ctx,
                              with_pop=True)
        ctx.close()
        want = oracle.deoct(oracle.dataset_from_X(X, y, 4), 3,
                            oracle.de_params(128, 15, 0.5, 0.9, 2), warm=warm, with_pop=True)
        for k in ("feat", "tau", "label"):
            np.testing.assert_array_equal(t2[k], want[k])
        for k in ("pop", "pop_cost"):
            np.testing.assert_array_equal(t2[k].view(np.uint64), want[k].view(np.uint64))
        assert t2["correct"] == want["correct"] >= t1["correct"]
        if first is None:
            first = t2
        else:
            np.testing.assert_array_equal(first["feat"], t2["feat"])
