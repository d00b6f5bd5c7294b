"""GPU parity of CART (Gini; reading R15) and of the moving horizon's warm
starts (Algorithm 2's warm-start branch; the warm-start factors of Section
4's ablation table) against the oracle.  Bar: bit-exact trees, counts and
f64 costs; the sequential and batched forms return the same tree."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


@pytest.mark.parametrize("seed,n,F,K,levels,D", [
    (1, 1, 2, 2, None, 2),          # one sample
    (2, 40, 3, 2, None, 3),
    (3, 500, 4, 3, 7, 4),           # many ties
    (4, 5000, 6, 5, None, 5),
    (5, 3000, 3, 2, 2, 6),          # binary features: thresholds run out
    (6, 200, 9, 4, 30, 10),         # depth 10: most nodes empty
    (7, 20_000, 40, 7, 50, 4),      # many (feature, threshold) candidates
    (8, 777, 255, 3, 5, 3),         # the largest feature count
    (9, 0, 4, 3, None, 3),          # empty dataset
    (10, 300_001, 7, 3, 90, 3),     # level counts and key build over several chunks per block
])
def test_cart_matches_oracle(mh, seed, n, F, K, levels, D):
    X, y = synth.random_small(seed, n, F, K, levels)
    want = oracle.cart(oracle.dataset_from_X(X, y, K), D)
    feat, tau = mh.cart(mh.dataset(X, y, K), D)
    np.testing.assert_array_equal(feat, want[0])
    np.testing.assert_array_equal(tau, want[1])


def test_cart_subsets_pure_and_constant(mh):
    X, y = synth.random_small(17, 4000, 5, 3, 25)
    ods = oracle.dataset_from_X(X, y, 3)
    ds = mh.dataset(X, y, 3)
    rng = np.random.default_rng(0)
    for size in (1, 2, 17, 999, 3999):
        idx = rng.choice(4000, size=size, replace=False).astype(np.uint32)
        for D in (1, 3):
            got = mh.cart(ds, D, idx=dev(idx))
            want = oracle.cart(ods, D, idx=idx)
            np.testing.assert_array_equal(got[0], want[0])
            np.testing.assert_array_equal(got[1], want[1])
    pure = np.nonzero(y == 1)[0].astype(np.uint32)
    feat, tau = mh.cart(ds, 3, idx=dev(pure))
    assert not feat.any() and not tau.any()
    Xc = np.repeat(X[:1], 50, axis=0)
    yc = (np.arange(50) % 3).astype(np.uint8)
    feat, tau = mh.cart(mh.dataset(Xc, yc, 3), 4)
    assert not feat.any() and not tau.any()


def _planted(seed, n, F=12, K=3):
    rng = np.random.default_rng(seed)
    X = rng.random((n, F)).astype(np.float32)
    y = np.where(X[:, 0] < 0.5, np.where(X[:, 1] < 0.3, 0, 1), np.where(X[:, 2] < 0.6, 2, 0))
    y = np.where(rng.random(n) < 0.05, rng.integers(K, size=n), y)
    return X, y.astype(np.uint8)


def _same(a, b):
    np.testing.assert_array_equal(a["feat"], b["feat"])
    np.testing.assert_array_equal(a["tau"], b["tau"])
    np.testing.assert_array_equal(a["label"], b["label"])
    assert a["correct"] == b["correct"] and a["cost"] == b["cost"]


WS = {"cart": 2, "deoct": 4, "deoct_cart": 12, "all": 14, "deoct_and_cart": 6}


@pytest.mark.parametrize("ws", list(WS))
@pytest.mark.parametrize("seed,n,F,K,D,D_MH,P,G", [
    (1, 3000, 6, 3, 4, 2, 16, 6),
    (2, 2500, 5, 4, 5, 3, 12, 4),
    (3, 4000, 12, 3, 7, 3, 8, 3),    # whole-tree run at depth 7 (the walk kernel)
])
def test_mh_warm_starts_match_oracle(mh, ws, seed, n, F, K, D, D_MH, P, G):
    """Sequential and batched moving horizon with each combination of warm
    starts equal the oracle's tree (Algorithm 2)."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(seed, n, F, K, levels=40) if seed != 3 else _planted(seed, n, F, K)
    flags = WS[ws]
    want = oracle.mh_train(oracle.dataset_from_X(X, y, K), D, D_MH,
                           oracle.de_params(P, G, 0.5, 0.9, 300 + seed), flags=flags)
    ctx = capi.Context(0)
    ds = mh.dataset(X, y, K, ctx=ctx)
    prm = mh.de_params(P, G, 0.5, 0.9, 300 + seed)
    seq = mh.mh_train(ds, D, D_MH, prm, batched=False, ctx=ctx, warm=flags)
    bat = mh.mh_train(ds, D, D_MH, prm, batched=True, ctx=ctx, warm=flags)
    ctx.close()
    _same(seq, want)
    _same(bat, want)


def test_mh_warm_start_flags_rejected(mh):
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(4, 100, 3, 2)
    ds = mh.dataset(X, y, 2)
    prm = mh.de_params(8, 2, 0.5, 0.9, 1)
    for bad in (capi.MH_WS_DEOCT_CART, 16, 1 << 31):
        with pytest.raises(mh.MhError) as ei:
            mh.mh_train(ds, 3, 2, prm, warm=bad)
        assert ei.value.code == capi.MH_EINVAL
    with pytest.raises(mh.MhError) as ei:
        mh.cart(ds, 11)
    assert ei.value.code == capi.MH_EINVAL
