"""A seeded sweep of moving-horizon shapes against the oracle (Algorithm 2):
depths 2 to 8, horizons 1 to 4, every combination of warm starts, penalised
objectives, 2 to 9 classes; the node-by-node and the level-batched forms both
equal the oracle's tree, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


def _shapes(seed=77, count=30):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        D = int(rng.integers(2, 9))
        H = int(rng.integers(1, 5))
        F = int(rng.choice([2, 5, 12, 40]))
        K = int(rng.integers(2, 10))
        n = int(rng.integers(50, 5000))
        P = int(rng.choice([4, 9, 16, 32]))
        G = int(rng.integers(1, 5))
        flags = int(rng.choice([0, 2, 4, 6, 12, 14]))
        n_min = int(rng.choice([1, 1, 15]))
        alpha = float(rng.choice([0.0, 0.0, 5.0]))
        levels = [None, 6, 60][int(rng.integers(0, 3))]
        out.append((i, n, F, K, D, H, P, G, flags, n_min, alpha, levels))
    return out


SHAPES = _shapes()


@pytest.mark.parametrize("shape", SHAPES, ids=[f"m{s[0]}" for s in SHAPES])
def test_mh_random_shapes(mh, shape):
    from paper_2311_06952_amd import capi
    i, n, F, K, D, H, P, G, flags, n_min, alpha, levels = shape
    X, y = synth.random_small(900 + i, n, F, K, levels)
    seed = 4000 + i
    want = oracle.mh_train(oracle.dataset_from_X(X, y, K), D, H,
                           oracle.de_params(P, G, 0.5, 0.9, seed, n_min, alpha), flags=flags)
    ctx = capi.Context(0)
    ds = mh.dataset(X, y, K, ctx=ctx)
    prm = mh.de_params(P, G, 0.5, 0.9, seed, n_min, alpha)
    forms = [False] + ([True] if min(D, H) <= 5 else [])
    for batched in forms:
        got = mh.mh_train(ds, D, H, prm, batched=batched, ctx=ctx, warm=flags)
        np.testing.assert_array_equal(got["feat"], want["feat"])
        np.testing.assert_array_equal(got["tau"], want["tau"])
        np.testing.assert_array_equal(got["label"], want["label"])
        assert got["correct"] == want["correct"] and got["cost"] == want["cost"]
    ctx.close()
