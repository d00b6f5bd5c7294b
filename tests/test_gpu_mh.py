"""GPU parity of the exact depth-1 split and the moving-horizon trainer
(Algorithm 2) against the oracle; the level-batched form must return the same
tree as the node-by-node form.  Bar: bit-exact (integer trees and counts,
exactly rounded f64 costs)."""
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


@pytest.mark.parametrize("seed,n,F,K,levels", [(1, 1, 2, 2, None), (2, 40, 3, 2, None),
                                               (3, 500, 4, 3, 7), (4, 5000, 6, 5, None),
                                               (5, 3000, 3, 2, 2), (6, 200, 9, 4, 30),
                                               # several 256-sample chunks per block of the
                                               # key build, a ragged last block, F not a
                                               # power of two
                                               (8, 300_001, 7, 3, None),
                                               # more than 16 classes: the class counts'
                                               # per-element LDS adds
                                               (11, 50_000, 5, 40, None)])
def test_split1_all(mh, seed, n, F, K, levels):
    X, y = synth.random_small(seed, n, F, K, levels)
    want = oracle.split1(oracle.dataset_from_X(X, y, K))
    assert mh.split1(mh.dataset(X, y, K)) == want


def test_split1_subsets_and_pure(mh):
    X, y = synth.random_small(7, 4000, 5, 3, 25)
    ods = oracle.dataset_from_X(X, y, 3)
    ds = mh.dataset(X, y, 3)
    rng = np.random.default_rng(0)
    for size in (1, 2, 17, 999, 3999):
        idx = rng.choice(4000, size=size, replace=False).astype(np.uint32)
        assert mh.split1(ds, idx=dev(idx)) == oracle.split1(ods, idx=idx)
    pure = np.nonzero(y == 1)[0].astype(np.uint32)
    assert mh.split1(ds, idx=dev(pure)) == oracle.split1(ods, idx=pure) == (0, 0, len(pure))


def test_split1_subsets_large(mh):
    """Subsets of a dataset large enough that the key build's blocks take
    several 256-sample chunks each (about two blocks per CU)."""
    X, y = synth.random_small(9, 400_000, 5, 4, 60)
    ods = oracle.dataset_from_X(X, y, 4)
    ds = mh.dataset(X, y, 4)
    rng = np.random.default_rng(1)
    for size in (1, 513, 150_000, 399_999):
        idx = np.sort(rng.choice(400_000, size=size, replace=False)).astype(np.uint32)
        assert mh.split1(ds, idx=dev(idx)) == oracle.split1(ods, idx=idx)


def _mh_both(mh, X, y, K, D, D_MH, P, G, seed, M=0.5, CR=0.9, n_min=1, alpha=0.0, ctx=None,
             want=None):
    if want is None:
        ods = oracle.dataset_from_X(X, y, K)
        want = oracle.mh_train(ods, D, D_MH, oracle.de_params(P, G, M, CR, seed, n_min, alpha))
    ds = mh.dataset(X, y, K, ctx=ctx)
    prm = mh.de_params(P, G, M, CR, seed, n_min, alpha)
    seq = mh.mh_train(ds, D, D_MH, prm, batched=False, ctx=ctx)
    bat = mh.mh_train(ds, D, D_MH, prm, batched=True, ctx=ctx)
    return want, seq, bat


def _same(a, b):
    np.testing.assert_array_equal(a["feat"], b["feat"])
    np.testing.assert_array_equal(a["tau"], b["tau"])
    np.testing.assert_array_equal(a["label"], b["label"])
    assert a["correct"] == b["correct"] and a["cost"] == b["cost"]


@pytest.mark.parametrize("seed,n,F,K,D,D_MH,P,G", [
    (1, 2000, 5, 3, 3, 2, 16, 8),
    (2, 3000, 4, 2, 4, 3, 12, 6),
    (3, 1500, 6, 4, 2, 2, 10, 5),
    (4, 2500, 5, 3, 5, 1, 8, 3),     # horizon 1: exact splits only
    (5, 800, 3, 2, 6, 3, 8, 4),
])
def test_mh_train_matches_oracle(mh, seed, n, F, K, D, D_MH, P, G):
    X, y = synth.random_small(seed, n, F, K, levels=40)
    want, seq, bat = _mh_both(mh, X, y, K, D, D_MH, P, G, 100 + seed)
    _same(seq, want)
    _same(bat, want)


@pytest.mark.parametrize("n_min,alpha", [(60, 0.0), (30, 12.5), (1, 400.0)])
def test_mh_train_penalised(mh, n_min, alpha):
    """Moving horizon under the penalised objective: n_min also decides which
    nodes of a level are solved (more than n_min samples of two or more
    classes), alpha prices each split in every subproblem."""
    X, y = synth.random_small(9, 3000, 5, 3, levels=40)
    want, seq, bat = _mh_both(mh, X, y, 3, 4, 2, 16, 6, 77, n_min=n_min, alpha=alpha)
    _same(seq, want)
    _same(bat, want)


_FORMS = {"default": {}, "staged": {"MHDEOCT_PERSIST": "1", "MHDEOCT_PERSIST_RESIDENT": "0"},
          "per_generation": {"MHDEOCT_PERSIST": "0"}}
_depth8_want = {}


@pytest.mark.parametrize("form", list(_FORMS))
@pytest.mark.parametrize("n,P,G", [(20_000, 16, 5), (200_000, 16, 3)])
def test_mh_depth8_launch_forms(mh, monkeypatch, form, n, P, G):
    """The batched moving-horizon workload's shape (Gaussian mixture, F = 20,
    K = 3, depth 8, horizon 3) in each launch form of a level: the default
    choice, the whole-level kernel with tiles staged from memory every
    generation (the form the levels take at n = 10^6, where a block's tiles do
    not fit its LDS), and the per-generation kernels (the form a level is
    redone in after a grid barrier gave up).  Sequential and batched runs
    equal the oracle's tree (Algorithm 2)."""
    from paper_2311_06952_amd import capi
    w = synth.batched_mh(1, n=n)
    key = (n, P, G)
    if key not in _depth8_want:
        _depth8_want[key] = oracle.mh_train(oracle.dataset_from_X(w.X, w.y, w.K), 8, 3,
                                            oracle.de_params(P, G, 0.5, 0.9, 1001))
    for k, v in _FORMS[form].items():
        monkeypatch.setenv(k, v)
    ctx = capi.Context(0)
    want, seq, bat = _mh_both(mh, w.X, w.y, w.K, 8, 3, P, G, 1001, ctx=ctx,
                              want=_depth8_want[key])
    _same(seq, want)
    _same(bat, want)
    ctx.close()


def test_mh_large_population_per_generation(mh, monkeypatch):
    """Moving horizon with P = 256 per subproblem on the per-generation kernels
    (the DE generation of every node of a level split over the chip) equals
    the oracle's tree."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(31, 6000, 5, 3, levels=40)
    monkeypatch.setenv("MHDEOCT_PERSIST", "0")
    ctx = capi.Context(0)
    want, seq, bat = _mh_both(mh, X, y, 3, 5, 3, 256, 4, 99, M=-1.0, ctx=ctx)
    _same(seq, want)
    _same(bat, want)
    ctx.close()
