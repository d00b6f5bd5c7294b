"""GPU parity of applying a trained tree to held-out rows (Section 2 split
rule with the Section 3.1 threshold sets; the 75/25 train/test protocol and
test accuracy of Section 4; reading R13): thresholds bit-equal to the
oracle's, predictions and correct counts equal."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


def _split(X, y, seed):
    """75/25 split of the rows."""
    perm = np.random.default_rng(seed).permutation(len(y))
    cut = (3 * len(y)) // 4
    a, b = perm[:cut], perm[cut:]
    return X[a], y[a], X[b], y[b]


def _check(mh, ds, Xtr, tree, Xte, yte):
    thr = mh.tree_thresholds(ds, Xtr, tree)
    want_thr = oracle.tree_thresholds(Xtr, tree["feat"], tree["tau"], tree["D"])
    np.testing.assert_array_equal(thr.cpu().numpy(), want_thr)
    pred, correct = mh.predict(Xte, tree, thr, y=yte)
    want_pred, want_correct = oracle.predict(Xte, tree["feat"], want_thr, tree["label"],
                                             tree["D"], y=yte)
    np.testing.assert_array_equal(pred.cpu().numpy(), want_pred)
    assert correct == want_correct
    return thr, correct


@pytest.mark.parametrize("seed,n,F,K,D,levels", [(1, 4000, 6, 3, 3, None), (2, 9001, 8, 2, 4, 30),
                                                 (3, 2500, 5, 4, 2, 4), (4, 130, 3, 5, 5, None)])
def test_trained_tree_on_held_out_rows(mh, seed, n, F, K, D, levels):
    X, y = synth.random_small(seed, n, F, K, levels)
    Xtr, ytr, Xte, yte = _split(X, y, seed)
    ds = mh.dataset(Xtr, ytr, K)
    tree = mh.subtree_solve(ds, D, mh.de_params(64, 20, 0.5, 0.9, seed))
    thr, _ = _check(mh, ds, Xtr, tree, Xte, yte)
    # on its own training rows the tree scores its training correct count
    _, c_train = mh.predict(Xtr, tree, thr, y=ytr)
    assert c_train == tree["correct"]


@pytest.mark.parametrize("D", [1, 2, 3, 6, 8, 10])
def test_random_trees_every_threshold_kind(mh, D):
    """Random trees with tau = 0, interior tau, tau = n_f, feat = 0 and a
    feature past F, on tied data; held-out rows with a ragged count, values
    outside the training range and NaNs."""
    X, y = synth.random_small(20 + D, 7000, 7, 3, levels=12)
    Xtr, ytr, Xte, yte = _split(X, y, D)
    Xte = Xte.copy()
    Xte[::37, 2] = np.nan
    Xte[5::41, 1] = 1e30
    Xte[7::43, 3] = -1e30
    ds = mh.dataset(Xtr, ytr, 3)
    nu = ds.n_unique.cpu().numpy()
    rng = np.random.default_rng(D)
    SB = (1 << D) - 1
    for _ in range(3):
        feat = rng.integers(0, 9, size=SB).astype(np.uint8)  # 8 = F + 1: no split
        tau = np.array([[0, nu[f - 1], rng.integers(0, nu[f - 1] + 1)][rng.integers(0, 3)]
                        if 0 < f <= 7 else rng.integers(0, 5) for f in feat], dtype=np.uint32)
        label = rng.integers(0, 3, size=SB + 1).astype(np.uint8)
        tree = dict(D=D, feat=feat, tau=tau, label=label)
        _check(mh, ds, Xtr, tree, Xte[: len(yte) - 3], yte[: len(yte) - 3])


@pytest.mark.parametrize("F,n,D", [(100, 5003, 4), (255, 3001, 3), (1, 777, 5), (63, 20000, 6)])
def test_wide_and_narrow_rows(mh, F, n, D):
    """Row widths that change how many rows one staged tile holds (F = 255:
    16 rows, F = 100: 40, F = 63: 64, F = 1: 256), with ragged last tiles."""
    X, y = synth.random_small(40 + F, n, F, 4, levels=50)
    Xtr, ytr, Xte, yte = _split(X, y, F)
    ds = mh.dataset(Xtr, ytr, 4)
    nu = ds.n_unique.cpu().numpy()
    rng = np.random.default_rng(F)
    SB = (1 << D) - 1
    feat = rng.integers(0, F + 1, size=SB).astype(np.uint8)
    tau = np.array([rng.integers(0, nu[f - 1] + 1) if f else 0 for f in feat], dtype=np.uint32)
    tree = dict(D=D, feat=feat, tau=tau, label=rng.integers(0, 4, size=SB + 1).astype(np.uint8))
    _check(mh, ds, Xtr, tree, Xte, yte)
    _check(mh, ds, Xtr, tree, Xtr, ytr)


def test_full_size_split(mh):
    """The DEOCT workload's shape (n = 10^5, F = 16, K = 3, depth 3) split
    75/25, and a depth-10 random tree on 10^6 held-out rows."""
    X, y = synth.random_small(99, 100_000, 16, 3)
    Xtr, ytr, Xte, yte = _split(X, y, 99)
    ds = mh.dataset(Xtr, ytr, 3)
    tree = mh.subtree_solve(ds, 3, mh.de_params(256, 30, 0.5, 0.9, 99))
    _check(mh, ds, Xtr, tree, Xte, yte)
    rng = np.random.default_rng(5)
    nu = ds.n_unique.cpu().numpy()
    SB = 1023
    feat = rng.integers(1, 17, size=SB).astype(np.uint8)
    tau = np.array([rng.integers(0, nu[f - 1] + 1) for f in feat], dtype=np.uint32)
    tree = dict(D=10, feat=feat, tau=tau, label=rng.integers(0, 3, size=1024).astype(np.uint8))
    Xbig, ybig = synth.random_small(98, 1_000_000, 16, 3)
    _check(mh, ds, Xtr, tree, Xbig, ybig)


def test_unaligned_rows_take_the_word_path(mh):
    """F = 8 rows starting 4 bytes past a 16-byte boundary: the float4 form
    does not apply, the per-word form must give the same result."""
    import torch
    X, y = synth.random_small(61, 5000, 8, 3, levels=20)
    ds = mh.dataset(X, y, 3)
    tree = mh.subtree_solve(ds, 4, mh.de_params(32, 10, 0.5, 0.9, 61))
    thr = mh.tree_thresholds(ds, X, tree)
    buf = torch.empty(X.size + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.as_tensor(X.ravel()).cuda()
    Xv = buf[1:].view(X.shape)
    assert Xv.data_ptr() % 16 == 4
    pred, correct = mh.predict(Xv, tree, thr, y=y)
    want_pred, want_correct = oracle.predict(X, tree["feat"], thr.cpu().numpy(), tree["label"],
                                             4, y=y)
    np.testing.assert_array_equal(pred.cpu().numpy(), want_pred)
    assert correct == want_correct == tree["correct"]


def test_empty_and_single_rows(mh):
    X, y = synth.random_small(7, 300, 4, 2)
    ds = mh.dataset(X, y, 2)
    tree = mh.subtree_solve(ds, 2, mh.de_params(16, 5, 0.5, 0.9, 7))
    thr = mh.tree_thresholds(ds, X, tree)
    pred, correct = mh.predict(X[:0], tree, thr, y=y[:0])
    assert pred.numel() == 0 and correct == 0
    _check(mh, ds, X, tree, X[:1], y[:1])
    # a tree over an empty training set: thresholds from n_f = 0
    ds0 = mh.dataset(X[:0], y[:0], 2)
    tree0 = dict(D=2, feat=np.array([1, 2, 0], np.uint8), tau=np.array([0, 0, 0], np.uint32),
                 label=np.array([1, 0, 1, 0], np.uint8))
    _check(mh, ds0, X[:0], tree0, X, y)


def test_argument_errors(mh):
    import torch
    from paper_2311_06952_amd import capi
    ctx = capi.default_context()
    X = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    feat = torch.zeros(3, dtype=torch.uint8, device="cuda")
    thr = torch.zeros(3, dtype=torch.float64, device="cuda")
    label = torch.zeros(4, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
    # correct without y (n > 0), depth 0, depth 11; no rows needs no y
    assert ctx.lib.mh_predict(ctx.h, None, 0, 3, p(feat), p(thr), p(label), 2, None, None,
                              p(cnt)) == capi.MH_OK
    assert ctx.lib.mh_predict(ctx.h, p(X), 10, 3, p(feat), p(thr), p(label), 2, None, None,
                              p(cnt)) == capi.MH_EINVAL
    assert ctx.lib.mh_predict(ctx.h, p(X), 10, 3, p(feat), p(thr), p(label), 0, None, None,
                              None) == capi.MH_EINVAL
    assert ctx.lib.mh_predict(ctx.h, p(X), 10, 3, p(feat), p(thr), p(label), 11, None, None,
                              None) == capi.MH_EINVAL
