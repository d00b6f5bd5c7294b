"""Pins of the oracle's threshold sets (rank encoding, reading R1) and
decoding (eq. aenc, eq. benc; readings R3, R4)."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth


@pytest.mark.parametrize("seed,n,F,levels", [(1, 50, 3, None), (2, 200, 5, 7), (3, 1, 2, None),
                                             (4, 300, 1, 2)])
def test_rank_encode_matches_numpy_unique(seed, n, F, levels):
    X, _ = synth.random_small(seed, n, F, 2, levels)
    ranks, nu = oracle.rank_encode(X)
    for f in range(F):
        u, inv = np.unique(X[:, f], return_inverse=True)
        assert nu[f] == len(u)
        np.testing.assert_array_equal(ranks[f], inv.ravel())


def test_rank_encode_signed_zero_and_nan():
    X = np.array([[0.0], [-0.0], [1.0], [-1.0]], dtype=np.float32)
    ranks, nu = oracle.rank_encode(X)
    assert nu[0] == 3
    assert list(ranks[0]) == [1, 1, 2, 0]
    Xn = np.array([[0.0], [np.nan]], dtype=np.float32)
    with pytest.raises(ValueError):
        oracle.rank_encode(Xn)


def test_rank_encode_extremes():
    big = np.finfo(np.float32).max
    X = np.array([[np.inf], [-np.inf], [big], [-big], [1e-45]], dtype=np.float32)
    ranks, nu = oracle.rank_encode(X)
    assert nu[0] == 5
    assert list(ranks[0]) == [4, 0, 3, 1, 2]


def test_golden_hand_worked_decode(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "hand_worked_depth2.json")))
    X = np.array(g["X"], dtype=np.float32)
    ranks, nu = oracle.rank_encode(X)
    np.testing.assert_array_equal(ranks, np.array(g["ranks"]))
    np.testing.assert_array_equal(nu, np.array(g["n_unique"]))
    for tr in g["trees"]:
        feat, tau = oracle.decode(np.array(tr["genes"]), g["D"], X.shape[1], nu)
        assert list(feat[0]) == tr["feat"]
        assert list(tau[0]) == tr["tau"]


def _decode1(a, b, F, nf, D=1):
    genes = np.array([[a, b]], dtype=np.float64)
    feat, tau = oracle.decode(genes, D, F, np.array([nf] * F, dtype=np.uint32))
    return int(feat[0, 0]), int(tau[0, 0])


def test_decode_feature_floor_and_clamp():
    F = 5
    for a, want in [(0.0, 0), (0.999, 0), (1.0, 1), (3.7, 3), (5.0, 5), (5.999, 5),
                    (6.0, 5), (1e9, 5), (-3.0, 0), (float("nan"), 0)]:
        assert _decode1(a, 0.5, F, 10)[0] == want, a


def test_decode_no_split_forces_zero_threshold():
    for b in (0.0, 0.3, 0.999, 1.0):
        assert _decode1(0.5, b, 4, 10) == (0, 0)


def test_decode_threshold_interior_matches_exact_rational():
    # eq. benc: i = floor(b (n_p + 1)) + 1, tau = i - 1 (clamped to n_p).
    # Away from the interval ends the f64 product cannot cross an integer,
    # so exact rational arithmetic gives the same index.
    rng = np.random.default_rng(0)
    for nf in (1, 2, 3, 10, 999, 65535, 1_000_000):
        for b in rng.random(200):
            x = Fraction(float(b)) * (nf + 1)
            if abs(x - round(x)) < Fraction(1, 10**9):
                continue
            want = min(math.floor(x), nf)
            assert _decode1(2.5, float(b), 3, nf)[1] == want


def test_decode_threshold_interval_ends():
    # b exactly at k/(n_p+1) in binary (n_p + 1 a power of two) gives k; one
    # ulp below gives k - 1; b = 1 (the closed end after clamping) gives n_p.
    for nf in (1, 3, 7, 255, 4095):
        for k in range(0, nf + 1, max(1, nf // 7)):
            b = k / (nf + 1)
            assert _decode1(1.2, b, 2, nf)[1] == k
            if k > 0:
                assert _decode1(1.2, np.nextafter(b, 0.0), 2, nf)[1] == k - 1
        assert _decode1(1.2, 1.0, 2, nf)[1] == nf
        assert _decode1(1.2, np.nextafter(1.0, 0.0), 2, nf)[1] == nf
        assert _decode1(1.2, -0.5, 2, nf)[1] == 0
        assert _decode1(1.2, float("nan"), 2, nf)[1] == 0


def test_decode_uses_the_selected_features_set_size():
    # tau is scaled by n_p of the selected feature (eq. benc)
    genes = np.array([[1.5, 2.5, 3.5, 0.5, 0.5, 0.5]])
    nu = np.array([3, 9, 99], dtype=np.uint32)
    feat, tau = oracle.decode(genes, 2, 3, nu)
    assert list(feat[0]) == [1, 2, 3]
    assert list(tau[0]) == [2, 5, 50]
