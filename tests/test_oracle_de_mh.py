"""Pins of the oracle's differential evolution (Section 2 eqs. mutation,
crossover, selection; Section 3.3; Algorithm 4; reading R8) and the
moving-horizon driver (Algorithm 2; reading R9).  The paper prints no DE
trajectory, so trajectories are pinned by properties only."""
import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth


def test_pick_distinct_and_uniform():
    P, m = 7, 6
    seen = np.zeros((P, P, P), dtype=np.int64)
    qs = np.zeros(m, dtype=np.int64)
    for g in range(1, 400):
        for r in range(P):
            r1, r2, q = oracle.de_pick(P, m, 3, 5, g, r)
            assert r1 != r and r2 != r and r2 != r1
            assert 0 <= r1 < P and 0 <= r2 < P and 0 <= q < m
            seen[r, r1, r2] += 1
            qs[q] += 1
    # every ordered pair (r1, r2) is reachable for each r, roughly uniformly
    for r in range(P):
        cnt = seen[r][(np.arange(P)[:, None] != r) & (np.arange(P)[None, :] != r)
                      & (np.arange(P)[:, None] != np.arange(P)[None, :])]
        assert cnt.min() > 0
        exp = 399 / ((P - 1) * (P - 2))
        assert np.sum((cnt - exp) ** 2 / exp) < 3 * len(cnt)
    assert qs.min() > 0


def test_init_ranges_and_warm_starts():
    D, F, P = 2, 5, 20
    warm = np.full((3, 6), 0.25)
    pop = oracle.de_init(P, D, F, 42, 0, warm)
    np.testing.assert_array_equal(pop[:3], warm)
    assert (pop[3:, :3] >= 0).all() and (pop[3:, :3] < F + 1).all()
    assert (pop[3:, 3:] >= 0).all() and (pop[3:, 3:] < 1).all()
    np.testing.assert_array_equal(pop, oracle.de_init(P, D, F, 42, 0, warm))
    assert not np.array_equal(pop, oracle.de_init(P, D, F, 42, 1, warm))


def _chi2(counts):
    counts = np.asarray(counts, dtype=np.float64)
    exp = counts.sum() / len(counts)
    return float(np.sum((counts - exp) ** 2 / exp))


def test_init_genes_cover_their_ranges_uniformly():
    """Algorithm 4 draws the initial population inside the range limits, and
    eq. aenc / eq. benc give the range of the feature gene as [0, F + 1) (so
    that floor picks "no split" or one of the F features) and of the
    threshold gene as [0, 1]: over 14,336 initial individuals' nodes the
    decoded feature hits every value 0..F with equal frequency and the
    threshold gene fills [0, 1) evenly (chi-square at far below the 0.1 %
    level for these degrees of freedom).  A scale of U * F would never select
    feature F."""
    D, F, P = 3, 6, 512
    SB = (1 << D) - 1
    a = np.concatenate([oracle.de_init(P, D, F, 77, prob)[:, :SB].ravel() for prob in range(4)])
    b = np.concatenate([oracle.de_init(P, D, F, 77, prob)[:, SB:].ravel() for prob in range(4)])
    assert a.size == 4 * P * SB >= 10_000
    assert (a >= 0).all() and (a < F + 1).all() and (b >= 0).all() and (b < 1).all()
    feat_hist = np.bincount(np.floor(a).astype(int), minlength=F + 1)
    assert len(feat_hist) == F + 1 and feat_hist.min() > 0
    assert _chi2(feat_hist) < 22.5           # 6 degrees of freedom, p = 0.001
    thr_hist = np.bincount(np.floor(b * 10).astype(int), minlength=10)
    assert _chi2(thr_hist) < 27.9            # 9 degrees of freedom, p = 0.001
    # the decoded features (eq. aenc) of one population follow the same law
    nu = np.full(F, 50, dtype=np.uint32)
    feat, _ = oracle.decode(oracle.de_init(P, D, F, 78, 0), D, F, nu)
    assert set(np.unique(feat)) == set(range(F + 1))


def test_random_mutation_factor_is_one_draw_per_individual():
    """With M < 0 the mutation factor is drawn from U[0, 1) (Section 3.3),
    once per individual and generation (reading R8): for CR = 1 every trial
    gene is the mutant v_q = s_best,q + M_r (s_r1,q - s_r2,q), so where no
    clamp bit, (v_q - s_best,q) / (s_r1,q - s_r2,q) is the same number for all
    genes q of an individual, lies in [0, 1), and is uniform over the
    individuals of a generation and across generations.  A draw per gene or
    per generation fails these checks."""
    D, F, P = 2, 4, 400
    m = 2 * ((1 << D) - 1)
    SB = m // 2
    hi = np.array([F + 1.0] * SB + [1.0] * SB)
    pop = oracle.de_init(P, D, F, 5, 0)
    best = 17
    Ms = []
    for g in range(1, 26):
        trial = oracle.de_trial(pop, D, F, -1.0, 1.0, 5, 0, g, best)
        gen = []
        for r in range(P):
            r1, r2, _ = oracle.de_pick(P, m, 5, 0, g, r)
            d = pop[r1] - pop[r2]
            ok = (trial[r] > 0) & (trial[r] < hi) & (np.abs(d) > 1e-3)
            if ok.sum() < 2:
                continue
            ratio = (trial[r][ok] - pop[best][ok]) / d[ok]
            assert ratio.max() - ratio.min() < 1e-9
            gen.append(ratio.mean())
        gen = np.array(gen)
        assert len(gen) > 300 and (gen > -1e-9).all() and (gen < 1.0).all()
        assert gen.std() > 0.2          # not one factor for the whole generation
        Ms.append(gen)
    Ms = np.concatenate(Ms)
    hist = np.bincount(np.clip(np.floor(Ms * 10), 0, 9).astype(int), minlength=10)
    assert _chi2(hist) < 27.9           # 9 degrees of freedom, p = 0.001
    # a fixed M >= 0 gives that factor exactly where no clamp bit
    trial = oracle.de_trial(pop, D, F, 0.5, 1.0, 5, 0, 3, best)
    r1, r2, _ = oracle.de_pick(P, m, 5, 0, 3, 0)
    d = pop[r1] - pop[r2]
    ok = (trial[0] > 0) & (trial[0] < hi) & (np.abs(d) > 1e-3)
    np.testing.assert_allclose((trial[0][ok] - pop[best][ok]) / d[ok], 0.5, rtol=0, atol=1e-9)


def test_trial_cr_zero_changes_only_q_rand():
    D, F, P = 3, 4, 12
    m = 2 * ((1 << D) - 1)
    pop = oracle.de_init(P, D, F, 1, 0)
    trial = oracle.de_trial(pop, D, F, 0.5, 0.0, 1, 0, 1, 2)
    for r in range(P):
        _, _, q = oracle.de_pick(P, m, 1, 0, 1, r)
        diff = np.nonzero(trial[r] != pop[r])[0]
        assert set(diff) <= {q}


def test_trial_m_zero_copies_best():
    D, F, P = 2, 4, 10
    pop = oracle.de_init(P, D, F, 9, 0)
    trial = oracle.de_trial(pop, D, F, 0.0, 1.0, 9, 0, 1, 3)
    np.testing.assert_array_equal(trial, np.repeat(pop[3:4], P, axis=0))


def test_trial_mutation_formula_and_clamp():
    D, F, P = 1, 3, 8
    m = 2
    rng = np.random.default_rng(0)
    pop = np.column_stack([rng.random(P) * 4, rng.random(P)])
    best = 5
    for M in (0.5, 1.7):
        trial = oracle.de_trial(pop, D, F, M, 1.0, 4, 0, 2, best)
        for r in range(P):
            r1, r2, _ = oracle.de_pick(P, m, 4, 0, 2, r)
            v = pop[best] + M * (pop[r1] - pop[r2])
            v = np.clip(v, 0.0, [F + 1.0, 1.0])
            np.testing.assert_array_equal(trial[r], v)


def test_selection_ties_go_to_trial():
    pop = np.zeros((3, 2))
    trial = np.ones((3, 2))
    cost = np.array([5.0, 5.0, 5.0])
    oracle.de_select(pop, cost, trial, np.array([4.0, 5.0, 6.0]))
    np.testing.assert_array_equal(pop, [[1, 1], [1, 1], [0, 0]])
    np.testing.assert_array_equal(cost, [4.0, 5.0, 5.0])
    assert oracle.argmin(np.array([3.0, 1.0, 1.0, 2.0])) == 1


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_deoct_plain_small_below_exhaustive_optimum(seed):
    # The small plain workload (n = 1000, F = 4, K = 2, depth 2, P = 32, 50
    # generations): DEOCT's training correct never exceeds the exact depth-2
    # optimum, and its best never gets worse across generations.
    w = synth.plain_small(seed)
    ds = oracle.dataset_from_X(w.X, w.y, w.K)
    prm = oracle.de_params(w.P, w.G, w.M, w.CR, 1000 + seed)
    res = oracle.deoct(ds, w.D, prm, with_trace=True)
    opt, _, _ = oracle.opt2(ds)
    assert res["correct"] <= opt
    assert (np.diff(res["trace"]) <= 0).all()
    assert res["cost"] == w.n - res["correct"] == res["trace"][-1]
    # the reported tree is the decoded best individual
    f, t = oracle.decode(res["genes"], w.D, w.F, ds.n_unique)
    np.testing.assert_array_equal(f[0], res["feat"])
    np.testing.assert_array_equal(t[0], res["tau"])


def _encode(feat, tau, n_unique):
    # inverse of the decoding: a^ = feat + 0.5, b^ = (tau + 0.5) / (n_f + 1)
    a = feat.astype(np.float64) + 0.5
    b = np.array([(t + 0.5) / (n_unique[f - 1] + 1) if f else 0.5 for f, t in zip(feat, tau)])
    return np.concatenate([a, b])


def test_warm_start_with_the_optimum_returns_it():
    w = synth.plain_small(2, n=300)
    ds = oracle.dataset_from_X(w.X, w.y, w.K)
    opt, f3, t3 = oracle.opt2(ds)
    genes = _encode(f3, t3, ds.n_unique)
    fd, td = oracle.decode(genes, 2, w.F, ds.n_unique)
    np.testing.assert_array_equal(fd[0], f3)
    np.testing.assert_array_equal(td[0], t3)
    prm = oracle.de_params(16, 10, 0.5, 0.9, 7)
    res = oracle.deoct(ds, 2, prm, warm=genes[None])
    assert res["correct"] == opt


def test_deoct_deterministic_and_problem_keyed():
    w = synth.plain_small(3, n=200)
    ds = oracle.dataset_from_X(w.X, w.y, w.K)
    prm = oracle.de_params(12, 8, -1.0, 0.5, 5)
    a = oracle.deoct(ds, 2, prm, prob=0, with_pop=True)
    b = oracle.deoct(ds, 2, prm, prob=0, with_pop=True)
    c = oracle.deoct(ds, 2, prm, prob=1, with_pop=True)
    np.testing.assert_array_equal(a["pop"], b["pop"])
    assert not np.array_equal(a["pop"], c["pop"])


@pytest.mark.parametrize("seed,D", [(1, 2), (2, 3), (3, 4), (4, 3)])
def test_mh_horizon1_is_the_greedy_tree(seed, D):
    X, y = synth.random_small(seed, 400, 4, 3, levels=12)
    ds = oracle.dataset_from_X(X, y, 3)
    prm = oracle.de_params(8, 3, 0.5, 0.9, seed)
    mh = oracle.mh_train(ds, D, 1, prm)
    gf, gt = oracle.greedy_tree(ds, D)
    np.testing.assert_array_equal(mh["feat"], gf)
    np.testing.assert_array_equal(mh["tau"], gt)
    _, correct, label, _ = oracle.fitness(ds, gf[None], gt[None], D)
    assert mh["correct"] == correct[0]
    np.testing.assert_array_equal(mh["label"], label[0])


def test_mh_root_comes_from_deoct_with_problem_id_one():
    w = synth.plain_small(4, n=300)
    ds = oracle.dataset_from_X(w.X, w.y, w.K)
    prm = oracle.de_params(16, 12, 0.5, 0.9, 77)
    mh = oracle.mh_train(ds, 2, 2, prm)
    de = oracle.deoct(ds, 2, prm, prob=1)
    assert (mh["feat"][0], mh["tau"][0]) == (de["feat"][0], de["tau"][0])
    # depth-1 children are exact splits of their subsets (horizon 2 -> 1)
    f0, t0 = mh["feat"][0], mh["tau"][0]
    left = np.nonzero((f0 != 0) & (ds.ranks[max(f0, 1) - 1] < t0))[0]
    right = np.setdiff1d(np.arange(300), left)
    for node, idx in ((1, left), (2, right)):
        if len(idx) > 1 and len(np.unique(w.y[idx])) > 1:
            f, t, _ = oracle.split1(ds, idx=idx)
            assert (mh["feat"][node], mh["tau"][node]) == (f, t)
        else:
            assert (mh["feat"][node], mh["tau"][node]) == (0, 0)


def test_mh_pure_node_gets_artificial_node():
    X = np.array([[0.1], [0.2], [0.3], [0.4]], dtype=np.float32)
    y = np.array([1, 1, 1, 1], dtype=np.uint8)
    ds = oracle.dataset_from_X(X, y, 2)
    mh = oracle.mh_train(ds, 3, 2, oracle.de_params(4, 2, 0.5, 0.9, 1))
    assert (mh["feat"] == 0).all() and mh["correct"] == 4
