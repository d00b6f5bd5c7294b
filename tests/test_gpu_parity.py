"""GPU parity: every step of the HIP path against the oracle, element by
element, on seeded inputs.  All results are integers or exactly rounded f64,
so the bar is bit-exact equality."""
import numpy as np
import pytest

import oracle
from gpu_helpers import dev, np_, random_trees, u32
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


def gpu_ds(mh, X, y, K):
    return mh.dataset(X, y, K)


# ---------------------------------------------------------------- rank encode
@pytest.mark.parametrize("seed,n,F,levels", [(1, 1, 1, None), (2, 63, 3, None), (3, 64, 2, 5),
                                             (4, 1000, 4, 17), (5, 4097, 7, None),
                                             (6, 100_000, 16, None), (7, 20_000, 33, 300)])
def test_rank_encode(mh, seed, n, F, levels):
    X, y = synth.random_small(seed, n, F, 3, levels)
    want_r, want_nu = oracle.rank_encode(X)
    ds = gpu_ds(mh, X, y, 3)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :n], want_r)


@pytest.mark.parametrize("coop,R", [("1", None), ("0", None), ("1", "256"), ("1", "8192")])
@pytest.mark.parametrize("seed,n,F,levels", [(8, 1, 3, None), (9, 257, 5, 4), (10, 20_000, 7, None),
                                             (11, 100_000, 16, 1000)])
def test_rank_encode_forms(mh, monkeypatch, coop, R, seed, n, F, levels):
    """The cooperative launch (several samples-per-block choices) and the
    separate launches give the oracle's ranks."""
    from paper_2311_06952_amd import capi
    monkeypatch.setenv("MHDEOCT_RANK_COOP", coop)
    if R:
        monkeypatch.setenv("MHDEOCT_RANK_R", R)
    ctx = capi.Context(0)
    X, y = synth.random_small(seed, n, F, 3, levels)
    want_r, want_nu = oracle.rank_encode(X)
    ds = mh.dataset(X, y, 3, ctx=ctx)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :n], want_r)
    Xn = X.copy()
    Xn[n // 2, F - 1] = np.nan
    with pytest.raises(mh.MhError):
        mh.dataset(Xn, y, 3, ctx=ctx)
    ctx.close()


@pytest.mark.parametrize("seed,n,F,levels", [(12, 64, 2, 3), (13, 65, 3, 2), (14, 1024, 2, 7),
                                             (15, 4096, 3, 1), (16, 8193, 4, 2), (17, 12_289, 2, 40)])
def test_rank_encode_separate_launch_boundaries(mh, monkeypatch, seed, n, F, levels):
    """The separate launches at sizes that end exactly on, or one past, a
    64-lane chunk, a wave's span (1,024) and a block (4,096), with runs of
    equal values that cross those boundaries (one to forty distinct values)."""
    from paper_2311_06952_amd import capi
    monkeypatch.setenv("MHDEOCT_RANK_COOP", "0")
    ctx = capi.Context(0)
    X, y = synth.random_small(seed, n, F, 3, levels)
    X = np.sort(X, axis=0)  # long sorted runs: equal values meet at the boundaries
    want_r, want_nu = oracle.rank_encode(X)
    ds = mh.dataset(X, y, 3, ctx=ctx)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :n], want_r)
    ctx.close()


@pytest.mark.parametrize("seed,n,F,levels", [(18, 600_001, 3, None), (19, 1_000_000, 2, 5000)])
def test_rank_encode_two_halves(mh, monkeypatch, seed, n, F, levels):
    """Rows of ranks of 2 to 8 MB: the separate launches write the ranks of
    the two halves of the sample ids in two passes of the rank scatter."""
    from paper_2311_06952_amd import capi
    monkeypatch.setenv("MHDEOCT_RANK_COOP", "0")
    ctx = capi.Context(0)
    X, y = synth.random_small(seed, n, F, 3, levels)
    want_r, want_nu = oracle.rank_encode(X)
    ds = mh.dataset(X, y, 3, ctx=ctx)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :n], want_r)
    ctx.close()


def test_rank_encode_signed_zero_and_nan(mh):
    X = np.array([[0.0, 1.0], [-0.0, 1.0], [-2.5, np.inf], [3.0, -np.inf]], dtype=np.float32)
    want_r, want_nu = oracle.rank_encode(X)
    ds = gpu_ds(mh, X, np.zeros(4, np.uint8), 2)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :4], want_r)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    Xn = X.copy()
    Xn[2, 1] = np.nan
    with pytest.raises(mh.MhError):
        gpu_ds(mh, Xn, np.zeros(4, np.uint8), 2)


# --------------------------------------------------------------------- decode
def test_decode_edges(mh):
    rng = np.random.default_rng(0)
    F, D = 5, 3
    SB = (1 << D) - 1
    nu = np.array([1, 2, 7, 255, 100_000], dtype=np.uint32)
    P = 400
    genes = np.column_stack([rng.random((P, SB)) * 7 - 0.5, rng.random((P, SB)) * 1.2 - 0.1])
    # interval ends, one ulp either side, range ends, NaN
    for r in range(0, P, 4):
        f = rng.integers(1, F + 1)
        k = rng.integers(0, nu[f - 1] + 1)
        b = k / (nu[f - 1] + 1.0)
        genes[r, 0] = f + 0.25
        genes[r, SB] = [b, np.nextafter(b, 0), np.nextafter(b, 2), 1.0][r % 4]
    genes[1, 1] = np.nan
    genes[2, SB + 1] = np.nan
    genes[3, 2] = F + 1.0
    genes[5, 3] = -0.0
    want_f, want_t = oracle.decode(genes, D, F, nu)
    gf, gt = mh.tree_decode(dev(genes), D, F, dev(nu))
    np.testing.assert_array_equal(np_(gf), want_f)
    np.testing.assert_array_equal(u32(gt), want_t)


# -------------------------------------------------------------------- fitness
FIT_CASES = [
    # seed, n, F, K, D, P, levels
    (1, 1, 2, 2, 1, 1, None),
    (2, 63, 3, 2, 2, 3, None),
    (3, 64, 3, 3, 3, 64, 4),
    (4, 127, 4, 5, 4, 65, None),
    (5, 5000, 6, 4, 5, 130, 50),
    (6, 3001, 8, 1, 3, 256, None),
    (7, 20_000, 16, 3, 3, 300, None),
    (8, 2000, 5, 3, 6, 20, 30),      # walk path
    (9, 1500, 4, 2, 8, 5, None),     # walk path
    (10, 700, 90, 3, 2, 40, None),   # F > 80: walk path
]


@pytest.mark.parametrize("seed,n,F,K,D,P,levels", FIT_CASES)
def test_fitness(mh, seed, n, F, K, D, P, levels):
    X, y = synth.random_small(seed, n, F, K, levels)
    ods = oracle.dataset_from_X(X, y, K)
    rng = np.random.default_rng(seed)
    feat, tau = random_trees(rng, P, D, F, ods.n_unique)
    want = oracle.fitness(ods, feat, tau, D)
    ds = gpu_ds(mh, X, y, K)
    got = mh.fitness_eval(ds, dev(feat), dev(tau), D)
    np.testing.assert_array_equal(u32(got[0]), want[0])
    np.testing.assert_array_equal(u32(got[1]), want[1])
    np.testing.assert_array_equal(np_(got[2]), want[2])
    np.testing.assert_array_equal(np_(got[3]), want[3])


# (seed, n, F, K, D, P, subset, huge_tau): the walk kernel's forms --
# staged tiles with several trees per block, ranks read from memory when the
# feature set is wide, histograms in memory when they do not fit in LDS,
# thresholds above every rank, subsets, fewer trees than the tile kernel
# takes, ragged tails
WALK_CASES = [
    (21, 5000, 16, 3, 8, 37, False, False),
    (22, 4099, 6, 4, 7, 100, True, True),
    (23, 3000, 60, 3, 6, 9, False, True),      # 60 features: ranks from memory
    (24, 2500, 5, 200, 10, 6, True, False),    # 2^10 leaves x 200 classes: counts in memory
    (25, 1, 3, 2, 9, 3, False, False),
    (26, 30_000, 12, 5, 4, 2, False, True),    # two trees: walk kernel at depth 4
    (27, 777, 100, 3, 3, 1, True, False),      # one tree, wide data
]


@pytest.mark.parametrize("seed,n,F,K,D,P,subset,huge", WALK_CASES)
def test_walk_kernel_forms(mh, seed, n, F, K, D, P, subset, huge):
    X, y = synth.random_small(seed, n, F, K, levels=None if seed % 2 else 50)
    ods = oracle.dataset_from_X(X, y, K)
    rng = np.random.default_rng(seed)
    feat, tau = random_trees(rng, P, D, F, ods.n_unique)
    if huge:  # thresholds past every rank send every sample left
        tau[rng.random(tau.shape) < 0.2] = 0xFFFFFFFF
    idx = np.sort(rng.choice(n, size=max(1, n // 3), replace=False)).astype(np.uint32) \
        if subset else None
    want = oracle.fitness(ods, feat, tau, D, idx=idx, n_min=2, alpha=1.5)
    ds = gpu_ds(mh, X, y, K)
    got = mh.fitness_eval(ds, dev(feat), dev(tau), D, idx=None if idx is None else dev(idx),
                          n_min=2, alpha=1.5)
    np.testing.assert_array_equal(u32(got[0]), want[0])
    np.testing.assert_array_equal(u32(got[1]), want[1])
    np.testing.assert_array_equal(np_(got[2]), want[2])
    np.testing.assert_array_equal(np_(got[3]), want[3])


@pytest.mark.parametrize("D", [2, 4, 6])
def test_fitness_subset_and_penalties(mh, D):
    X, y = synth.random_small(11, 3000, 5, 3, 40)
    ods = oracle.dataset_from_X(X, y, 3)
    rng = np.random.default_rng(D)
    feat, tau = random_trees(rng, 70, D, 5, ods.n_unique)
    idx = np.sort(rng.choice(3000, size=1234, replace=False)).astype(np.uint32)
    want = oracle.fitness(ods, feat, tau, D, idx=idx, n_min=7, alpha=0.375)
    ds = gpu_ds(mh, X, y, 3)
    got = mh.fitness_eval(ds, dev(feat), dev(tau), D, idx=dev(idx), n_min=7, alpha=0.375)
    np.testing.assert_array_equal(u32(got[0]), want[0])
    np.testing.assert_array_equal(np_(got[2]), want[2])
    np.testing.assert_array_equal(np_(got[3]), want[3])


def test_fitness_empty_subset(mh):
    X, y = synth.random_small(12, 100, 3, 2)
    ds = gpu_ds(mh, X, y, 2)
    feat = np.ones((4, 3), np.uint8)
    tau = np.ones((4, 3), np.uint32)
    idx = dev(np.zeros(0, np.uint32))
    got = mh.fitness_eval(ds, dev(feat), dev(tau), 2, idx=idx)
    assert u32(got[0]).sum() == 0 and (u32(got[1]) == 0).all()
    assert (np_(got[3]) == 0).all()


def test_tileset_reuse_matches(mh):
    X, y = synth.random_small(13, 9000, 6, 4, None)
    ods = oracle.dataset_from_X(X, y, 4)
    rng = np.random.default_rng(1)
    ds = gpu_ds(mh, X, y, 4)
    ts = mh.TileSet(ds)
    for D in (1, 3, 5):
        feat, tau = random_trees(rng, 100, D, 6, ods.n_unique)
        want = oracle.fitness(ods, feat, tau, D)
        import torch
        SL = 1 << D
        out = (torch.zeros((100, SL, 4), dtype=torch.int32, device="cuda"),
               torch.zeros(100, dtype=torch.int32, device="cuda"),
               torch.zeros((100, SL), dtype=torch.uint8, device="cuda"),
               torch.zeros(100, dtype=torch.float64, device="cuda"))
        for _ in range(2):  # the counters are re-zeroed by each call
            ts.fitness(dev(feat), dev(tau), D, out=out)
            np.testing.assert_array_equal(u32(out[0]), want[0])
            np.testing.assert_array_equal(np_(out[3]), want[3])


# ------------------------------------------------------------------------- DE
def test_de_init_and_steps(mh):
    P, D, F = 37, 3, 6
    SB = (1 << D) - 1
    rng = np.random.default_rng(4)
    warm = rng.random((3, 2 * SB))
    want = oracle.de_init(P, D, F, 99, 5, warm)
    got = mh.de_init(P, D, F, 99, 5, warm=dev(warm))
    np.testing.assert_array_equal(np_(got), want)
    prm = mh.de_params(P, 10, M=0.7, CR=0.3, seed=99)
    cost = rng.integers(0, 5, size=P).astype(np.float64)
    pop = want.copy()
    gpop, gcost = got, dev(cost)
    for g in range(1, 5):
        trial = oracle.de_trial(pop, D, F, 0.7, 0.3, 99, 5, g, oracle.argmin(cost))
        tcost = rng.integers(0, 5, size=P).astype(np.float64)
        # device: selection of the previous trial is done by the next step
        best, gtrial = mh.de_step(prm, D, F, 5, g, gpop, gcost)
        assert int(np_(best)[0]) == oracle.argmin(cost)
        np.testing.assert_array_equal(np_(gtrial), trial)
        oracle.de_select(pop, cost, trial, tcost)
        mh.de_step(prm, D, F, 5, g, gpop, gcost, trial=gtrial, trial_cost=dev(tcost),
                   make_trial=False)
        np.testing.assert_array_equal(np_(gpop), pop)
        np.testing.assert_array_equal(np_(gcost), cost)


def test_de_random_mutation_factor(mh):
    P, D, F = 50, 2, 4
    pop = oracle.de_init(P, D, F, 3, 0)
    want = oracle.de_trial(pop, D, F, -1.0, 0.5, 3, 0, 7, 11)
    cost = np.full(P, 9.0)
    cost[11] = 1.0
    prm = mh.de_params(P, 10, M=-1.0, CR=0.5, seed=3)
    _, gtrial = mh.de_step(prm, D, F, 0, 7, dev(pop), dev(cost))
    np.testing.assert_array_equal(np_(gtrial), want)


# -------------------------------------------------------------------- DEOCT
def _deoct_both(mh, w, seed, G=None, idx=None, P=None, prob=0, warm=None):
    G = w.G if G is None else G
    P = w.P if P is None else P
    ods = oracle.dataset_from_X(w.X, w.y, w.K)
    prm_o = oracle.de_params(P, G, w.M, w.CR, seed)
    want = oracle.deoct(ods, w.D, prm_o, idx=idx, warm=warm, prob=prob, with_pop=True)
    ds = gpu_ds(mh, w.X, w.y, w.K)
    prm = mh.de_params(P, G, w.M, w.CR, seed)
    got = mh.subtree_solve(ds, w.D, prm, idx=None if idx is None else dev(idx), warm=warm,
                           prob=prob, with_pop=True)
    return want, got, ods


def _same_tree(want, got):
    """The best tree, its labels, correct count and cost; and, when either
    side carries it, the whole final population (float64 genes, bit for bit)
    and every individual's cost."""
    np.testing.assert_array_equal(got["feat"], want["feat"])
    np.testing.assert_array_equal(got["tau"], want["tau"])
    np.testing.assert_array_equal(got["label"], want["label"])
    assert got["correct"] == want["correct"]
    assert got["cost"] == want["cost"]
    for key in ("pop", "pop_cost"):
        if key in got or key in want:
            a, b = np.asarray(got[key]), np.asarray(want[key])
            assert a.shape == b.shape
            np.testing.assert_array_equal(a.view(np.uint64), b.view(np.uint64))


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_subtree_solve_plain_small(mh, seed):
    """n = 1000, F = 4, K = 2, depth 2, P = 32, 50 generations (M = 0.5,
    CR = 0.9): identical to the oracle and never above the exact optimum."""
    w = synth.plain_small(seed)
    want, got, ods = _deoct_both(mh, w, 1000 + seed)
    _same_tree(want, got)
    assert got["correct"] <= oracle.opt2(ods)[0]


def test_async_rank_status(mh):
    """Rank encoding that does not wait: its status word, carried by the
    dataset, is read with subtree_solve's result (NaN -> MH_EINVAL) and
    before mh_train and mh_autotune start; valid data solve as usual."""
    import torch
    from paper_2311_06952_amd import capi
    w = synth.plain_small(7)
    Xd = torch.as_tensor(w.X).cuda()
    yd = torch.as_tensor(w.y).cuda()
    status = torch.full((1,), 77, dtype=torch.int32, device="cuda")
    prm = mh.de_params(w.P, w.G, w.M, w.CR, 1007)
    ranks, nu = mh.rank_encode(Xd, status=status)
    got = mh.subtree_solve(mh.Dataset(ranks, yd, nu, w.n, w.F, w.K, status), w.D, prm,
                           with_pop=True)
    assert int(status.item()) == 0
    want = oracle.deoct(oracle.dataset_from_X(w.X, w.y, w.K), w.D,
                        oracle.de_params(w.P, w.G, w.M, w.CR, 1007), with_pop=True)
    _same_tree(want, got)
    Xn = Xd.clone()
    Xn[w.n // 3, 1] = float("nan")
    ranks, nu = mh.rank_encode(Xn, status=status)
    bad = mh.Dataset(ranks, yd, nu, w.n, w.F, w.K, status)
    for call in (lambda: mh.subtree_solve(bad, w.D, prm, with_pop=True),
                 lambda: mh.mh_train(bad, 3, 2, prm),
                 lambda: mh.autotune(bad, w.D, prm, generations=2)):
        with pytest.raises(mh.MhError) as ei:
            call()
        assert ei.value.code == capi.MH_EINVAL
    assert int(status.item()) & 1 == 1


def test_subtree_solve_subset_warm_and_random_m(mh):
    w = synth.plain_small(6, n=2000)
    w.M = -1.0
    rng = np.random.default_rng(0)
    idx = np.sort(rng.choice(2000, 1500, replace=False)).astype(np.uint32)
    warm = rng.random((2, 6)) * [5, 5, 5, 1, 1, 1]
    want, got, _ = _deoct_both(mh, w, 77, G=20, idx=idx, warm=warm, prob=9)
    _same_tree(want, got)


def test_subtree_solve_plain_scale_full_n(mh):
    """n = 100,000, F = 16, K = 3, depth 3, P = 256 at full size, 5
    generations (the oracle's share of the run is a few seconds)."""
    w = synth.plain_scale(1)
    want, got, _ = _deoct_both(mh, w, 1001, G=5)
    _same_tree(want, got)


def test_plain_large_full_size(mh):
    """The large plain configuration at its full size (n = 10^6, F = 32, K = 4,
    depth 4, P = 512): ranks, the fitness of 16 random trees, and a DEOCT run
    cut to G = 1 (the oracle's full run would take hours), all equal to the
    oracle's."""
    w = synth.plain_large(1)
    ods = oracle.dataset_from_X(w.X, w.y, w.K)
    ds = gpu_ds(mh, w.X, w.y, w.K)
    np.testing.assert_array_equal(u32(ds.n_unique), ods.n_unique)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :w.n], ods.ranks)
    rng = np.random.default_rng(5)
    feat, tau = random_trees(rng, 16, w.D, w.F, ods.n_unique)
    want = oracle.fitness(ods, feat, tau, w.D)
    got = mh.fitness_eval(ds, dev(feat), dev(tau), w.D)
    for i in range(4):
        np.testing.assert_array_equal(np_(got[i]) if i >= 2 else u32(got[i]), want[i])
    prm = (w.P, 1, w.M, w.CR, 77)
    got = mh.subtree_solve(ds, w.D, mh.de_params(*prm), with_pop=True)
    _same_tree(oracle.deoct(ods, w.D, oracle.de_params(*prm), with_pop=True), got)


@pytest.mark.parametrize("mode,n,P,G", [("normal", 2000, 100, 600), ("long", 400, 200, 4000)])
def test_paper_parameter_modes(mh, mode, n, P, G):
    """DEOCT with the paper's parameter modes (Section 4: Normal P = 100,
    G = 600; Long P = 200, G = 4000; CR = 0.1 and a mutation factor drawn per
    individual and generation): equal to the oracle's run."""
    X, y = synth.random_small(300 + P, n, 6, 3)
    prm = (P, G, -1.0, 0.1, 4242)
    got = mh.subtree_solve(gpu_ds(mh, X, y, 3), 3, mh.de_params(*prm), with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, 3), 3, oracle.de_params(*prm), with_pop=True)
    _same_tree(want, got)


def test_tile_sort_wide_keys(mh):
    """Over 2^26 samples with ranks past 2^26: the tile sort's composite
    (rank << 6 | position) keys are 64 bits wide.  The values are positive
    finite float32 bit patterns drawn uniformly, so nearly all are distinct.
    DEOCT equals the oracle's run."""
    n = (1 << 26) + (1 << 22)
    rng = np.random.default_rng(2626)
    bits = rng.integers(1, 0x7F000000, size=n, dtype=np.uint32)
    X = bits.view(np.float32).reshape(n, 1)
    y = ((bits > 0x3F800000) ^ (rng.random(n) < 0.25)).astype(np.uint8)
    ods = oracle.dataset_from_X(X, y, 2)
    assert int(ods.n_unique[0]) > (1 << 26)
    prm = (8, 2, 0.5, 0.9, 77)
    got = mh.subtree_solve(gpu_ds(mh, X, y, 2), 2, mh.de_params(*prm), with_pop=True)
    want = oracle.deoct(ods, 2, oracle.de_params(*prm), with_pop=True)
    _same_tree(want, got)


def test_subtree_solve_depth6_walk_path(mh):
    w = synth.plain_small(7, n=1500)
    w.D = 6
    want, got, _ = _deoct_both(mh, w, 5, G=6, P=12)
    _same_tree(want, got)


@pytest.mark.parametrize("D,n,P,G,M", [(8, 5000, 32, 10, 0.5), (8, 3001, 100, 6, -1.0),
                                       (10, 2000, 16, 4, 0.5)])
def test_whole_tree_deep_deoct(mh, D, n, P, G, M):
    """Whole-tree DEOCT at depth 8 (510 genes) and 10 (2046 genes), the deep
    setting DEOCT alone is compared in (Section 4), equal to the oracle's."""
    X, y = synth.random_small(900 + D, n, 9, 4, levels=60)
    prm = (P, G, M, 0.9, 31 + D)
    got = mh.subtree_solve(gpu_ds(mh, X, y, 4), D, mh.de_params(*prm), with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, 4), D, oracle.de_params(*prm), with_pop=True)
    _same_tree(want, got)


def test_fused_and_separate_de_step_agree(mh, monkeypatch):
    """The fused launch (DE step run by the block that completes the counts)
    and the separate DE-step launch give the same DEOCT run."""
    from paper_2311_06952_amd import capi
    w = synth.plain_small(8, n=5000)
    monkeypatch.setenv("MHDEOCT_FUSE_DE", "0")
    ctx_sep = capi.Context(0)
    monkeypatch.delenv("MHDEOCT_FUSE_DE")
    ctx_fus = capi.Context(0)
    out = []
    for ctx in (ctx_sep, ctx_fus):
        ds = mh.dataset(w.X, w.y, w.K, ctx=ctx)
        out.append(mh.subtree_solve(ds, w.D, mh.de_params(100, 30, 0.5, 0.9, 3), ctx=ctx,
                                    with_pop=True))
    _same_tree(out[0], out[1])
    ctx_sep.close()
    ctx_fus.close()


@pytest.mark.parametrize("D,P,K,M", [(1, 12, 2, 0.5), (2, 64, 5, -1.0), (3, 300, 3, 0.5),
                                     (4, 128, 7, 0.5), (5, 40, 4, 0.5)])
def test_persistent_and_per_generation_deoct_agree(mh, monkeypatch, D, P, K, M):
    """The whole-run cooperative kernel and the per-generation kernels give the
    same DEOCT run (and the oracle's)."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(40 + D, 6000, 9, K)
    monkeypatch.setenv("MHDEOCT_PERSIST", "0")
    ctx_gen = capi.Context(0)
    monkeypatch.setenv("MHDEOCT_PERSIST", "1")
    ctx_per = capi.Context(0)
    out = []
    for ctx in (ctx_gen, ctx_per):
        ds = mh.dataset(X, y, K, ctx=ctx)
        out.append(mh.subtree_solve(ds, D, mh.de_params(P, 12, M, 0.9, 5 + D), prob=3, ctx=ctx,
                                    with_pop=True))
    _same_tree(out[0], out[1])
    want = oracle.deoct(oracle.dataset_from_X(X, y, K), D, oracle.de_params(P, 12, M, 0.9, 5 + D),
                        prob=3, with_pop=True)
    _same_tree(want, out[1])
    ctx_gen.close()
    ctx_per.close()


@pytest.mark.parametrize("D,P,K,n_min,alpha", [(2, 64, 3, 40, 150.0), (3, 128, 4, 25, 33.5),
                                             (4, 96, 2, 200, 0.25), (3, 64, 5, 1, 1e9)])
def test_penalised_objective_deoct(mh, monkeypatch, D, P, K, n_min, alpha):
    """DEOCT under the penalised objective (Section 3: a per-split cost alpha
    and leaves below n_min samples treated as infeasible), whole-run kernel and
    per-generation kernels against the oracle. With n_min = 1 the cost is the
    misclassified count plus alpha per split node."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(70 + D, 5000, 8, K)
    out = []
    for persist in ("0", "1"):
        monkeypatch.setenv("MHDEOCT_PERSIST", persist)
        ctx = capi.Context(0)
        ds = mh.dataset(X, y, K, ctx=ctx)
        out.append(mh.subtree_solve(ds, D, mh.de_params(P, 15, 0.5, 0.9, 9 + D, n_min, alpha),
                                    ctx=ctx, with_pop=True))
        ctx.close()
    want = oracle.deoct(oracle.dataset_from_X(X, y, K), D,
                        oracle.de_params(P, 15, 0.5, 0.9, 9 + D, n_min, alpha), with_pop=True)
    _same_tree(want, out[0])
    _same_tree(want, out[1])
    if n_min == 1:
        nsplit = int(np.count_nonzero(np.asarray(want["feat"])))
        assert want["cost"] == (len(y) - want["correct"]) + alpha * nsplit


_GROUP_SHAPES = [(1, 12, 2, 3000, 5), (3, 256, 3, 20000, 16), (3, 100, 6, 7000, 9),
                 (4, 128, 3, 9000, 12), (5, 64, 2, 5000, 7), (2, 256, 40, 12000, 8),
                 (2, 40, 3, 6000, 40)]
_group_want = {}


@pytest.mark.parametrize("halves", ["1", "2", "4"])
@pytest.mark.parametrize("resident", ["0", "1"])
@pytest.mark.parametrize("D,P,K,n,F", _GROUP_SHAPES)
def test_persistent_wave_groups_agree(mh, monkeypatch, halves, resident, D, P, K, n, F):
    """One, two or four tile streams (wave groups) per block, tiles resident
    in LDS or staged each generation (whole records below 16 features, the
    compact form with the masks rebuilt in LDS from 16 on; at F = 40 and one
    wave per group part of a tile is staged without prefetch): the whole-run
    kernel gives the oracle's DEOCT run (the groups only change the order in
    which counts are added)."""
    from paper_2311_06952_amd import capi
    key = (D, P, K, n, F)
    X, y = synth.random_small(110 + D + K, n, F, K)
    prm = (P, 5, 0.5, 0.9, 17 + D)
    if key not in _group_want:
        _group_want[key] = oracle.deoct(oracle.dataset_from_X(X, y, K), D,
                                        oracle.de_params(*prm), prob=4, with_pop=True)
    monkeypatch.setenv("MHDEOCT_PERSIST", "1")
    monkeypatch.setenv("MHDEOCT_PERSIST_HALVES", halves)
    monkeypatch.setenv("MHDEOCT_PERSIST_RESIDENT", resident)
    ctx = capi.Context(0)
    ds = mh.dataset(X, y, K, ctx=ctx)
    got = mh.subtree_solve(ds, D, mh.de_params(*prm), prob=4, ctx=ctx, with_pop=True)
    _same_tree(_group_want[key], got)
    ctx.close()


@pytest.mark.parametrize("D,P,K,n", [(1, 3, 2, 1), (2, 3, 20, 500), (3, 65, 9, 0), (2, 200, 3, 64),
                                     (4, 256, 2, 6300), (3, 129, 255, 3000)])
def test_persistent_deoct_edge_shapes(mh, D, P, K, n):
    """Smallest population, many classes, empty and single-sample data, ragged
    populations: the whole-run kernel agrees with the oracle."""
    X, y = synth.random_small(70 + D + n, n, 5, K)
    ds = mh.dataset(X, y, K)
    got = mh.subtree_solve(ds, D, mh.de_params(P, 7, 0.5, 0.9, 11), prob=1, with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, K), D, oracle.de_params(P, 7, 0.5, 0.9, 11),
                        prob=1, with_pop=True)
    _same_tree(want, got)


@pytest.mark.parametrize("D,P,F,K", [(4, 512, 32, 4), (4, 128, 4, 6), (5, 200, 30, 3)])
def test_persistent_large_lds_shapes(mh, monkeypatch, D, P, F, K):
    """Populations whose DE rows need more than 64 KiB of LDS, and narrow
    data whose tile buffer is smaller than the node exchange: whole-run kernel
    (where the device allows it) and per-generation kernels agree with the
    oracle."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(90 + D + F, 4000, F, K)
    want = oracle.deoct(oracle.dataset_from_X(X, y, K), D, oracle.de_params(P, 6, 0.5, 0.9, 13),
                        prob=2, with_pop=True)
    for persist in ("1", "0"):
        monkeypatch.setenv("MHDEOCT_PERSIST", persist)
        ctx = capi.Context(0)
        ds = mh.dataset(X, y, K, ctx=ctx)
        got = mh.subtree_solve(ds, D, mh.de_params(P, 6, 0.5, 0.9, 13), prob=2, ctx=ctx,
                               with_pop=True)
        _same_tree(want, got)
        ctx.close()


def test_barrier_give_up_recovery(mh, monkeypatch):
    """A cooperative grid whose barrier gives up (forced from the host with a
    zero time limit, so that waits end at once) is recorded, and the work is
    redone with another launch form: the rank encoding and the DEOCT run still
    give the oracle's results."""
    from paper_2311_06952_amd import capi
    monkeypatch.setenv("MHDEOCT_WAIT_TICKS", "0")
    ctx = capi.Context(0)
    X, y = synth.random_small(123, 20000, 8, 3)
    ds = mh.dataset(X, y, 3, ctx=ctx)
    want_r, want_nu = oracle.rank_encode(X)
    np.testing.assert_array_equal(u32(ds.n_unique), want_nu)
    np.testing.assert_array_equal(u32(ds.ranks)[:, :20000], want_r)
    got = mh.subtree_solve(ds, 3, mh.de_params(64, 6, 0.5, 0.9, 9), ctx=ctx, with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, 3), 3, oracle.de_params(64, 6, 0.5, 0.9, 9),
                        with_pop=True)
    _same_tree(want, got)
    ctx.close()


def test_autotune_keeps_results(mh):
    """The autotuner picks a launch configuration for the shape; runs with it
    still equal the oracle."""
    from paper_2311_06952_amd import capi
    w = synth.plain_small(3, n=30000)
    ctx = capi.Context(0)
    ds = mh.dataset(w.X, w.y, w.K, ctx=ctx)
    prm = mh.de_params(64, 15, 0.5, 0.9, 21)
    tuned = mh.autotune(ds, w.D, prm, generations=5, ctx=ctx)
    assert tuned["persist"] in (0, 1) and tuned["halves"] in (1, 2, 4)
    assert len(tuned["ms"]) == 12 and all(t > 0 for t in tuned["ms"])
    got = mh.subtree_solve(ds, w.D, prm, ctx=ctx, with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(w.X, w.y, w.K), w.D,
                        oracle.de_params(64, 15, 0.5, 0.9, 21), with_pop=True)
    _same_tree(want, got)
    ctx.close()



@pytest.mark.parametrize("D,P,K,M,n_min,alpha", [(1, 256, 2, 0.5, 1, 0.0), (3, 300, 3, -1.0, 1, 0.0),
                                                 (4, 512, 4, 0.5, 20, 7.5), (5, 1024, 3, 0.5, 1, 0.0),
                                                 (2, 257, 6, -1.0, 3, 0.0)])
def test_large_population_generation_split(mh, monkeypatch, D, P, K, M, n_min, alpha):
    """From P = 256 on, a generation's DE work on the per-generation path runs
    as a selection launch and a mutation launch spread over the chip; the run
    (final population included) equals the oracle's."""
    from paper_2311_06952_amd import capi
    X, y = synth.random_small(500 + D + P, 7000, 7, K)
    monkeypatch.setenv("MHDEOCT_PERSIST", "0")
    ctx = capi.Context(0)
    ds = mh.dataset(X, y, K, ctx=ctx)
    prm = (P, 6, M, 0.9, 41 + D, n_min, alpha)
    got = mh.subtree_solve(ds, D, mh.de_params(*prm), prob=5, ctx=ctx, with_pop=True)
    want = oracle.deoct(oracle.dataset_from_X(X, y, K), D, oracle.de_params(*prm), prob=5,
                        with_pop=True)
    _same_tree(want, got)
    ctx.close()
