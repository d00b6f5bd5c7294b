"""fitness_eval_static, the fitness entry point that allocates nothing (its
scratch is a static device array): through the C ABI its outputs equal
fitness_eval's on the same inputs, element by element, on two calls in a
row whose second input is smaller than the first (the array keeps the
first call's contents), on the tile path and on the walk path; an input
whose scratch would exceed the array is refused with MH_EINVAL."""
import ctypes as C

import numpy as np
import pytest

import oracle
from gpu_helpers import dev, np_, random_trees, u32
from paper_2311_06952_amd import capi, synth

pytestmark = pytest.mark.gpu


def _both(mh, ctx, ds, feat, tau, D, idx=None, n_min=1, alpha=0.0):
    a = mh.fitness_eval(ds, dev(feat), dev(tau), D, idx=idx, n_min=n_min, alpha=alpha, ctx=ctx)
    b = mh.fitness_eval(ds, dev(feat), dev(tau), D, idx=idx, n_min=n_min, alpha=alpha, ctx=ctx,
                        static=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np_(x), np_(y))
    return b


# (seed, n, F, K, D, P): tile path (depth <= 5) and walk path (depth 8)
@pytest.mark.parametrize("first,second", [
    ((1, 40_000, 12, 4, 4, 256), (2, 3_001, 5, 3, 3, 64)),
    ((3, 30_000, 9, 3, 8, 40), (4, 2_500, 6, 5, 6, 17)),
])
def test_static_equals_fitness_eval_twice(first, second):
    import paper_2311_06952_amd as mh
    ctx = capi.Context(0)
    for seed, n, F, K, D, P in (first, second):
        X, y = synth.random_small(seed, n, F, K, levels=None if seed % 2 else 40)
        ds = mh.dataset(X, y, K, ctx=ctx)
        rng = np.random.default_rng(seed)
        nu = u32(ds.n_unique)
        feat, tau = random_trees(rng, P, D, F, nu)
        got = _both(mh, ctx, ds, feat, tau, D, n_min=3, alpha=0.5)
        # and against the oracle, on a sample of the trees
        ods = oracle.Dataset(u32(ds.ranks)[:, :n], nu, y, K)
        pick = np.arange(0, P, max(1, P // 5))
        want = oracle.fitness(ods, feat[pick], tau[pick], D, n_min=3, alpha=0.5)
        np.testing.assert_array_equal(u32(got[0])[pick], want[0])
        np.testing.assert_array_equal(np_(got[3])[pick], want[3])
        # a subset through idx (ragged)
        idx = np.sort(rng.choice(n, n // 3 + 7, replace=False)).astype(np.uint32)
        _both(mh, ctx, ds, feat, tau, D, idx=dev(idx))
    ctx.close()


def test_static_refuses_what_does_not_fit():
    import torch
    import paper_2311_06952_amd as mh
    ctx = capi.Context(0)
    # the walk path's counts alone: 1024 trees x 2^10 leaves x 255 classes x 4 B = 1 GiB
    X, y = synth.random_small(9, 1000, 4, 255)
    ds = mh.dataset(X, y, 255, ctx=ctx)
    P, D = 1024, 10
    feat = torch.zeros((P, (1 << D) - 1), dtype=torch.uint8, device="cuda")
    tau = torch.zeros((P, (1 << D) - 1), dtype=torch.int32, device="cuda")
    cost = torch.zeros(P, dtype=torch.float64, device="cuda")
    dsc = ds.cstruct()
    rc = ctx.lib.fitness_eval_static(ctx.h, C.byref(dsc), None, 1000, C.c_void_p(feat.data_ptr()),
                                     C.c_void_p(tau.data_ptr()), P, D, 1, 0.0, None, None, None,
                                     C.c_void_p(cost.data_ptr()))
    assert rc == capi.MH_EINVAL
    assert "static" in ctx.lib.mh_last_error(ctx.h).decode()
    # a call that fits still works after the refusal
    rng = np.random.default_rng(1)
    f2, t2 = random_trees(rng, 32, 3, 4, u32(ds.n_unique))
    _both(mh, ctx, ds, f2, t2, 3)
    ctx.close()
