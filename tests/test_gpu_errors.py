"""Invalid arguments at every entry point of the C ABI (include/mhdeoct.h):
each call returns its documented error code, leaves a message in
mh_last_error, queues nothing that could fail later, and leaves the context
usable (a valid call on it afterwards still gives the oracle's result)."""
import ctypes as C

import numpy as np
import pytest

import oracle
from gpu_helpers import dev, np_, u32
from paper_2311_06952_amd import capi, synth

pytestmark = pytest.mark.gpu

EINVAL, ENOMEM, EBUSY = capi.MH_EINVAL, capi.MH_ENOMEM, capi.MH_EBUSY


@pytest.fixture(scope="module")
def env():
    import torch
    import paper_2311_06952_amd as mh
    ctx = capi.Context(0)
    X, y = synth.random_small(5, 700, 4, 3, levels=20)
    ds = mh.dataset(X, y, 3, ctx=ctx)
    yield dict(mh=mh, torch=torch, ctx=ctx, lib=ctx.lib, X=X, y=y, ds=ds,
               Xd=torch.as_tensor(X).cuda(), yd=torch.as_tensor(y).cuda())
    ctx.close()


def _ds(ds, **kw):
    d = ds.cstruct()
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def _prm(P=16, G=3, M=0.5, CR=0.9, n_min=1, alpha=0.0):
    return capi.DEParamsC(P, G, M, CR, 7, n_min, alpha)


def _p(t):
    return C.c_void_p(t.data_ptr())


def _expect(env, rc, code=EINVAL):
    assert rc == code
    assert env["lib"].mh_last_error(env["ctx"].h).decode()


def _still_usable(env):
    """A valid DEOCT run on the same context equals the oracle's."""
    mh = env["mh"]
    got = mh.subtree_solve(env["ds"], 2, mh.de_params(16, 4, 0.5, 0.9, 3), ctx=env["ctx"])
    want = oracle.deoct(oracle.dataset_from_X(env["X"], env["y"], 3), 2,
                        oracle.de_params(16, 4, 0.5, 0.9, 3))
    np.testing.assert_array_equal(got["feat"], want["feat"])
    np.testing.assert_array_equal(got["tau"], want["tau"])
    assert got["correct"] == want["correct"]


def test_context_calls(env):
    lib = env["lib"]
    h = C.c_void_p()
    assert lib.mh_ctx_create(-1, None, C.byref(h)) != 0
    assert lib.mh_last_error(None).decode()
    assert lib.mh_ctx_create(0, None, None) == EINVAL
    assert lib.mh_ctx_profile(None, 1) == EINVAL
    assert lib.mh_ctx_stats(None, None, None, None, None, 0) == EINVAL
    assert lib.mh_version().decode()
    lib.mh_ctx_destroy(None)  # a null handle is ignored


def test_rank_encode_decode_encode(env):
    lib, ctx, torch = env["lib"], env["ctx"].h, env["torch"]
    X = env["Xd"]
    ranks = torch.empty((4, 768), dtype=torch.int32, device="cuda")
    nu = torch.empty(4, dtype=torch.int32, device="cuda")
    _expect(env, lib.mh_rank_encode(ctx, _p(X), 700, 0, 768, _p(ranks), _p(nu), None))
    _expect(env, lib.mh_rank_encode(ctx, _p(X), 700, 256, 768, _p(ranks), _p(nu), None))
    _expect(env, lib.mh_rank_encode(ctx, _p(X), 700, 4, 699, _p(ranks), _p(nu), None))
    _expect(env, lib.mh_rank_encode(ctx, None, 700, 4, 768, _p(ranks), _p(nu), None))
    _expect(env, lib.mh_rank_encode(ctx, _p(X), 700, 4, 768, _p(ranks), None, None))
    genes = torch.zeros((8, 6), dtype=torch.float64, device="cuda")
    feat = torch.zeros((8, 3), dtype=torch.uint8, device="cuda")
    tau = torch.zeros((8, 3), dtype=torch.int32, device="cuda")
    nu0 = env["ds"].n_unique
    for D, F in ((0, 4), (11, 4), (2, 0), (2, 256)):
        _expect(env, lib.tree_decode(ctx, _p(genes), 8, D, F, _p(nu0), _p(feat), _p(tau)))
        _expect(env, lib.tree_encode(ctx, _p(feat), _p(tau), 8, D, F, _p(nu0), _p(genes)))
    _expect(env, lib.tree_decode(ctx, None, 8, 2, 4, _p(nu0), _p(feat), _p(tau)))
    _expect(env, lib.tree_encode(ctx, _p(feat), _p(tau), 8, 2, 4, _p(nu0), None))
    _still_usable(env)


def test_fitness_and_tiles(env):
    lib, ctx, torch = env["lib"], env["ctx"].h, env["torch"]
    ds = env["ds"]
    feat = torch.zeros((4, 3), dtype=torch.uint8, device="cuda")
    tau = torch.zeros((4, 3), dtype=torch.int32, device="cuda")
    cost = torch.zeros(4, dtype=torch.float64, device="cuda")

    def fe(d, P=4, D=2, n_sub=700, n_min=1, alpha=0.0, f=feat, c=cost):
        return lib.fitness_eval(ctx, C.byref(d), None, n_sub, _p(f) if f is not None else None,
                                _p(tau), P, D, n_min, alpha, None, None, None,
                                _p(c) if c is not None else None)
    good = ds.cstruct()
    _expect(env, lib.fitness_eval(ctx, None, None, 700, _p(feat), _p(tau), 4, 2, 1, 0.0, None,
                                  None, None, _p(cost)))
    for bad in (dict(F=0), dict(F=256), dict(K=0), dict(K=256), dict(ld=699), dict(ranks=None),
                dict(labels=None), dict(n_unique=None)):
        _expect(env, fe(_ds(ds, **bad)))
    for kw in (dict(P=0), dict(P=1025), dict(D=0), dict(D=11), dict(n_sub=701), dict(n_min=0),
               dict(alpha=-1.0), dict(alpha=float("nan")), dict(f=None), dict(c=None)):
        _expect(env, fe(good, **kw))
    nb = C.c_size_t()
    assert lib.mh_tileset_bytes(700, 0, 3, C.byref(nb)) == EINVAL
    assert lib.mh_tileset_bytes(700, 4, 0, C.byref(nb)) == EINVAL
    assert lib.mh_tileset_bytes(700, 4, 3, None) == EINVAL
    assert lib.mh_tileset_bytes(700, 4, 3, C.byref(nb)) == 0
    buf = torch.empty(nb.value + 512, dtype=torch.uint8, device="cuda")
    off = (-buf.data_ptr()) % 256
    base = C.c_void_p(buf.data_ptr() + off)
    _expect(env, lib.mh_tileset_build(ctx, C.byref(good), None, 700, base, nb.value - 1))
    _expect(env, lib.mh_tileset_build(ctx, C.byref(good), None, 700,
                                      C.c_void_p(buf.data_ptr() + off + 16), nb.value))
    _expect(env, lib.mh_tileset_build(ctx, C.byref(good), None, 700, None, nb.value))
    _expect(env, lib.mh_tileset_build(ctx, C.byref(good), None, 701, base, nb.value))
    # a buffer that holds no tile set
    buf.zero_()
    _expect(env, lib.fitness_eval_tiles(ctx, base, _p(ds.n_unique), _p(feat), _p(tau), 4, 2, 1,
                                        0.0, None, None, None, _p(cost)))
    _expect(env, lib.fitness_eval_tiles(ctx, None, _p(ds.n_unique), _p(feat), _p(tau), 4, 2, 1,
                                        0.0, None, None, None, _p(cost)))
    # a real tile set, asked for a depth the tile kernel does not have
    assert lib.mh_tileset_build(ctx, C.byref(good), None, 700, base, nb.value) == 0
    f6 = torch.zeros((4, 63), dtype=torch.uint8, device="cuda")
    t6 = torch.zeros((4, 63), dtype=torch.int32, device="cuda")
    _expect(env, lib.fitness_eval_tiles(ctx, base, _p(ds.n_unique), _p(f6), _p(t6), 4, 6, 1, 0.0,
                                        None, None, None, _p(cost)))
    _still_usable(env)


def test_de_calls(env):
    lib, ctx, torch = env["lib"], env["ctx"].h, env["torch"]
    pop = torch.zeros((16, 6), dtype=torch.float64, device="cuda")
    cost = torch.zeros(16, dtype=torch.float64, device="cuda")
    best = torch.zeros(1, dtype=torch.int32, device="cuda")
    _expect(env, lib.de_init(ctx, 16, 0, 4, 1, 0, None, 0, _p(pop)))
    _expect(env, lib.de_init(ctx, 16, 2, 4, 1, 0, None, 17, _p(pop)))
    _expect(env, lib.de_init(ctx, 16, 2, 4, 1, 0, None, 2, _p(pop)))
    _expect(env, lib.de_init(ctx, 1025, 2, 4, 1, 0, None, 0, _p(pop)))
    _expect(env, lib.de_init(ctx, 16, 2, 4, 1, 0, None, 0, None))
    for prm in (_prm(P=2), _prm(P=1025), _prm(CR=1.5), _prm(CR=float("nan")),
                _prm(M=float("nan")), _prm(G=1 << 24), _prm(alpha=-2.0), _prm(n_min=0)):
        _expect(env, lib.de_step(ctx, C.byref(prm), 2, 4, 0, 1, _p(pop), _p(cost), None, None,
                                 _p(best), None))
    prm = _prm()
    _expect(env, lib.de_step(ctx, None, 2, 4, 0, 1, _p(pop), _p(cost), None, None, _p(best), None))
    _expect(env, lib.de_step(ctx, C.byref(prm), 2, 4, 0, 1, None, _p(cost), None, None, _p(best),
                             None))
    _expect(env, lib.de_step(ctx, C.byref(prm), 2, 4, 0, 1, _p(pop), _p(cost), _p(pop), None,
                             _p(best), None))
    _expect(env, lib.de_step(ctx, C.byref(prm), 2, 4, 0, 1 << 24, _p(pop), _p(cost), None, None,
                             _p(best), None))
    _still_usable(env)


def test_solve_train_split(env):
    lib, ctx = env["lib"], env["ctx"].h
    ds = env["ds"]
    good = ds.cstruct()
    out = capi.TreeC()
    tune = capi.TuneC()
    prm = _prm()
    for p in (_prm(P=2), _prm(CR=-0.1)):
        _expect(env, lib.subtree_solve(ctx, C.byref(good), None, 700, 2, C.byref(p), None, 0, 0,
                                       C.byref(out)))
    for D in (0, 11):
        _expect(env, lib.subtree_solve(ctx, C.byref(good), None, 700, D, C.byref(prm), None, 0, 0,
                                       C.byref(out)))
    _expect(env, lib.subtree_solve(ctx, C.byref(good), None, 701, 2, C.byref(prm), None, 0, 0,
                                   C.byref(out)))
    _expect(env, lib.subtree_solve(ctx, C.byref(good), None, 700, 2, C.byref(prm), None, 0, 0,
                                   None))
    _expect(env, lib.subtree_solve(ctx, C.byref(good), None, 700, 2, C.byref(prm), None, 2, 0,
                                   C.byref(out)))
    _expect(env, lib.subtree_solve(ctx, C.byref(_ds(ds, K=0)), None, 700, 2, C.byref(prm), None,
                                   0, 0, C.byref(out)))
    _expect(env, lib.subtree_solve_pop(ctx, C.byref(good), None, 700, 2, C.byref(_prm(P=2)),
                                       None, 0, 0, C.byref(out), None, None))
    _expect(env, lib.mh_autotune(ctx, C.byref(good), 2, C.byref(prm), 0, C.byref(tune)))
    _expect(env, lib.mh_autotune(ctx, C.byref(good), 2, C.byref(prm), 5, None))
    _expect(env, lib.mh_train(ctx, C.byref(good), 3, 0, C.byref(prm), 0, C.byref(out)))
    _expect(env, lib.mh_train(ctx, C.byref(good), 0, 2, C.byref(prm), 0, C.byref(out)))
    _expect(env, lib.mh_train(ctx, C.byref(good), 3, 2, C.byref(prm), 0x80, C.byref(out)))
    _expect(env, lib.mh_train(ctx, C.byref(good), 3, 2, C.byref(prm), 0, None))
    f, t, c = C.c_uint8(), C.c_uint32(), C.c_uint32()
    _expect(env, lib.split1(ctx, C.byref(good), None, 701, C.byref(f), C.byref(t), C.byref(c)))
    _expect(env, lib.split1(ctx, C.byref(good), None, 700, None, C.byref(t), C.byref(c)))
    _still_usable(env)


def test_thresholds_and_predict(env):
    lib, ctx, torch = env["lib"], env["ctx"].h, env["torch"]
    ds = env["ds"]
    good = ds.cstruct()
    feat = torch.zeros(3, dtype=torch.uint8, device="cuda")
    tau = torch.zeros(3, dtype=torch.int32, device="cuda")
    thr = torch.zeros(3, dtype=torch.float64, device="cuda")
    lab = torch.zeros(4, dtype=torch.uint8, device="cuda")
    X = env["Xd"]
    _expect(env, lib.mh_tree_thresholds(ctx, None, _p(X), _p(feat), _p(tau), 2, _p(thr)))
    _expect(env, lib.mh_tree_thresholds(ctx, C.byref(good), _p(X), _p(feat), _p(tau), 0, _p(thr)))
    _expect(env, lib.mh_tree_thresholds(ctx, C.byref(good), None, _p(feat), _p(tau), 2, _p(thr)))
    _expect(env, lib.mh_tree_thresholds(ctx, C.byref(good), _p(X), _p(feat), _p(tau), 2, None))
    corr = torch.zeros(1, dtype=torch.int32, device="cuda")
    pred = torch.zeros(700, dtype=torch.uint8, device="cuda")
    _expect(env, lib.mh_predict(ctx, _p(X), 700, 0, _p(feat), _p(thr), _p(lab), 2, None,
                                _p(pred), None))
    _expect(env, lib.mh_predict(ctx, _p(X), 700, 4, _p(feat), _p(thr), _p(lab), 11, None,
                                _p(pred), None))
    _expect(env, lib.mh_predict(ctx, _p(X), 700, 4, None, _p(thr), _p(lab), 2, None, _p(pred),
                                None))
    _expect(env, lib.mh_predict(ctx, _p(X), 700, 4, _p(feat), _p(thr), _p(lab), 2, None,
                                _p(pred), _p(corr)))
    _expect(env, lib.mh_predict(ctx, None, 700, 4, _p(feat), _p(thr), _p(lab), 2, None, _p(pred),
                                None))
    _still_usable(env)


def test_server_calls(env, monkeypatch):
    """Server creation and submission limits; the queue limit refuses a
    request with MH_EBUSY without queuing it."""
    lib = env["lib"]
    mh = env["mh"]
    ctx = capi.Context(0)
    h = C.c_void_p()
    assert lib.mh_server_create(ctx.h, 1 << 20, 0, C.byref(h)) == EINVAL
    assert lib.mh_server_create(ctx.h, 1 << 20, 257, C.byref(h)) == EINVAL
    assert lib.mh_server_create(ctx.h, 100, 2, C.byref(h)) == EINVAL
    assert lib.mh_server_create(None, 1 << 20, 2, C.byref(h)) == EINVAL
    b = C.c_uint64()
    for shape in ((1000, 0, 2, 2, 16), (1000, 81, 2, 2, 16), (1000, 4, 0, 2, 16),
                  (1000, 4, 2, 0, 16), (1000, 4, 2, 6, 16), (1000, 4, 2, 2, 2),
                  (1000, 4, 2, 2, 513)):
        assert lib.mh_server_footprint(*shape, C.byref(b)) == EINVAL
    assert lib.mh_server_footprint(1000, 4, 2, 2, 16, None) == EINVAL
    srv = mh.Server(1 << 28, 2, ctx=ctx)
    X, y = env["Xd"], env["yd"]
    prm = _prm()
    for n, F, K, D, p in ((700, 0, 3, 2, prm), (700, 81, 3, 2, prm), (700, 4, 0, 2, prm),
                          (700, 4, 3, 6, prm), (700, 4, 3, 2, _prm(P=513)),
                          (700, 4, 3, 2, _prm(P=2))):
        rc = lib.mh_server_submit(srv.h, 1, _p(X), _p(y), n, F, K, D, C.byref(p))
        assert rc == EINVAL and lib.mh_last_error(ctx.h).decode()
    assert lib.mh_server_submit(srv.h, 1, None, _p(y), 700, 4, 3, 2, C.byref(prm)) == EINVAL
    k = C.c_uint32()
    assert lib.mh_server_poll(srv.h, None, 4, C.byref(k)) == EINVAL
    assert lib.mh_server_poll(srv.h, None, 0, None) == EINVAL
    assert lib.mh_server_cancel(srv.h, 12345) == EINVAL
    assert lib.mh_server_pump(None, 1, None, None) == EINVAL
    # back-pressure: two may wait, the third is refused and not queued
    srv.set_limits(max_queued=2)
    for rid in (1, 2):
        srv.submit(rid, X, y, 3, 2, mh.de_params(16, 3, 0.5, 0.9, 7))
    rc = lib.mh_server_submit(srv.h, 3, _p(X), _p(y), 700, 4, 3, 2, C.byref(prm))
    assert rc == EBUSY and "queue" in lib.mh_last_error(ctx.h).decode()
    res = {r["req_id"]: r for r in srv.drain()}
    assert sorted(res) == [1, 2] and all(r["status"] == 0 for r in res.values())
    srv.close()
    ctx.close()
