"""GPU parity of the served form: a request's result from the continuous-
batching server equals the same request solved alone (subtree_solve on its
own context) and the oracle's DEOCT, bit for bit, whatever else shares its
launches; admission follows submission order under slot and HBM limits."""
import numpy as np
import pytest

import oracle
from paper_2311_06952_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mh():
    import paper_2311_06952_amd as m
    return m


# (rid, n, F, K, D, P, G, M): mixed sizes, depths, populations and classes;
# ragged tails, a single sample, an empty dataset, depth 1 and depth 5
REQUESTS = [
    (0, 1000, 4, 2, 2, 32, 20, 0.5),
    (1, 3000, 7, 3, 3, 64, 15, 0.5),
    (2, 12000, 16, 5, 4, 128, 10, 0.5),
    (3, 500, 32, 10, 2, 128, 25, 0.5),
    (4, 40000, 12, 4, 3, 100, 8, 0.5),
    (5, 63, 5, 2, 1, 16, 30, 0.5),
    (6, 1, 3, 2, 3, 8, 5, 0.5),
    (7, 20000, 20, 3, 5, 200, 6, 0.5),
    (8, 7000, 9, 6, 4, 128, 12, -1.0),
    (9, 0, 6, 3, 3, 32, 4, 0.5),
    (10, 2500, 80, 4, 3, 512, 5, 0.5),
    (11, 250_000, 10, 3, 3, 64, 4, 0.5),   # a large request (runs whole by default)
]


def _data(rid, n, F, K):
    return synth.Request(rid, 0.0, n, F, K, 2, seed=500 + rid).data()


def _prm(mh, P, G, M, rid):
    return mh.de_params(P, G, M, 0.9, 7000 + rid)


def _same(a, b):
    np.testing.assert_array_equal(a["feat"], b["feat"])
    np.testing.assert_array_equal(a["tau"], b["tau"])
    np.testing.assert_array_equal(a["label"], b["label"])
    assert a["correct"] == b["correct"]
    assert a["cost"] == b["cost"]


def _submit(mh, srv, req):
    import torch
    rid, n, F, K, D, P, G, M = req
    X, y = _data(rid, n, F, K)
    Xd = torch.as_tensor(X).cuda()
    yd = torch.as_tensor(y).cuda()
    srv.submit(rid, Xd, yd, K, D, _prm(mh, P, G, M, rid))


@pytest.mark.parametrize("solo", [None, "1", "0"])
def test_served_equals_alone_and_oracle(mh, monkeypatch, solo):
    """solo: requests from this many tiles up run whole as one cooperative
    launch (None: the server's default, two tiles per CU; "1": every request;
    "0": none, all stepped generation by generation in the batched launches)."""
    from paper_2311_06952_amd import capi
    if solo is not None:
        monkeypatch.setenv("MHDEOCT_SERVE_SOLO_TILES", solo)
    big = max(mh.server_footprint(n, F, K, D, P) for _, n, F, K, D, P, _, _ in REQUESTS)
    # room for about two of the largest requests, three slots: requests
    # wait for both, and later ones are admitted while others run
    srv_ctx = capi.Context(0)
    srv = mh.Server(2 * big + (1 << 20), 3, ctx=srv_ctx)
    for req in REQUESTS[:5]:
        _submit(mh, srv, req)
    srv.pump(3)
    for req in REQUESTS[5:]:
        _submit(mh, srv, req)
    results = {r["req_id"]: r for r in srv.drain()}
    srv.close()
    assert sorted(results) == [r[0] for r in REQUESTS]

    alone_ctx = capi.Context(0)
    for rid, n, F, K, D, P, G, M in REQUESTS:
        res = results[rid]
        assert res["status"] == 0
        assert (res["n"], res["F"], res["K"]) == (n, F, K)
        assert res["t_submit_ns"] <= res["t_admit_ns"] <= res["t_done_ns"]
        X, y = _data(rid, n, F, K)
        ds = mh.dataset(X, y, K, ctx=alone_ctx)
        alone = mh.subtree_solve(ds, D, _prm(mh, P, G, M, rid), ctx=alone_ctx)
        _same(res["tree"], alone)
        ods = oracle.dataset_from_X(X, y, K)
        want = oracle.deoct(ods, D, oracle.de_params(P, G, M, 0.9, 7000 + rid))
        _same(res["tree"], want)
    alone_ctx.close()
    # admission in submission order
    admits = [results[r[0]]["t_admit_ns"] for r in REQUESTS]
    assert admits == sorted(admits)


def test_served_penalised_objective(mh):
    """Requests with their own n_min and alpha share the server's launches and
    each still equals the oracle's DEOCT under its own objective."""
    import torch
    from paper_2311_06952_amd import capi
    reqs = [(60, 4000, 6, 3, 3, 64, 10, 40, 25.0), (61, 2500, 5, 2, 2, 32, 12, 1, 0.0),
            (62, 6000, 8, 4, 4, 96, 8, 150, 3.5)]
    ctx = capi.Context(0)
    srv = mh.Server(1 << 30, 3, ctx=ctx)
    for rid, n, F, K, D, P, G, n_min, alpha in reqs:
        X, y = _data(rid, n, F, K)
        srv.submit(rid, torch.as_tensor(X).cuda(), torch.as_tensor(y).cuda(), K, D,
                   mh.de_params(P, G, 0.5, 0.9, 7000 + rid, n_min, alpha))
    res = {r["req_id"]: r for r in srv.drain()}
    srv.close()
    ctx.close()
    for rid, n, F, K, D, P, G, n_min, alpha in reqs:
        assert res[rid]["status"] == 0
        X, y = _data(rid, n, F, K)
        want = oracle.deoct(oracle.dataset_from_X(X, y, K), D,
                            oracle.de_params(P, G, 0.5, 0.9, 7000 + rid, n_min, alpha))
        _same(res[rid]["tree"], want)


def test_server_rejects_oversized_and_reports_nan(mh):
    import torch
    from paper_2311_06952_amd import capi
    small = (0, 1000, 4, 2, 2, 32, 10, 0.5)
    ctx = capi.Context(0)
    budget = mh.server_footprint(1000, 4, 2, 2, 32) + 4096
    srv = mh.Server(budget, 2, ctx=ctx)
    X = torch.zeros((100_000, 8), dtype=torch.float32, device="cuda")
    y = torch.zeros(100_000, dtype=torch.uint8, device="cuda")
    with pytest.raises(mh.MhError) as ei:
        srv.submit(99, X, y, 2, 3, mh.de_params(32, 5, 0.5, 0.9, 1))
    assert ei.value.code == capi.MH_ENOMEM
    # a NaN request fails alone; the next one is unaffected
    Xn, yn = _data(50, 1000, 4, 2)
    Xn = Xn.copy()
    Xn[17, 2] = np.nan
    srv.submit(50, torch.as_tensor(Xn).cuda(), torch.as_tensor(yn).cuda(), 2, 2,
               mh.de_params(32, 10, 0.5, 0.9, 1))
    _submit(mh, srv, small)
    res = {r["req_id"]: r for r in srv.drain()}
    srv.close()
    assert res[50]["status"] == capi.MH_EINVAL
    assert res[0]["status"] == 0
    X0, y0 = _data(0, 1000, 4, 2)
    want = oracle.deoct(oracle.dataset_from_X(X0, y0, 2), 2, oracle.de_params(32, 10, 0.5, 0.9,
                                                                              7000))
    _same(res[0]["tree"], want)
    ctx.close()


def test_server_cancel_and_time_limit(mh, monkeypatch):
    """Failure handling of the served form: a queued request cancelled before
    admission, a resident request cancelled between its generations, a
    whole-request run cancelled after its launch, and requests past the
    server's time limit all come back with MH_ECANCELED; the slots and pool
    room they held serve later requests, whose results still equal the
    oracle's."""
    import torch
    from paper_2311_06952_amd import capi

    def sub(srv, rid, n, F, K, D, P, G):
        X, y = _data(rid, n, F, K)
        srv.submit(rid, torch.as_tensor(X).cuda(), torch.as_tensor(y).cuda(), K, D,
                   _prm(mh, P, G, 0.5, rid))

    def oracle_tree(rid, n, F, K, D, P, G):
        X, y = _data(rid, n, F, K)
        return oracle.deoct(oracle.dataset_from_X(X, y, K), D,
                            oracle.de_params(P, G, 0.5, 0.9, 7000 + rid))

    # stepped generation by generation: one slot, so the others queue
    monkeypatch.setenv("MHDEOCT_SERVE_SOLO_TILES", "0")
    ctx = capi.Context(0)
    srv = mh.Server(1 << 28, 1, ctx=ctx)
    sub(srv, 20, 3000, 5, 3, 3, 32, 60)
    sub(srv, 21, 2000, 4, 2, 2, 32, 10)
    srv.cancel(21)                      # still queued
    srv.pump(3)                         # 20 admitted and stepped
    srv.cancel(20)                      # resident, between generations
    with pytest.raises(mh.MhError) as ei:
        srv.cancel(20)                  # already cancelled
    assert ei.value.code == capi.MH_EINVAL
    sub(srv, 22, 2500, 6, 3, 3, 32, 8)  # gets the freed slot
    res = {r["req_id"]: r for r in srv.drain()}
    assert res[20]["status"] == capi.MH_ECANCELED
    assert res[21]["status"] == capi.MH_ECANCELED and res[21]["t_admit_ns"] == 0
    assert res[22]["status"] == 0
    _same(res[22]["tree"], oracle_tree(22, 2500, 6, 3, 3, 32, 8))
    with pytest.raises(mh.MhError):
        srv.cancel(22)                  # finished: no longer cancellable
    # a time limit of one nanosecond cancels everything at the next round
    srv.set_limits(0, 1)
    sub(srv, 23, 1500, 4, 2, 2, 16, 5)
    res = {r["req_id"]: r for r in srv.drain()}
    assert res[23]["status"] == capi.MH_ECANCELED
    srv.set_limits(0, 0)
    sub(srv, 24, 1500, 4, 2, 2, 16, 5)
    res = {r["req_id"]: r for r in srv.drain()}
    assert res[24]["status"] == 0
    _same(res[24]["tree"], oracle_tree(24, 1500, 4, 2, 2, 16, 5))
    srv.close()
    ctx.close()

    # a whole-request run (large request, default threshold) cancelled after
    # its launch finishes on the device and is reported cancelled
    monkeypatch.delenv("MHDEOCT_SERVE_SOLO_TILES")
    ctx = capi.Context(0)
    srv = mh.Server(1 << 30, 2, ctx=ctx)
    sub(srv, 30, 100_000, 8, 3, 3, 64, 20)
    sub(srv, 31, 2000, 4, 2, 2, 16, 6)
    srv.pump(1)
    srv.cancel(30)
    res = {r["req_id"]: r for r in srv.drain()}
    assert res[30]["status"] == capi.MH_ECANCELED and res[30]["t_admit_ns"] > 0
    assert res[31]["status"] == 0
    _same(res[31]["tree"], oracle_tree(31, 2000, 4, 2, 2, 16, 6))
    srv.close()
    ctx.close()
