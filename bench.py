"""Benchmark: sample-tree evaluations per second of the MH-DEOCT fitness path
on one MI355X.

A step is one DEOCT run (Algorithm 4) on the large plain workload: n =
1,000,000 samples, F = 32 float32 features (16 from a 4-component Gaussian
mixture, 16 uniform noise), K = 4 classes from a planted depth-5 tree with 5 %
label flips, depth-4 trees, P = 512, G = 100 generations (M = 0.5, CR = 0.9):
rank encoding of the resident float32 features, the tiled sample layout,
initialisation and G + 1 population evaluations with the DE step between
them, all on the device.  value = P * n * (G + 1) / (seconds per step).

Prints one JSON line.  --gpus N > 1 is refused: the library runs on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

VALU_PEAK = 256 * 64 * 2.4e9      # int32 lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
HBM_PEAK = 8.0e12                 # bytes/s
CSRC = os.path.join(ROOT, "paper_2311_06952_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")

# the dominant kernel of each form, the sources its code comes from, and the
# committed counter summary of it
KERNELS = {
    "per_generation": dict(
        sources=("fitness.hip", "fitness_core.h", "epilogue.h", "device_common.h", "de_body.h",
                 "internal.h"),
        counters="k_fitness_bits_plain_large_counters.txt"),
    "persistent": dict(
        sources=("persist.hip", "fitness_core.h", "epilogue.h", "device_common.h", "grid_sync.h",
                 "internal.h"),
        counters=None),
}
C2_TRAFFIC = os.path.join(PROFILES, "k_deoct_persist_plain_scale_traffic.txt")
C2_SOURCES = KERNELS["persistent"]["sources"]


def source_hash(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_summary(path, sources):
    """Key: value lines of a committed counter summary, or None when it is
    missing or the kernel's sources changed since the counters were taken."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != source_hash(sources):
            return None
        return kv
    except OSError:
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, seconds=15.0):
    """The oracle on the host cores (its fitness loop over individuals on
    OpenMP threads): DEOCT runs on the same workload with G = 1, 2, 4, ... as
    many as fit in about `seconds` (at least one)."""
    import oracle
    ods = oracle.dataset_from_X(w.X, w.y, w.K)
    evals = 0
    G = 1
    t0 = time.perf_counter()
    while True:
        prm = oracle.de_params(w.P, G, w.M, w.CR, 1001)
        t1 = time.perf_counter()
        oracle.deoct(ods, w.D, prm)
        dt = time.perf_counter() - t1
        evals += w.P * w.n * (G + 1) + w.n  # + the final re-evaluation of the best tree
        if time.perf_counter() - t0 > seconds or dt * 2 > seconds:
            break
        G *= 2
    el = time.perf_counter() - t0
    thr = oracle.threads()
    return dict(value=evals / el, unit="sample-tree evals/s", cores=thr, kind="oracle",
                sample=f"oracle DEOCT runs with G = 1, 2, 4, ... on the full {w.name} workload "
                       f"(rank encoding excluded), {evals:.3g} evals in {el:.1f} s on {thr} "
                       f"OpenMP threads of {os.cpu_count()} visible CPUs ({cpu_model()})")


def ds_of(mh, Xd, yd, w, ctx):
    ranks, nu = mh.rank_encode(Xd, ctx)
    return mh.Dataset(ranks, yd, nu, w.n, w.F, w.K)


def kernel_name(w, form, tuned):
    waves = min(8, max(1, (w.P + 63) // 64))
    waves = 8 if waves > 4 else (4 if waves > 2 else waves)
    if form == "persistent":
        return f"k_deoct_persist<{w.D},{waves},{tuned['halves']},...>"
    return f"k_fitness_bits<{w.D},{waves},false>"


def roofline(w, kernel_ms, launches_per_step, form, kname):
    """The dominant kernel against the int32 VALU roof: D compare-and-descend
    steps and one count per sample-tree evaluation (Algorithm 1).  Per
    generation the kernel is launched once per population evaluation; the
    whole-run form covers all G + 1 of them in one launch.  Beside it: the
    kernel's own VALU instruction rate and its HBM bytes from the committed
    counter summary (null once the kernel's sources changed)."""
    evals_launch = w.P * w.n * (w.G + 1) // launches_per_step
    ops_per_eval = w.D + 1
    sec = kernel_ms * 1e-3
    achieved = ops_per_eval * evals_launch / sec
    bytes_launch = (4 * w.F + 1) / w.P * evals_launch
    out = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
           "unit": "TOP/s", "frac": achieved / VALU_PEAK, "traffic": None,
           "kernel": kname, "kernel_ms_avg": kernel_ms, "launches_per_step": launches_per_step,
           "ops_per_eval": ops_per_eval, "evals_per_launch": evals_launch,
           "algorithmic_bytes_per_launch": bytes_launch,
           "hbm_equiv": {"GB_s": bytes_launch / sec / 1e9, "frac": bytes_launch / sec / HBM_PEAK}}
    k = KERNELS[form]
    kv = read_summary(os.path.join(PROFILES, k["counters"]), k["sources"]) if k["counters"] else None
    if kv:
        traffic = float(kv["traffic_bytes_per_launch"])
        valu = float(kv["sq_insts_valu_per_launch"]) * 64
        out["traffic"] = traffic
        out["counters"] = {
            "source": k["counters"],
            "hbm_GB_s": traffic / sec / 1e9, "hbm_frac": traffic / sec / HBM_PEAK,
            "valu_lane_ops_per_s": valu / sec, "valu_frac": valu / sec / VALU_PEAK,
            "lds_insts_per_launch": float(kv["sq_insts_lds_per_launch"]),
            "lds_bank_conflict_cycles_per_cu": float(kv["lds_bank_conflict_cycles_per_cu"]),
            "note": "rates use this run's kernel duration with the counted per-launch totals"}
    return out


def kernel_only(args):
    """Counter runs: one plain device copy of known size (the calibration for
    the byte counters), then --steps DEOCT runs of --gens generations on the
    resident workload (the large plain one by default).  Prints one JSON
    line."""
    import torch
    import paper_2311_06952_amd as mh
    from paper_2311_06952_amd import synth
    w = synth.plain_scale(1) if args.workload == "plain_scale" else synth.plain_large(1)
    G = args.gens if args.gens > 0 else w.G
    ctx = mh.default_context(0)
    dev = torch.device("cuda", 0)
    copy_bytes = 256 << 20
    a = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    Xd = torch.as_tensor(w.X).to(dev)
    yd = torch.as_tensor(w.y).to(dev)
    ds = ds_of(mh, Xd, yd, w, ctx)
    prm = mh.de_params(w.P, G, w.M, w.CR, 1001)
    ctx.stats(reset=True)
    ctx.profile(True)
    for _ in range(args.steps):
        mh.subtree_solve(ds, w.D, prm, ctx=ctx)
    ctx.profile(False)
    st = ctx.stats(reset=True)
    print(json.dumps({"workload": w.name, "generations": G, "launches": int(st["launches"]),
                      "kernel_ms_avg": st["ms"] / max(st["launches"], 1),
                      "copy_bytes": copy_bytes,
                      "per_generation_sha256_16": source_hash(KERNELS["per_generation"]["sources"]),
                      "persistent_sha256_16": source_hash(KERNELS["persistent"]["sources"])}),
          flush=True)


def timed_steps(mh, ctx, w, Xd, yd, steps, warmup, tune=True):
    """W untimed and K timed steps (rank encoding with an asynchronous status
    word, tile layout, the whole DEOCT run, the result read-back), then the
    same K steps again with the fitness launches timed by HIP events on the
    library's stream.  Returns (ms per step, result of the last step, event
    milliseconds per fitness launch, fitness launches per step, tuned)."""
    import torch
    dev = Xd.device
    prm = mh.de_params(w.P, w.G, w.M, w.CR, 1001)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    enc = mh.rank_encode(Xd, ctx)  # output buffers, written again by every step

    def step():
        # the rank encoding's NaN check is read back with the solved tree, so
        # a step waits for the device once
        ranks, nu = mh.rank_encode(Xd, ctx, status=status, out=enc)
        return mh.subtree_solve(mh.Dataset(ranks, yd, nu, w.n, w.F, w.K, status), w.D, prm,
                                ctx=ctx)

    # launch configuration for this shape, timed on short runs (it changes
    # timing only)
    if tune:
        tuned = mh.autotune(ds_of(mh, Xd, yd, w, ctx), w.D, prm, generations=10, ctx=ctx)
    else:
        tuned = {"persist": 1, "halves": int(os.environ.get("MHDEOCT_PERSIST_HALVES", "2")),
                 "persist_blocks_per_cu": 0, "fit_blocks_per_cu": 2, "untuned": True}
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # fitness-kernel duration: the population-evaluation launches record
    # start/stop events themselves (kept out of the timed steps above because
    # event-carrying launches cost about 3 us each)
    ctx.stats(reset=True)
    ctx.profile(True)
    for _ in range(steps):
        step()
    ctx.profile(False)
    st = ctx.stats(reset=True)
    kernel_ms = st["ms"] / max(st["launches"], 1)
    lps = max(1, round(st["launches"] / steps))
    return el / steps * 1e3, res, kernel_ms, lps, tuned, int(st["launches"])


def plain_scale(mh, ctx, steps=5, warmup=1):
    """The plain-scale workload (n = 100,000, F = 16, K = 3, depth 3, P = 256,
    G = 200): the whole run is one grid-synchronising launch with the tiles
    resident in LDS."""
    import torch
    from paper_2311_06952_amd import synth
    w = synth.plain_scale(1)
    dev = torch.device("cuda", 0)
    Xd = torch.as_tensor(w.X).to(dev)
    yd = torch.as_tensor(w.y).to(dev)
    ms, res, kms, lps, tuned, nl = timed_steps(mh, ctx, w, Xd, yd, steps, warmup)
    form = "persistent" if lps == 1 else "per_generation"
    roof = roofline(w, kms, lps, form, kernel_name(w, form, tuned))
    kv = read_summary(C2_TRAFFIC, C2_SOURCES) if form == "persistent" else None
    roof["traffic"] = float(kv["traffic_bytes_per_launch"]) if kv else None
    return {"workload": w.name, "ms_per_step": ms,
            "evals_per_s": w.P * w.n * (w.G + 1) / (ms * 1e-3), "best_correct": res["correct"],
            "roofline": roof,
            "launch_config": {k: tuned[k] for k in ("persist", "halves", "persist_blocks_per_cu",
                                                    "fit_blocks_per_cu")}}, (w, Xd, yd, res)


def _device_requests(torch, reqs):
    """Request datasets generated on the device: a Gaussian mixture with K
    class means ~ N(0, 2I), y uniform, x ~ N(mu_y, I), from torch's Philox
    generator seeded with the request's seed."""
    out = []
    for q in reqs:
        g = torch.Generator(device="cuda")
        g.manual_seed(q.seed)
        mu = torch.randn((q.K, q.F), generator=g, device="cuda") * (2.0 ** 0.5)
        y = torch.randint(q.K, (q.n,), generator=g, device="cuda")
        X = (mu[y] + torch.randn((q.n, q.F), generator=g, device="cuda")).contiguous()
        out.append((X, y.to(torch.uint8)))
    torch.cuda.synchronize()
    return out


def serving(mh, count=96, seed=11, n_hi=1e7, slots=64):
    """Served subtree solves: `count` requests (n log-uniform in [1e3, n_hi],
    F in 4..32, K in 2..10, D in 2..4, P = 128, G = 100).  The same requests
    are solved (1) one after another with subtree_solve, (2) through the
    server all submitted at once (its capacity), (3) through the server with
    Poisson arrivals at 0.8x that capacity (latency)."""
    import torch
    from paper_2311_06952_amd import capi, synth
    reqs = synth.request_stream(seed, count, 1.0, n_hi=n_hi)
    data = _device_requests(torch, reqs)
    evals = sum(q.n * q.P * (q.G + 1) for q in reqs)
    prm = [mh.de_params(q.P, q.G, 0.5, 0.9, 5000 + q.rid) for q in reqs]

    # (1) plain: one request at a time on one context (the rank encoding's
    # NaN check is read with the result)
    ctx = capi.Context(0)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    t0 = time.perf_counter()
    for q, (X, y), p in zip(reqs, data, prm):
        ranks, nu = mh.rank_encode(X, ctx, status=status)
        mh.subtree_solve(mh.Dataset(ranks, y, nu, q.n, q.F, q.K, status), q.D, p, ctx=ctx)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.close()

    budget = 96 << 30

    def run(arrivals):
        sctx = capi.Context(0)
        srv = mh.Server(budget, slots, ctx=sctx)
        t0 = time.monotonic_ns()
        nxt, done = 0, []
        while len(done) < count:
            now = time.monotonic_ns() - t0
            while nxt < count and arrivals[nxt] <= now:
                q = reqs[nxt]
                srv.submit(q.rid, data[nxt][0], data[nxt][1], q.K, q.D, prm[nxt])
                nxt += 1
            act, queued = srv.pump(1)
            done += srv.poll(256)
            if act == 0 and queued == 0 and nxt < count:
                time.sleep(max(0.0, (arrivals[nxt] - (time.monotonic_ns() - t0)) * 1e-9))
        el = (time.monotonic_ns() - t0) * 1e-9
        srv.close()
        sctx.close()
        lat = sorted((r["t_done_ns"] - (t0 + arrivals[r["req_id"]])) * 1e-6 for r in done)
        bad = [r["req_id"] for r in done if r["status"] != 0]
        return el, lat, bad

    el_c, _, bad_c = run([0] * count)
    cap = count / el_c
    rate = 0.8 * cap
    arr = [int(q.arrival / rate * 1e9) for q in reqs]   # the unit-rate stream rescaled
    el_o, lat, bad_o = run(arr)
    pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100 * (len(lat) - 1))))]
    return {
        "workload": f"{count} requests, n log-uniform [1e3, {n_hi:.0e}], F 4..32, K 2..10, "
                    f"D 2..4, P 128, G 100, Gaussian mixtures generated on the device",
        "server": {"hbm_budget_bytes": budget, "max_slots": slots},
        "evals": evals,
        "plain": {"s": t_plain, "evals_per_s": evals / t_plain, "solves_per_s": count / t_plain},
        "served_all_at_once": {"s": el_c, "evals_per_s": evals / el_c, "solves_per_s": cap},
        "served_poisson": {"rate_per_s": rate, "s": el_o, "evals_per_s": evals / el_o,
                           "solves_per_s": count / el_o, "p50_ms": pct(50), "p99_ms": pct(99),
                           "max_ms": lat[-1]},
        "failed": bad_c + bad_o,
    }


def _gen_request(torch, q, stream):
    """One request's dataset generated on the device on `stream` (torch's
    Philox generator seeded with the request's seed): K class means ~ N(0,
    2I), y uniform, x ~ N(mu_y, I).  Returns (X, y, event recorded after)."""
    with torch.cuda.stream(stream):
        g = torch.Generator(device="cuda")
        g.manual_seed(q.seed)
        mu = torch.randn((q.K, q.F), generator=g, device="cuda") * (2.0 ** 0.5)
        y = torch.randint(q.K, (q.n,), generator=g, device="cuda")
        X = (mu[y] + torch.randn((q.n, q.F), generator=g, device="cuda")).contiguous()
        y8 = y.to(torch.uint8)
        ev = torch.cuda.Event()
        ev.record(stream)
    return X, y8, ev


def serving_full(mh, count=2000, seed=21, rates=(0.5, 0.8, 1.2), slots=64):
    """The served configuration at its stated size: `count` requests (n
    log-uniform in [1e3, 1e7], F 4..32, K 2..10, D 2..4, P = 128, G = 100),
    each request's data generated on the device when it is submitted (on a
    stream of its own, which the solving stream waits for).  Forms: (1) one
    request after another with subtree_solve (the plain form); (2) the server
    fed as fast as it admits (at most 2 x slots waiting: its capacity); (3)
    Poisson arrivals at each of `rates` x that capacity (latency from arrival
    to the result).  Then the moving-horizon run on n = 10^7, F = 8, K = 2,
    depth 8, horizon 3, batched and node by node."""
    import torch
    from paper_2311_06952_amd import capi, synth
    reqs = synth.request_stream(seed, count, 1.0, n_hi=1e7)
    evals = sum(q.n * q.P * (q.G + 1) for q in reqs)
    prm = [mh.de_params(q.P, q.G, 0.5, 0.9, 5000 + q.rid) for q in reqs]
    gen_stream = torch.cuda.Stream()
    out = {"workload": f"{count} requests, n log-uniform [1e3, 1e7], F 4..32, K 2..10, D 2..4, "
                       f"P 128, G 100; data generated on the device at submit time",
           "evals": evals}

    # (1) plain
    run_stream = torch.cuda.Stream()
    ctx = capi.Context(0, stream=run_stream)
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for q, p in zip(reqs, prm):
        X, y, ev = _gen_request(torch, q, gen_stream)
        run_stream.wait_event(ev)
        X.record_stream(run_stream)  # freed only after the solving stream is done with it
        y.record_stream(run_stream)
        if q.rid % 250 == 0:
            print(f"serving_full: plain, request {q.rid}", file=sys.stderr, flush=True)
        with torch.cuda.stream(run_stream):
            ranks, nu = mh.rank_encode(X, ctx, status=status)
            mh.subtree_solve(mh.Dataset(ranks, y, nu, q.n, q.F, q.K, status), q.D, p, ctx=ctx)
        del X, y, ranks, nu
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    ctx.close()
    out["plain"] = {"s": t_plain, "evals_per_s": evals / t_plain, "solves_per_s": count / t_plain}

    budget = 96 << 30

    def run(arrivals, max_wait=None):
        srv_stream = torch.cuda.Stream()
        sctx = capi.Context(0, stream=srv_stream)
        srv = mh.Server(budget, slots, ctx=sctx)
        torch.cuda.synchronize()
        t0 = time.monotonic_ns()
        nxt, done, queued = 0, [], 0
        while len(done) < count:
            now = time.monotonic_ns() - t0
            while nxt < count and (arrivals is None or arrivals[nxt] <= now) and \
                    (max_wait is None or queued < max_wait):
                q = reqs[nxt]
                X, y, ev = _gen_request(torch, q, gen_stream)
                srv_stream.wait_event(ev)
                srv.submit(q.rid, X, y, q.K, q.D, prm[nxt])
                nxt += 1
                queued += 1
                if nxt % 250 == 0:
                    print(f"serving_full: served, {nxt} submitted, {len(done)} done",
                          file=sys.stderr, flush=True)
            act, queued = srv.pump(1)
            done += srv.poll(256)
            if act == 0 and queued == 0 and nxt < count and arrivals is not None:
                time.sleep(max(0.0, (arrivals[nxt] - (time.monotonic_ns() - t0)) * 1e-9))
        el = (time.monotonic_ns() - t0) * 1e-9
        srv.close()
        sctx.close()
        arr = arrivals if arrivals is not None else [0] * count
        lat = sorted((r["t_done_ns"] - (t0 + arr[r["req_id"]])) * 1e-6 for r in done)
        bad = [r["req_id"] for r in done if r["status"] != 0]
        pct = lambda p: lat[min(len(lat) - 1, int(round(p / 100 * (len(lat) - 1))))]
        return el, {"p50_ms": pct(50), "p99_ms": pct(99), "max_ms": lat[-1]}, bad

    el_c, _, bad = run(None, max_wait=2 * slots)
    cap = count / el_c
    out["server"] = {"hbm_budget_bytes": budget, "max_slots": slots}
    out["served_capacity"] = {"s": el_c, "evals_per_s": evals / el_c, "solves_per_s": cap}
    out["failed"] = bad
    out["poisson"] = []
    for f in rates:
        rate = f * cap
        arr = [int(q.arrival / rate * 1e9) for q in reqs]   # the unit-rate stream rescaled
        el, lat, bad = run(arr)
        out["poisson"].append({"load": f, "rate_per_s": rate, "s": el,
                               "evals_per_s": evals / el, "solves_per_s": count / el, **lat})
        out["failed"] += bad
    # the moving-horizon run of the served configuration
    print("serving_full: moving horizon", file=sys.stderr, flush=True)
    w = synth.served_mh(1)
    ctx = mh.default_context(0)
    ds = mh.dataset(w.X, w.y, w.K, ctx=ctx)
    p = mh.de_params(w.P, w.G, w.M, w.CR, 1001)
    mhr = {"workload": w.name}
    trees = {}
    for name, batched in (("batched", True), ("sequential", False)):
        mh.mh_train(ds, w.D, w.D_MH, p, batched=batched, ctx=ctx)
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trees[name] = mh.mh_train(ds, w.D, w.D_MH, p, batched=batched, ctx=ctx)
        el = time.perf_counter() - t0
        st = ctx.stats(reset=True)
        mhr[name] = {"s": el, "evals": int(st["evals"]), "evals_per_s": st["evals"] / el}
    mhr["same_tree"] = bool(all((trees["batched"][k] == trees["sequential"][k]).all()
                                for k in ("feat", "tau", "label")))
    mhr["correct"] = trees["batched"]["correct"]
    out["moving_horizon"] = mhr
    return out


def moving_horizon(mh, ctx):
    """Moving-horizon training of a depth-8 tree with horizon 3 on n = 10^6,
    F = 20, K = 3 (P = 128, G = 100): the level-batched form against the
    node-by-node form; both build the identical tree."""
    import torch
    from paper_2311_06952_amd import synth
    w = synth.batched_mh(1)
    ds = mh.dataset(w.X, w.y, w.K, ctx=ctx)
    prm = mh.de_params(w.P, w.G, w.M, w.CR, 1001)
    out = {"workload": w.name}
    trees = {}
    for name, batched in (("batched", True), ("sequential", False)):
        # one untimed run first (buffer allocation and the first launches'
        # set-up), then the timed one
        mh.mh_train(ds, w.D, w.D_MH, prm, batched=batched, ctx=ctx)
        ctx.stats(reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trees[name] = mh.mh_train(ds, w.D, w.D_MH, prm, batched=batched, ctx=ctx)
        el = time.perf_counter() - t0
        st = ctx.stats(reset=True)
        out[name] = {"s": el, "evals": int(st["evals"]), "evals_per_s": st["evals"] / el}
    out["same_tree"] = bool(all((trees["batched"][k] == trees["sequential"][k]).all()
                                for k in ("feat", "tau", "label")))
    out["correct"] = trees["batched"]["correct"]
    return out


def deep_whole_tree(mh, ctx, w, Xd, yd):
    """Whole-tree DEOCT at depth 8 (510 genes) on the plain-scale data with
    the paper's Normal setting (P = 100, G = 600, CR = 0.1, a mutation factor
    drawn per individual and generation): one untimed short run, then the
    timed one."""
    import torch
    ds = ds_of(mh, Xd, yd, w, ctx)
    D, P, G = 8, 100, 600
    mh.subtree_solve(ds, D, mh.de_params(P, 2, -1.0, 0.1, 7), ctx=ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = mh.subtree_solve(ds, D, mh.de_params(P, G, -1.0, 0.1, 7), ctx=ctx)
    el = time.perf_counter() - t0
    return {"workload": f"plain-scale data, depth {D}, P {P}, G {G}, CR 0.1, M ~ U[0,1)",
            "s": el, "evals_per_s": P * w.n * (G + 1) / el, "correct": r["correct"]}


def alpha_sweep(mh, ctx, w, alphas=(0.0, 3.0, 10.0, 30.0, 100.0, 300.0, 1000.0), D=4):
    """Choosing the per-split penalty alpha by validation (the sweep of
    Section 3.2's penalised objective): the plain-scale data split 75/25 into
    training and validation rows, a depth-4 tree solved per alpha (P = 256,
    G = 200), scored on the validation rows; the chosen tree's accuracy on the
    10^6 held-out rows.  Every solve and score runs on the device."""
    import numpy as np
    from paper_2311_06952_amd import synth
    perm = np.random.default_rng(3).permutation(w.n)
    cut = (3 * w.n) // 4
    Xtr, ytr = w.X[perm[:cut]], w.y[perm[:cut]]
    Xva, yva = w.X[perm[cut:]], w.y[perm[cut:]]
    ds = mh.dataset(Xtr, ytr, w.K, ctx=ctx)
    rows = []
    best = None
    for a in alphas:
        t = mh.subtree_solve(ds, D, mh.de_params(w.P, w.G, w.M, w.CR, 1001, 1, a), ctx=ctx)
        thr = mh.tree_thresholds(ds, Xtr, t, ctx=ctx)
        _, cv = mh.predict(Xva, t, thr, y=yva, ctx=ctx)
        rows.append({"alpha": a, "splits": int(np.count_nonzero(t["feat"])),
                     "train_acc": t["correct"] / cut, "val_acc": cv / len(yva)})
        if best is None or cv > best[0]:
            best = (cv, a, t, thr)
    Xh, yh = synth.plain_scale_heldout(1, 1_000_000)
    _, ch = mh.predict(Xh, best[2], best[3], y=yh, ctx=ctx)
    return {"depth": D, "sweep": rows, "chosen_alpha": best[1], "heldout_acc": ch / len(yh)}


def ablation(mh, ctx, n=100_000, depths=((2, 2), (4, 3), (8, 3))):
    """The warm-start ablation in the layout of Section 4's ablation table on
    synthetic data: the plain-large generator (F = 32, K = 4, labels from a
    planted depth-5 tree with 5 % flips) at 2n rows, split in half into
    training and test rows.  Rows: 1 CART; 2-3 whole-tree DEOCT without and
    with the CART warm start; 4-5 the same with 1,800 generations; 6-11 the
    batched moving horizon (horizon 2 at depth 2, 3 at depths 4 and 8) with
    the warm-start factors "CART WS in DE" (MH_WS_DEOCT_CART), "DE WS"
    (MH_WS_DEOCT) and "CART WS" (MH_WS_CART).  DE in the paper's Normal
    setting: P = 100, G = 600, CR = 0.1, a mutation factor drawn per
    individual and generation.  Each timed run follows an untimed two-
    generation run of the same configuration; times include computing the
    warm starts."""
    import numpy as np
    import torch
    from paper_2311_06952_amd import capi, synth
    w = synth.plain_large(3, n=2 * n)
    perm = np.random.default_rng(5).permutation(2 * n)
    Xtr, ytr = np.ascontiguousarray(w.X[perm[:n]]), w.y[perm[:n]]
    Xte, yte = np.ascontiguousarray(w.X[perm[n:]]), w.y[perm[n:]]
    ds = mh.dataset(Xtr, ytr, w.K, ctx=ctx)
    P, G, CR = 100, 600, 0.1
    dev = torch.device("cuda", ctx.device)

    def accs(tree):
        thr = mh.tree_thresholds(ds, Xtr, tree, ctx=ctx)
        _, ct = mh.predict(Xte, tree, thr, y=yte, ctx=ctx)
        return tree["correct"] / n, ct / n

    def cart_tree(D):
        feat, tau = mh.cart(ds, D, ctx=ctx)
        fd = torch.as_tensor(feat).to(dev)
        td = torch.as_tensor(tau.view(np.int32)).to(dev)
        _, corr, lab, cost = mh.fitness_eval(ds, fd, td, D, ctx=ctx, want_counts=False)
        return {"D": D, "feat": feat, "tau": tau, "label": lab[0].cpu().numpy(),
                "correct": int(corr[0].item()), "cost": float(cost[0].item())}

    def deoct(D, g, ws):
        t = None
        if ws:
            t = cart_tree(D)
            genes = mh.tree_encode(t["feat"], t["tau"], D, w.F, ds.n_unique, ctx=ctx)
            t = genes.cpu().numpy()
        return mh.subtree_solve(ds, D, mh.de_params(P, g, -1.0, CR, 11), warm=t, ctx=ctx)

    def timed(fn, warm_fn):
        warm_fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tree = fn()
        torch.cuda.synchronize()
        return tree, time.perf_counter() - t0

    rows = []

    def add(no, method, D, tree, s):
        tr, te = accs(tree)
        rows.append({"no": no, "method": method, "D": D, "train_acc": tr, "test_acc": te,
                     "s": s})

    ws_rows = ((6, 0), (7, capi.MH_WS_CART), (8, capi.MH_WS_DEOCT),
               (9, capi.MH_WS_DEOCT | capi.MH_WS_CART),
               (10, capi.MH_WS_DEOCT_CART | capi.MH_WS_DEOCT),
               (11, capi.MH_WS_DEOCT_CART | capi.MH_WS_DEOCT | capi.MH_WS_CART))
    for D, H in depths:
        tree, s = timed(lambda: cart_tree(D), lambda: cart_tree(D))
        add(1, "CART", D, tree, s)
        for no, g, ws in ((2, G, False), (3, G, True), (4, 3 * G, False), (5, 3 * G, True)):
            if no >= 4 and D == 2:
                continue
            tree, s = timed(lambda: deoct(D, g, ws), lambda: deoct(D, 2, ws))
            add(no, "DEOCT" + (" + CART WS" if ws else "") + (" (1800 gens)" if no >= 4 else ""),
                D, tree, s)
        for no, fl in ws_rows:
            prm = mh.de_params(P, G, -1.0, CR, 11)
            short = mh.de_params(P, 2, -1.0, CR, 11)
            tree, s = timed(lambda: mh.mh_train(ds, D, H, prm, batched=True, ctx=ctx, warm=fl),
                            lambda: mh.mh_train(ds, D, H, short, batched=True, ctx=ctx, warm=fl))
            add(no, f"MH-DEOCT (horizon {H}, warm starts {fl:#x})", D, tree, s)
        print(f"ablation: depth {D} done", file=sys.stderr, flush=True)
    return {"workload": f"plain-large generator, {n} training + {n} test rows, F {w.F}, K {w.K}",
            "de": {"P": P, "G": G, "CR": CR, "M": "U[0,1) per individual and generation"},
            "rows": rows}


def predict_bench(mh, ctx, w, Xd, yd, tree, reps=16, launches=20):
    """The trained tree on 10^6 held-out rows of the same mixture (test
    accuracy), and k_predict's duration on those rows tiled reps times
    (HIP events on the library's stream, which is torch's current one)."""
    import torch
    from paper_2311_06952_amd import synth
    Xh, yh = synth.plain_scale_heldout(1, 1_000_000)
    thr = mh.tree_thresholds(ds_of(mh, Xd, yd, w, ctx), Xd, tree, ctx=ctx)
    _, c_test = mh.predict(Xh, tree, thr, y=yh, ctx=ctx)
    dev = Xd.device
    Xb = torch.as_tensor(Xh).to(dev).repeat(reps, 1).contiguous()
    yb = torch.as_tensor(yh).to(dev).repeat(reps).contiguous()
    n = int(Xb.shape[0])
    feat = torch.as_tensor(tree["feat"]).to(dev)
    label = torch.as_tensor(tree["label"]).to(dev)
    pred = torch.empty(n, dtype=torch.uint8, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)

    def launch():
        ctx.check(ctx.lib.mh_predict(ctx.h, Xb.data_ptr(), n, w.F, feat.data_ptr(),
                                     thr.data_ptr(), label.data_ptr(), w.D, yb.data_ptr(),
                                     pred.data_ptr(), cnt.data_ptr()))

    launch()
    torch.cuda.synchronize()
    assert int(cnt.item()) == reps * c_test
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(launches):
        launch()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / launches
    bytes_row = 4 * w.F + 2  # the row, its label, its prediction
    return {"heldout_rows": len(yh), "test_accuracy": c_test / len(yh),
            "train_accuracy": tree["correct"] / w.n, "rows_per_launch": n,
            "ms_per_launch": ms, "rows_per_s": n / (ms * 1e-3),
            "algorithmic_bytes_per_row": bytes_row,
            "GB_s": bytes_row * n / (ms * 1e-3) / 1e9,
            "hbm_frac": bytes_row * n / (ms * 1e-3) / HBM_PEAK,
            "note": "ms per launch includes the zeroing of the count (one small launch)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-configuration tuning (size rules and environment)")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (plain-scale, serving, moving horizon, ...)")
    ap.add_argument("--extra-only", action="store_true",
                    help="only the serving and moving-horizon measurements (for profiler runs)")
    ap.add_argument("--predict-only", action="store_true",
                    help="only one solve and the held-out predict measurement (for profiler runs)")
    ap.add_argument("--alpha-only", action="store_true",
                    help="only the alpha sweep with validation")
    ap.add_argument("--deep-only", action="store_true",
                    help="only the depth-8 whole-tree DEOCT run (for profiler runs)")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only a calibration copy and --steps DEOCT runs (for counter runs)")
    ap.add_argument("--serving-full", action="store_true",
                    help="only the served configuration at its stated size (2,000 requests at "
                         "three loads, and the 10^7-sample moving-horizon run)")
    ap.add_argument("--ablation", action="store_true",
                    help="only the warm-start ablation (CART, DEOCT, moving-horizon variants)")
    ap.add_argument("--workload", default="plain_large", choices=("plain_large", "plain_scale"),
                    help="workload of --kernel-only")
    ap.add_argument("--gens", type=int, default=10,
                    help="generations per DEOCT run of --kernel-only (0: the workload's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.kernel_only:
        kernel_only(args)
        return
    if args.ablation:
        import paper_2311_06952_amd as mh
        print(json.dumps({"ablation": ablation(mh, mh.default_context(0))}), flush=True)
        return
    if args.serving_full:
        import paper_2311_06952_amd as mh
        print(json.dumps({"serving_full": serving_full(mh)}), flush=True)
        return
    if args.extra_only:
        import paper_2311_06952_amd as mh
        print(json.dumps({"serving": serving(mh),
                          "serving_small": serving(mh, count=256, seed=12, n_hi=2e4, slots=256),
                          "moving_horizon": moving_horizon(mh, mh.default_context(0))}),
              flush=True)
        return

    import torch
    import paper_2311_06952_amd as mh
    from paper_2311_06952_amd import synth

    ctx = mh.default_context(0)
    dev = torch.device("cuda", 0)
    if args.predict_only or args.alpha_only or args.deep_only:
        w2 = synth.plain_scale(1)
        X2 = torch.as_tensor(w2.X).to(dev)
        y2 = torch.as_tensor(w2.y).to(dev)
        if args.alpha_only:
            print(json.dumps({"alpha_sweep": alpha_sweep(mh, ctx, w2)}), flush=True)
        elif args.deep_only:
            print(json.dumps({"deep_whole_tree": deep_whole_tree(mh, ctx, w2, X2, y2)}),
                  flush=True)
        else:
            t = mh.subtree_solve(ds_of(mh, X2, y2, w2, ctx), w2.D,
                                 mh.de_params(w2.P, w2.G, w2.M, w2.CR, 1001), ctx=ctx)
            print(json.dumps({"predict": predict_bench(mh, ctx, w2, X2, y2, t)}), flush=True)
        return

    w = synth.plain_large(1)
    Xd = torch.as_tensor(w.X).to(dev)
    yd = torch.as_tensor(w.y).to(dev)
    ms, res, kernel_ms, lps, tuned, nlaunch = timed_steps(mh, ctx, w, Xd, yd, args.steps,
                                                          args.warmup, tune=not args.no_tune)
    evals_per_step = w.P * w.n * (w.G + 1)
    form = "persistent" if lps == 1 else "per_generation"
    roof = roofline(w, kernel_ms, lps, form, kernel_name(w, form, tuned))
    roof["timed_launches"] = nlaunch
    out = {
        "metric": "sample-tree evals/s (fitness)",
        "value": evals_per_step / (ms * 1e-3),
        "unit": "sample-tree evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "F": w.F, "K": w.K, "D": w.D, "P": w.P,
                   "G": w.G, "M": w.M, "CR": w.CR,
                   "form": ("plain DEOCT, the whole run in one grid-synchronising launch"
                            if form == "persistent" else
                            "plain DEOCT, one fitness launch and two DE launches per generation")},
        "kernel_evals_per_s": roof["evals_per_launch"] / (kernel_ms * 1e-3),
        "subtree_solves_per_s": 1e3 / ms,
        "best_correct": res["correct"],
        "roofline": roof,
        "launch_config": dict(
            {k: tuned[k] for k in ("persist", "halves", "persist_blocks_per_cu",
                                   "fit_blocks_per_cu")},
            note="persist = 1 allows the whole-run kernel; the library still runs the "
                 "per-generation kernels where they keep more waves resident (the form above)"),
    }
    del Xd, yd
    if not args.no_extra:
        c2, (w2, X2, y2, res2) = plain_scale(mh, ctx)
        out["plain_scale"] = c2
        out["predict"] = predict_bench(mh, ctx, w2, X2, y2, res2)
        out["deep_whole_tree"] = deep_whole_tree(mh, ctx, w2, X2, y2)
        out["alpha_sweep"] = alpha_sweep(mh, ctx, w2)
        out["serving"] = serving(mh)
        # the same forms on a stream of small requests (n log-uniform in
        # [1e3, 2e4]), where a request alone cannot fill the GPU
        out["serving_small"] = serving(mh, count=256, seed=12, n_hi=2e4, slots=256)
        out["moving_horizon"] = moving_horizon(mh, ctx)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
