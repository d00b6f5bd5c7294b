"""Benchmark: sample-tree evaluations per second of the MH-DEOCT fitness path
on one MI355X.

A step is one DEOCT run (Algorithm 4) on the plain-scale workload: n = 100,000
samples, F = 16 Gaussian-mixture features, K = 3 classes, depth-3 trees,
P = 256, G = 200 generations (M = 0.5, CR = 0.9): rank encoding of the
resident float32 features, the tiled sample layout, initialisation and
G + 1 population evaluations with the DE step between them, all on the device.
value = P * n * (G + 1) / (seconds per step).

Prints one JSON line.  --gpus N > 1 is refused: this build runs on one GPU.
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


def cpu_baseline(w, seconds=15.0):
    """The oracle on the host: DEOCT generations on the same workload, as many
    as fit in about `seconds` (at least one)."""
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
    return dict(value=evals / el, unit="sample-tree evals/s", cores=1, kind="oracle",
                sample=f"oracle DEOCT runs with G = 1, 2, 4, ... on the full n={w.n} "
                       f"workload, {evals:.3g} evals in {el:.1f} s, single thread")


KERNEL = "k_fitness_bits<3,4,false>"
KERNEL_SOURCES = ("fitness.hip", "epilogue.h", "de_body.h", "device_common.h", "internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fitness_bits_plain_scale_traffic.txt")


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2311_06952_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fitness kernel from the committed counter
    summary, or None when it is missing or the kernel sources changed since
    the counters were taken."""
    try:
        kv = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                if ":" in line and not line.startswith(" "):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def ds_of(mh, Xd, yd, w, ctx):
    ranks, nu = mh.rank_encode(Xd, ctx)
    return mh.Dataset(ranks, yd, nu, w.n, w.F, w.K)


def fitness_kernel_loop(mh, ctx, ds, w, launches):
    """Average duration (ms) of the fitness kernel over `launches` population
    evaluations of a freshly initialised population on the tiled layout."""
    import torch
    ts = mh.TileSet(ds, ctx=ctx)
    pop = mh.de_init(w.P, w.D, w.F, 1001, 0, ctx=ctx)
    feat, tau = mh.tree_decode(pop, w.D, w.F, ds.n_unique, ctx)
    out = (None, None, None, torch.zeros(w.P, dtype=torch.float64, device=pop.device))
    ts.fitness(feat, tau, w.D, out=out)
    ctx.stats(reset=True)
    ctx.profile(True)
    for _ in range(launches):
        ts.fitness(feat, tau, w.D, out=out)
    st = ctx.stats(reset=True)
    ctx.profile(False)
    return st["ms"] / max(st["launches"], 1), st


def roofline(w, kernel_ms):
    """The fitness kernel against the int32 VALU roof: D compare-and-descend
    steps and one count per sample-tree evaluation (Algorithm 1)."""
    evals_launch = w.P * w.n
    ops_per_eval = w.D + 1
    achieved = ops_per_eval * evals_launch / (kernel_ms * 1e-3)
    bytes_eval = (4 * w.F + 1) / w.P
    traffic = measured_traffic()
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "TOP/s", "frac": achieved / VALU_PEAK, "traffic": traffic,
            "kernel": KERNEL, "kernel_ms_avg": kernel_ms,
            "ops_per_eval": ops_per_eval, "evals_per_launch": evals_launch,
            "algorithmic_bytes_per_launch": bytes_eval * evals_launch,
            "hbm_equiv": {"GB_s": bytes_eval * evals_launch / (kernel_ms * 1e-3) / 1e9,
                          "frac": bytes_eval * evals_launch / (kernel_ms * 1e-3) / HBM_PEAK}}


def kernel_only(args):
    """Counter runs: one plain device copy of known size (the calibration for
    the byte counters), then the fitness-kernel loop.  Prints one JSON line."""
    import torch
    import paper_2311_06952_amd as mh
    from paper_2311_06952_amd import synth
    w = synth.plain_scale(1)
    ctx = mh.default_context(0)
    dev = torch.device("cuda", 0)
    copy_bytes = 256 << 20
    a = torch.ones(copy_bytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    Xd = torch.as_tensor(w.X).to(dev)
    yd = torch.as_tensor(w.y).to(dev)
    kernel_ms, st = fitness_kernel_loop(mh, ctx, ds_of(mh, Xd, yd, w, ctx), w, args.steps)
    print(json.dumps({"kernel": KERNEL, "workload": w.name, "launches": int(st["launches"]),
                      "kernel_ms_avg": kernel_ms, "copy_bytes": copy_bytes,
                      "kernel_source_sha256_16": kernel_source_hash(),
                      "roofline": roofline(w, kernel_ms)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="only a calibration copy and --steps fitness-kernel launches "
                         "(for counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    if args.kernel_only:
        kernel_only(args)
        return

    import torch
    import paper_2311_06952_amd as mh
    from paper_2311_06952_amd import synth

    w = synth.plain_scale(1)
    ctx = mh.default_context(0)
    dev = torch.device("cuda", 0)
    Xd = torch.as_tensor(w.X).to(dev)
    yd = torch.as_tensor(w.y).to(dev)
    prm = mh.de_params(w.P, w.G, w.M, w.CR, 1001)

    def step():
        ranks, nu = mh.rank_encode(Xd, ctx)
        ds = mh.Dataset(ranks, yd, nu, w.n, w.F, w.K)
        return mh.subtree_solve(ds, w.D, prm, ctx=ctx)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / args.steps * 1e3
    evals_per_step = w.P * w.n * (w.G + 1)
    value = evals_per_step * args.steps / el

    # fitness-kernel duration: the same steps again with HIP events that the
    # population-evaluation launches record themselves on the library's
    # stream (read back after the region; kept out of the timed steps above
    # because event-carrying launches cost about 3 us each)
    ctx.stats(reset=True)
    ctx.profile(True)
    for _ in range(args.steps):
        step()
    ctx.profile(False)
    st = ctx.stats(reset=True)
    kernel_ms = st["ms"] / max(st["launches"], 1)
    roof = roofline(w, kernel_ms)
    roof["timed_launches"] = int(st["launches"])
    out = {
        "metric": "sample-tree evals/s (fitness)",
        "value": value,
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
                   "G": w.G, "M": w.M, "CR": w.CR, "form": "plain DEOCT, one launch per "
                   "population evaluation"},
        "kernel_evals_per_s": w.P * w.n / (kernel_ms * 1e-3),
        "fitness_launches_per_step": w.G + 2,  # G + 1 population evaluations + the best tree
        "subtree_solves_per_s": args.steps / el,
        "best_correct": res["correct"],
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
