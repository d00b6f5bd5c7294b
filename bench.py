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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-only", action="store_true",
                    help="time only the fitness kernel (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

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

    # fitness-kernel duration with HIP events on the library's stream
    ctx.profile(True)
    ctx.stats(reset=True)
    ranks, nu = mh.rank_encode(Xd, ctx)
    ds = mh.Dataset(ranks, yd, nu, w.n, w.F, w.K)
    mh.subtree_solve(ds, w.D, prm, ctx=ctx)
    st = ctx.stats(reset=True)
    ctx.profile(False)
    # the last launch evaluates the single best tree; the others the population
    pop_launches = st["launches"] - 1
    kernel_ms = st["ms"] / max(st["launches"], 1)
    evals_launch = w.P * w.n
    ops_per_eval = w.D + 1          # D compare-and-descend steps + 1 count
    achieved = ops_per_eval * evals_launch / (kernel_ms * 1e-3)
    bytes_eval = (4 * w.F + 1) / w.P
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK / 1e12,
            "unit": "TOP/s", "frac": achieved / VALU_PEAK, "traffic": None,
            "kernel": "k_fitness_bits<3,4>", "kernel_ms_avg": kernel_ms,
            "ops_per_eval": ops_per_eval, "evals_per_launch": evals_launch,
            "hbm_equiv": {"GB_s": bytes_eval * evals_launch / (kernel_ms * 1e-3) / 1e9,
                          "frac": bytes_eval * evals_launch / (kernel_ms * 1e-3) / HBM_PEAK}}
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
        "kernel_evals_per_s": evals_launch / (kernel_ms * 1e-3),
        "fitness_launches_per_step": int(st["launches"]),
        "subtree_solves_per_s": args.steps / el,
        "best_correct": res["correct"],
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
