"""Benchmark of the p-median hot path on one MI355X.

Workload (one step): a random connected graph with n = m = 900 vertices and
16200 edges, integer weights uniform in 1..100, distances = all-pairs
shortest paths (int32, resident in HBM before timing), p = 90.  A step
preprocesses it (Section 2.1 tables) and runs the genetic algorithm with a
population of 1024 (NB = 4 groups of NT = 256) for 500 generations, every
fitness evaluation on the GPU.  The reported value is client x chromosome
fitness evaluations per second over the whole step.

Also reported: the evaluation kernel's algorithmic bandwidth against the HBM
peak (HIP events around each of its launches in the first generations of
every timed step), and the CPU oracle's rate on the same workload, timed on
this host's cores.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure

WORKLOAD = {
    "workload": "G900 plain GA: random connected graph n=m=900, 16200 edges, "
                "weights U{1..100}, APSP int32 distances, p=90, population 1024 "
                "(NB=4 x NT=256), 500 generations; step = preprocess + GA run",
    "n": 900, "m": 900, "p": 90, "edges": 16200, "population": 1024,
    "group_size": 256, "generations": 500,
}
PROFILE_GENS = 10
METRIC = ("client×chromosome fitness evals/s; time-to-best, plain vs "
          "learned-proposal GA")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(d, p, P, NT, budget_s):
    """The oracle GA on the same instance and parameters, a bounded number of
    generations, on all host cores it is allowed."""
    import oracle
    n = d.shape[0]
    st = oracle.GaState(n, d.shape[1], p, P, NT, 10_000, seed=12345)
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    oracle.ga_run(d, st, 1)
    one = time.perf_counter() - t0
    more = max(0, min(40, int(budget_s / max(one, 1e-3)) - 1))
    if more:
        oracle.ga_run(d, st, more)
    dt = time.perf_counter() - t0
    gens = 1 + more
    pairs = int(st.state[oracle.ST_CHROM_EVALS]) * n
    return {"value": pairs / dt, "unit": "client×chromosome evals/s",
            "cores": threads, "kind": "oracle",
            "sample": f"{gens} generations of the oracle GA on the same G900 instance "
                      f"(P={P}, NT={NT}), {pairs} client x chromosome evaluations "
                      f"in {dt:.1f} s"}


def bench_batch(args, specs, ds):
    """256 ragged instances (population 256 each): all preprocessed, then
    `--batch-generations` generations of every GA run, (a) in one persistent
    launch per step replayed from a hipGraph, (b) instance by instance with
    pmp_ga_step.  Reports instances per second of (a) and (b)."""
    import torch
    import paper_1610_10061_amd as pm
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    G = args.batch_generations
    dd = [torch.from_numpy(d).cuda() for d in ds]

    def run(batched, seed0):
        t0 = time.perf_counter()
        insts = [pm.Instance(d, s["p"], stream) for s, d in zip(specs, dd)]
        gas = [pm.GA(i, 256, 256, G, seed0 + s["index"]) for i, s in zip(insts, specs)]
        for g in gas:
            g.autotune(stream)
        t1 = time.perf_counter()
        if batched:
            bt = pm.Batch(gas)
            bt.step(G, stream)
            bt.check(stream)
        else:
            for g in gas:
                g.step(G, stream)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        pairs = 0
        costs = []
        for g in gas:
            _, c, st = g.best(stream)
            pairs += st["pair_evals"]
            costs.append(c)
        if batched:
            bt.close()
        return t1 - t0, t2 - t1, pairs, costs

    log("warm-up ...")
    run(True, 10_000)
    log("batched ...")
    prep_b, evo_b, pairs_b, costs_b = run(True, 0)
    log("one launch per instance ...")
    prep_s, evo_s, pairs_s, costs_s = run(False, 0)
    assert costs_b == costs_s, "batched and per-instance runs must agree"
    out = {
        "metric": "instances/s, 256 ragged instances x %d generations" % G,
        "value": 256 / (prep_b + evo_b),
        "unit": "instances/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batch of 256: n=m log-uniform [100,2000], p U[5,n/4], "
                               "half graphs (4n edges, weights 1..100), half Euclidean; "
                               "population 256 (NT=256), %d generations" % G},
        "batched": {"preprocess_s": prep_b, "evolve_s": evo_b,
                    "instances_per_s_evolve": 256 / evo_b,
                    "pair_evals_per_s": pairs_b / evo_b},
        "per_instance_launches": {"preprocess_s": prep_s, "evolve_s": evo_s,
                                  "instances_per_s_evolve": 256 / evo_s,
                                  "pair_evals_per_s": pairs_s / evo_s},
        "speedup_evolve": evo_s / evo_b,
        "identical_results": costs_b == costs_s,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--generations", type=int, default=WORKLOAD["generations"])
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="no per-launch events (the GA then replays hipGraphs)")
    ap.add_argument("--workload", choices=["g900", "batch"], default="g900",
                    help="g900: the headline configuration; batch: 256 ragged "
                         "instances in one launch vs one launch per instance")
    ap.add_argument("--batch-generations", type=int, default=100)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the path "
              "would shard by population across GPUs, which this build does not run.",
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "batch":
        # instances are built before anything touches the GPU (worker
        # processes must not inherit a GPU context)
        import pmp_inputs as gi
        from concurrent.futures import ProcessPoolExecutor
        specs = gi.batch_specs(256)
        log("generating 256 instances ...")
        with ProcessPoolExecutor(max_workers=8) as ex:
            ds = list(ex.map(gi.batch_instance, specs))
        return bench_batch(args, specs, ds)

    import numpy as np
    import torch

    if args.calibrate_copy:
        # 256 MiB read + 256 MiB written per copy, 4 copies
        x = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(4):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": x.numel() * 4, "copies": 4}))
        return

    import paper_1610_10061_amd as pm
    import pmp_inputs as gi

    n, p, P, NT = WORKLOAD["n"], WORKLOAD["p"], WORKLOAD["population"], WORKLOAD["group_size"]
    G = args.generations
    log(f"generating G900 instance ...")
    d = gi.graph_instance(n, WORKLOAD["edges"], seed=0)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_dev = torch.from_numpy(d).to(dev)
    stream = torch.cuda.current_stream()
    pm.lib()

    def step(seed, record):
        inst = pm.Instance(d_dev, p, stream)
        ga = pm.GA(inst, P, NT, G, seed)
        # events bracket the evaluation launches of the first PROFILE_GENS
        # generations only: an event between every pair of kernels would
        # slow the whole run down
        pg = 0 if args.no_profile else min(PROFILE_GENS, G)
        prof = None
        if pg:
            ga.profile(True)
            ga.step(pg, stream)
            prof = ga.profile_read(stream)
            ga.profile(False)
        ga.step(G - pg, stream)
        _, cost, stats = ga.best(stream)
        ga.close()
        inst.close()
        if record is not None:
            record.append((stats, prof, cost))

    for w in range(args.warmup):
        log(f"warmup step {w}")
        step(1000 + w, None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, rec)
        log(f"step {k} done: best {rec[-1][2]}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    pairs = sum(s["pair_evals"] for s, _, _ in rec)
    profs = [pr for _, pr, _ in rec if pr]
    ev_ms = sum(pr["eval_ms"] for pr in profs)
    ev_n = sum(pr["eval_launches"] for pr in profs)
    ev_bytes = sum(pr["eval_bytes"] for pr in profs)
    achieved = ev_bytes / (ev_ms / 1e3) / 1e9 if ev_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": pairs / dt,
        "unit": "client×chromosome evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / max(args.steps, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": dict(WORKLOAD, generations=G),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_eval (population evaluation)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "launches": ev_n,
            "avg_launch_us": ev_ms * 1e3 / max(ev_n, 1),
            "bytes_per_launch": ev_bytes / max(ev_n, 1),
            "sampled": f"evaluation launches of the first {PROFILE_GENS} generations of each timed step",
        },
        "best_costs": [int(c) for _, _, c in rec],
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(d, p, P, NT, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
