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

After the timed region the same run measures the other configurations
(--legs, default all): the evaluation kernel alone on Euclidean n = m = 5000
(p = 10, 100, 500; random and evolved populations of 4096), plain vs
learned-proposal GA time-to-best on fresh Euclidean n = m = 2000 seeds, and
256 ragged instances in one batched launch vs one launch sequence per
instance.  Their numbers go into the same JSON line.

The evaluation kernel's roofline is its VALU issue rate: the rocprofv3
SQ_INSTS_VALU count per (client, chromosome) pair of the same workload (the
committed counter summary, used while the kernel's sources match it) times
the pairs the sampled launches evaluated, over their measured time, against
1024 SIMDs x 2.4 GHz / 4 cycles per wave64 VALU instruction.  The bytes the
paper's untiled walk would read (2 s* + 4 per pair) are reported beside it,
labelled as such: the tiled kernel reads each row chunk once per 64
chromosomes, so they are not HBM traffic; the measured HBM traffic is.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs e5000,learned,batch|none]
python bench.py --workload batch     256 ragged instances, one launch vs many
python bench.py --workload learned   plain vs learned-proposal GA at equal
                                     wall time (Euclidean n=m=2000, p=200)
python bench.py --workload e5000     the evaluation kernel alone at E5000
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
# VALU issue: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD every
# 4 cycles (16 lanes per SIMD), 2.4 GHz peak engine clock
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9
VALU_PEAK_GIPS = SIMDS * CLOCK_HZ / 4 / 1e9  # 614.4 G wave-instructions/s

WORKLOAD = {
    "workload": "G900 plain GA: random connected graph n=m=900, 16200 edges, "
                "weights U{1..100}, APSP int32 distances, p=90, population 1024 "
                "(NB=4 x NT=256), 500 generations; step = preprocess + GA run",
    "n": 900, "m": 900, "p": 90, "edges": 16200, "population": 1024,
    "group_size": 256, "generations": 500,
}
PROFILE_GENS = 4
BATCH_PROFILE_GENS = 2  # batch generations whose evaluation launches are timed
METRIC = ("client×chromosome fitness evals/s; time-to-best, plain vs "
          "learned-proposal GA")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


COUNTERS = os.path.join(ROOT, "profiles", "k_eval_counters.json")
# sources of the evaluation kernels (k_eval, and k_stage_eval: a crossover
# stage fused with its evaluation): a change to them voids their counters
# (the summary also records the client tiles the dispatches used)
EVAL_SOURCES = ("eval_device.hpp", "k_eval.hip", "k_ga.hip", "ga_device.hpp")


def eval_sources_digest():
    """Digest of the evaluation kernel's source files."""
    import hashlib
    h = hashlib.sha256()
    for f in EVAL_SOURCES:
        with open(os.path.join(ROOT, "paper_1610_10061_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def eval_counters(case):
    """Per-dispatch counter averages of the evaluation kernel for one
    workload case from the committed rocprofv3 summary (VALU and LDS
    instructions, LDS bank-conflict cycles, HBM bytes scaled by a plain
    copy's readings, pairs per dispatch), or None when the summary is absent
    or the kernel's sources changed since it was taken."""
    try:
        with open(COUNTERS) as fh:
            c = json.load(fh)
    except (OSError, ValueError):
        return None
    if c.get("eval_sources_digest") != eval_sources_digest():
        return None
    return c.get("cases", {}).get(case)


def valu_roofline(ctr, pairs, seconds, launches):
    """VALU-issue roofline of the evaluation kernel from the counters'
    instructions per pair, the pairs evaluated and their measured time."""
    if not ctr or not seconds or not pairs:
        return {"bound": "alu", "achieved": None, "peak": VALU_PEAK_GIPS,
                "unit": "G wave64 VALU instructions/s", "frac": None, "traffic": None,
                "note": "no counter summary matching the kernel's sources and tile"}
    per_pair = ctr["SQ_INSTS_VALU"] / ctr["pairs"]
    achieved = per_pair * pairs / seconds / 1e9
    out = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GIPS,
           "unit": "G wave64 VALU instructions/s", "frac": achieved / VALU_PEAK_GIPS,
           "traffic": ctr.get("hbm_bytes")}
    avg_s = seconds / max(launches, 1)
    if ctr.get("hbm_bytes") is not None:
        gbs = ctr["hbm_bytes"] / avg_s / 1e9
        out["hbm_measured"] = {"GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    if ctr.get("SQ_INSTS_LDS"):
        out["lds"] = {"instructions_per_dispatch": ctr["SQ_INSTS_LDS"],
                      "bank_conflict_cycles_per_lds_instruction":
                          ctr.get("SQ_LDS_BANK_CONFLICT", 0) / ctr["SQ_INSTS_LDS"]}
    return out


def host_info():
    """CPU model and core count of this host."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc": usable, "os_cpu_count": os.cpu_count()}


def cpu_baseline(d, p, P, NT, budget_s):
    """The oracle on this host's cores, on the same G900 instance and GA
    parameters: the oracle GA on all cores it is allowed (the reported
    value) and on one thread, each for a bounded number of generations; the
    paper's walk of Section 4.2 on the CPU (one thread) over the population
    the GA left; and the preprocessing of Section 2.1 (the oracle's sort, and
    numpy's stable argsort, one thread)."""
    import numpy as np
    import oracle
    n, m = d.shape
    threads = oracle.default_threads()

    def ga_rate(nthreads, seconds, seed):
        st = oracle.GaState(n, m, p, P, NT, 10_000, seed=seed)
        t0 = time.perf_counter()
        oracle.ga_run(d, st, 1, threads=nthreads)
        one = time.perf_counter() - t0
        more = max(0, min(400, int(seconds / max(one, 1e-3)) - 1))
        if more:
            oracle.ga_run(d, st, more, threads=nthreads)
        dt = time.perf_counter() - t0
        pairs = int(st.state[oracle.ST_CHROM_EVALS]) * n
        return pairs / dt, 1 + more, pairs, dt, st

    rate, gens, pairs, dt, st = ga_rate(0, budget_s, 12345)
    rate1, gens1, pairs1, dt1, _ = ga_rate(1, budget_s / 3, 12345)
    out = {"value": rate, "unit": "client×chromosome evals/s",
           "cores": threads, "kind": "oracle",
           "sample": f"{gens} generations of the oracle GA on the same G900 instance "
                     f"(P={P}, NT={NT}), {pairs} client x chromosome evaluations "
                     f"in {dt:.1f} s on {threads} threads",
           "host": host_info(),
           "one_thread": {"value": rate1, "unit": "client×chromosome evals/s", "cores": 1,
                          "sample": f"{gens1} generations of the same oracle GA, "
                                    f"{pairs1} evaluations in {dt1:.1f} s"}}
    # the paper's walk on the CPU: Pi'/Delta' tables, scan to the first open
    pi, de, _ = oracle.tables(d, p)
    pop = st.pop
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.bc_eval(pi, de, pop, m)
        reps += 1
        if time.perf_counter() - t0 > 1.0:
            break
    dts = time.perf_counter() - t0
    out["pi_scan"] = {"value": reps * pop.shape[0] * n / dts,
                      "unit": "client×chromosome evals/s", "cores": 1,
                      "sample": f"{reps} walks of Section 4.2 over the {pop.shape[0]} "
                                f"chromosomes the oracle GA left, in {dts:.2f} s"}
    # preprocessing, one thread
    t0 = time.perf_counter()
    oracle.tables(d, p)
    dtp = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.tables_numpy(d, p)
    dtn = time.perf_counter() - t0
    out["preprocess"] = {"oracle_rows_per_s": n / dtp, "numpy_argsort_rows_per_s": n / dtn,
                         "cores": 1,
                         "sample": f"tables of the {n} rows of the G900 instance: oracle "
                                   f"sort {dtp * 1e3:.1f} ms, numpy stable argsort + diff "
                                   f"{dtn * 1e3:.1f} ms"}
    return out


def leg_batch(args, specs, ds):
    """256 ragged instances (population 256 each): all preprocessed, then
    `--batch-generations` generations of every GA run, (a) batched (one
    batch-wide kernel per phase, a step replayed from a hipGraph; the batch
    evaluation's client tiling timed by the batch autotuner, counted with the
    per-run tuning in the set-up time), (b) instance by instance with
    pmp_ga_step.  Reports instances per second of
    (a) and (b), and the roofline of the batch evaluation kernel from the
    first BATCH_PROFILE_GENS generations of (a), whose evaluation launches
    are timed with HIP events.  --batch-only runs (a) alone, without the
    warm-up (the command the counter runs profile)."""
    import torch
    import paper_1610_10061_amd as pm
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    G = args.batch_generations
    dd = [torch.from_numpy(d).cuda() for d in ds]

    def run(batched, seed0, profile=False):
        t0 = time.perf_counter()
        # preprocessing back to back on the device, checked once it is done
        insts = [pm.Instance(d, s["p"], stream, asynchronous=True) for s, d in zip(specs, dd)]
        gas = [pm.GA(i, 256, 256, G, seed0 + s["index"]) for i, s in zip(insts, specs)]
        for i in insts:
            i.check(stream)
        for g in gas:
            g.autotune(stream)
        common = None
        if batched:
            bt = pm.Batch(gas)
            common = bt.autotune(stream)
        t1 = time.perf_counter()
        prof = None
        if batched:
            pg = min(BATCH_PROFILE_GENS, G) if profile else 0
            if pg:
                bt.profile(True)
                bt.step(pg, stream)
                prof = bt.profile_read(stream)
                bt.profile(False)
            if G > pg:
                bt.step(G - pg, stream)
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
        return t1 - t0, t2 - t1, pairs, costs, prof, common

    if args.batch_only:
        log("batched (alone) ...")
        prep_b, evo_b, pairs_b, costs_b, prof_b, common_b = run(True, 0, profile=True)
        return {"batch_only": True, "evolve_s": evo_b, "eval_ms": prof_b[0],
                "eval_launches": prof_b[1], "batch_clients": common_b}
    log("warm-up ...")
    run(True, 10_000)
    log("batched ...")
    prep_b, evo_b, pairs_b, costs_b, prof_b, common_b = run(True, 0, profile=True)
    log("one launch per instance ...")
    prep_s, evo_s, pairs_s, costs_s, _, _ = run(False, 0)
    assert costs_b == costs_s, "batched and per-instance runs must agree"
    return {
        "metric": "instances/s, 256 ragged instances x %d generations" % G,
        "value": 256 / (prep_b + evo_b),
        "unit": "instances/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "batch of 256: n=m log-uniform [100,2000], p U[5,n/4], "
                               "half graphs (4n edges, weights 1..100), half Euclidean; "
                               "population 256 (NT=256), %d generations" % G},
        "batched": {"preprocess_s": prep_b, "evolve_s": evo_b,
                    "batch_clients": common_b,
                    "instances_per_s_evolve": 256 / evo_b,
                    "pair_evals_per_s": pairs_b / evo_b},
        "per_instance_launches": {"preprocess_s": prep_s, "evolve_s": evo_s,
                                  "instances_per_s_evolve": 256 / evo_s,
                                  "pair_evals_per_s": pairs_s / evo_s},
        "speedup_evolve": evo_s / evo_b,
        "identical_results": costs_b == costs_s,
        "roofline": batch_eval_roofline(prof_b, common_b),
    }


def batch_eval_roofline(prof, clients):
    """VALU-issue roofline of the batch evaluation kernel (k_batch_eval): the
    VALU instructions per launch that rocprofv3 counted for the same launches
    (the first BATCH_PROFILE_GENS generations of the same batched run with the
    same client tiling, case batch_eval@<clients> of the committed counter
    summary) over the launches' time
    measured here."""
    ms, launches = prof if prof else (0.0, 0)
    # counters are taken per common client tiling (a run's own tuning varies
    # from process to process, so a batch tiled by it has none)
    ctr = eval_counters(f"batch_eval@{clients}") if clients else None
    out = {"kernel": "k_batch_eval", "bound": "alu", "peak": VALU_PEAK_GIPS,
           "unit": "G wave64 VALU instructions/s", "launches": launches,
           "avg_launch_us": ms * 1e3 / max(launches, 1),
           "sampled": f"evaluation launches of the first {BATCH_PROFILE_GENS} generations of "
                      "the timed batched run (HIP events recorded by each dispatch)"}
    if not ctr or not ms or not launches or ctr.get("dispatches") != launches:
        out.update({"achieved": None, "frac": None, "traffic": None,
                    "note": "no counter summary matching the kernel's sources, the batch's "
                            f"client tiling ({clients} clients per workgroup) and launches"})
        return out
    achieved = ctr["SQ_INSTS_VALU"] * launches / (ms / 1e3) / 1e9
    out.update({"achieved": achieved, "frac": achieved / VALU_PEAK_GIPS,
                "traffic": ctr.get("hbm_bytes"),
                "counters": f"profiles/k_eval_counters.json (case batch_eval@{clients})"})
    if ctr.get("hbm_bytes") is not None:
        gbs = ctr["hbm_bytes"] / (ms / 1e3 / launches) / 1e9
        out["hbm_measured"] = {"GBps": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


LEARNED = {
    "workload": "learned proposal: Euclidean n=m=2000 on the 10^4 x 10^4 integer grid, "
                "p=200, population 1024 (NB=4 x NT=256); network trained online on "
                "training seeds, then plain vs learned GA at equal wall time on fresh seeds",
    "n": 2000, "p": 200, "population": 1024, "group_size": 256,
    "candidates": 64, "learned_iters": 4, "explore_permille": 50, "history": 4,
    "lr": 1e-3,
}


def _run_timed(pm, inst, seed, params, seconds, chunk, stream, learn_kw):
    """Step a GA (learned, starting from network parameters `params`, when
    given) for `seconds` of wall time in chunks of `chunk` generations;
    returns [(t, best, generations)] after every chunk."""
    import torch

    def make():
        ga = pm.GA(inst, LEARNED["population"], LEARNED["group_size"], 1 << 30, seed)
        model = None
        if params is not None:
            model = pm.Model(0)
            model.set_params(params)
            ga.set_model(model, **learn_kw)
        return ga, model

    ga, model = make()  # first launches (code loading) outside the clock
    ga.step(chunk, stream)
    ga.best(stream)
    ga.close()
    ga, model = make()
    torch.cuda.synchronize()
    trace = []
    t0 = time.perf_counter()
    while True:
        ga.step(chunk, stream)
        _, best, stats = ga.best(stream)
        t = time.perf_counter() - t0
        trace.append((t, best, stats["generations"]))
        if t >= seconds:
            break
    ga.close()
    return trace


def leg_learned(args):
    """Train the network online on `--train-seeds` instances, then on each
    fresh seed run the plain and the learned GA for the same wall time;
    report the time the learned GA needs to reach the plain GA's best."""
    import numpy as np
    import torch
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n, p = LEARNED["n"], LEARNED["p"]
    kw = {k: LEARNED[k] for k in ("candidates", "learned_iters", "explore_permille",
                                  "history", "lr")}
    model = pm.Model(1)
    t0 = time.perf_counter()
    for s in range(args.train_seeds):
        d = torch.from_numpy(gi.euclid_instance(n, s)).cuda()
        inst = pm.Instance(d, p, stream)
        ga = pm.GA(inst, LEARNED["population"], LEARNED["group_size"], 1 << 30, s)
        ga.set_model(model, train_every=1, **kw)
        ga.step(args.train_generations, stream)
        _, best, st = ga.best(stream)
        log(f"training seed {s}: best {best}, swaps taken {st['swap_taken']}"
            f"/{st['swap_tried']}")
        ga.close()
        inst.close()
    train_s = time.perf_counter() - t0
    rows = []
    for s in range(100, 100 + args.eval_seeds):
        d = torch.from_numpy(gi.euclid_instance(n, s)).cuda()
        inst = pm.Instance(d, p, stream)
        plain = _run_timed(pm, inst, s, None, args.seconds, 8, stream, kw)
        learned = _run_timed(pm, inst, s, model.params(), args.seconds, 8, stream,
                             dict(kw, train_every=1))
        target = plain[-1][1]
        reach = next((t for t, b, _ in learned if b <= target), None)
        rows.append({"seed": s, "plain_best": plain[-1][1], "learned_best": learned[-1][1],
                     "plain_time_s": plain[-1][0], "learned_time_s": learned[-1][0],
                     "plain_generations": plain[-1][2], "learned_generations": learned[-1][2],
                     "learned_reaches_plain_best_s": reach})
        log(json.dumps(rows[-1]))
        inst.close()
    speed = [r["plain_time_s"] / r["learned_reaches_plain_best_s"]
             for r in rows if r["learned_reaches_plain_best_s"]]
    gap = [(r["plain_best"] - r["learned_best"]) / r["plain_best"] for r in rows]
    q = lambda v: [float(np.percentile(v, x)) for x in (25, 50, 75)] if v else None  # noqa
    # network throughput: forward over a device batch of P x C rows
    X = torch.randn(1024 * 64, 32, device="cuda")
    model.forward(X)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        model.forward(X)
    e1.record()
    torch.cuda.synchronize()
    fwd_s = e0.elapsed_time(e1) / 1e3 / 20
    flops_row = 2 * (32 * 128 + 128 * 128 + 128)
    out = {
        "metric": "time-to-best, plain vs learned-proposal GA: plain GA's wall time / "
                  "learned GA's time to reach the plain GA's best (median over fresh seeds)",
        "value": q(speed)[1] if speed else None,
        "unit": "x",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32 eval / bf16-fp32 network",
        "data": "synthetic",
        "config": dict(LEARNED, train_seeds=args.train_seeds,
                       train_generations=args.train_generations,
                       eval_seeds=args.eval_seeds, seconds_per_run=args.seconds),
        "speedup_iqr": q(speed),
        "reached": f"{len(speed)}/{len(rows)}",
        "relative_gap_at_equal_time_iqr": q(gap),
        "training_s": train_s,
        "per_seed": rows,
        "mlp_forward": {"rows": X.shape[0], "seconds": fwd_s,
                        "tflops": X.shape[0] * flops_row / fwd_s / 1e12,
                        "peak_tflops_bf16": 2500.0},
    }
    if not args.no_cpu_baseline:
        import oracle.learned as OL
        Xc = X[:8192].cpu().numpy()
        t1 = time.perf_counter()
        OL.forward(model.params(), Xc)
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": Xc.shape[0] / dt, "unit": "network rows/s",
                               "cores": oracle_threads(), "kind": "oracle",
                               "sample": "oracle forward (numpy float64) of 8192 rows"}
    return out


def leg_e5000(args):
    """The evaluation kernel alone on the Euclidean n = m = 5000 instance,
    p in {10, 100, 500}, population 4096: a uniform random population, then
    the population a GA run (P = 4096, NT = 256) leaves after
    --evolve-generations generations; median of 20 timed launches (HIP
    events on the launch stream) after 3 warm-ups.  Also the preprocessing
    time of each instance.  Per case: pairs/s, the VALU-issue roofline from
    the committed counters of the same launches, the measured HBM traffic,
    and the bytes the paper's untiled walk would read."""
    import numpy as np
    import torch
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    n, P = 5000, 4096
    d = gi.euclid_instance(n, 0)
    dd = torch.from_numpy(d).cuda()
    W = gi.words_for(n)
    res = []

    def timed(inst, masks, p, kind, prep_ms):
        fit = torch.empty(P, dtype=torch.int64, device="cuda")
        scan = torch.empty(P, dtype=torch.int64, device="cuda")
        for _ in range(3):
            inst.eval(masks, fit, scan, stream, asynchronous=True)
        times = []
        for _ in range(20):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            inst.eval(masks, fit, scan, stream, asynchronous=True)
            b.record()
            times.append((a, b))
        inst.check(stream)
        ms = float(np.median([a.elapsed_time(b) for a, b in times]))
        s_tot = int(scan.sum().item())
        pairs = P * n
        byts = 2 * s_tot + 4 * pairs + P * (8 * W + 8)
        case = f"e5000_p{p}_{kind}"
        row = {"case": case, "p": p, "population": kind, "eval_ms": ms,
               "pair_evals_per_s": pairs / (ms / 1e3),
               "mean_scan": s_tot / pairs, "expected_scan_random": (n + 1) / (p + 1),
               "roofline": valu_roofline(eval_counters(case), pairs, ms / 1e3, 1),
               "paper_form_bytes": {"GBps": byts / (ms / 1e3) / 1e9,
                                    "vs_hbm_peak": byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS},
               "preprocess_ms": prep_ms, "preprocess_rows_per_s": n / (prep_ms / 1e3)}
        if kind == "random":
            import oracle
            sub = masks[:8].cpu().numpy()
            oc, os_ = oracle.objective(d, sub, p, scan=True)
            assert np.array_equal(oc, fit[:8].cpu().numpy())
            assert np.array_equal(os_, scan[:8].cpu().numpy())
        log(json.dumps(row))
        res.append(row)

    for p in (10, 100, 500):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        pm.Instance(dd, p, stream).close()  # first use outside the clock
        torch.cuda.synchronize()
        e0.record()
        inst = pm.Instance(dd, p, stream)
        e1.record()
        torch.cuda.synchronize()
        prep_ms = e0.elapsed_time(e1)
        rnd = torch.from_numpy(gi.random_population(P, n, p, 1)).cuda()
        timed(inst, rnd, p, "random", prep_ms)
        ga = pm.GA(inst, P, 256, args.evolve_generations, 0)
        ga.step(args.evolve_generations, stream)
        evolved = torch.from_numpy(ga.state()[0]).cuda()
        ga.close()
        timed(inst, evolved, p, "evolved", prep_ms)
        inst.close()
    out = {
        "metric": "client×chromosome fitness evals/s (evaluation kernel alone)",
        "value": float(np.median([r["pair_evals_per_s"] for r in res])),
        "unit": "client×chromosome evals/s",
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "E5000: Euclidean n=m=5000 on the 10^4 x 10^4 integer grid, "
                               "p in {10,100,500}, population 4096, random and evolved "
                               "(%d generations) populations" % args.evolve_generations},
        "cases": res,
    }
    if not args.no_cpu_baseline:
        import oracle
        sub = rnd[:256].cpu().numpy()
        t0 = time.perf_counter()
        oracle.objective(d, sub, 500)
        dt = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.objective(d, sub[:32], 500, threads=1)
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 256 * n / dt, "unit": "client×chromosome evals/s",
                               "cores": oracle.default_threads(), "kind": "oracle",
                               "sample": "oracle objective of 256 chromosomes (p=500)",
                               "one_thread": {"value": 32 * n / dt1, "cores": 1,
                                              "sample": "32 chromosomes (p=500)"}}
    return out


ALU_INT32_OPS = 256 * 64 * 2.4e9   # 256 CUs x 64 int32 VALU lanes x 2.4 GHz


def bench_ablation(args):
    """The three thread mappings of the evaluation (tiled; one thread per
    chromosome, the paper's choice; one thread per client, its "n threads"
    scenario) on the same random populations: G900 (p = 90, population
    1024) and E5000 (p in {10, 100, 500}, population 4096).  Median of the
    timed launches (HIP events on the launch stream); all three must give
    the same costs.  Also the load-balance statistics behind the paper's
    argument, from the exact scan lengths of a sample of chromosomes: for
    one thread per client, the mean over waves (64 clients of one
    chromosome) of the longest scan over the mean scan; for one thread per
    chromosome, the same over 64 chromosomes' total scans."""
    import numpy as np
    import torch
    import oracle
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    cases = [("G900", gi.graph_instance(900, 16200, 0), 90, 1024)]
    e5 = gi.euclid_instance(5000, 0)
    cases += [("E5000", e5, p, 4096) for p in (10, 100, 500)]
    rows = []
    for name, d, p, P in cases:
        n, m = d.shape
        W = gi.words_for(m)
        inst = pm.Instance(torch.from_numpy(d).cuda(), p, stream)
        host_masks = gi.random_population(P, m, p, 1)
        masks = torch.from_numpy(host_masks.view(np.int64)).cuda().view(torch.uint64)
        ref = None
        row = {"instance": name, "n": n, "p": p, "population": P}
        for scheme in ("tiled", "per_chromosome", "per_client"):
            fit = torch.empty(P, dtype=torch.int64, device="cuda")
            scan = torch.empty(P, dtype=torch.int64, device="cuda")
            pm.pmp_eval_population(inst.handle, masks, fit, scan, stream, True, scheme)
            inst.check(stream)
            times = []
            reps = 10
            for r in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                pm.pmp_eval_population(inst.handle, masks, fit, scan, stream, True, scheme)
                b.record()
                times.append((a, b))
                if r == 0:
                    b.synchronize()
                    if a.elapsed_time(b) > 300.0:  # slow mapping: three launches do
                        reps = 3
                if r + 1 >= reps:
                    break
            inst.check(stream)
            ms = float(np.median([a.elapsed_time(b) for a, b in times]))
            f = fit.cpu().numpy()
            if ref is None:
                ref = f
                s_tot = int(scan.sum().item())
                sub = host_masks[:8]
                oc = oracle.objective(d, sub, p)
                assert np.array_equal(oc, f[:8]), "tiled evaluation disagrees with the oracle"
            assert np.array_equal(f, ref), f"{scheme} disagrees with the tiled evaluation"
            byts = 2 * s_tot + 4 * P * n + P * (8 * W + 8)
            row[scheme] = {"ms": ms, "pair_evals_per_s": P * n / (ms / 1e3),
                           "algorithmic_GBps": byts / (ms / 1e3) / 1e9,
                           "frac_of_hbm_peak": byts / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}
            log(f"{name} p={p} {scheme}: {ms:.3f} ms")
        # exact scan lengths of 8 chromosomes: s*[c, i] = position of the
        # first open facility in client i's order (1-based)
        pi, _, _ = oracle.tables(d, p)
        bits = gi.unpack_masks(host_masks[:64], m)
        sstar = np.stack([np.argmax(bits[c][pi], axis=1) + 1 for c in range(8)])
        waves = sstar[:, : (n // 64) * 64].reshape(8, -1, 64)
        row["mean_scan"] = float(sstar.mean())
        row["per_client_wave_max_over_mean"] = float(waves.max(axis=2).mean() / sstar.mean())
        tot = np.stack([np.sum(np.argmax(bits[c][pi], axis=1) + 1) for c in range(64)])
        row["per_chromosome_wave_max_over_mean"] = float(tot.max() / tot.mean())
        row["tiled_speedup_vs_per_client"] = row["per_client"]["ms"] / row["tiled"]["ms"]
        row["tiled_speedup_vs_per_chromosome"] = row["per_chromosome"]["ms"] / row["tiled"]["ms"]
        rows.append(row)
        inst.close()
    gm = float(np.exp(np.mean([np.log(r["tiled_speedup_vs_per_client"]) for r in rows])))
    out = {"metric": "evaluation time, one thread per client / tiled (geometric mean)",
           "value": gm, "unit": "x", "n_gpus": 1, "higher_is_better": True,
           "dtype": "int32", "data": "synthetic",
           "config": {"workload": "thread-mapping ablation of the evaluation: G900 (p=90, "
                                  "population 1024) and E5000 (p in {10,100,500}, population "
                                  "4096), uniform random populations"},
           "cases": rows}
    print(json.dumps(out), flush=True)


def bench_apsp(args):
    """All-pairs shortest paths of the workloads' graphs on the GPU (blocked
    Floyd-Warshall): n = 900 with 16200 edges (G900), n = 2000 with 8000
    edges (the largest batch graph) and n = 4096 with 16384 edges.  Wall time
    of pmp_apsp on device buffers (median of 5 after a warm-up); the
    algorithmic work is n^3 min-plus updates of one add and one min each,
    against the int32 vector ALU peak.  Results are checked against the
    input generator's Dijkstra distances (n <= 2000); the CPU baseline is
    the oracle's Floyd-Warshall at n = 900."""
    import numpy as np
    import torch
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    peak = ALU_INT32_OPS / 2  # updates/s
    rows = []
    specs = [(900, 16200, 0), (2000, 8000, 7), (4096, 16384, 1)]
    for n, e, seed in specs:
        w = gi.graph_weights(n, e, seed)
        wd = torch.from_numpy(w).cuda()
        dd = torch.empty_like(wd)
        pm.pmp_apsp(wd, dd)
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pm.pmp_apsp(wd, dd)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        if n <= 2000:
            assert np.array_equal(dd.cpu().numpy(), gi.graph_instance(n, e, seed)), "APSP mismatch"
        upd = float(n) ** 3
        rows.append({"n": n, "edges": e, "ms": t * 1e3, "updates_per_s": upd / t,
                     "frac_of_alu_peak": upd / t / peak})
        log(json.dumps(rows[-1]))
    big = rows[-1]
    out = {"metric": "min-plus updates/s (all-pairs shortest paths)",
           "value": big["updates_per_s"], "unit": "updates/s", "n_gpus": 1,
           "higher_is_better": True, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "APSP of random connected graphs (weights U{1..100}): "
                                  "n=900/16200 edges, n=2000/8000, n=4096/16384"},
           "roofline": {"bound": "alu", "kernel": "k_fw_rest (with k_fw_panels)",
                        "achieved": big["updates_per_s"] * 2 / 1e12, "peak": ALU_INT32_OPS / 1e12,
                        "unit": "Tops/s (int32)", "frac": big["frac_of_alu_peak"],
                        "traffic": None},
           "cases": rows}
    if not args.no_cpu_baseline:
        import oracle
        w = gi.graph_weights(900, 16200, 0)
        t0 = time.perf_counter()
        od = oracle.apsp(w)
        dt = time.perf_counter() - t0
        assert np.array_equal(od, gi.graph_instance(900, 16200, 0))
        out["cpu_baseline"] = {"value": 900.0 ** 3 / dt, "unit": "updates/s", "cores": 1,
                               "kind": "oracle", "sample": "oracle Floyd-Warshall, n = 900"}
    print(json.dumps(out), flush=True)


def bench_hbp(args):
    """The reduced Hammer-Beresnev polynomial against the plain walk: for
    G900 (p = 90), E5000 (p = 100) and a clustered-demand instance (5000
    clients at 500 distinct sites, 500 candidate facilities, p = 50: every
    site's 10 clients give identical rows), the reduction's term counts and
    kept rows, its construction time, and the evaluation of a random
    population by both walks (median of 20 launches after 3 warm-ups, HIP
    events on the launch stream).  Algorithmic bytes: plain 2 s* + 4 per
    (client, chromosome) pair; reduced 2 s + 8 per (kept row, chromosome)
    pair (s = positions read, int64 running sums)."""
    import numpy as np
    import torch
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    sites = gi.euclid_instance(500, 9)
    clustered = np.repeat(sites, 10, axis=0)
    cases = [("G900", gi.graph_instance(900, 16200, 0), 90, 1024),
             ("E5000", gi.euclid_instance(5000, 0), 100, 4096),
             ("clustered 5000x500", clustered, 50, 4096)]
    rows = []

    def timed(fn):
        for _ in range(3):
            fn()
        ts = []
        for _ in range(20):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            ts.append((a, b))
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ts]))

    for name, d, p, P in cases:
        n, m = d.shape
        W = gi.words_for(m)
        inst = pm.Instance(torch.from_numpy(np.ascontiguousarray(d)).cuda(), p, stream)
        pm.Hbp(inst, stream).close()  # first use outside the clock
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = pm.Hbp(inst, stream)
        reduce_ms = (time.perf_counter() - t0) * 1e3
        const, T, kept, maxlen = h.info()
        _, _, _, rl = h.terms()
        masks = torch.from_numpy(gi.random_population(P, m, p, 1).view(np.int64)).cuda().view(torch.uint64)
        f1 = torch.empty(P, dtype=torch.int64, device="cuda")
        s1 = torch.empty(P, dtype=torch.int64, device="cuda")
        f2 = torch.empty_like(f1)
        s2 = torch.empty_like(s1)
        ms_plain = timed(lambda: inst.eval(masks, f1, s1, stream, asynchronous=True))
        ms_red = timed(lambda: h.eval(masks, f2, s2, stream, asynchronous=True))
        inst.check(stream)
        assert torch.equal(f1, f2), "reduced evaluation disagrees with the plain walk"
        b_plain = 2 * int(s1.sum().item()) + 4 * P * n + P * (8 * W + 8)
        b_red = 2 * int(s2.sum().item()) + 8 * P * kept + P * (8 * W + 8)
        row = {"instance": name, "n": n, "m": m, "p": p, "population": P,
               "terms_full": n * (m - p + 1), "terms_reduced": T + 1,
               "rows_kept": kept, "mean_row_len_kept": float(rl[rl > 0].mean()) if kept else 0.0,
               "reduce_ms": reduce_ms,
               "plain_ms": ms_plain, "reduced_ms": ms_red, "speedup": ms_plain / ms_red,
               "plain_bytes": b_plain, "reduced_bytes": b_red,
               "plain_GBps": b_plain / ms_plain / 1e6, "reduced_GBps": b_red / ms_red / 1e6}
        log(json.dumps(row))
        rows.append(row)
        h.close()
        inst.close()
    out = {"metric": "evaluation time, plain walk / reduced-polynomial walk",
           "value": rows[-1]["speedup"], "unit": "x", "n_gpus": 1, "higher_is_better": True,
           "dtype": "int32 / int64", "data": "synthetic",
           "config": {"workload": "reduced Hammer-Beresnev polynomial: G900 p=90 (population "
                                  "1024), E5000 p=100 and clustered demand 5000 clients at 500 "
                                  "sites x 500 facilities p=50 (population 4096); value = the "
                                  "clustered case"},
           "cases": rows}
    print(json.dumps(out), flush=True)


def bench_g100(args):
    """G100 (n = m = 100, 200 edges, p = 5; the shape of pmed1): the exact
    optimum of instance seeds 0-9 by GPU enumeration of all C(100, 5)
    subsets (the first three cross-checked with the CPU oracle), then the
    plain GA (population 64, NT 64, 100 generations, GA seed = instance seed)
    and the learned-proposal GA stepped one generation at a time until their
    best equals the optimum: generations and wall time to the optimum."""
    import numpy as np
    import torch
    import paper_1610_10061_amd as pm
    import pmp_inputs as gi
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    rows = []
    enum_s, pairs = 0.0, 0
    for s in range(args.g100_instances):
        d = gi.graph_instance(100, 200, s)
        inst = pm.Instance(torch.from_numpy(d).cuda(), 5, stream)
        if s == 0:
            pm.pmp_exhaustive(inst.handle, stream)  # first use outside the clock
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        opt, mask, count = pm.pmp_exhaustive(inst.handle, stream)
        enum_s += time.perf_counter() - t0
        pairs += count * 100
        row = {"seed": s, "optimum": opt, "subsets": count}
        if s < 3 and not args.no_cpu_baseline:
            import oracle
            t1 = time.perf_counter()
            ocost, omask, _ = oracle.exhaustive(d, 5)
            row["oracle_exhaustive_s"] = time.perf_counter() - t1
            assert ocost == opt and np.array_equal(omask, mask), "enumeration disagrees"
        for kind in ("plain", "learned"):
            ga = pm.GA(inst, 64, 64, 100, s)
            if kind == "learned":
                model = pm.Model(s)
                ga.set_model(model, candidates=64, learned_iters=3, explore_permille=50,
                             train_every=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            reached = None
            for gen in range(1, 101):
                ga.step(1, stream)
                _, best, _ = ga.best(stream)
                if best == opt:
                    reached = (gen, time.perf_counter() - t0)
                    break
            row[kind + "_generations"] = reached[0] if reached else None
            row[kind + "_ms"] = reached[1] * 1e3 if reached else None
            row[kind + "_best"] = best
            ga.close()
        log(json.dumps(row))
        rows.append(row)
        inst.close()
    med = lambda v: float(np.median(v)) if v else None  # noqa: E731
    pl = [r["plain_ms"] for r in rows if r["plain_ms"] is not None]
    le = [r["learned_ms"] for r in rows if r["learned_ms"] is not None]
    out = {
        "metric": "time to the exact optimum, plain vs learned-proposal GA (G100)",
        "value": med(pl), "unit": "ms (median over instances that reached it)",
        "n_gpus": 1, "higher_is_better": False, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "G100: random connected graph n=m=100, 200 edges, weights "
                               "U{1..100}, APSP int32, p=5, population 64 (NT=64), 100 "
                               "generations; instance and GA seeds 0-%d" % (args.g100_instances - 1)},
        "plain_reached": f"{len(pl)}/{len(rows)}", "learned_reached": f"{len(le)}/{len(rows)}",
        "learned_median_ms": med(le),
        "plain_median_generations": med([r["plain_generations"] for r in rows
                                         if r["plain_generations"] is not None]),
        "learned_median_generations": med([r["learned_generations"] for r in rows
                                           if r["learned_generations"] is not None]),
        "enumeration": {"subsets_per_instance": rows[0]["subsets"] if rows else None,
                        "seconds_per_instance": enum_s / max(len(rows), 1),
                        "pair_evals_per_s": pairs / enum_s if enum_s else None},
        "per_instance": rows,
    }
    print(json.dumps(out), flush=True)


def oracle_threads():
    import oracle
    return oracle.default_threads()


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
    ap.add_argument("--g100-instances", type=int, default=10)
    ap.add_argument("--workload", choices=["g900", "batch", "learned", "e5000", "g100",
                                           "ablation", "apsp", "hbp"],
                    default="g900",
                    help="g900: the headline configuration (plus --legs); batch: 256 "
                         "ragged instances in one launch vs one launch per instance; "
                         "learned: plain vs learned-proposal GA at equal wall time; "
                         "e5000: the evaluation kernel alone")
    ap.add_argument("--legs", default="e5000,learned,batch",
                    help="configurations measured after the headline's timed region "
                         "(comma list of e5000, learned, batch; or none)")
    ap.add_argument("--train-seeds", type=int, default=20)
    ap.add_argument("--train-generations", type=int, default=100)
    ap.add_argument("--eval-seeds", type=int, default=10)
    ap.add_argument("--evolve-generations", type=int, default=20)
    ap.add_argument("--seconds", type=float, default=2.0,
                    help="wall time of each plain / learned run (learned workload)")
    ap.add_argument("--batch-generations", type=int, default=100)
    ap.add_argument("--batch-only", action="store_true",
                    help="batch workload: the batched run alone, no warm-up or "
                         "per-instance run (what the counter runs profile)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (scales the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); runs on several "
              "GPUs are not implemented (the path would shard by population).",
              file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    for x in legs:
        if x not in ("e5000", "learned", "batch"):
            ap.error(f"unknown leg {x}")

    batch_inputs = None
    if args.workload == "batch" or (args.workload == "g900" and "batch" in legs):
        # instances are built before anything touches the GPU (worker
        # processes must not inherit a GPU context)
        import pmp_inputs as gi
        from concurrent.futures import ProcessPoolExecutor
        specs = gi.batch_specs(256)
        log("generating 256 instances ...")
        with ProcessPoolExecutor(max_workers=8) as ex:
            ds = list(ex.map(gi.batch_instance, specs))
        batch_inputs = (specs, ds)
    if args.workload == "batch":
        print(json.dumps(leg_batch(args, *batch_inputs)), flush=True)
        return
    if args.workload == "learned":
        print(json.dumps(leg_learned(args)), flush=True)
        return
    if args.workload == "e5000":
        print(json.dumps(leg_e5000(args)), flush=True)
        return
    if args.workload == "g100":
        return bench_g100(args)
    if args.workload == "ablation":
        return bench_ablation(args)
    if args.workload == "apsp":
        return bench_apsp(args)
    if args.workload == "hbp":
        return bench_hbp(args)

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
        tile = ga.autotune(stream)  # timed once per process, then cached
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
            record.append((stats, prof, cost, tile))

    for w in range(args.warmup):
        log(f"warmup step {w}")
        step(1000 + w, None)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(k, rec)
        log(f"step {k} done: best {rec[-1][2]} (tile {rec[-1][3][0]} clients, "
            f"{rec[-1][3][1]} waves)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    pairs = sum(r[0]["pair_evals"] for r in rec)
    profs = [r[1] for r in rec if r[1]]
    ev_ms = sum(pr["eval_ms"] for pr in profs)
    ev_n = sum(pr["eval_launches"] for pr in profs)
    ev_bytes = sum(pr["eval_bytes"] for pr in profs)
    ev_pairs = sum(pr["eval_pairs"] for pr in profs)
    # counters are taken per client tile of the plain evaluation (the
    # autotuner's choice; the fused launches' tile follows from the shape)
    tile = rec[0][3] if rec else (0, 0)
    roof = valu_roofline(eval_counters(f"g900_ga@{tile[0]}x{tile[1]}"), ev_pairs, ev_ms / 1e3,
                         ev_n)
    roof = dict({"bound": roof.pop("bound"),
                 "kernel": "k_stage_eval + k_eval (the crossover stages fused with their "
                           "evaluations, the population's and the mutants' evaluations)"},
                **roof)
    paper_gbs = ev_bytes / (ev_ms / 1e3) / 1e9 if ev_ms > 0 else 0.0
    roof.update({
        "launches": ev_n,
        "avg_launch_us": ev_ms * 1e3 / max(ev_n, 1),
        "pairs_per_launch": ev_pairs / max(ev_n, 1),
        "sampled": f"evaluation launches of the first {PROFILE_GENS} generations of each "
                   "timed step (HIP events recorded by each dispatch)",
        "counters": f"profiles/k_eval_counters.json (case g900_ga@{tile[0]}x{tile[1]}: this "
                    "run's tile; null fields when the evaluation kernels changed since or the "
                    "tile has no counters)",
        "paper_form_bytes": {
            "bytes_per_launch": ev_bytes / max(ev_n, 1), "GBps": paper_gbs,
            "vs_hbm_peak": paper_gbs / HBM_PEAK_GBS,
            "note": "2 s* + 4 B per pair plus 8W + 8 per chromosome, what the untiled walk "
                    "of Section 4.2 would read; the tiled kernel reads each row chunk once "
                    "per 64 chromosomes, so this is not HBM traffic; s* from the kernel's "
                    "own scan count (checked against the oracle by the parity tests)"},
    })
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
        "roofline": roof,
        "best_costs": [int(r[2]) for r in rec],
        "eval_tile": {"clients": rec[0][3][0], "waves": rec[0][3][1]} if rec else None,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(d, p, P, NT, args.cpu_seconds)
    # the other configurations, outside the timed region
    out["legs"] = {}
    if "e5000" in legs:
        log("E5000 evaluation leg ...")
        out["legs"]["e5000"] = leg_e5000(argparse.Namespace(**dict(
            vars(args), no_cpu_baseline=True)))
    if "learned" in legs:
        log("learned-proposal leg ...")
        out["legs"]["learned"] = leg_learned(argparse.Namespace(**dict(
            vars(args), train_seeds=4, train_generations=60, eval_seeds=5, seconds=1.0,
            no_cpu_baseline=True)))
        out["time_to_best"] = {k: out["legs"]["learned"].get(k) for k in
                               ("metric", "value", "unit", "speedup_iqr", "reached",
                                "relative_gap_at_equal_time_iqr")}
    if "batch" in legs:
        log("batch leg ...")
        out["legs"]["batch"] = leg_batch(args, *batch_inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
