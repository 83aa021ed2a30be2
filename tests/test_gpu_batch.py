"""Batched GA (one persistent launch for many instances) and the evaluation
tile autotuner, on the GPU.

A batch step must leave every run exactly as stepping it alone would: same
Philox streams, same integer decisions.  Each batched run is compared with
the same run stepped on its own (per-step kernels) and, where the oracle
finishes in seconds, with the oracle GA.
"""
import os

import numpy as np
import pytest

import oracle
import pmp_inputs as gi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1610_10061_amd as pm
    pm.lib()
    return pm


def _say(*a):
    print(*a, flush=True)


def _state(ga):
    pop, fit, gm, gc = ga.state()
    mask, cost, stats = ga.best()
    return pop, fit, gm, gc, mask, cost, stats


def _assert_same(a, b):
    for x, y in zip(a[:6], b[:6]):
        np.testing.assert_array_equal(x, y)
    for k in ("generations", "saturation_count", "done", "chromosome_evals",
              "crossover_fail", "crossover_taken", "mutation_taken", "scan_total"):
        assert a[6][k] == b[6][k], k


def _mini_batch():
    """Ragged shapes: graph and Euclidean, n != m, small and large p, p = 1
    (no crossover), several group sizes and stage counts, m past 64, both
    migration variants, both ways of generating chromosomes."""
    rng = np.random.default_rng(3)
    cases = []
    for k, (kind, n, m, p, P, NT, X, Y, sat, mig, init) in enumerate([
            ("graph", 60, 60, 4, 64, 16, 0, 0, 0, 1, 1),
            ("euclid", 90, 90, 9, 128, 64, 0, 0, 3, 0, 0),
            ("rand", 37, 150, 20, 64, 32, 5, 2, 0, 0, 0),
            ("euclid", 200, 200, 1, 32, 8, 0, 0, 0, 1, 0),
            ("graph", 130, 130, 30, 256, 256, 0, 0, 0, 0, 0),
            ("rand", 20, 300, 150, 64, 64, 2, 9, 0, 0, 0),
            ("euclid", 70, 70, 5, 8, 1, 0, 0, 2, 0, 1),
            ("graph", 80, 80, 6, 256, 8, 0, 0, 0, 1, 1)]):
        if kind == "graph":
            d = gi.graph_instance(n, 2 * n, 100 + k)
        elif kind == "euclid":
            d = gi.euclid_instance(n, 100 + k)
        else:
            d = rng.integers(0, 500, size=(n, m)).astype(np.int32)
        cases.append((d, p, P, NT, X, Y, sat, 7 + k, mig, init))
    return cases


def _make(pm, cases, G):
    insts, gas = [], []
    for d, p, P, NT, X, Y, sat, seed, mig, init in cases:
        inst = pm.Instance(d, p)
        insts.append(inst)
        gas.append(pm.GA(inst, P, NT, G, seed, sat, X, Y, mig, init))
    return insts, gas


@pytest.mark.parametrize("graph", ["1", "0"])
@pytest.mark.parametrize("bmode", ["kernels", "persistent"])
def test_batch_equals_single_runs_and_oracle(pm, graph, bmode):
    old = {k: os.environ.get(k) for k in ("PMP_BATCH_GRAPH", "PMP_GA_MODE", "PMP_BATCH_MODE")}
    os.environ["PMP_BATCH_GRAPH"] = graph
    os.environ["PMP_GA_MODE"] = "kernels"
    os.environ["PMP_BATCH_MODE"] = bmode
    try:
        cases = _mini_batch()
        G = 6
        _say("mini batch of", len(cases), "graph", graph, "mode", bmode)
        insts, gas = _make(pm, cases, G)
        batch = pm.Batch(gas)
        batch.step(3)
        batch.step(3)  # the same generation count replays the captured graph
        batch.check()
        rinsts, refs = _make(pm, cases, G)
        for r in refs:
            r.step(G)
        for (d, p, P, NT, X, Y, sat, seed, mig, init), ga, ref in zip(cases, gas, refs):
            a, b = _state(ga), _state(ref)
            _assert_same(a, b)
            st = oracle.GaState(d.shape[0], d.shape[1], p, P, NT, G, seed, sat, X, Y, mig, init)
            oracle.ga_run(d, st, G)
            np.testing.assert_array_equal(a[0], st.pop)
            assert a[5] == st.best_cost
        batch.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_batch_small_grid_loops_every_phase(pm):
    old = os.environ.get("PMP_GA_BLOCKS")
    os.environ["PMP_GA_BLOCKS"] = "8"
    os.environ["PMP_BATCH_MODE"] = "persistent"
    try:
        cases = _mini_batch()
        insts, gas = _make(pm, cases, 4)
        batch = pm.Batch(gas)
        batch.step(4)
        assert batch.check() == 8
        rinsts, refs = _make(pm, cases, 4)
        for r in refs:
            r.step(4)
        for ga, ref in zip(gas, refs):
            _assert_same(_state(ga), _state(ref))
        batch.close()
    finally:
        os.environ.pop("PMP_BATCH_MODE", None)
        if old is None:
            os.environ.pop("PMP_GA_BLOCKS", None)
        else:
            os.environ["PMP_GA_BLOCKS"] = old


def test_step_batch_convenience_and_stopped_runs(pm):
    cases = _mini_batch()[:3]
    insts, gas = _make(pm, cases, 2)  # EvolveLimit 2: stepping 5 stops at 2
    pm.pmp_ga_step_batch([g.handle for g in gas], 5)
    for ga in gas:
        _, _, stats = ga.best()
        assert stats["generations"] == 2 and stats["done"] == 1


def test_autotune_keeps_results(pm):
    d = gi.euclid_instance(700, 5)
    inst = pm.Instance(d, 40)
    a = pm.GA(inst, 512, 128, 3, seed=1)
    chosen, waves = a.autotune()
    # the shape's default tile, or one of the timed candidates
    assert 1 <= chosen <= 700 and waves in (4, 8, 16)
    b = pm.GA(inst, 512, 128, 3, seed=1)
    os.environ["PMP_CLIENTS_PER_BLOCK"] = "4"
    try:
        b.autotune()  # forced tile
    finally:
        os.environ.pop("PMP_CLIENTS_PER_BLOCK")
    a.step(3)
    b.step(3)
    _assert_same(_state(a), _state(b))
    with pytest.raises(pm.PmpError):
        a.autotune()  # after the first generation


def test_full_batch_config(pm):
    """The ragged 256-instance configuration (n = m log-uniform in
    [100, 2000], p uniform in [5, n/4], half graphs with 4n edges, half
    Euclidean, population 256) stepped in one launch per call, as the
    benchmark runs it.  Every run is compared with the same run stepped
    alone, and 16 runs spread over the range of n with the oracle GA."""
    specs = gi.batch_specs(256)
    _say("generating 256 instances")
    ds = [gi.batch_instance(s) for s in specs]
    G = 2
    insts, gas = [], []
    for s, d in zip(specs, ds):
        inst = pm.Instance(d, s["p"])
        insts.append(inst)
        ga = pm.GA(inst, 256, 256, 100, seed=s["index"])
        ga.autotune()
        gas.append(ga)
    _say("batch autotune")
    batch = pm.Batch(gas)
    clients = batch.autotune()
    _say("batch step, clients per workgroup", clients)
    batch.step(G)
    batch.check()
    by_n = sorted(range(256), key=lambda b: specs[b]["n"])
    # 16 runs at evenly spaced ranks of n, smallest and largest included
    with_oracle = {by_n[round(k * 255 / 15)] for k in range(16)}
    for b in range(256):
        s = specs[b]
        ref_inst = pm.Instance(ds[b], s["p"])
        ref = pm.GA(ref_inst, 256, 256, 100, seed=b)
        ref.step(G)
        a = _state(gas[b])
        _assert_same(a, _state(ref))
        ref.close()
        ref_inst.close()
        if b in with_oracle:
            _say("oracle run", b, "n", s["n"], "p", s["p"], s["kind"])
            st = oracle.GaState(s["n"], s["n"], s["p"], 256, 256, 100, b)
            oracle.ga_run(ds[b], st, G)
            np.testing.assert_array_equal(a[0], st.pop)
            np.testing.assert_array_equal(a[1], st.fit)
            assert a[5] == st.best_cost
            assert a[6]["chromosome_evals"] == st.state[oracle.ST_CHROM_EVALS]
    batch.close()


@pytest.mark.parametrize("how", ["autotuned", "common512", "common96_persistent"])
def test_batch_client_tiling_keeps_results(pm, how):
    """The batch evaluation's client tiling (each run's own tuning, or a
    common count of clients per workgroup, timed by the batch autotuner or
    set by hand) changes no run: every batched run equals the run stepped
    alone.  The autotuner applies a cached choice at any time and refuses to
    time a batch past its first step."""
    keys = ("PMP_BATCH_CLIENTS", "PMP_BATCH_MODE")
    old = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ.pop(k, None)
    if how == "common512":
        os.environ["PMP_BATCH_CLIENTS"] = "512"
    elif how == "common96_persistent":
        os.environ["PMP_BATCH_CLIENTS"] = "96"
        os.environ["PMP_BATCH_MODE"] = "persistent"
    try:
        cases = _mini_batch()
        G = 5
        insts, gas = _make(pm, cases, G)
        for g in gas:
            g.autotune()
        batch = pm.Batch(gas)
        clients = batch.autotune()
        _say(how, "clients per workgroup", clients)
        if how == "autotuned":
            assert clients in (0, 64, 96, 128, 192, 256, 384, 512)
        else:
            assert clients == int(os.environ["PMP_BATCH_CLIENTS"])
        batch.step(2)
        batch.step(3)
        batch.check()
        if how == "autotuned":
            # a cached choice applies between steps; a choice to be timed
            # needs runs before their first generation
            assert batch.autotune() == clients
            sub_insts, sub = _make(pm, cases[:3], G)
            sb = pm.Batch(sub)
            sb.step(1)
            with pytest.raises(pm.PmpError) as e:
                sb.autotune()
            assert e.value.status == pm.PMP_EINVAL
            sb.close()
        rinsts, refs = _make(pm, cases, G)
        for r in refs:
            r.step(G)
        for ga, ref in zip(gas, refs):
            _assert_same(_state(ga), _state(ref))
        batch.close()
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_batch_profiled_steps_keep_results(pm):
    """Profiled batch steps (launched directly, the evaluation launches
    bracketed by events) evolve every run as the unprofiled ones, and count
    one evaluation launch per stage and generation."""
    old = os.environ.get("PMP_BATCH_MODE")
    os.environ.pop("PMP_BATCH_MODE", None)
    try:
        cases = _mini_batch()
        G = 5
        _say("profiled mini batch of", len(cases))
        insts, gas = _make(pm, cases, G)
        batch = pm.Batch(gas)
        batch.profile(True)
        batch.step(2)
        ms, launches = batch.profile_read()
        batch.profile(False)
        batch.step(3)
        batch.check()
        # every generation launches the same number of evaluations
        assert ms > 0 and launches >= 2 and launches % 2 == 0
        rinsts, refs = _make(pm, cases, G)
        for r in refs:
            r.step(G)
        for ga, ref in zip(gas, refs):
            _assert_same(_state(ga), _state(ref))
        batch.close()
    finally:
        if old is not None:
            os.environ["PMP_BATCH_MODE"] = old
