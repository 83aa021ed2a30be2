"""GPU parity of the genetic algorithm (pmp_ga_step) with the oracle GA.

Both sides draw every random choice from the same Philox counters and take
every decision on exact integer fitness, so after k generations the whole
state (population, fitness, group bests, global best and counters) must be
identical bit for bit.
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


# launch schemes: per-step kernels replayed from a hipGraph of 2 generations
# (the default scheme, with a chunk small enough to replay here), the same
# with every chromosome's mutants made by one wave, per-step kernels launched
# one by one, the per-step kernels with the mutation cycle run attempt by
# attempt instead of at once, one persistent cooperative kernel, and the same
# with a grid of 8 workgroups (every phase loops)
MODES = {"graph": {"PMP_GA_GRAPH_GENS": "2"},
         "graph_16_waves": {"PMP_GA_GRAPH_GENS": "2", "PMP_EVAL_WAVES": "16"},
         "kernels_8_waves": {"PMP_GA_MODE": "kernels", "PMP_EVAL_WAVES": "8"},
         "graph_mutants_1_wave": {"PMP_GA_GRAPH_GENS": "2", "PMP_MUTANTS_PER_WAVE": "64"},
         "kernels": {"PMP_GA_MODE": "kernels"},
         "sequential": {"PMP_GA_GRAPH_GENS": "2", "PMP_GA_SPEC": "0"},
         "persistent": {"PMP_GA_MODE": "persistent"},
         "persistent_8wg": {"PMP_GA_MODE": "persistent", "PMP_GA_BLOCKS": "8"}}
_ENV = ("PMP_GA_MODE", "PMP_GA_BLOCKS", "PMP_GA_GRAPH_GENS", "PMP_GA_SPEC",
        "PMP_MUTANTS_PER_WAVE", "PMP_EVAL_WAVES")


@pytest.fixture(params=list(MODES))
def mode(request):
    old = {k: os.environ.get(k) for k in _ENV}
    for k in old:
        os.environ.pop(k, None)
    os.environ.update(MODES[request.param])
    yield request.param
    for k, v in old.items():
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = v


def _compare(pm, d, p, P, NT, G, seed, steps, sat=0, X=0, Y=0, mig=0, init=0):
    n, m = d.shape
    print("case", d.shape, "p", p, "P", P, "NT", NT, "steps", steps, "seed", seed,
          "migration", mig, "init", init, "mode", {k: os.environ.get(k) for k in _ENV},
          flush=True)
    inst = pm.Instance(d, p)
    ga = pm.GA(inst, P, NT, G, seed, sat, X, Y, mig, init)
    st = oracle.GaState(n, m, p, P, NT, G, seed, sat, X, Y, mig, init)
    for k in steps:
        ga.step(k)
        oracle.ga_run(d, st, k)
    pop, fit, gm, gc = ga.state()
    mask, cost, stats = ga.best()
    np.testing.assert_array_equal(pop, st.pop)
    np.testing.assert_array_equal(fit, st.fit)
    np.testing.assert_array_equal(gm, st.gbest_mask)
    np.testing.assert_array_equal(gc, st.gbest_cost)
    np.testing.assert_array_equal(mask, st.best_mask)
    assert cost == st.best_cost
    assert stats["generations"] == st.state[oracle.ST_GEN]
    assert stats["saturation_count"] == st.state[oracle.ST_SAT]
    assert stats["done"] == st.state[oracle.ST_DONE]
    assert stats["chromosome_evals"] == st.state[oracle.ST_CHROM_EVALS]
    assert stats["crossover_fail"] == st.state[oracle.ST_XO_FAIL]
    assert stats["crossover_taken"] == st.state[oracle.ST_XO_TAKEN]
    assert stats["mutation_taken"] == st.state[oracle.ST_MUT_TAKEN]
    assert stats["pair_evals"] == stats["chromosome_evals"] * n
    # the reported best is what its mask costs
    assert oracle.objective(d, mask[None], p)[0] == cost
    return stats


def test_ga_g100_config(pm, mode):
    """Graph n = m = 100, 200 edges, p = 5, population 64 (one group)."""
    d = gi.graph_instance(100, 200, 0)
    _compare(pm, d, 5, 64, 64, 100, seed=1, steps=[4])


def test_ga_g20_groups_saturation(pm, mode):
    d = gi.graph_instance(20, 40, 0)
    s = _compare(pm, d, 4, 32, 8, 500, seed=7, steps=[40, 40], sat=6)
    assert s["done"] == 1


def test_ga_example1_tiny(pm, mode):
    _compare(pm, gi.example1_matrix(), 2, 8, 4, 5, seed=3, steps=[2, 3])


def test_ga_p1_has_no_crossover(pm, mode):
    d = gi.euclid_instance(70, 3)
    s = _compare(pm, d, 1, 16, 16, 3, seed=2, steps=[3])
    assert s["crossover_taken"] == 0 and s["crossover_fail"] == 0


def test_ga_preset_iteration_counts(pm, mode):
    """More crossover stages than lg NT cycle the strides again."""
    d = gi.euclid_instance(150, 8)
    _compare(pm, d, 12, 64, 16, 4, seed=5, steps=[2], X=9, Y=2)


def test_ga_ragged_m_and_resume(pm, mode):
    d = np.random.default_rng(4).integers(0, 50, size=(77, 131)).astype(np.int32)
    _compare(pm, d, 17, 128, 32, 8, seed=11, steps=[1, 2, 4])


def test_ga_g900_full_config(pm, mode):
    """Graph n = m = 900, 16200 edges, p = 90, population 1024 (NT = 256),
    the benchmark's configuration, two generations."""
    d = gi.graph_instance(900, 16200, 0)
    _compare(pm, d, 90, 1024, 256, 500, seed=0, steps=[2])


def test_ga_euclid_1000(pm, mode):
    d = gi.euclid_instance(1000, 1)
    _compare(pm, d, 50, 512, 128, 3, seed=9, steps=[1])


def test_solve_returns_consistent_best(pm):
    d = gi.graph_instance(20, 40, 1)
    open_, cost, stats = pm.pmp_solve(d, 4, 32, 8, 30, seed=2, saturation=5)
    assert open_.sum() == 4
    mask = gi.pack_masks(open_[None].astype(bool), 20)
    assert oracle.objective(d, mask, 4)[0] == cost
    best, _, _ = oracle.exhaustive(d, 4)
    assert cost >= best


def test_ga_m4096_two_words_per_lane(pm, mode):
    """m above 4096: each lane of the operator waves owns two words."""
    d = np.random.default_rng(12).integers(0, 1000, size=(40, 4500)).astype(np.int32)
    _compare(pm, d, 300, 64, 16, 3, seed=4, steps=[2])


def test_ga_group_of_one(pm, mode):
    """NT = 1: no crossover, no mutation (lg NT = 0); random restarts with
    migration only."""
    d = gi.euclid_instance(60, 2)
    s = _compare(pm, d, 6, 8, 1, 4, seed=6, steps=[4])
    assert s["crossover_taken"] == 0 and s["mutation_taken"] == 0


@pytest.mark.parametrize("P,NT", [(128, 32), (64, 8), (256, 8)],
                         ids=["NB<NT", "NB=NT", "NB>NT"])
def test_ga_migration_to_one_block(pm, mode, P, NT):
    """The other migration variant: every group best goes to slots 0..NB-1
    (one block when NB <= NT, the first NB / NT blocks otherwise)."""
    d = gi.graph_instance(100, 200, 2)
    _compare(pm, d, 5, P, NT, 20, seed=13, steps=[1, 3, 2], mig=1)


def test_ga_rejects_unknown_migration(pm):
    inst = pm.Instance(gi.graph_instance(20, 40, 0), 4)
    with pytest.raises(pm.PmpError):
        pm.GA(inst, 32, 8, 5, 1, migration=2)


def test_ga_init_by_rank(pm, mode):
    """Chromosomes generated from uniform lexicographic ranks (Section 4.1)
    in every launch scheme: fresh slots each generation, with migrants."""
    d = gi.graph_instance(100, 200, 4)
    _compare(pm, d, 5, 128, 16, 10, seed=17, steps=[1, 4], init=1)


@pytest.mark.parametrize("n,m,p", [(40, 62, 31), (40, 300, 4), (40, 130, 127),
                                   (32, 5000, 3), (30, 67, 1)],
                         ids=["C(62,31)", "m=300", "p=m-3", "m=5000", "p=1"])
def test_ga_init_by_rank_shapes(pm, n, m, p):
    """Ranks up to 4.7e17, candidates that run past one 64-lane batch, subsets
    that fill almost every slot, and words past 64 (the second word register
    of each lane)."""
    d = np.random.default_rng(m * 7 + p).integers(0, 300, size=(n, m)).astype(np.int32)
    _compare(pm, d, p, 64, 8, 3, seed=31, steps=[2], init=1)


def test_ga_init_by_rank_rejects(pm):
    inst = pm.Instance(gi.graph_instance(100, 200, 0), 50)
    with pytest.raises(pm.PmpError):  # C(100, 50) is past 2^63
        pm.GA(inst, 32, 8, 5, 1, init=1)
    with pytest.raises(pm.PmpError):
        pm.GA(inst, 32, 8, 5, 1, init=2)


@pytest.mark.parametrize("m,p", [(150, 147), (130, 129), (200, 129)],
                         ids=["p=m-3", "p=m-1", "p=129"])
def test_ga_dense_subsets(pm, m, p):
    """Populations where most of Floyd's draws collide: chains of repeated
    draws inside and across the sampler's 64-draw batches."""
    d = np.random.default_rng(m + p).integers(0, 200, size=(40, m)).astype(np.int32)
    _compare(pm, d, p, 64, 16, 3, seed=21, steps=[2])


def test_mutation_cycle_at_once_counts(pm, mode):
    """Evaluating the mutation cycle at once evaluates mutants beyond the
    first improvement (counted apart); attempt by attempt it does not.  The
    algorithm's own counters match the oracle either way (_compare)."""
    d = gi.graph_instance(100, 200, 3)
    s = _compare(pm, d, 5, 128, 32, 10, seed=2, steps=[3])
    if mode in ("graph", "graph_mutants_1_wave", "kernels", "graph_16_waves", "kernels_8_waves"):
        assert s["speculative_evals"] > 0
    else:
        assert s["speculative_evals"] == 0


def test_ga_paper_preset_counts(pm, mode):
    """The preset iteration counts of the paper's runs (60 crossover stages,
    20 mutation attempts): crossover strides cycle, and the mutation cycle
    evaluated at once takes 32 lanes per chromosome."""
    d = gi.graph_instance(60, 150, 5)
    _compare(pm, d, 6, 64, 16, 3, seed=8, steps=[2], X=60, Y=20)


def test_ga_paired_walk_with_long_scans(pm):
    """The GA with the two-clients-per-chunk walk forced on an instance whose
    rows often reach past 32 entries (G100, p = 5)."""
    old = os.environ.get("PMP_EVAL_PAIRED")
    os.environ["PMP_EVAL_PAIRED"] = "1"
    try:
        d = gi.graph_instance(100, 200, 6)
        _compare(pm, d, 5, 128, 32, 6, seed=4, steps=[3])
    finally:
        if old is None:
            os.environ.pop("PMP_EVAL_PAIRED", None)
        else:
            os.environ["PMP_EVAL_PAIRED"] = old


def test_ga_population_made_ahead_across_launch_schemes(pm):
    """The per-step schedule makes each next generation's population in the
    launch of the current one's resolve step (the cycle at once, even X and
    X + Y).  Runs that switch to the batch kernels, re-tune the evaluation
    tile or replay graphs in between must still match the oracle bit for bit
    (the batch kernels make their own populations; the autotuner samples
    generation 0 before the run)."""
    old = os.environ.get("PMP_GA_GRAPH_GENS")
    os.environ["PMP_GA_GRAPH_GENS"] = "2"
    try:
        d = gi.graph_instance(100, 200, 7)
        n, m = d.shape
        p, P, NT, G, seed = 5, 256, 64, 50, 23  # X = Y = lg 64 = 6
        print("case G100 p", p, "P", P, "NT", NT, "seed", seed, flush=True)
        inst = pm.Instance(d, p)
        ga = pm.GA(inst, P, NT, G, seed)
        st = oracle.GaState(n, m, p, P, NT, G, seed, 0, 0, 0, 0, 0)
        ga.autotune()                            # samples generation 0
        ga.step(3)                               # graph replay + one generation
        pm.pmp_ga_step_batch([ga.handle], 2)     # the batch kernels
        ga.step(1)
        ga.step(4)                               # graphs again
        oracle.ga_run(d, st, 10)
        pop, fit, gm, gc = ga.state()
        np.testing.assert_array_equal(pop, st.pop)
        np.testing.assert_array_equal(fit, st.fit)
        np.testing.assert_array_equal(gm, st.gbest_mask)
        np.testing.assert_array_equal(gc, st.gbest_cost)
        mask, cost, stats = ga.best()
        np.testing.assert_array_equal(mask, st.best_mask)
        assert cost == st.best_cost
        assert stats["generations"] == st.state[oracle.ST_GEN] == 10
        assert stats["chromosome_evals"] == st.state[oracle.ST_CHROM_EVALS]
    finally:
        if old is None:
            os.environ.pop("PMP_GA_GRAPH_GENS", None)
        else:
            os.environ["PMP_GA_GRAPH_GENS"] = old
