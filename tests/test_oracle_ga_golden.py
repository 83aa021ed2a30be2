"""The oracle GA against a worked derivation of whole generations
(tests/golden/ga_generation.json, written by derive_ga_generation.py next to
it, which shares nothing with oracle/): every random word is re-checked
against numpy's Philox, every bounded draw against exact integer
arithmetic, every operator of the oracle against the recorded parameters and
offspring, and the oracle's state after each generation against the recorded
one.  This pins the GA trajectory from outside the oracle (Section 3.2
Evolve steps 1-8, Sections 4.1, 4.3-4.5): drawing a pair's parameters from
the wrong slot, accepting equal costs, or reading a partner that was already
replaced in the same stage each changes a recorded decision.

Also Lemire's bounded draw in its rejection branch, against a big-integer
reference fed by numpy's Philox words.
"""
import json
import os

import numpy as np
import pytest

import oracle
import pmp_inputs as gi

HERE = os.path.dirname(os.path.abspath(__file__))
M64 = (1 << 64) - 1


@pytest.fixture(scope="module")
def golden():
    with open(os.path.join(HERE, "golden", "ga_generation.json")) as f:
        return json.load(f)


def _numpy_block(key, ctr):
    c = sum(int(w) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & M64 for k in range(4)], dtype=np.uint64)
    g = np.random.Philox(counter=words, key=np.array(key, dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


def _stream_words(rec, count):
    key, c3 = rec["stream"]["key"], rec["stream"]["counter"]
    out, blk = [], 0
    while len(out) < count:
        out += _numpy_block(key, c3 + [blk])
        blk += 1
    return out[:count]


def _records(case):
    for g in case["trace"]:
        for r in g["population"]:
            if "draws" in r:
                yield r
        for st in g["crossover"]:
            yield from st["pairs"]
        for at in g["mutation"]:
            yield from at["slots"]


def _mask(opened, m):
    return gi.pack_masks([opened], m)[0]


def test_golden_draws_are_numpy_philox_and_lemire(golden):
    n_draws = 0
    for case in golden["cases"]:
        for rec in _records(case):
            words = [int(w, 16) for d in rec["draws"] for w in d["words"]]
            assert words == _stream_words(rec, len(words))
            for d in rec["draws"]:
                r, x = d["bound"], int(d["words"][-1], 16)
                assert d["value"] == (x * r) >> 64
                assert (x * r) & M64 >= ((1 << 64) - r) % r
                n_draws += 1
    assert n_draws > 300


def test_golden_costs_are_the_papers_objective(golden):
    """Example 1's recorded costs are the values of its printed polynomial
    (Section 2.1): {1,2} 43, {1,3} 37, {1,4} 35, {2,3} 46, {2,4} 40, {3,4} 44
    (1-based)."""
    printed = {(0, 1): 43, (0, 2): 37, (0, 3): 35, (1, 2): 46, (1, 3): 40, (2, 3): 44}
    case = golden["cases"][0]
    assert case["name"] == "example1"
    seen = 0
    for g in case["trace"]:
        for r, f in zip(g["population"], g["fitness_after_population"]):
            assert printed[tuple(r["open"])] == f
            seen += 1
        for rec in _records(case):
            if rec.get("offspring_cost") is not None:
                assert printed[tuple(rec["offspring"])] == rec["offspring_cost"]
                seen += 1
    assert seen > 20


def test_golden_holds_the_decisions_that_pin_the_trajectory(golden):
    """The recorded run contains what tells the plausible mistakes apart:
    offspring exactly as cheap as their parents (not taken), pairs whose
    upper partner would get another offspring from parameters drawn from
    its own stream, and pairs whose lower partner's offspring is taken (a
    stage run slot by slot would hand the upper partner that offspring)."""
    ties = own_differs = lower_taken = 0
    for case in golden["cases"]:
        m, p = len(case["d"][0]), case["p"]
        for g in case["trace"]:
            for st in g["crossover"]:
                start = _stage_start(g, st["stage"])
                by_slot = {x["slot"]: x for x in st["pairs"]}
                for x in st["pairs"]:
                    if x.get("offspring_cost") is not None and \
                            x["offspring_cost"] == x["parent_cost"]:
                        ties += 1
                    if x["slot"] < x["partner"]:
                        continue
                    lower_taken += bool(by_slot[x["partner"]].get("taken"))
                    w = _numpy_block([case["seed"], 2],
                                     [g["generation"], x["slot"],
                                      (2 << 32) | st["stage"], 0])
                    r1, i = (w[0] * m) >> 64, 1 + ((w[1] * (p // 2)) >> 64)
                    ok, F = oracle.crossover(_mask(start[x["slot"]], m),
                                             _mask(start[x["partner"]], m), m, r1, i)
                    rec = x["offspring"]
                    if ok != (rec is not None) or (ok and not np.array_equal(F, _mask(rec, m))):
                        own_differs += 1
    assert ties >= 5 and lower_taken >= 5 and own_differs >= 3, \
        (ties, lower_taken, own_differs)


@pytest.mark.parametrize("ci", [0, 1])
def test_oracle_operators_match_golden(golden, ci):
    case = golden["cases"][ci]
    m, p, seed = len(case["d"][0]), case["p"], case["seed"]
    for g in case["trace"]:
        gen = g["generation"]
        for r in g["population"]:
            if "draws" in r:
                got = oracle.sample_subset(seed, gen, r["slot"], m, p)
                np.testing.assert_array_equal(got, _mask(r["open"], m))
        for st in g["crossover"]:
            pop = _stage_start(g, st["stage"])   # parents as the stage found them
            for x in st["pairs"]:
                A, B = _mask(pop[x["slot"]], m), _mask(pop[x["partner"]], m)
                ok, F = oracle.crossover(A, B, m, x["r1"], x["i"])
                assert ok == (x["offspring"] is not None)
                if ok:
                    np.testing.assert_array_equal(F, _mask(x["offspring"], m))
        parent = {c: o for c, o in enumerate(g["crossover"][-1]["after"]["population"])}
        for at in g["mutation"]:
            for x in at["slots"]:
                F, desc = oracle.mutate(seed, gen, x["slot"], at["attempt"],
                                        _mask(parent[x["slot"]], m), m)
                np.testing.assert_array_equal(F, _mask(x["offspring"], m))
                mv = x["move"]
                if mv["kind"] == "circular":
                    assert desc[0] == 0 and desc[4] == mv["s"]
                else:
                    assert desc[0] == 1 and desc[2:] == (mv["a"], mv["b"], mv["s"])
                assert desc[1] == (0 if mv["dir"] == "right" else 1)


def _stage_start(g, k):
    if k == 0:
        return [r["open"] for r in g["population"]]
    return g["crossover"][k - 1]["after"]["population"]


@pytest.mark.parametrize("ci", [0, 1])
def test_oracle_ga_run_matches_golden(golden, ci):
    case = golden["cases"][ci]
    d = np.array(case["d"], np.int32)
    n, m = d.shape
    st = oracle.GaState(n, m, case["p"], case["P"], case["NT"], case["generations"],
                        seed=case["seed"])
    for g in case["trace"]:
        oracle.ga_run(d, st, 1)
        end = g["end"]
        want = np.stack([_mask(o, m) for o in end["population"]])
        np.testing.assert_array_equal(st.pop, want)
        np.testing.assert_array_equal(st.fit, end["fitness"])
        np.testing.assert_array_equal(st.gbest_cost, [x["cost"] for x in end["group_bests"]])
        np.testing.assert_array_equal(
            st.gbest_mask, np.stack([_mask(x["open"], m) for x in end["group_bests"]]))
        assert st.best_cost == end["global_best"]["cost"]
        np.testing.assert_array_equal(st.best_mask, _mask(end["global_best"]["open"], m))
        c = end["counters"]
        assert st.state[oracle.ST_CHROM_EVALS] == c["evals"]
        assert st.state[oracle.ST_XO_FAIL] == c["xo_fail"]
        assert st.state[oracle.ST_XO_TAKEN] == c["xo_taken"]
        assert st.state[oracle.ST_MUT_TAKEN] == c["mut_taken"]


# ------------------------------------------------- Lemire's rejection branch
def _lemire_reference(words, bounds):
    """Bounded draws by multiply-and-reject (Lemire, ACM TOMACS 2019) with
    Python integers: for bound r take words x until (x r mod 2^64) is not
    below (2^64 - r) mod r; the draw is floor(x r / 2^64)."""
    it = iter(words)
    out, rejected = [], 0
    for r in bounds:
        x = next(it)
        while (x * r) & M64 < ((1 << 64) - r) % r:
            rejected += 1
            x = next(it)
        out.append((x * r) >> 64)
    return out, rejected


@pytest.mark.parametrize("r", [2**63 + 1, 2**63 + 12345, 3 * 2**62 + 7])
def test_bounded_draws_reject_like_big_integer_reference(r):
    seed, role, gen, chrom, tag, stage = 99, 2, 5, 17, 3, 1
    count = 200
    got = oracle.stream_draws(seed, role, gen, chrom, tag, stage, [r] * count)
    # enough raw words of the same stream for every rejection
    words = []
    blk = 0
    while len(words) < 4 * count:
        words += _numpy_block([seed, role], [gen, chrom, (tag << 32) | stage, blk])
        blk += 1
    want, rejected = _lemire_reference(words, [r] * count)
    assert [int(v) for v in got] == want
    # the bound sits where about half (a third for 3 * 2^62) of the words
    # are rejected: the branch really runs
    assert rejected > count // 5
    assert all(v < r for v in want)
