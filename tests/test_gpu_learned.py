"""Learned swap proposal on the GPU against the oracle (oracle/learned.py).

* features: bit-exact (integer sums, one double-rounded normalisation);
* network: initial parameters bit-exact; scores within the 2e-2 relative
  tolerance the design states (BF16 operands, FP32 accumulation on the matrix
  cores, versus the oracle's float64 sums); gradients per parameter block
  within a normwise 2e-2 (the kernel also rounds the backward signals to
  BF16 for the matrix products); the first Adam step moves each parameter
  by lr against the sign of its gradient;
* learned GA: every evaluated swap of generation 0 checked against the
  oracle (candidate draws, input row, exact change of cost, target) and the
  choice checked against the ranking of the GPU's own scores (a decision
  floating point makes, so only its validity is checked); populations,
  fitness and stop rules as the plain GA's invariants;
* a trained network's proposals succeed more often than an untrained one's,
  and the learned GA beats the plain GA on fresh instances.
"""
import os

import numpy as np
import pytest

import oracle
import oracle.learned as OL
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


FEATURE_CASES = [
    # name, d builder, p, P
    ("example1", lambda: gi.example1_matrix(), 2, 6),
    ("graph90", lambda: gi.graph_instance(90, 180, 1), 7, 8),
    ("euclid200", lambda: gi.euclid_instance(200, 2), 20, 6),
    ("rand37x150", lambda: np.random.default_rng(3).integers(0, 40, (37, 150)).astype(np.int32),
     20, 5),
    ("p1", lambda: gi.euclid_instance(70, 4), 1, 4),
    ("p_m-1", lambda: np.random.default_rng(5).integers(0, 9, (30, 12)).astype(np.int32),
     11, 4),
    ("euclid300_m>256", lambda: gi.euclid_instance(300, 6), 30, 3),
]


@pytest.mark.parametrize("name,make,p,P", FEATURE_CASES, ids=[c[0] for c in FEATURE_CASES])
def test_features_match_oracle(pm, name, make, p, P):
    d = make()
    n, m = d.shape
    _say("features", name, n, m, p, P)
    masks = gi.random_population(P, m, p, 11)
    if name == "example1":
        masks[0] = gi.pack_masks([[0, 3]], m)[0]
    inst = pm.Instance(d, p)
    got = pm.pmp_features(inst.handle, masks, 0.375)
    static = OL.static_sums(d, p)
    for c, bits in enumerate(gi.unpack_masks(masks, m)):
        ref = OL.features(d, bits, p, 0.375, static)
        np.testing.assert_array_equal(got[c], ref, err_msg=f"chromosome {c}")


def test_features_reject_infeasible(pm):
    d = gi.euclid_instance(50, 1)
    inst = pm.Instance(d, 5)
    bad = gi.pack_masks([[0, 1, 2]], 50)
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_features(inst.handle, bad)
    assert e.value.status == 4


def test_model_init_matches_oracle(pm):
    for seed in (0, 12345):
        model = pm.Model(seed)
        np.testing.assert_array_equal(model.params(), OL.init_params(seed))


def _rel_ok(got, ref, tol=2e-2, floor_frac=0.1):
    """Relative tolerance tol where |ref| >= floor = floor_frac * mean |ref|,
    and |got - ref| <= tol * floor below it.  A score near zero is a
    difference of large terms: one first-layer activation whose FP32 sum
    rounds to the other neighbouring BF16 value than its float64 sum moves
    the score by about |w3_k| 2^-8 |h_k|, however small the score is, so
    a pure relative bound cannot hold there."""
    floor = floor_frac * np.abs(ref).mean() + 1e-30
    err = np.abs(got - ref)
    big = np.abs(ref) >= floor
    return np.where(big, err <= tol * np.abs(ref), err <= tol * floor)


@pytest.mark.parametrize("rows", [1, 17, 1000, 4099])
def test_forward_matches_oracle(pm, rows):
    _say("forward rows", rows)
    rng = np.random.default_rng(rows)
    q = (rng.standard_normal(OL.N_PARAMS) * 0.15).astype(np.float32)
    X = (rng.standard_normal((rows, 32)) * 1.5).astype(np.float32)
    model = pm.Model(1)
    model.set_params(q)
    y = model.forward(X)
    ref, _ = OL.forward(q, X)
    ok = _rel_ok(y.astype(np.float64), ref)
    assert ok.all(), (np.abs(y - ref).max(), ref[~ok][:5], y[~ok][:5])
    # far inside the bound in practice
    assert np.abs(y - ref).max() <= 5e-3 * (np.abs(ref).max() + 1)


def test_forward_zero_rows_and_device_buffers(pm):
    import torch
    model = pm.Model(2)
    model.forward(np.zeros((0, 32), np.float32))  # no work, no error
    X = torch.randn(300, 32, device="cuda")
    y = model.forward(X)
    ref = model.forward(X.cpu().numpy())
    np.testing.assert_array_equal(y.cpu().numpy(), ref)


@pytest.mark.parametrize("rows", [64, 1000, 9000])
def test_grad_matches_oracle(pm, rows):
    _say("grad rows", rows)
    rng = np.random.default_rng(rows + 1)
    q = (rng.standard_normal(OL.N_PARAMS) * 0.12).astype(np.float32)
    X = rng.standard_normal((rows, 32)).astype(np.float32)
    T = rng.standard_normal(rows).astype(np.float32)
    w = (rng.random(rows) < 0.75).astype(np.float32)
    model = pm.Model(3)
    model.set_params(q)
    g, loss = model.grad(X, T, w)
    ref, rloss = OL.backward(q, X, T.astype(np.float64), w.astype(np.float64))
    assert abs(loss - rloss) <= 1e-2 * abs(rloss)
    for lo, hi, name in ((OL.OFF_W1, OL.OFF_B1, "W1"), (OL.OFF_B1, OL.OFF_W2, "b1"),
                         (OL.OFF_W2, OL.OFF_B2, "W2"), (OL.OFF_B2, OL.OFF_W3, "b2"),
                         (OL.OFF_W3, OL.OFF_B3, "w3"), (OL.OFF_B3, OL.N_PARAMS, "b3")):
        a, b = g[lo:hi].astype(np.float64), ref[lo:hi]
        err = np.linalg.norm(a - b) / (np.linalg.norm(b) + 1e-30)
        assert err <= 2e-2, (name, err)


def test_train_step_moves_by_lr_against_gradient_sign(pm):
    rng = np.random.default_rng(9)
    q = (rng.standard_normal(OL.N_PARAMS) * 0.1).astype(np.float32)
    X = rng.standard_normal((2000, 32)).astype(np.float32)
    T = rng.standard_normal(2000).astype(np.float32)
    model = pm.Model(4)
    model.set_params(q)
    lr = 1e-3
    model.train(X, T, lr=lr, steps=1)
    after = model.params().astype(np.float64)
    ref, _ = OL.backward(q, X, T.astype(np.float64))
    # Adam's first step: -lr m/(sqrt(v) + eps) = -lr sign(g) up to eps
    strong = np.abs(ref) > 1e-3 * np.abs(ref).max()
    step = after - q.astype(np.float64)
    np.testing.assert_allclose(step[strong], -lr * np.sign(ref[strong]), rtol=1e-2,
                               atol=1e-6)


def test_training_fits_a_function(pm):
    """Many steps on y = x0 - 2 x1 + relu(x2): the loss falls far."""
    rng = np.random.default_rng(10)
    X = rng.standard_normal((4096, 32)).astype(np.float32)
    T = (X[:, 0] - 2 * X[:, 1] + np.maximum(X[:, 2], 0)).astype(np.float32)
    model = pm.Model(5)
    first = model.train(X, T, lr=3e-3, steps=1)
    last = model.train(X, T, lr=3e-3, steps=300)
    assert last < 0.05 * first, (first, last)


def _learned_ga(pm, d, p, P, NT, G, seed, model, **kw):
    inst = pm.Instance(d, p)
    ga = pm.GA(inst, P, NT, G, seed)
    ga.set_model(model, **kw)
    return inst, ga


@pytest.mark.parametrize("case", ["graph120", "euclid260", "euclid2000_config"])
def test_learned_generation0_against_oracle(pm, case):
    sample = None
    if case == "graph120":
        d, p, P, NT, C, L, expl = gi.graph_instance(120, 240, 3), 9, 64, 16, 16, 4, 300
    elif case == "euclid260":
        d, p, P, NT, C, L, expl = gi.euclid_instance(260, 4), 26, 32, 32, 24, 3, 0
    else:
        # the learned workload's configuration: Euclidean n = m = 2000, p =
        # 200, population 1024 (NT 256), 64 candidates, 4 scored swaps, 5 %
        # exploration; 24 chromosomes checked swap by swap
        d, p, P, NT, C, L, expl = gi.euclid_instance(2000, 100), 200, 1024, 256, 64, 4, 50
        sample = np.concatenate([[0, P - 1], np.random.default_rng(5).choice(
            np.arange(1, P - 1), 22, replace=False)])
    n, m = d.shape
    seed, G = 21, 50
    _say("learned generation 0", case)
    model = pm.Model(8)
    inst, ga = _learned_ga(pm, d, p, P, NT, G, seed, model, candidates=C, learned_iters=L,
                           explore_permille=expl, train_every=0)
    ga.step(1)
    rep = ga.replay()
    pop, fit, _, _ = ga.state()
    np.testing.assert_array_equal(fit, oracle.objective(d, pop, p))
    parent, pfit = OL.population_after_crossover(d, p, P, NT, seed)
    pbits = gi.unpack_masks(parent, m)
    static = OL.static_sums(d, p)
    checked = 0
    for c in (range(P) if sample is None else sample):
        feats = OL.features(d, pbits[c], p, 0.0, static)
        cands = OL.candidates(seed, 0, c, pbits[c], p, C)
        rows = np.stack([np.concatenate([feats[j], feats[k]]) for j, k in cands])
        scores = rep["scores"][c]  # what the proposal kernel computed
        ref_scores, _ = OL.forward(model.params(), rows)
        assert _rel_ok(scores.astype(np.float64), ref_scores).all()
        np.testing.assert_allclose(model.forward(OL.bf16(rows)), scores, rtol=1e-6,
                                   atol=1e-6)
        order = sorted(range(C), key=lambda t: (scores[t], t))
        improved = False
        for a in range(L):
            r = a * P + c  # generation 0 -> ring slot h = 0
            if improved:
                assert rep["weight"][r] == 0
                continue
            assert rep["weight"][r] == 1, (c, a)
            e, u = OL.explore_draws(seed, 0, c, a, C)
            pick = u if e < expl else order[a]
            j, k = cands[pick]
            assert tuple(rep["swap"][r]) == (j, k), (c, a)
            np.testing.assert_array_equal(rep["x"][r], OL.bf16_bits(rows[pick]))
            child = pbits[c].copy()
            child[j], child[k] = False, True
            cf = int(oracle.objective(d, gi.pack_masks(child[None], m), p)[0])
            assert rep["delta"][r][1] == pfit[c]
            assert rep["delta"][r][0] == cf - pfit[c]
            assert rep["target"][r] == OL.target(cf - pfit[c], pfit[c], p)
            improved = cf < pfit[c]
            checked += 1
    if sample is not None:
        assert checked >= len(sample)
        return
    assert checked >= P
    _, cost, stats = ga.best()
    assert stats["swap_tried"] == checked
    assert stats["swap_taken"] == sum(
        1 for c in range(P) for a in range(L)
        if rep["weight"][a * P + c] == 1 and rep["delta"][a * P + c][0] < 0)


def test_learned_ga_invariants_graph_replay_and_determinism(pm):
    d = gi.euclid_instance(300, 7)
    p, P, NT, G = 30, 128, 32, 40
    runs = []
    # the graph-replayed and kernel-by-kernel schedules, and the mutation
    # cycle attempt by attempt instead of at once: all must agree
    for mode, spec in (("graph", "1"), ("kernels", "1"), ("graph", "1"), ("graph", "0"),
                       ("kernels", "0")):
        old = os.environ.get("PMP_GA_MODE")
        old_spec = os.environ.get("PMP_GA_SPEC")
        os.environ["PMP_GA_MODE"] = mode
        os.environ["PMP_GA_SPEC"] = spec
        try:
            model = pm.Model(9)
            inst, ga = _learned_ga(pm, d, p, P, NT, G, 5, model, candidates=32,
                                   learned_iters=2, explore_permille=50, train_every=1,
                                   lr=2e-3)
            trace = []
            for _ in range(5):
                ga.step(8)
                trace.append(ga.best()[1])
            pop, fit, gm, gc = ga.state()
            runs.append((trace, pop, fit, gm, gc, model.params(), ga.best()[2]))
        finally:
            if old is None:
                os.environ.pop("PMP_GA_MODE", None)
            else:
                os.environ["PMP_GA_MODE"] = old
            if old_spec is None:
                os.environ.pop("PMP_GA_SPEC", None)
            else:
                os.environ["PMP_GA_SPEC"] = old_spec
        np.testing.assert_array_equal(fit, oracle.objective(d, pop, p))
        assert all(a >= b for a, b in zip(trace, trace[1:]))
        assert np.all(gi.unpack_masks(pop, 300).sum(axis=1) == p)
    for other in runs[1:]:
        assert runs[0][0] == other[0]
        for x, y in zip(runs[0][1:6], other[1:6]):
            np.testing.assert_array_equal(x, y)
        for k in ("chromosome_evals", "swap_tried", "swap_taken", "mutation_taken",
                  "crossover_taken", "scan_total"):
            assert runs[0][6][k] == other[6][k], k
    st = runs[0][6]
    assert st["generations"] == G and st["done"] == 1
    assert st["swap_tried"] > 0 and st["swap_taken"] > 0


def test_set_model_rejects(pm):
    d = gi.euclid_instance(100, 1)
    inst = pm.Instance(d, 10)
    ga = pm.GA(inst, 64, 16, 5, 1)
    model = pm.Model(1)
    for kw in ({"candidates": 65}, {"learned_iters": 5}, {"candidates": 3, "learned_iters": 4},
               {"explore_permille": 1001}, {"train_every": -1}, {"lr": -1.0}):
        with pytest.raises(pm.PmpError) as e:
            ga.set_model(model, **kw)
        assert e.value.status == 1, kw
    ga.set_model(model)
    with pytest.raises(pm.PmpError):
        pm.Batch([ga])
    ga.set_model(None)  # plain again
    ga.step(2)
    big = np.random.default_rng(0).integers(0, 9, (3, 4100)).astype(np.int32)
    binst = pm.Instance(big, 2000)
    bga = pm.GA(binst, 64, 16, 5, 1)
    with pytest.raises(pm.PmpError) as e:
        bga.set_model(model)
    assert e.value.status == 5


def _success(pm, d, p, model, seed, explore):
    """Attempt-0 success rate and mean target of one frozen-model generation."""
    inst, ga = _learned_ga(pm, d, p, 256, 64, 10, seed, model, candidates=32,
                           learned_iters=3, explore_permille=explore, train_every=0)
    ga.step(1)
    rep = ga.replay()
    first = rep["delta"][:256, 0]
    return float((first < 0).mean()), float(rep["target"][:256].mean())


def test_trained_network_gains(pm):
    """Online training on three instances, then on a fresh one: the trained
    network's first proposals improve chromosomes more often than an
    untrained network's and than a uniform choice among the candidates; and
    the learned GA ends below the plain GA after the same generations."""
    p, n = 40, 400
    model = pm.Model(11)
    for s in range(3):
        d = gi.euclid_instance(n, 50 + s)
        inst, ga = _learned_ga(pm, d, p, 256, 64, 60, s, model, candidates=32,
                               learned_iters=3, explore_permille=100, train_every=1,
                               lr=2e-3)
        ga.step(60)
        _say("training instance", s, "best", ga.best()[1])
    fresh = gi.euclid_instance(n, 99)
    trained = pm.Model(0)
    trained.set_params(model.params())
    rate_t, tgt_t = _success(pm, fresh, p, trained, 7, 0)
    rate_u, tgt_u = _success(pm, fresh, p, pm.Model(12), 7, 0)
    rate_r, tgt_r = _success(pm, fresh, p, pm.Model(12), 7, 1000)
    _say("success trained/untrained/random", rate_t, rate_u, rate_r, tgt_t, tgt_u, tgt_r)
    # success rates are capped at 1: compare by margins
    assert rate_t >= max(rate_u, rate_r) + 0.1
    assert tgt_t <= min(tgt_u, tgt_r) - 0.3
    # same generations, fresh seed: learned GA (continuing to train) vs plain
    G = 40
    inst, lga = _learned_ga(pm, fresh, p, 256, 64, G, 3, trained, candidates=32,
                            learned_iters=3, explore_permille=50, train_every=1, lr=1e-3)
    lga.step(G)
    pga = pm.GA(inst, 256, 64, G, 3)
    pga.step(G)
    lbest, pbest = lga.best()[1], pga.best()[1]
    _say("learned vs plain best", lbest, pbest)
    assert lbest < pbest
    mask, cost, _ = lga.best()
    assert cost == oracle.objective(fresh, mask[None], p)[0]


@pytest.mark.parametrize("case", ["euclid300", "rand_p3", "short_rows", "far_overflow",
                                  "unstaged", "wide_m4000", "ragged_P96"])
def test_two_pass_walk_equals_one_pass(pm, case):
    """The two-pass proposal walk (first two open positions per chromosome
    and client, then each candidate facility's index entries; positions past
    the index walked directly) gives the one-pass walk's slot sums: the same
    features, scores, swaps, training and runs, bit for bit.  Cases: common
    rows, rows whose second open facility often lies past the index (p = 3),
    rows shorter than the index (K < 64), more rows past the index than a
    chromosome's list holds (256: the rest walked by the wave that finds
    them), more clients than the per-chromosome LDS staging takes (4096:
    client data read from device memory), m = 4000 (the first pass's widest
    mask staging), and a population of 96 (a last chromosome tile of 32)."""
    if case == "euclid300":
        d, p = gi.euclid_instance(300, 7), 30
    elif case == "rand_p3":
        d, p = np.random.default_rng(3).integers(1, 500, size=(40, 150)).astype(np.int32), 3
    elif case == "far_overflow":
        d, p = np.random.default_rng(4).integers(1, 900, size=(700, 300)).astype(np.int32), 3
    elif case == "unstaged":
        d, p = np.random.default_rng(5).integers(1, 3000, size=(4200, 120)).astype(np.int32), 12
    elif case == "wide_m4000":  # 63 mask words: the widest staging of the first pass
        d, p = np.random.default_rng(6).integers(1, 5000, size=(300, 4000)).astype(np.int32), 40
    elif case == "ragged_P96":  # a last chromosome tile of 32
        d, p = gi.euclid_instance(210, 8), 20
    else:
        d, p = gi.euclid_instance(70, 2), 30
    P, NT, G = (96 if case == "ragged_P96" else 128), 32, 20
    runs = []
    old = os.environ.get("PMP_WALK")
    try:
        for walk in ("0", "2"):
            os.environ["PMP_WALK"] = walk
            _say("walk", walk, case)
            model = pm.Model(11)
            inst, ga = _learned_ga(pm, d, p, P, NT, G, 3, model, candidates=32,
                                   learned_iters=2, explore_permille=50, train_every=1,
                                   lr=2e-3)
            ga.step(6)
            rep = ga.replay()
            pop, fit, gm, gc = ga.state()
            runs.append((pop, fit, gm, gc, model.params(), rep["x"], rep["delta"],
                         rep["scores"], ga.best()[2]))
    finally:
        if old is None:
            os.environ.pop("PMP_WALK", None)
        else:
            os.environ["PMP_WALK"] = old
    a, b = runs
    for x, y in zip(a[:8], b[:8]):
        np.testing.assert_array_equal(x, y)
    for k in ("swap_tried", "swap_taken", "chromosome_evals"):
        assert a[8][k] == b[8][k], k
    assert a[8]["swap_tried"] > 0
