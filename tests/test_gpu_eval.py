"""GPU parity of the preprocessing and population-evaluation kernels with the
CPU oracle, through the C ABI.

Bar: bit-exact.  The tables are integer data; fitness values are exact
int64 sums of int32 distances; scan lengths are integer counts.  The oracle
computes costs straight from d (never through the tables) and scan lengths
by counting, so agreement checks the GPU tables and walk end to end.
"""
import itertools
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


def _rand(n, m, hi, seed):
    return np.random.default_rng(seed).integers(0, hi, size=(n, m)).astype(np.int32)


INSTANCES = {
    "example1": lambda: (gi.example1_matrix(), 2),
    "g20": lambda: (gi.graph_instance(20, 40, 0), 4),
    "g100": lambda: (gi.graph_instance(100, 200, 0), 5),
    "g900": lambda: (gi.graph_instance(900, 16200, 0), 90),
    "rect_37x150": lambda: (_rand(37, 150, 1000, 1), 20),
    "ties_p1": lambda: (_rand(60, 65, 4, 2), 1),
    "ties_pm1": lambda: (_rand(30, 64, 4, 3), 63),
    "euclid_64": lambda: (gi.euclid_instance(64, 4), 7),
    "euclid_129": lambda: (gi.euclid_instance(129, 5), 3),
    "wide_2x700": lambda: (_rand(2, 700, 50, 6), 350),
    "m2": lambda: (_rand(5, 2, 10, 7), 1),
    # distances at and past 2^16: rows sort on 64-bit keys, the others on
    # 32-bit keys, row by row
    "wide_d": lambda: (_rand(40, 300, 2**31 - 1, 8), 30),
    "mixed_rows": lambda: (_mixed_rows(), 10),
    "edge_65535": lambda: (_rand(20, 100, 2, 10) + 65534, 5),
}


def _mixed_rows():
    d = _rand(24, 200, 60000, 9)
    d[3, 5] = 70000
    d[17, 150] = 65536
    d[20, :] = 65535
    return d


@pytest.mark.parametrize("name", list(INSTANCES))
def test_tables_bit_exact(pm, name):
    d, p = INSTANCES[name]()
    _say("case", name, d.shape, "p", p)
    inst = pm.Instance(d, p)
    pi, de, ds = inst.tables()
    opi, ode, ods = oracle.tables(d, p)
    np.testing.assert_array_equal(pi.astype(np.int32), opi)
    np.testing.assert_array_equal(de, ode)
    np.testing.assert_array_equal(ds, ods)


@pytest.mark.parametrize("name,P", [("example1", 6), ("g20", 200), ("g100", 64), ("g100", 1),
                                    ("g900", 1024), ("rect_37x150", 131), ("ties_p1", 70),
                                    ("ties_pm1", 65), ("euclid_64", 127), ("euclid_129", 64),
                                    ("wide_2x700", 300), ("m2", 3), ("wide_d", 70),
                                    ("mixed_rows", 65), ("edge_65535", 33)])
def test_eval_bit_exact_host_path(pm, name, P):
    d, p = INSTANCES[name]()
    n, m = d.shape
    _say("case", name, d.shape, "p", p, "P", P)
    masks = gi.random_population(P, m, p, seed=P + n)
    inst = pm.Instance(d, p)
    fit = np.zeros(P, np.int64)
    scan = np.zeros(P, np.int64)
    pm.pmp_eval_population(inst.handle, masks, fit, scan)
    want, wscan = oracle.objective(d, masks, p, scan=True)
    np.testing.assert_array_equal(fit, want)
    np.testing.assert_array_equal(scan, wscan)


def test_eval_device_path_and_async(pm):
    import torch
    d, p = INSTANCES["g900"]()
    masks = gi.random_population(333, 900, p, seed=9)
    inst = pm.Instance(torch.from_numpy(d).cuda(), p)
    dm = torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)
    fit = torch.empty(333, dtype=torch.int64, device="cuda")
    scan = torch.empty(333, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population(inst.handle, dm, fit, scan)
    want, wscan = oracle.objective(d, masks, p, scan=True)
    np.testing.assert_array_equal(fit.cpu().numpy(), want)
    np.testing.assert_array_equal(scan.cpu().numpy(), wscan)
    fit2 = torch.full((333,), -5, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population(inst.handle, dm, fit2, None, asynchronous=True)
    inst.check()
    np.testing.assert_array_equal(fit2.cpu().numpy(), want)


def test_g20_all_subsets_min_is_exhaustive_optimum(pm):
    d, p = INSTANCES["g20"]()
    allsets = gi.pack_masks([list(s) for s in itertools.combinations(range(20), p)], 20)
    inst = pm.Instance(d, p)
    fit = inst.eval(allsets)
    assert len(fit) == 4845
    np.testing.assert_array_equal(fit, oracle.objective(d, allsets, p))
    best, _, _ = oracle.exhaustive(d, p)
    assert fit.min() == best


def test_example1_all_pairs_match_printed_costs(pm):
    d, p = INSTANCES["example1"]()
    sets = list(itertools.combinations(range(4), 2))
    fit = pm.Instance(d, p).eval(gi.pack_masks([list(s) for s in sets], 4))
    # costs of the six open pairs from the paper's reduced polynomial
    assert fit.tolist() == [43, 37, 35, 46, 40, 44]


@pytest.mark.parametrize("p", [10, 100, 500])
def test_e5000_full_size(pm, p):
    """Full E5000 shape (P = 4096) in the benchmark's launch configuration:
    every chromosome's fitness against the oracle's direct minimum, scan
    lengths of a sample (the oracle counts them in O(m) per client), and a
    sample of table rows."""
    import torch
    d = _e5000()
    _say("case e5000 p", p)
    inst = pm.Instance(torch.from_numpy(d).cuda(), p)
    masks = gi.random_population(4096, 5000, p, seed=p)
    dm = torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)
    fit = torch.empty(4096, dtype=torch.int64, device="cuda")
    scan = torch.empty(4096, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population(inst.handle, dm, fit, scan)
    fit, scan = fit.cpu().numpy(), scan.cpu().numpy()
    np.testing.assert_array_equal(fit, oracle.objective(d, masks, p))
    rng = np.random.default_rng(p)
    pick = np.concatenate([[0, 4095], rng.choice(4096, 46, replace=False)])
    want, wscan = oracle.objective(d, masks[pick], p, scan=True)
    np.testing.assert_array_equal(fit[pick], want)
    np.testing.assert_array_equal(scan[pick], wscan)
    # E[s*] = (m+1)/(p+1) for uniform random subsets
    mean = scan.sum() / (4096 * 5000)
    assert abs(mean - 5001 / (p + 1)) < 0.03 * 5001 / (p + 1)
    rows = rng.choice(5000, 40, replace=False)
    pi, de, ds = inst.tables()
    opi, ode, ods = oracle.tables(d[rows], p)
    np.testing.assert_array_equal(pi[rows].astype(np.int32), opi)
    np.testing.assert_array_equal(de[rows], ode)
    np.testing.assert_array_equal(ds[rows], ods)


@pytest.mark.parametrize("p", [10, 500])
def test_e5000_evolved_population(pm, p):
    """The population the E5000 benchmark times after evolving it (GA with
    P = 4096, NT = 256 for 20 generations): the evaluation of all 4096
    chromosomes against the oracle, and against the GA's own fitness."""
    import torch
    d = _e5000()
    _say("case e5000 evolved p", p)
    inst = pm.Instance(torch.from_numpy(d).cuda(), p)
    ga = pm.GA(inst, 4096, 256, 20, 0)
    ga.step(20)
    pop, gfit, _, _ = ga.state()
    dm = torch.from_numpy(pop.view(np.int64)).cuda().view(torch.uint64)
    fit = torch.empty(4096, dtype=torch.int64, device="cuda")
    scan = torch.empty(4096, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population(inst.handle, dm, fit, scan)
    fit, scan = fit.cpu().numpy(), scan.cpu().numpy()
    want = oracle.objective(d, pop, p)
    np.testing.assert_array_equal(fit, want)
    np.testing.assert_array_equal(gfit, want)
    pick = np.random.default_rng(p + 1).choice(4096, 24, replace=False)
    _, wscan = oracle.objective(d, pop[pick], p, scan=True)
    np.testing.assert_array_equal(scan[pick], wscan)


def test_e5000_ga_generation_bitwise(pm):
    """One generation of the E5000 GA configuration (p = 10, the long-scan
    walk; P = 4096, NT = 256, NB = 16) against the oracle GA, bit for bit:
    population, fitness, group bests, global best and counters."""
    d = _e5000()
    _say("case e5000 GA generation p 10")
    from test_gpu_ga import _compare
    _compare(pm, d, 10, 4096, 256, 200, seed=0, steps=[1])


_E5000 = {}


def _e5000():
    if "d" not in _E5000:
        _E5000["d"] = gi.euclid_instance(5000, 0)
    return _E5000["d"]


@pytest.mark.parametrize("m,p", [(8192, 2000), (8191, 3), (8192, 8191)],
                         ids=["m=8192 short scans", "m=8191 long scans", "p=m-1"])
def test_eval_at_the_facility_limit(pm, m, p):
    """m at PMP_MAX_FACILITIES (128 words per chromosome, the largest staging
    and facility-major tile) and one below it, with two chromosome tiles (the
    second ragged)."""
    n, P = 24, 70
    d = np.random.default_rng(m + p).integers(0, 10000, size=(n, m)).astype(np.int32)
    masks = gi.random_population(P, m, p, seed=5)
    print("case m", m, "p", p, "n", n, "P", P, flush=True)
    inst = pm.Instance(d, p)
    np.testing.assert_array_equal(inst.eval(masks), oracle.objective(d, masks, p))


@pytest.mark.parametrize("waves", ["4", "8", "16"])
@pytest.mark.parametrize("name,P", [("g900", 300), ("euclid_129", 130), ("wide_2x700", 70),
                                    ("ties_p1", 65), ("mixed_rows", 129)])
def test_waves_per_workgroup(pm, name, P, waves):
    """4, 8 or 16 waves sharing one staged chromosome tile: same results,
    for the single and paired walks and several tile sizes."""
    d, p = INSTANCES[name]()
    n, m = d.shape
    masks = gi.random_population(P, m, p, seed=P + 7)
    want, wscan = oracle.objective(d, masks, p, scan=True)
    old = {k: os.environ.get(k) for k in ("PMP_EVAL_WAVES", "PMP_CLIENTS_PER_BLOCK",
                                          "PMP_EVAL_PAIRED")}
    try:
        os.environ["PMP_EVAL_WAVES"] = waves
        for cpb, paired in (("0", "0"), ("0", "1"), ("5", "0"), ("37", "1"), ("900", "0")):
            _say("case", name, "P", P, "waves", waves, "clients", cpb, "paired", paired)
            if cpb == "0":
                os.environ.pop("PMP_CLIENTS_PER_BLOCK", None)
            else:
                os.environ["PMP_CLIENTS_PER_BLOCK"] = cpb
            os.environ["PMP_EVAL_PAIRED"] = paired
            inst = pm.Instance(d, p)
            fit = np.zeros(P, np.int64)
            scan = np.zeros(P, np.int64)
            pm.pmp_eval_population(inst.handle, masks, fit, scan)
            np.testing.assert_array_equal(fit, want)
            np.testing.assert_array_equal(scan, wscan)
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def test_tile_shape_does_not_change_results(pm):
    d, p = INSTANCES["g900"]()
    masks = gi.random_population(257, 900, p, seed=3)
    inst = pm.Instance(d, p)
    outs = []
    old = os.environ.get("PMP_CLIENTS_PER_BLOCK")
    try:
        for cpb in ("4", "12", "13", "64", "417", "900"):
            os.environ["PMP_CLIENTS_PER_BLOCK"] = cpb
            outs.append(inst.eval(masks).copy())
    finally:
        if old is None:
            os.environ.pop("PMP_CLIENTS_PER_BLOCK", None)
        else:
            os.environ["PMP_CLIENTS_PER_BLOCK"] = old
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    np.testing.assert_array_equal(outs[0], oracle.objective(d, masks, p))


def test_empty_population_is_a_no_op(pm):
    d, p = INSTANCES["g100"]()
    inst = pm.Instance(d, p)
    fit = np.zeros(0, np.int64)
    pm.pmp_eval_population(inst.handle, np.zeros((0, 2), np.uint64), fit)


@pytest.mark.parametrize("kind", ["fewer", "more", "stray"])
def test_infeasible_chromosomes_rejected(pm, kind):
    d, p = INSTANCES["euclid_129"]()
    m = 129
    masks = gi.random_population(10, m, p, seed=1)
    bits = gi.unpack_masks(masks, m)
    if kind == "fewer":
        bits[4, np.nonzero(bits[4])[0][0]] = False
        masks = gi.pack_masks(bits, m)
    elif kind == "more":
        bits[4, np.nonzero(~bits[4])[0][0]] = True
        masks = gi.pack_masks(bits, m)
    else:
        masks[4, 2] |= np.uint64(1) << np.uint64(5)  # bit 133 >= m
    inst = pm.Instance(d, p)
    with pytest.raises(pm.PmpError) as e:
        inst.eval(masks)
    assert e.value.status == pm.PMP_EINFEASIBLE
    # the instance stays usable; a feasible call succeeds afterwards
    ok = gi.random_population(10, m, p, seed=2)
    np.testing.assert_array_equal(inst.eval(ok), oracle.objective(d, ok, p))


def test_negative_distance_rejected_on_device(pm):
    import torch
    d = _rand(10, 12, 9, 8)
    d[3, 7] = -2
    with pytest.raises(pm.PmpError) as e:
        pm.Instance(torch.from_numpy(d).cuda(), 3)
    assert e.value.status == pm.PMP_EINVAL
    # asynchronous preprocessing: the same error, from the instance check
    inst = pm.Instance(torch.from_numpy(d).cuda(), 3, asynchronous=True)
    with pytest.raises(pm.PmpError) as e:
        inst.check()
    assert e.value.status == pm.PMP_EINVAL


@pytest.mark.parametrize("name", ["g100", "g900", "euclid_129", "wide_2x700", "ties_p1"])
def test_asynchronous_preprocessing_same_tables(pm, name):
    """Instances preprocessed back to back without waiting (PMP_ASYNC) hold
    the oracle's tables and evaluate like synchronously made ones; the
    learned features, which read the sum of d back on first use, agree."""
    import torch
    d, p = INSTANCES[name]()
    dd = torch.from_numpy(d).cuda()
    insts = [pm.Instance(dd, p, asynchronous=True) for _ in range(3)]
    for inst in insts:
        inst.check()
    opi, ode, ods = oracle.tables(d, p)
    masks = gi.random_population(70, d.shape[1], p, seed=4)
    want = oracle.objective(d, masks, p)
    for inst in insts:
        pi, de, ds = inst.tables()
        np.testing.assert_array_equal(pi.astype(np.int32), opi)
        np.testing.assert_array_equal(de, ode)
        np.testing.assert_array_equal(ds, ods)
        np.testing.assert_array_equal(inst.eval(masks), want)
    sync = pm.Instance(d, p)
    np.testing.assert_array_equal(pm.pmp_features(insts[0].handle, masks[:5], 0.25),
                                  pm.pmp_features(sync.handle, masks[:5], 0.25))


SCHEME_CASES = [("example1", 6), ("g20", 200), ("g100", 64), ("g900", 257),
                ("rect_37x150", 131), ("ties_p1", 70), ("ties_pm1", 65),
                ("euclid_129", 64), ("wide_2x700", 30), ("m2", 3)]


@pytest.mark.parametrize("scheme", ["per_chromosome", "per_client"])
@pytest.mark.parametrize("name,P", SCHEME_CASES)
def test_eval_schemes_bit_exact(pm, scheme, name, P):
    """The other thread mappings (one thread per chromosome, one per client)
    give the same exact costs and scan lengths."""
    d, p = INSTANCES[name]()
    n, m = d.shape
    _say("case", name, d.shape, "p", p, "P", P, "scheme", scheme)
    masks = gi.random_population(P, m, p, seed=P + n + 1)
    inst = pm.Instance(d, p)
    fit = np.zeros(P, np.int64)
    scan = np.zeros(P, np.int64)
    pm.pmp_eval_population(inst.handle, masks, fit, scan, scheme=scheme)
    want, wscan = oracle.objective(d, masks, p, scan=True)
    np.testing.assert_array_equal(fit, want)
    np.testing.assert_array_equal(scan, wscan)
    fit2 = np.zeros(P, np.int64)
    pm.pmp_eval_population(inst.handle, masks, fit2, None, scheme=scheme)
    np.testing.assert_array_equal(fit2, want)


@pytest.mark.parametrize("scheme", ["per_chromosome", "per_client"])
@pytest.mark.parametrize("kind", ["fewer", "stray"])
def test_eval_schemes_reject_infeasible(pm, scheme, kind):
    d, p = INSTANCES["euclid_129"]()
    m = 129
    masks = gi.random_population(10, m, p, seed=3)
    if kind == "fewer":
        bits = gi.unpack_masks(masks, m)
        bits[7, np.nonzero(bits[7])[0][0]] = False
        masks = gi.pack_masks(bits, m)
    else:
        masks[7, 2] |= np.uint64(1) << np.uint64(9)  # bit 137 >= m
    _say("infeasible", kind, "scheme", scheme)
    inst = pm.Instance(d, p)
    fit = np.zeros(10, np.int64)
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_eval_population(inst.handle, masks, fit, scheme=scheme)
    assert e.value.status == pm.PMP_EINFEASIBLE


def test_eval_both_scheme_flags_rejected(pm):
    d, p = INSTANCES["g20"]()
    inst = pm.Instance(d, p)
    masks = gi.random_population(4, 20, p, seed=1)
    fit = np.zeros(4, np.int64)
    rc = pm.lib().pmp_eval_population(inst.handle, masks.ctypes.data_as(pm._vp), 4,
                                      fit.ctypes.data_as(pm._vp), None,
                                      pm.PMP_EVAL_PER_CHROMOSOME | pm.PMP_EVAL_PER_CLIENT, None)
    assert rc == pm.PMP_EINVAL


@pytest.mark.parametrize("paired", ["1", "0"])
@pytest.mark.parametrize("name,P", [("g100", 130), ("euclid_129", 64), ("ties_p1", 70),
                                    ("g900", 257), ("ties_pm1", 65), ("m2", 3),
                                    ("rect_37x150", 131), ("wide_2x700", 300)])
def test_eval_paired_and_single_chunks(pm, paired, name, P):
    """Both walks of the tiled kernel - two clients per 32-entry chunk, or
    one client per 64-entry chunk - on short scans, long scans (rows finish
    in the tail walk) and rows shorter than 32 entries."""
    d, p = INSTANCES[name]()
    n, m = d.shape
    _say("case", name, d.shape, "p", p, "P", P, "paired", paired)
    old = os.environ.get("PMP_EVAL_PAIRED")
    os.environ["PMP_EVAL_PAIRED"] = paired
    try:
        masks = gi.random_population(P, m, p, seed=P + 3)
        inst = pm.Instance(d, p)
        fit = np.zeros(P, np.int64)
        scan = np.zeros(P, np.int64)
        pm.pmp_eval_population(inst.handle, masks, fit, scan)
        want, wscan = oracle.objective(d, masks, p, scan=True)
        np.testing.assert_array_equal(fit, want)
        np.testing.assert_array_equal(scan, wscan)
    finally:
        if old is None:
            os.environ.pop("PMP_EVAL_PAIRED", None)
        else:
            os.environ["PMP_EVAL_PAIRED"] = old
