"""GPU parity of instances wider than one workgroup's LDS staging
(8192 < m <= 65535) with the CPU oracle, through the C ABI.

Rows of such instances are sorted in device memory (chunks in LDS, larger
bitonic strides as passes over a scratch array) and the chromosome tiles are
turned facility-major into device memory before the walk.  Bar: bit-exact,
as for the narrow instances: the tables are integer data, fitness values
exact int64 sums, scan lengths integer counts; the oracle computes costs
straight from d and counts scan lengths itself.
"""
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


# the first width past the staged limit, the widest one, a middle one whose
# padded row (32768 keys) is not the widest, distances past 2^16 and heavy
# ties (the order of equal distances is by facility index), p from 1 to
# about m / 2
WIDE = {
    "m8193_p5": lambda: (_rand(37, 8193, 1000, 21), 5),
    "m8193_p4000_big_d": lambda: (_rand(37, 8193, 2**31 - 1, 22), 4000),
    "m20000_ties_p7": lambda: (_rand(50, 20000, 4, 23), 7),
    "m16385_p1": lambda: (_rand(9, 16385, 70000, 26), 1),
    "m65535_p3": lambda: (_rand(12, 65535, 100000, 24), 3),
    "m65535_p30000": lambda: (_rand(12, 65535, 2**20, 25), 30000),
}
_CACHE = {}


def _case(name):
    if name not in _CACHE:
        _CACHE[name] = WIDE[name]()
    return _CACHE[name]


@pytest.mark.parametrize("name", list(WIDE))
def test_wide_tables_bit_exact(pm, name):
    d, p = _case(name)
    _say("case", name, d.shape, "p", p)
    inst = pm.Instance(d, p)
    assert inst.W == (d.shape[1] + 63) // 64
    pi, de, ds = inst.tables()
    opi, ode, ods = oracle.tables(d, p)
    np.testing.assert_array_equal(pi.astype(np.int32), opi)
    np.testing.assert_array_equal(de, ode)
    np.testing.assert_array_equal(ds, ods)


@pytest.mark.parametrize("name,P", [("m8193_p5", 131), ("m8193_p4000_big_d", 64),
                                    ("m20000_ties_p7", 200), ("m16385_p1", 70),
                                    ("m65535_p3", 65), ("m65535_p30000", 65)])
def test_wide_eval_bit_exact(pm, name, P):
    """Fitness and scan lengths of ragged populations (P not a multiple of
    the 64-chromosome tile) against the oracle's direct minimum."""
    d, p = _case(name)
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
    # a smaller population next (the tile buffer is reused), without scans
    fit2 = inst.eval(masks[:17])
    np.testing.assert_array_equal(fit2, want[:17])


def test_wide_device_path_async_and_growth(pm):
    """Device tensors, an asynchronous call checked afterwards, and a larger
    population than the first call (the tile buffer grows)."""
    import torch
    d, p = _case("m8193_p5")
    m = d.shape[1]
    inst = pm.Instance(torch.from_numpy(d).cuda(), p)
    for P, seed in ((70, 1), (300, 2)):
        _say("device path P", P)
        masks = gi.random_population(P, m, p, seed=seed)
        dm = torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)
        fit = torch.full((P,), -1, dtype=torch.int64, device="cuda")
        pm.pmp_eval_population(inst.handle, dm, fit, None, asynchronous=True)
        inst.check()
        np.testing.assert_array_equal(fit.cpu().numpy(), oracle.objective(d, masks, p))


@pytest.mark.parametrize("kind", ["fewer", "more", "stray"])
def test_wide_infeasible_chromosomes_rejected(pm, kind):
    d, p = _case("m8193_p5")
    m = d.shape[1]
    masks = gi.random_population(80, m, p, seed=5)
    bits = gi.unpack_masks(masks, m)
    if kind == "fewer":
        bits[66, np.nonzero(bits[66])[0][0]] = False
        masks = gi.pack_masks(bits, m)
    elif kind == "more":
        bits[66, np.nonzero(~bits[66])[0][0]] = True
        masks = gi.pack_masks(bits, m)
    else:
        masks[66, 128] |= np.uint64(1) << np.uint64(7)  # bit 8199 >= m
    _say("infeasible", kind)
    inst = pm.Instance(d, p)
    with pytest.raises(pm.PmpError) as e:
        inst.eval(masks)
    assert e.value.status == pm.PMP_EINFEASIBLE
    ok = gi.random_population(80, m, p, seed=6)
    np.testing.assert_array_equal(inst.eval(ok), oracle.objective(d, ok, p))


def test_wide_rejects_what_takes_m_up_to_8192(pm):
    """The GA, the other evaluation schemes, the no-allocation evaluation and
    the reduced polynomial keep the m <= 8192 limit and say so."""
    import torch
    d, p = _case("m8193_p5")
    m = d.shape[1]
    inst = pm.Instance(d, p)
    masks = gi.random_population(8, m, p, seed=7)
    fit = np.zeros(8, np.int64)
    for scheme in ("per_chromosome", "per_client"):
        with pytest.raises(pm.PmpError) as e:
            pm.pmp_eval_population(inst.handle, masks, fit, scheme=scheme)
        assert e.value.status == pm.PMP_EUNSUPPORTED
    dm = torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)
    dfit = torch.empty(8, dtype=torch.int64, device="cuda")
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_eval_population_noalloc(inst.handle, dm, dfit)
    assert e.value.status == pm.PMP_EUNSUPPORTED
    with pytest.raises(pm.PmpError) as e:
        pm.GA(inst, 64, 16, 3, 1)
    assert e.value.status == pm.PMP_EUNSUPPORTED
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_hbp_reduce(inst.handle)
    assert e.value.status == pm.PMP_EUNSUPPORTED
