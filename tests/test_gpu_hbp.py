"""GPU construction and evaluation of the reduced Hammer-Beresnev polynomial
(pmp_hbp_*) against the oracle (oracle.hbp): the constant, every merged
monomial (owner row, degree, coefficient), the kept row lengths, and the
evaluation, bit for bit; at full size through properties that hold at any
size."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import pmp_inputs as gi
from oracle import hbp

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def pm():
    import torch
    assert torch.cuda.is_available()
    import paper_1610_10061_amd as pm
    pm.lib()
    return pm


def _walk_scan(d, p, masks, K_rows):
    """Positions the truncated walks read: sum over kept rows of
    min(first open position + 1, K_i)."""
    pi, _, _ = oracle.tables(d, p)
    bits = gi.unpack_masks(masks, d.shape[1])
    out = []
    for c in range(len(masks)):
        f = np.argmax(bits[c][pi], axis=1)
        out.append(int(np.where(K_rows > 0, np.minimum(f + 1, K_rows), 0).sum()))
    return np.array(out, np.int64)


def _check(pm, d, p, P=64, seed=0):
    n, m = d.shape
    inst = pm.Instance(d, p)
    h = pm.Hbp(inst)
    const, T, rows, maxlen = h.info()
    row, deg, coef, rl = h.terms()
    oc, ocoef, _ = hbp.hbp_reduce(d, p)
    _, K_rows, _ = hbp.hbp_rows(d, p)
    want = hbp.hbp_terms_canonical(d, p)
    assert const == oc
    assert T == len(ocoef) == len(want)
    assert list(zip(row.tolist(), deg.tolist(), coef.tolist())) == want
    np.testing.assert_array_equal(rl, K_rows)
    assert rows == int((K_rows > 0).sum())
    assert maxlen == (int(K_rows.max()) if rows else 0)
    masks = gi.random_population(P, m, p, seed=seed)
    fit = np.zeros(P, np.int64)
    scan = np.zeros(P, np.int64)
    pm.pmp_hbp_eval(h.handle, masks, fit, scan)
    np.testing.assert_array_equal(fit, oracle.objective(d, masks, p))
    np.testing.assert_array_equal(scan, _walk_scan(d, p, masks, K_rows))
    return h, inst


def test_example1(pm):
    with open(os.path.join(HERE, "golden", "example1.json")) as f:
        g = json.load(f)
    d = np.array(g["C"], np.int32)
    h, inst = _check(pm, d, 2, P=6)
    const, T, rows, maxlen = h.info()
    assert (const, T, rows, maxlen) == (33, 6, 4, 3)
    # every open pair
    bits = np.zeros((6, 4), bool)
    for r, s in enumerate(itertools.combinations(range(4), 2)):
        bits[r, list(s)] = True
    masks = gi.pack_masks(bits, 4)
    np.testing.assert_array_equal(h.eval(masks), oracle.objective(d, masks, 2))


def _dup(n, m, seed):
    rng = np.random.default_rng(seed)
    base = rng.integers(0, 60, size=(max(1, n // 4), m)).astype(np.int32)
    return base[rng.integers(0, len(base), size=n)]


CASES = {
    "ties_30x40": lambda: (np.random.default_rng(1).integers(0, 4, (30, 40)).astype(np.int32), 5),
    "dup_200x70": lambda: (_dup(200, 70, 2), 7),
    "rand_37x150": lambda: (np.random.default_rng(3).integers(0, 1000, (37, 150)).astype(np.int32), 20),
    "G100": lambda: (gi.graph_instance(100, 200, 0), 5),
    "E129": lambda: (gi.euclid_instance(129, 5), 3),
    "wide_3x700": lambda: (np.random.default_rng(6).integers(0, 9, (3, 700)).astype(np.int32), 350),
    "G300": lambda: (gi.graph_instance(300, 600, 4), 30),
}


@pytest.mark.parametrize("name", list(CASES))
def test_reduced_polynomial_matches_oracle(pm, name):
    d, p = CASES[name]()
    print("hbp case", name, d.shape, "p", p, flush=True)
    _check(pm, d, p, P=130, seed=len(name))


def test_g900_full_size(pm):
    """The G900 instance: monomials, rows and the evaluation of a population
    of 1024, all against the oracle."""
    d = gi.graph_instance(900, 16200, 0)
    print("hbp G900", flush=True)
    _check(pm, d, 90, P=1024, seed=11)


def test_e5000_full_size_properties(pm):
    """n = m = 5000, p = 100: the constant and the coefficient sum are fixed
    by the tables; sampled fitness values by the oracle's objective."""
    d = gi.euclid_instance(5000, 0)
    p = 100
    print("hbp E5000", flush=True)
    inst = pm.Instance(d, p)
    h = pm.Hbp(inst)
    const, T, rows, maxlen = h.info()
    _, _, ds = oracle.tables(d, p)
    row, deg, coef, rl = h.terms()
    assert const == int(ds[:, 0].astype(np.int64).sum())
    assert int(coef.sum()) == int((ds[:, -1].astype(np.int64) - ds[:, 0]).sum())
    assert (coef > 0).all() and len(coef) == T and rows == int((rl > 0).sum())
    assert (np.diff(row) >= 0).all() and (deg >= 1).all() and (deg < rl[row]).all()
    masks = gi.random_population(256, 5000, p, seed=3)
    fit = h.eval(masks)
    np.testing.assert_array_equal(fit[:16], oracle.objective(d, masks[:16], p))
    np.testing.assert_array_equal(fit, inst.eval(masks))


def test_all_rows_constant(pm):
    d = np.full((5, 6), 7, np.int32)
    inst = pm.Instance(d, 2)
    h = pm.Hbp(inst)
    assert h.info() == (35, 0, 0, 0)
    masks = gi.random_population(9, 6, 2, seed=1)
    np.testing.assert_array_equal(h.eval(masks), np.full(9, 35))
    bits = gi.unpack_masks(masks, 6)
    bits[3] = False
    bits[3, 0] = True
    with pytest.raises(pm.PmpError) as e:
        h.eval(gi.pack_masks(bits, 6))
    assert e.value.status == pm.PMP_EINFEASIBLE


def test_device_buffers_and_rejects(pm):
    import torch
    d, p = CASES["G100"]()
    inst = pm.Instance(d, p)
    h = pm.Hbp(inst)
    masks = gi.random_population(100, 100, p, seed=5)
    dm = torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)
    fit = torch.empty(100, dtype=torch.int64, device="cuda")
    pm.pmp_hbp_eval(h.handle, dm, fit, None, asynchronous=True)
    inst.check()
    np.testing.assert_array_equal(fit.cpu().numpy(), oracle.objective(d, masks, p))
    # m past 8128 (more than 127 words per chromosome) is served too
    dw = np.random.default_rng(0).integers(0, 9, (2, 8150)).astype(np.int32)
    wide = pm.Instance(dw, 5)
    hw = pm.Hbp(wide)
    mw = gi.random_population(3, 8150, 5, seed=1)
    fw = np.zeros(3, np.int64)
    pm.pmp_hbp_eval(hw.handle, mw, fw)
    np.testing.assert_array_equal(fw, oracle.objective(dw, mw, 5))
    with pytest.raises(pm.PmpError) as e:  # a chromosome with the wrong count
        pm.pmp_hbp_eval(hw.handle, gi.random_population(1, 8150, 6, seed=1), fw[:1])
    assert e.value.status == pm.PMP_EINFEASIBLE


def test_reduced_eval_at_the_facility_limit(pm):
    """m = PMP_MAX_FACILITIES: the reduced walk's stop needs no staged word
    beyond the chromosome's 128, so the largest tile serves it too."""
    n, m, p, P = 20, 8192, 1500, 70
    d = np.random.default_rng(4).integers(0, 50, size=(n, m)).astype(np.int32)
    print("case hbp m", m, "p", p, flush=True)
    inst = pm.Instance(d, p)
    h = pm.Hbp(inst)
    masks = gi.random_population(P, m, p, seed=2)
    fit = np.zeros(P, np.int64)
    scan = np.zeros(P, np.int64)
    pm.pmp_hbp_eval(h.handle, masks, fit, scan)
    np.testing.assert_array_equal(fit, oracle.objective(d, masks, p))
