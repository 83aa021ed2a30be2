"""The no-allocation evaluation entry point (pmp_eval_population_noalloc)
against pmp_eval_population, through the C ABI.

Bar: bit-exact (int64 fitness, integer scan sums).  Each case makes two calls
in a row into the library's fixed workspace, the second with a smaller input,
so stale partial sums of the first call would show in the second.  The
oracle's direct-min objective is checked beside them on the small cases.
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


def _dev_masks(masks):
    import torch
    return torch.from_numpy(masks.view(np.int64)).cuda().view(torch.uint64)


def _both(pm, inst, masks):
    """(fitness, scan) from the allocating entry point and from the
    no-allocation one, on the same device masks."""
    import torch
    dm = _dev_masks(masks)
    P = masks.shape[0]
    f0 = torch.empty(P, dtype=torch.int64, device="cuda")
    s0 = torch.empty(P, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population(inst.handle, dm, f0, s0)
    f1 = torch.full((P,), -7, dtype=torch.int64, device="cuda")
    s1 = torch.full((P,), -7, dtype=torch.int64, device="cuda")
    pm.pmp_eval_population_noalloc(inst.handle, dm, f1, s1)
    torch.cuda.synchronize()
    return f0.cpu().numpy(), s0.cpu().numpy(), f1.cpu().numpy(), s1.cpu().numpy()


CASES = [
    # (name, instance builder, p, P of the first call, P of the second)
    ("g100", lambda: gi.graph_instance(100, 200, 0), 5, 700, 37),
    ("g900", lambda: gi.graph_instance(900, 16200, 0), 90, 1024, 65),
    ("euclid1200_p10", lambda: gi.euclid_instance(1200, 3), 10, 300, 1),
]


@pytest.mark.parametrize("name,make,p,P1,P2", CASES)
def test_two_calls_match_the_allocating_entry_point(pm, name, make, p, P1, P2):
    d = make()
    n, m = d.shape
    inst = pm.Instance(d, p)
    for call, P in enumerate((P1, P2)):
        _say("case", name, "call", call, "P", P)
        masks = gi.random_population(P, m, p, seed=11 + call)
        f0, s0, f1, s1 = _both(pm, inst, masks)
        np.testing.assert_array_equal(f1, f0)
        np.testing.assert_array_equal(s1, s0)
        np.testing.assert_array_equal(f1, oracle.objective(d, masks, p))


def _tiled_population(P, m, p, seed, distinct=1024):
    """P chromosomes: `distinct` random p-subsets repeated (cheap to make at
    large P)."""
    base = gi.random_population(distinct, m, p, seed=seed)
    reps = (P + distinct - 1) // distinct
    return np.ascontiguousarray(np.tile(base, (reps, 1))[:P])


def test_widened_tiles_then_a_smaller_call(pm):
    # Long scans (mean (m+1)/(p+1) = 273): the default tiling would take 47
    # client tiles of 64 clients x 16384 chromosomes, more cells than the
    # workspace holds, so the tiles are widened to 94 clients (32 tiles).
    # The next call (another instance, fewer chromosomes) reuses the cells.
    d = gi.euclid_instance(3000, 21)
    p = 10
    inst = pm.Instance(d, p)
    P = 16384
    _say("case widened tiles, P", P)
    masks = _tiled_population(P, 3000, p, seed=5)
    f0, s0, f1, s1 = _both(pm, inst, masks)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(f1[:1024], oracle.objective(d, masks[:1024], p))

    d2 = gi.graph_instance(90, 300, 2)
    inst2 = pm.Instance(d2, 9)
    masks2 = gi.random_population(130, 90, 9, seed=6)
    _say("case widened, second call P 130")
    f0, s0, f1, s1 = _both(pm, inst2, masks2)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(f1, oracle.objective(d2, masks2, 9))


def test_workspace_limit_then_a_smaller_call(pm):
    # P = PMP_NOALLOC_CELLS: one client tile of all n clients
    d = gi.euclid_instance(200, 22)
    p = 12
    inst = pm.Instance(d, p)
    P = pm.PMP_NOALLOC_CELLS
    _say("case workspace limit, P", P)
    masks = _tiled_population(P, 200, p, seed=7, distinct=2048)
    f0, s0, f1, s1 = _both(pm, inst, masks)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(s1, s0)
    np.testing.assert_array_equal(f1[:2048], oracle.objective(d, masks[:2048], p))
    masks2 = masks[:999].copy()
    _say("case workspace limit, second call P 999")
    f0, s0, f1, s1 = _both(pm, inst, masks2)
    np.testing.assert_array_equal(f1, f0)
    np.testing.assert_array_equal(s1, s0)


def test_fitness_only_and_async(pm):
    import torch
    d = gi.graph_instance(300, 1200, 4)
    p = 30
    inst = pm.Instance(d, p)
    masks = gi.random_population(257, 300, p, seed=8)
    dm = _dev_masks(masks)
    f = torch.empty(257, dtype=torch.int64, device="cuda")
    _say("case fitness only, async")
    pm.pmp_eval_population_noalloc(inst.handle, dm, f, None, asynchronous=True)
    pm.pmp_instance_check(inst.handle)
    np.testing.assert_array_equal(f.cpu().numpy(), oracle.objective(d, masks, p))


def test_rejects(pm):
    import torch
    d = gi.graph_instance(100, 200, 0)
    p = 5
    inst = pm.Instance(d, p)
    masks = gi.random_population(10, 100, p, seed=1)
    dm = _dev_masks(masks)
    f = torch.empty(10, dtype=torch.int64, device="cuda")
    L = pm.lib()
    import ctypes as C
    # host pointers (no PMP_ON_DEVICE)
    fh = np.zeros(10, np.int64)
    st = L.pmp_eval_population_noalloc(inst.handle, masks.ctypes.data_as(C.c_void_p), 10,
                                       fh.ctypes.data_as(C.c_void_p), None, 0, None)
    assert st == pm.PMP_EINVAL
    # a scheme flag
    st = L.pmp_eval_population_noalloc(inst.handle, C.c_void_p(dm.data_ptr()), 10,
                                       C.c_void_p(f.data_ptr()), None,
                                       pm.PMP_ON_DEVICE | pm.PMP_EVAL_PER_CLIENT, None)
    assert st == pm.PMP_EINVAL
    # more chromosomes than the workspace holds (rejected before any access)
    st = L.pmp_eval_population_noalloc(inst.handle, C.c_void_p(dm.data_ptr()),
                                       pm.PMP_NOALLOC_CELLS + 1, C.c_void_p(f.data_ptr()),
                                       None, pm.PMP_ON_DEVICE, None)
    assert st == pm.PMP_EINVAL
    # an infeasible chromosome
    bad = masks.copy()
    w0 = int(bad[3, 0])
    j = next(j for j in range(64) if not (w0 >> j) & 1)
    bad[3, 0] = np.uint64(w0 | (1 << j))  # p + 1 open facilities
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_eval_population_noalloc(inst.handle, _dev_masks(bad), f)
    assert e.value.status == pm.PMP_EINFEASIBLE
    # and a good call after it
    pm.pmp_eval_population_noalloc(inst.handle, dm, f)
    np.testing.assert_array_equal(f.cpu().numpy(), oracle.objective(d, masks, p))
