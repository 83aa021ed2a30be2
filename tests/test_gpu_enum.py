"""GPU exhaustive enumeration (pmp_exhaustive) against the oracle's
exhaustive search: the least cost, the lexicographically first open set
attaining it (the tie rule matters on instances with many equal costs) and
the count C(m, p), bit for bit."""
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


CASES = [
    ("example1", lambda: gi.example1_matrix(), 2),
    ("G20", lambda: gi.graph_instance(20, 40, 0), 4),
    ("ties9x12", lambda: np.random.default_rng(1).integers(0, 4, (9, 12)).astype(np.int32), 3),
    ("ties7x15_p1", lambda: np.random.default_rng(2).integers(0, 3, (7, 15)).astype(np.int32), 1),
    ("p_m-1", lambda: np.random.default_rng(3).integers(0, 5, (10, 9)).astype(np.int32), 8),
    ("graph70_two_words", lambda: gi.graph_instance(70, 140, 4), 2),
    ("graph40_three_batches", lambda: gi.graph_instance(40, 80, 1), 5),
    ("G100_pmed1_shape", lambda: gi.graph_instance(100, 200, 0), 5),
]


@pytest.mark.parametrize("name,make,p", CASES, ids=[c[0] for c in CASES])
def test_exhaustive_matches_oracle(pm, name, make, p):
    d = make()
    print("enumerate", name, d.shape, p, flush=True)
    inst = pm.Instance(d, p)
    cost, mask, count = pm.pmp_exhaustive(inst.handle)
    ocost, omask, ocount = oracle.exhaustive(d, p)
    assert count == ocount
    assert cost == ocost
    np.testing.assert_array_equal(mask, omask)
    assert oracle.objective(d, mask[None], p)[0] == cost
    if name == "example1":
        assert cost == 35 and gi.unpack_masks(mask[None], 4)[0].tolist() == [1, 0, 0, 1]


def test_exhaustive_rejects_huge(pm):
    d = np.random.default_rng(0).integers(0, 9, (3, 200)).astype(np.int32)
    inst = pm.Instance(d, 100)
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_exhaustive(inst.handle)
    assert e.value.status == 5
