"""GPU all-pairs shortest paths (pmp_apsp, blocked Floyd-Warshall) against
the oracle's plain Floyd-Warshall, bit for bit, on ragged tile counts,
directed graphs with unreachable pairs and zero-weight arcs, and the graph
instances of the workloads (whose distance matrices the input generator
also measures with scipy's Dijkstra)."""
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


def _digraph(n, density, wmax, seed):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, wmax + 1, size=(n, n)).astype(np.int32)
    w[rng.random((n, n)) >= density] = -1
    w[(rng.random((n, n)) < 0.05) & (w >= 0)] = 0
    return w


@pytest.mark.parametrize("n,density,wmax,seed", [
    (1, 1.0, 9, 0), (2, 0.5, 9, 1), (5, 0.4, 9, 2), (63, 0.05, 1000, 3),
    (64, 0.05, 1000, 4), (65, 0.05, 1000, 5), (129, 0.02, 100000, 6),
    (300, 0.01, 1000, 7), (200, 0.002, 50, 8)])
def test_apsp_matches_oracle(pm, n, density, wmax, seed):
    print("apsp digraph", n, density, wmax, seed, flush=True)
    w = _digraph(n, density, wmax, seed)
    np.testing.assert_array_equal(pm.pmp_apsp(w), oracle.apsp(w))


@pytest.mark.parametrize("n,e,seed", [(100, 200, 0), (900, 16200, 0), (2000, 8000, 7)])
def test_apsp_graph_instances(pm, n, e, seed):
    """The workloads' graphs: G100, G900 and the largest batch graph."""
    print("apsp graph", n, e, seed, flush=True)
    w = gi.graph_weights(n, e, seed)
    d = pm.pmp_apsp(w)
    np.testing.assert_array_equal(d, gi.graph_instance(n, e, seed))
    if n <= 900:
        np.testing.assert_array_equal(d, oracle.apsp(w))


def test_apsp_device_tensors(pm):
    import torch
    w = gi.graph_weights(300, 1200, 3)
    wd = torch.from_numpy(w).cuda()
    dd = pm.pmp_apsp(wd)
    np.testing.assert_array_equal(dd.cpu().numpy(), oracle.apsp(w))
    out = torch.full((300, 300), 7, dtype=torch.int32, device="cuda")
    pm.pmp_apsp(wd, out)
    np.testing.assert_array_equal(out.cpu().numpy(), oracle.apsp(w))


def test_apsp_rejects(pm):
    big = np.full((3, 3), -1, np.int32)
    big[0, 1] = big[1, 2] = 2**30
    with pytest.raises(pm.PmpError) as e:
        pm.pmp_apsp(big)
    assert e.value.status == pm.PMP_EUNSUPPORTED
    with pytest.raises(ValueError):
        pm.pmp_apsp(np.zeros((3, 4), np.int32))
