"""Pins of the oracle's all-pairs shortest paths (oracle.apsp, Floyd 1962)
against routines and facts that do not share its code: scipy's
Floyd-Warshall and Dijkstra, brute force over all simple paths on tiny
graphs, and the metric properties of the result."""
import itertools

import numpy as np
import pytest
from scipy.sparse.csgraph import csgraph_from_dense, floyd_warshall

import oracle
import pmp_inputs as gi


def _random_digraph(n, density, wmax, seed, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    w = rng.integers(0, wmax + 1, size=(n, n)).astype(np.int32)
    w[rng.random((n, n)) >= density] = -1
    if zero_frac:
        w[(rng.random((n, n)) < zero_frac) & (w >= 0)] = 0
    return w


def _scipy(w):
    """scipy's Floyd-Warshall; zero-weight arcs go in as explicit edges
    (a dense array would read 0 as "no edge")."""
    dense = np.where(w >= 0, w.astype(np.float64), np.inf)
    g = csgraph_from_dense(dense, null_value=np.inf)
    out = floyd_warshall(g, directed=True)
    return np.where(np.isfinite(out), out, -1).astype(np.int64)


@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (2, 0.5, 1), (7, 0.3, 2),
                                            (40, 0.1, 3), (97, 0.05, 4), (150, 0.02, 5)])
def test_apsp_matches_scipy_floyd_warshall(n, density, seed):
    w = _random_digraph(n, density, 1000, seed, zero_frac=0.1)
    np.testing.assert_array_equal(oracle.apsp(w), _scipy(w))


def test_apsp_brute_force_simple_paths():
    for seed in range(30):
        n = 5
        w = _random_digraph(n, 0.45, 9, 100 + seed, zero_frac=0.15)
        got = oracle.apsp(w)
        for s, t in itertools.product(range(n), range(n)):
            best = 0 if s == t else None
            if s != t:
                others = [v for v in range(n) if v not in (s, t)]
                for r in range(len(others) + 1):
                    for mid in itertools.permutations(others, r):
                        path = (s,) + mid + (t,)
                        ws = [w[a, b] for a, b in zip(path, path[1:])]
                        if min(ws) >= 0 and (best is None or sum(ws) < best):
                            best = sum(ws)
            assert got[s, t] == (-1 if best is None else best), (seed, s, t)


def test_apsp_of_generated_graph_equals_its_distance_matrix():
    """graph_instance measures the same graph with scipy's Dijkstra."""
    for n, e, seed in [(100, 200, 0), (300, 900, 1), (64, 63, 2)]:
        w = gi.graph_weights(n, e, seed)
        d = oracle.apsp(w)
        np.testing.assert_array_equal(d, gi.graph_instance(n, e, seed))
        # a metric: symmetric, zero diagonal, triangle inequality
        assert (d == d.T).all() and (np.diag(d) == 0).all()
        if n <= 100:  # d[i, j] <= d[i, k] + d[k, j], indexed [i, k, j]
            assert (d[:, None, :] <= d[:, :, None] + d[None, :, :]).all()


def test_apsp_unreachable_and_overflow():
    w = np.full((3, 3), -1, np.int32)
    w[0, 1] = 5
    d = oracle.apsp(w)
    assert d[0, 1] == 5 and d[1, 0] == -1 and d[0, 2] == -1 and (np.diag(d) == 0).all()
    big = np.full((3, 3), -1, np.int32)
    big[0, 1] = big[1, 2] = 2**31 - 10
    with pytest.raises(oracle.OracleError):
        oracle.apsp(big)
