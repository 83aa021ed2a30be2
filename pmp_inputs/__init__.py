"""Seeded synthetic inputs for the p-median hot path.

This module is shared by the CPU oracle side and the GPU side.  It holds only
input construction: distance matrices shaped like the paper's benchmark
families, random populations of p-subsets, and the bit packing of a chromosome
(m bits, bit j set when facility j is open; Section 4.1).  It holds none of
the method's arithmetic: no orderings, no gap terms, no objective, no genetic
operators.

Instance families (the paper's benchmark files are not available; these
stand in for their shapes):

* ``graph_instance``: a random connected undirected graph with integer edge
  weights, distances = all-pairs shortest paths (the OR-Library pmed family
  of Table 1 is built this way).
* ``euclid_instance``: integer points on a square grid, distance = the
  Euclidean length rounded half-up to an integer, computed exactly.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import dijkstra

__all__ = [
    "graph_instance", "euclid_instance", "random_population", "pack_masks",
    "unpack_masks", "words_for", "batch_specs", "batch_instance", "batch_instances",
    "example1_matrix",
]


def words_for(m: int) -> int:
    """Number of 64-bit words of one chromosome of m facilities."""
    return (m + 63) // 64


def _graph_edges(n: int, n_edges: int, rng: np.random.Generator,
                 wmin: int, wmax: int):
    """Random connected simple graph: a random spanning tree over a random
    vertex order (vertex order[k] joins a uniformly chosen earlier vertex),
    then distinct extra edges drawn uniformly, kept in draw order, until
    n_edges."""
    if n_edges < n - 1:
        raise ValueError("a connected graph on n vertices needs n-1 edges")
    if n_edges > n * (n - 1) // 2:
        raise ValueError("too many edges for a simple graph")
    order = rng.permutation(n).astype(np.int64)
    if n > 1:
        earlier = rng.integers(0, np.arange(1, n))
        a, b = order[1:], order[earlier]
    else:
        a = b = np.zeros(0, np.int64)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    keys = lo * n + hi
    seen = set(keys.tolist())
    chosen = [keys]
    have = len(keys)
    while have < n_edges:
        need = n_edges - have
        cand = rng.integers(0, n, size=(2 * need + 16, 2))
        x, y = cand[:, 0], cand[:, 1]
        ok = x != y
        k2 = np.minimum(x, y)[ok] * n + np.maximum(x, y)[ok]
        # first occurrence of each new key, in draw order
        _, first = np.unique(k2, return_index=True)
        k2 = k2[np.sort(first)]
        fresh = np.fromiter((k not in seen for k in k2.tolist()), bool, len(k2))
        k2 = k2[fresh][:need]
        seen.update(k2.tolist())
        chosen.append(k2)
        have += len(k2)
    keys = np.concatenate(chosen)
    edges = np.stack([keys // n, keys % n], axis=1)
    w = rng.integers(wmin, wmax + 1, size=len(edges))
    return edges.astype(np.int64), w.astype(np.int64)


def graph_weights(n: int, n_edges: int, seed: int, wmin: int = 1,
                  wmax: int = 100) -> np.ndarray:
    """n x n int32 arc weights of the random connected graph that
    graph_instance(n, n_edges, seed) measures: both arcs of every edge carry
    its weight, -1 where there is no edge, 0 on the diagonal."""
    rng = np.random.default_rng([0x6772617068, seed, n, n_edges])
    e, w = _graph_edges(n, n_edges, rng, wmin, wmax)
    out = np.full((n, n), -1, np.int32)
    out[e[:, 0], e[:, 1]] = w
    out[e[:, 1], e[:, 0]] = w
    np.fill_diagonal(out, 0)
    return out


def graph_instance(n: int, n_edges: int, seed: int, wmin: int = 1,
                   wmax: int = 100) -> np.ndarray:
    """n x n int32 shortest-path distance matrix of a random connected graph.

    Shortest paths are unique as lengths, so the Dijkstra-per-source solver
    used here yields exactly the matrix Floyd-Warshall would.
    """
    rng = np.random.default_rng([0x6772617068, seed, n, n_edges])
    e, w = _graph_edges(n, n_edges, rng, wmin, wmax)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    vals = np.concatenate([w, w]).astype(np.float64)
    g = coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    dist = dijkstra(g, directed=True)
    if not np.all(np.isfinite(dist)):
        raise RuntimeError("generated graph is not connected")
    out = np.rint(dist).astype(np.int64)
    if out.max() >= 2**31:
        raise OverflowError("distance exceeds int32")
    return out.astype(np.int32)


def euclid_instance(n: int, seed: int, grid: int = 10_000) -> np.ndarray:
    """n x n int32 matrix of rounded Euclidean distances between n random
    integer points in [0, grid)^2 (the same points are clients and
    facilities).  Rounding is half-up, done exactly in integers:
    r = isqrt(s), d = r + (s - r*r > r)."""
    rng = np.random.default_rng([0x6575636C, seed, n, grid])
    pts = rng.integers(0, grid, size=(n, 2), dtype=np.int64)
    dx = pts[:, None, 0] - pts[None, :, 0]
    dy = pts[:, None, 1] - pts[None, :, 1]
    s = dx * dx + dy * dy
    r = np.floor(np.sqrt(s.astype(np.float64))).astype(np.int64)
    # repair the float estimate to the exact integer square root
    r -= (r * r > s)
    r += ((r + 1) * (r + 1) <= s)
    d = r + ((s - r * r) > r)
    return d.astype(np.int32)


def example1_matrix() -> np.ndarray:
    """The 5 x 4 cost matrix of the paper's Example 1 (Section 2.1), p = 2."""
    return np.array([[7, 10, 16, 11],
                     [15, 17, 7, 7],
                     [10, 4, 6, 6],
                     [7, 11, 18, 12],
                     [10, 22, 14, 8]], dtype=np.int32)


def pack_masks(open_sets, m: int) -> np.ndarray:
    """Pack a P x m 0/1 array (or a list of index lists) into P x W uint64."""
    if isinstance(open_sets, np.ndarray) and open_sets.ndim == 2 \
            and open_sets.shape[1] == m:
        bits = open_sets.astype(bool)
    else:
        bits = np.zeros((len(open_sets), m), dtype=bool)
        for r, s in enumerate(open_sets):
            bits[r, list(s)] = True
    P = bits.shape[0]
    W = words_for(m)
    padded = np.zeros((P, W * 64), dtype=np.uint8)
    padded[:, :m] = bits
    by = np.packbits(padded, axis=1, bitorder="little")
    return by.view(np.uint64).reshape(P, W).copy()


def unpack_masks(masks: np.ndarray, m: int) -> np.ndarray:
    """P x W uint64 -> P x m bool."""
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    by = masks.view(np.uint8).reshape(masks.shape[0], -1)
    bits = np.unpackbits(by, axis=1, bitorder="little")
    return bits[:, :m].astype(bool)


def random_population(P: int, m: int, p: int, seed: int) -> np.ndarray:
    """P uniformly random p-subsets of {0..m-1}, packed as P x W uint64."""
    rng = np.random.default_rng([0x706F70, seed, P, m, p])
    keys = rng.random((P, m))
    idx = np.argpartition(keys, p - 1, axis=1)[:, :p] if p < m else \
        np.tile(np.arange(m), (P, 1))
    bits = np.zeros((P, m), dtype=bool)
    np.put_along_axis(bits, idx, True, axis=1)
    return pack_masks(bits, m)


def batch_specs(count: int = 256, seed: int = 0, nmin: int = 100,
                nmax: int = 2000):
    """Shapes of the ragged batch: instance b has n = m drawn log-uniform in
    [nmin, nmax], p uniform in [5, n // 4]; even b is a shortest-path graph
    with 4n edges, odd b a Euclidean grid instance."""
    specs = []
    for b in range(count):
        rng = np.random.default_rng([0x6261746368, seed, b])
        n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
        p = int(rng.integers(5, n // 4 + 1))
        kind = "graph" if b % 2 == 0 else "euclid"
        specs.append({"index": b, "n": n, "m": n, "p": p, "kind": kind,
                      "seed": seed * 100003 + b})
    return specs


def batch_instance(spec) -> np.ndarray:
    if spec["kind"] == "graph":
        return graph_instance(spec["n"], 4 * spec["n"], spec["seed"])
    return euclid_instance(spec["n"], spec["seed"])


def batch_instances(specs, workers: int = 8):
    """All instances of a batch, built on a thread pool (the shortest-path
    and distance computations release the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(batch_instance, specs))
