"""Pins of the reduced Hammer-Beresnev polynomial (oracle.hbp): the reduced
polynomial printed for the paper's Example 1, brute force over every open set
of small instances (both the term-by-term value and the truncated walks equal
the cost of Eq. (1) computed straight from d), and the coefficient-sum
identity."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import pmp_inputs as gi
from oracle import hbp

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "example1.json")) as f:
        return json.load(f)


def test_example1_reduced_polynomial_as_printed():
    g = _golden()
    d = np.array(g["C"], np.int32)
    const, coef, first = hbp.hbp_reduce(d, g["p"])
    printed = g["reduced_polynomial"]["terms"]
    want_const = [a for a, s in printed if not s]
    want = {frozenset(j - 1 for j in s): a for a, s in printed if s}
    assert [const] == want_const == [33]
    assert coef == want
    assert 1 + len(coef) == 7 and g["entries"] == 15
    # truncated walks: client 3 (0-based) repeats client 0's monomials and
    # is dropped; client 1 keeps its zero first term to reach z3 z4
    c, K_rows, E = hbp.hbp_rows(d, g["p"])
    assert c == 33 and K_rows.tolist() == [3, 3, 2, 0, 3]
    assert E[1, :3].tolist() == [0, 0, 8] and E[0, :3].tolist() == [0, 7, 9]


def _small(kind, n, m, seed):
    rng = np.random.default_rng(seed)
    if kind == "ties":
        return rng.integers(0, 4, size=(n, m)).astype(np.int32)
    if kind == "dup":  # repeated clients: rows that merge completely
        base = rng.integers(0, 50, size=(max(1, n // 3), m)).astype(np.int32)
        return base[rng.integers(0, len(base), size=n)]
    return rng.integers(0, 100, size=(n, m)).astype(np.int32)


@pytest.mark.parametrize("kind,n,m,p,seed", [
    ("rand", 6, 7, 3, 0), ("ties", 7, 6, 2, 1), ("dup", 9, 7, 3, 2),
    ("ties", 5, 8, 1, 3), ("rand", 4, 8, 6, 4), ("dup", 12, 6, 4, 5)])
def test_brute_force_every_open_set(kind, n, m, p, seed):
    d = _small(kind, n, m, seed)
    const, coef, _ = hbp.hbp_reduce(d, p)
    rows = hbp.hbp_rows(d, p)
    sets = list(itertools.combinations(range(m), p))
    bits = np.zeros((len(sets), m), bool)
    for r, s in enumerate(sets):
        bits[r, list(s)] = True
    want = oracle.objective(d, gi.pack_masks(bits, m), p)
    for r in range(len(sets)):
        assert hbp.hbp_eval(const, coef, bits[r]) == want[r]
        assert hbp.hbp_walk_eval(d, p, bits[r], rows) == want[r]


@pytest.mark.parametrize("name,d,p", [
    ("G100", gi.graph_instance(100, 200, 0), 5),
    ("E120", gi.euclid_instance(120, 3), 12)])
def test_coefficient_sum_and_walk_on_larger_instances(name, d, p):
    pi, de, ds = oracle.tables(d, p)
    const, coef, first = hbp.hbp_reduce(d, p)
    assert const == int(ds[:, 0].astype(np.int64).sum())
    # every positive gap term is in exactly one merged coefficient
    assert sum(coef.values()) == int((ds[:, -1].astype(np.int64) - ds[:, 0]).sum())
    assert all(a > 0 for a in coef.values())
    # the first occurrence of a set sits at its degree, in the lowest row
    for s, (i, t) in first.items():
        assert t == len(s) and frozenset(pi[i, :t].tolist()) == s
    rows = hbp.hbp_rows(d, p)
    masks = gi.random_population(20, d.shape[1], p, seed=4)
    bits = gi.unpack_masks(masks, d.shape[1])
    want = oracle.objective(d, masks, p)
    for r in range(20):
        assert hbp.hbp_walk_eval(d, p, bits[r], rows) == want[r]
