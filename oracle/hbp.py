"""The reduced Hammer-Beresnev polynomial (Section 2.1, after Eq. (6), and
Example 1): TEST INFRASTRUCTURE ONLY, like the rest of this package.

Eq. (6) writes the cost as a sum over clients i of
    delta'_i1 + sum_{t>=1} delta'_{i,t+1} * prod_{r<=t} z_{pi'_ir}
(0-based here: term t of row i has coefficient delta'[i, t] and the monomial
"all of the first t facilities of row i are closed").  Monomials are sets, so
rows that share the set of their first t facilities give the same monomial;
the reduced polynomial adds their coefficients and drops monomials whose
coefficient is 0.  The constant collects every row's first term.

``hbp_reduce``   the reduced polynomial: constant, {set: coefficient}, and for
                 each set the first row (lowest index) where it occurs with a
                 positive coefficient, with its degree t.
``hbp_eval``     the reduced polynomial at an open set, term by term.
``hbp_rows``     the same polynomial as truncated walks: each set is charged
                 to its first row; row i keeps positions 0 .. K_i - 1 where
                 K_i - 1 is its last charged degree (rows charged nothing are
                 dropped) and E_i[f] = sum of its charged coefficients of
                 degree <= f.  A client then costs E_i[min(f_i, K_i - 1)] for
                 its first open position f_i, and the cost is
                 constant + sum over kept rows.
``hbp_walk_eval`` the cost from ``hbp_rows`` by that walk.

Parity: pinned by the reduced polynomial printed for Example 1, by brute
force over every open set of small instances (the reduced polynomial and the
walk both equal Eq. (1)), and by the coefficient-sum identity.
"""
from __future__ import annotations

import numpy as np

from . import tables


def hbp_reduce(d, p: int):
    """(constant, {frozenset: coefficient}, {frozenset: (row, degree)})."""
    pi, de, _ = tables(d, p)
    n, K = pi.shape
    const = int(de[:, 0].astype(np.int64).sum())
    coef: dict = {}
    first: dict = {}
    for i in range(n):
        for t in range(1, K):
            a = int(de[i, t])
            if a == 0:  # adds nothing; a set whose terms are all 0 is dropped
                continue
            s = frozenset(pi[i, :t].tolist())
            coef[s] = coef.get(s, 0) + a
            if s not in first:
                first[s] = (i, t)
    return const, coef, first


def hbp_eval(const: int, coef: dict, open_bits) -> int:
    """Reduced polynomial at an open set (bool vector over facilities): the
    constant plus every monomial none of whose facilities is open."""
    open_set = set(np.nonzero(np.asarray(open_bits))[0].tolist())
    return const + sum(a for s, a in coef.items() if not (s & open_set))


def hbp_rows(d, p: int):
    """(constant, K_rows (n,), E (n x K int64)) of the walk form; rows with
    K_rows[i] == 0 are dropped."""
    const, coef, first = hbp_reduce(d, p)
    pi, de, _ = tables(d, p)
    n, K = pi.shape
    charged = np.zeros((n, K), np.int64)
    for s, (i, t) in first.items():
        charged[i, t] = coef[s]
    K_rows = np.zeros(n, np.int64)
    for i in range(n):
        nz = np.nonzero(charged[i])[0]
        K_rows[i] = nz.max() + 1 if len(nz) else 0
    E = np.cumsum(charged, axis=1)
    return const, K_rows, E


def hbp_walk_eval(d, p: int, open_bits, rows=None) -> int:
    """The cost by the truncated walks of ``hbp_rows``."""
    const, K_rows, E = rows if rows is not None else hbp_rows(d, p)
    pi, _, _ = tables(d, p)
    ob = np.asarray(open_bits, bool)
    total = const
    for i in range(pi.shape[0]):
        if K_rows[i] == 0:
            continue
        f = 0
        while f < K_rows[i] - 1 and not ob[pi[i, f]]:
            f += 1
        total += int(E[i, f])
    return total


def hbp_terms_canonical(d, p: int):
    """The charged terms as (row, degree, coefficient), sorted by row then
    degree (the order the device lists them in)."""
    _, coef, first = hbp_reduce(d, p)
    return sorted((i, t, coef[s]) for s, (i, t) in first.items())
