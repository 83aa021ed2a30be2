"""CPU oracle for the p-median hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product library never imports
this package and this package never imports the product.

Thin ctypes wrappers around ``pmp_oracle.c`` (plain C, built with gcc), plus
``tables_numpy``, a second construction of the tables from numpy library
routines used to pin the C one.

Functions and the passages they follow:

* ``objective``      Eq. (1)-(3): cost = sum over clients of the least distance
                     to an open facility, straight from d; optional scan
                     lengths (position of the serving facility in Pi^i).
* ``tables``         Section 2.1: Pi, Delta, truncated to K = m-p+1 columns.
* ``bc_eval``        Eq. (6) evaluated by the walk of Section 4.2.
* ``exhaustive``     Eq. (1)-(3) minimised over all C(m,p) open sets.
* ``philox``         Philox4x64-10 (Salmon et al., SC 2011).
* ``stream_draws``   bounded draws (Lemire 2019) from one counter stream.
* ``sample_subset``  Section 4.1, read as a uniform p-subset (Floyd 1987).
* ``crossover``      Section 4.3.
* ``mutate``         Section 4.4.
* ``ga_run``         Section 3 (host steps 7-16, Evolve steps 1-8).
* ``apsp``           shortest-path cost matrix of a graph (Floyd 1962).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

ROLE_INIT = 1
ROLE_EVOLVE = 2
TAG_INIT = 1
TAG_XOVER = 2
TAG_MUT = 3

ST_GEN, ST_SAT, ST_DONE, ST_BEST, ST_CHROM_EVALS, ST_XO_FAIL, ST_XO_TAKEN, \
    ST_MUT_TAKEN, ST_COUNT = range(9)

_p = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_u64 = C.c_uint64


class OracleError(RuntimeError):
    pass


class _GaParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("population", C.c_int32),
                ("group_size", C.c_int32), ("generations", C.c_int32),
                ("saturation", C.c_int32), ("crossover_iters", C.c_int32),
                ("mutation_iters", C.c_int32), ("migration", C.c_int32),
                ("init", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_objective.argtypes = [_p, _i64, _i32, _i32, _i32, _p, _i32, _p, _p, _i32]
        L.orc_tables.argtypes = [_p, _i64, _i32, _i32, _i32, _i32, _p, _p, _p]
        L.orc_bc_eval.argtypes = [_p, _p, _i32, _i32, _i32, _p, _i32, _p, _p]
        L.orc_exhaustive.argtypes = [_p, _i64, _i32, _i32, _i32, _p, _p, _p, _i32]
        L.orc_philox4x64.argtypes = [_p, _p, _p]
        L.orc_apsp.argtypes = [_p, _i32, _p]
        L.orc_unrank.argtypes = [_u64, _i32, _i32, _p]
        L.orc_philox4x64.restype = None
        L.orc_stream_draws.argtypes = [_u64, _u64, _u64, _u64, _u64, _u64, _p, _i32, _p]
        L.orc_sample_subset.argtypes = [_u64, _u64, _u64, _i32, _i32, _p]
        L.orc_crossover.argtypes = [_p, _p, _i32, _i32, _i32, _p]
        L.orc_mutate.argtypes = [_u64, _u64, _u64, _u64, _p, _i32, _p, _p]
        L.orc_ga_run.argtypes = [_p, _i64, _i32, _i32, _i32, C.POINTER(_GaParams),
                                 _i32, _p, _p, _p, _p, _p, _p, _p, _i32]
        L.orc_default_threads.argtypes = []
        L.orc_default_threads.restype = C.c_int
        _lib = L
    return _lib


def default_threads() -> int:
    """Threads the oracle uses when a call passes threads=0."""
    return int(lib().orc_default_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _d(d):
    d = np.ascontiguousarray(d, dtype=np.int32)
    if d.ndim != 2:
        raise ValueError("d must be 2-D")
    return d


def _check(rc, what):
    if rc != 0:
        raise OracleError(f"{what}: oracle returned {rc}")


def objective(d, masks, p: int = 0, scan: bool = False, threads: int = 0,
              strict: bool = True):
    """Eq. (1)-(3): int64 cost of every chromosome (and, with scan=True, the
    summed scan lengths).  p > 0 also requires popcount == p."""
    d = _d(d)
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    P = masks.shape[0]
    n, m = d.shape
    cost = np.zeros(P, np.int64)
    st = np.zeros(P, np.int64) if scan else None
    rc = lib().orc_objective(_ptr(d), m, n, m, p, _ptr(masks), P, _ptr(cost),
                             _ptr(st) if scan else None, threads)
    if strict:
        _check(rc, "objective")
    return (cost, st) if scan else cost


def tables(d, p: int, ncols: int = 0):
    """Section 2.1: (pi, delta, dsorted), each n x K int32 (K = m-p+1 unless
    ncols is given)."""
    d = _d(d)
    n, m = d.shape
    K = ncols if ncols > 0 else m - p + 1
    pi = np.zeros((n, K), np.int32)
    de = np.zeros((n, K), np.int32)
    ds = np.zeros((n, K), np.int32)
    _check(lib().orc_tables(_ptr(d), m, n, m, p, K, _ptr(pi), _ptr(de),
                            _ptr(ds)), "tables")
    return pi, de, ds


def tables_numpy(d, p: int, ncols: int = 0):
    """The same tables from numpy library routines: a stable argsort orders
    equal distances by index; the gaps are a first difference."""
    d = np.asarray(d, dtype=np.int64)
    n, m = d.shape
    K = ncols if ncols > 0 else m - p + 1
    order = np.argsort(d, axis=1, kind="stable")
    srt = np.take_along_axis(d, order, axis=1)
    gaps = np.diff(srt, axis=1, prepend=0)
    return (order[:, :K].astype(np.int32), gaps[:, :K].astype(np.int32),
            srt[:, :K].astype(np.int32))


def bc_eval(pi, delta, masks, m: int, strict: bool = True):
    """Eq. (6) by the walk of Section 4.2.  Returns (cost, scan_total)."""
    pi = np.ascontiguousarray(pi, dtype=np.int32)
    delta = np.ascontiguousarray(delta, dtype=np.int32)
    masks = np.ascontiguousarray(masks, dtype=np.uint64)
    n, K = pi.shape
    P = masks.shape[0]
    cost = np.zeros(P, np.int64)
    st = np.zeros(P, np.int64)
    rc = lib().orc_bc_eval(_ptr(pi), _ptr(delta), n, K, m, _ptr(masks), P,
                           _ptr(cost), _ptr(st))
    if strict:
        _check(rc, "bc_eval")
    return cost, st


def exhaustive(d, p: int, threads: int = 0):
    """Least cost over all C(m,p) open sets; returns (cost, mask, count)."""
    d = _d(d)
    n, m = d.shape
    W = (m + 63) // 64
    best = np.zeros(1, np.int64)
    mask = np.zeros(W, np.uint64)
    cnt = np.zeros(1, np.int64)
    _check(lib().orc_exhaustive(_ptr(d), m, n, m, p, _ptr(best), _ptr(mask),
                                _ptr(cnt), threads), "exhaustive")
    return int(best[0]), mask, int(cnt[0])


def unrank(r: int, m: int, p: int):
    """The p-subset of lexicographic rank r (packed mask), Section 4.1."""
    mask = np.zeros((m + 63) // 64, np.uint64)
    _check(lib().orc_unrank(r, m, p, _ptr(mask)), "unrank")
    return mask


def apsp(w):
    """Shortest path lengths of the graph with arc weights w (n x n int32,
    negative = no arc), by Floyd-Warshall; -1 where there is no path."""
    w = _d(w)
    n = w.shape[0]
    if w.shape != (n, n):
        raise ValueError("w must be square")
    d = np.zeros((n, n), np.int32)
    _check(lib().orc_apsp(_ptr(w), n, _ptr(d)), "apsp")
    return d


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_ptr(c), _ptr(k), _ptr(out))
    return out


def stream_draws(seed, role, gen, chrom, tag, stage, bounds):
    """Consecutive draws from one stream; bound 0 means a raw 64-bit word."""
    b = np.ascontiguousarray(bounds, dtype=np.uint64)
    out = np.zeros(len(b), np.uint64)
    _check(lib().orc_stream_draws(seed, role, gen, chrom, tag, stage, _ptr(b),
                                  len(b), _ptr(out)), "stream_draws")
    return out


def sample_subset(seed, gen, chrom, m, p):
    mask = np.zeros((m + 63) // 64, np.uint64)
    _check(lib().orc_sample_subset(seed, gen, chrom, m, p, _ptr(mask)),
           "sample_subset")
    return mask


def crossover(a, b, m, r1, i):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    f = np.zeros_like(a)
    ok = lib().orc_crossover(_ptr(a), _ptr(b), m, r1, i, _ptr(f))
    if ok < 0:
        raise OracleError("crossover: bad arguments")
    return bool(ok), f


def mutate(seed, gen, chrom, attempt, a, m):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    f = np.zeros_like(a)
    desc = np.zeros(5, np.int32)
    _check(lib().orc_mutate(seed, gen, chrom, attempt, _ptr(a), m, _ptr(f),
                            _ptr(desc)), "mutate")
    return f, tuple(int(x) for x in desc)


class GaState:
    """Resumable GA state: everything the next generation depends on."""

    def __init__(self, n, m, p, population, group_size, generations, seed,
                 saturation=0, crossover_iters=0, mutation_iters=0, migration=0, init=0):
        self.n, self.m, self.p = n, m, p
        self.params = _GaParams(seed, population, group_size, generations,
                                saturation, crossover_iters, mutation_iters,
                                migration, init)
        W = (m + 63) // 64
        NB = population // group_size
        self.pop = np.zeros((population, W), np.uint64)
        self.fit = np.zeros(population, np.int64)
        self.gbest_mask = np.zeros((NB, W), np.uint64)
        self.gbest_cost = np.zeros(NB, np.int64)
        self.best_mask = np.zeros(W, np.uint64)
        self.state = np.zeros(ST_COUNT, np.int64)
        self.state[ST_BEST] = np.iinfo(np.int64).max

    @property
    def generation(self):
        return int(self.state[ST_GEN])

    @property
    def best_cost(self):
        return int(self.state[ST_BEST])

    @property
    def done(self):
        return bool(self.state[ST_DONE])


def ga_run(d, st: GaState, gens: int, threads: int = 0):
    """Advance the GA state by up to `gens` generations; returns the per
    generation best-cost trace of this call."""
    d = _d(d)
    n, m = d.shape
    trace = np.full(max(gens, 1), -1, np.int64)
    _check(lib().orc_ga_run(_ptr(d), m, n, m, st.p, C.byref(st.params), gens,
                            _ptr(st.pop), _ptr(st.fit), _ptr(st.gbest_mask),
                            _ptr(st.gbest_cost), _ptr(st.best_mask),
                            _ptr(st.state), _ptr(trace), threads), "ga_run")
    return trace[:gens]
