"""Oracle of the learned swap proposal (not in the paper).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU-baseline leg call it; the product never
does.  Plain numpy, written from the definitions (the same ones the C header
of the library states), sharing nothing with the GPU code.

* ``feature_sums`` / ``features``  the 16 per-facility features of a
  chromosome, straight from d: positions in a client's row are ranks under
  the key (d_ij, j) (the order of Section 2.1, ties to the lower index),
  truncated to K = m - p + 1 as after Eq. (6).
* ``static_sums``   column sums of d, near counts (j among the first
  L = ceil(m/p) of a row).
* ``candidates`` / ``explore_draws``  the Philox draws of the proposal.
* ``init_params``, ``forward``, ``backward``, ``adam``  the scoring network:
  32 -> 128 -> 128 -> 1 with ReLU; weights, inputs and the first hidden
  activations rounded to BF16 (nearest even); everything else in float64;
  the gradient treats the roundings as identity; Adam as Kingma & Ba (2015).
* ``target``        the training target of an evaluated swap.
* ``population_after_crossover``  generation 0 of the GA up to the end of its
  crossover stages (Section 3, Evolve steps 1-3), from the oracle's own
  sampler, objective and crossover.
"""
from __future__ import annotations

import math

import numpy as np

from . import objective, stream_draws, sample_subset, crossover, ROLE_EVOLVE

FEATURES = 16
N_IN, N_HID = 32, 128
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_HID * N_IN
OFF_W2 = OFF_B1 + N_HID
OFF_B2 = OFF_W2 + N_HID * N_HID
OFF_W3 = OFF_B2 + N_HID
OFF_B3 = OFF_W3 + N_HID
N_PARAMS = OFF_B3 + 1

ROLE_MODEL = 3
TAG_WEIGHTS = 4
TAG_PROPOSE = 5
TAG_EXPLORE = 6


# ---------------------------------------------------------------- features
def _ranks(d):
    """order[i] = facilities by (d_ij, j); rank[i, j] = position of j."""
    n, m = d.shape
    order = np.argsort(d, axis=1, kind="stable")
    rank = np.empty_like(order)
    rank[np.arange(n)[:, None], order] = np.arange(m)[None, :]
    return order, rank


def feature_sums(d, bits, p):
    """Integer sums of one chromosome (bits: m bools, exactly p true).

    Per client i: a_i, c1_i = first open facility and cost; b_i, c2_i = the
    second open facility and cost when its position is below K, else no b_i
    and c2_i = the K-th smallest d_i (position K - 1).  Returns a dict of
    int64 arrays (length m) and f."""
    d = np.asarray(d, dtype=np.int64)
    bits = np.asarray(bits, dtype=bool)
    n, m = d.shape
    K = m - p + 1
    order, rank = _ranks(d)
    rows = np.arange(n)
    R = np.where(bits[None, :], rank, m + 1)
    s1 = R.min(axis=1)
    a = order[rows, s1]
    c1 = d[rows, a]
    R2 = R.copy()
    R2[rows, a] = m + 1
    s2 = R2.min(axis=1)
    has_b = s2 < K
    b = np.where(has_b, order[rows, np.minimum(s2, m - 1)], -1)
    kth = d[rows, order[:, K - 1]]
    c2 = np.where(has_b, d[rows, np.maximum(b, 0)], kth)
    z = lambda: np.zeros(m, np.int64)  # noqa: E731
    count, served, loss, cnt2, c2share = z(), z(), z(), z(), z()
    np.add.at(count, a, 1)
    np.add.at(served, a, c1)
    np.add.at(loss, a, c2 - c1)
    np.add.at(cnt2, b[has_b], 1)
    np.add.at(c2share, b[has_b], (c2 - c1)[has_b])
    closed = ~bits[None, :]
    ahead_m = closed & (rank < s1[:, None])
    end = np.where(has_b, s2, K)
    between_m = closed & (rank > s1[:, None]) & (rank < end[:, None])
    ahead = ahead_m.sum(axis=0).astype(np.int64)
    gain = ((c1[:, None] - d) * ahead_m).sum(axis=0)
    bcount = between_m.sum(axis=0).astype(np.int64)
    bgain = ((c2[:, None] - d) * between_m).sum(axis=0)
    return {"count": count, "served": served, "loss": loss, "cnt2": cnt2,
            "c2share": c2share, "ahead": ahead, "gain": gain, "bcount": bcount,
            "bgain": bgain, "f": int(c1.sum())}


def static_sums(d, p):
    """(colsum, total, near, L): column sums of d, their total, and the
    number of rows holding j among their first L = ceil(m/p) positions."""
    d = np.asarray(d, dtype=np.int64)
    n, m = d.shape
    L = -(-m // p)
    _, rank = _ranks(d)
    near = (rank < L).sum(axis=0).astype(np.int64)
    colsum = d.sum(axis=0)
    return colsum, int(colsum.sum()), near, L


def _q(a, b, c):
    """(float)(a * b / c) in double, elementwise."""
    return (np.asarray(a, np.float64) * np.float64(b) / np.asarray(c, np.float64)
            ).astype(np.float32)


def features(d, bits, p, gen_frac, static=None):
    """The 16 features of every facility of one chromosome: m x 16 float32."""
    d = np.asarray(d, dtype=np.int64)
    n, m = d.shape
    bits = np.asarray(bits, dtype=bool)
    S = feature_sums(d, bits, p)
    colsum, total, near, L = static if static is not None else static_sums(d, p)
    F = float(max(S["f"], 1))
    T = float(max(total, 1))
    o = bits
    out = np.zeros((m, FEATURES), np.float32)
    zero = np.float32(0)
    out[:, 0] = np.where(o, 1.0, 0.0)
    out[:, 1] = np.where(o, _q(S["count"], p, n), zero)
    out[:, 2] = np.where(o, _q(S["served"], p, F), zero)
    out[:, 3] = np.where(o, _q(S["loss"], p, F), zero)
    out[:, 4] = np.where(o, _q(S["cnt2"], p, n), zero)
    out[:, 5] = np.where(o, _q(S["c2share"], p, F), zero)
    out[:, 6] = np.where(o, zero, _q(S["ahead"], p, n))
    out[:, 7] = np.where(o, zero, _q(S["gain"], p, F))
    out[:, 8] = np.where(o, zero, _q(S["bcount"], p, n))
    out[:, 9] = np.where(o, zero, _q(S["bgain"], p, F))
    out[:, 10] = _q(colsum, m, T)
    out[:, 11] = _q(near, m, float(n) * float(L))
    out[:, 12] = np.float32(np.float64(p) / np.float64(m))
    out[:, 13] = _q(S["f"], m, T)
    out[:, 14] = np.float32(gen_frac)
    out[:, 15] = 1.0
    return out


# ------------------------------------------------------- proposal draws
def _nth(bits, r, want):
    return int(np.flatnonzero(np.asarray(bits, bool) == want)[r])


def candidates(seed, gen, chrom, bits, p, C):
    """Candidate swaps (j open, k closed) of chromosome `chrom`: candidate t
    draws r_j in [0, p) and r_k in [0, m - p) from stream (seed, role 2;
    gen, chrom, tag 5, stage t); j / k = the r_j-th open / r_k-th closed
    facility in index order."""
    m = len(bits)
    out = []
    for t in range(C):
        rj, rk = stream_draws(seed, ROLE_EVOLVE, gen, chrom, TAG_PROPOSE, t, [p, m - p])
        out.append((_nth(bits, int(rj), True), _nth(bits, int(rk), False)))
    return out


def explore_draws(seed, gen, chrom, attempt, C):
    """(e, u) of attempt `attempt`: e in [0, 1000), u in [0, C)."""
    e, u = stream_draws(seed, ROLE_EVOLVE, gen, chrom, TAG_EXPLORE, attempt, [1000, C])
    return int(e), int(u)


def target(delta, f, p):
    """Normalised change of cost, clamped to [-4, 4]."""
    v = float(delta) * float(p) / float(f if f > 0 else 1)
    return np.float32(min(4.0, max(-4.0, v)))


# ------------------------------------------------------------- network
def bf16(x):
    """Round float32 values to the nearest BF16 (ties to even); float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of float32 values, rounded to nearest."""
    return (bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(h):
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32)


def split(params):
    q = np.asarray(params, dtype=np.float64)
    return (q[OFF_W1:OFF_B1].reshape(N_HID, N_IN), q[OFF_B1:OFF_W2],
            q[OFF_W2:OFF_B2].reshape(N_HID, N_HID), q[OFF_B2:OFF_W3],
            q[OFF_W3:OFF_B3], q[OFF_B3])


def init_params(seed):
    """Glorot-uniform weights (Glorot & Bengio 2010), zero biases: parameter
    k takes the first word x of stream (seed, role 3; 0, k, tag 4, 0),
    u = (x >> 40) / 2^24 and the value (2u - 1) a in float32, with
    a = sqrt(6 / (fan_in + fan_out))."""
    out = np.zeros(N_PARAMS, np.float32)
    spans = [(OFF_W1, OFF_B1, N_IN + N_HID), (OFF_W2, OFF_B2, N_HID + N_HID),
             (OFF_W3, OFF_B3, N_HID + 1)]
    for lo, hi, fan in spans:
        a = np.sqrt(np.float32(6.0) / np.float32(fan), dtype=np.float32)
        for k in range(lo, hi):
            x = int(stream_draws(seed, ROLE_MODEL, 0, k, TAG_WEIGHTS, 0, [0])[0])
            u = np.float32(x >> 40) * np.float32(1.0 / 16777216.0)
            out[k] = (np.float32(2.0) * u - np.float32(1.0)) * a
    return out


def forward(params, X, rounding=True):
    """Scores of rows X (rows x 32).  Returns (y, cache) in float64."""
    W1, b1, W2, b2, w3, b3 = split(params)
    r = (lambda v: bf16(np.asarray(v, np.float32)).astype(np.float64)) if rounding \
        else (lambda v: np.asarray(v, np.float64))
    x = r(X)
    W1r, W2r, w3r = r(W1), r(W2), r(w3)
    z1 = x @ W1r.T + b1
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ W2r.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3r + b3
    return y, (x, W1r, W2r, w3r, z1, h1, z2, h2)


def backward(params, X, T, w=None, rounding=True):
    """Gradient (N_PARAMS, float64) and loss of
    L = sum_r w_r (y_r - t_r)^2 / (2 sum_r w_r), roundings as identity."""
    y, (x, W1r, W2r, w3r, z1, h1, z2, h2) = forward(params, X, rounding)
    T = np.asarray(T, np.float64)
    w = np.ones(len(T)) if w is None else np.asarray(w, np.float64)
    N = w.sum()
    e = y - T
    loss = float((w * e * e).sum() / (2 * N))
    dy = w * e / N
    g = np.zeros(N_PARAMS)
    g[OFF_B3] = dy.sum()
    g[OFF_W3:OFF_B3] = h2.T @ dy
    dz2 = np.outer(dy, w3r) * (z2 > 0)
    g[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    g[OFF_W2:OFF_B2] = (dz2.T @ h1).ravel()
    dz1 = (dz2 @ W2r) * (z1 > 0)
    g[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    g[OFF_W1:OFF_B1] = (dz1.T @ x).ravel()
    return g, loss


def adam(params, m1, m2, grad, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns (params, m1, m2) in float64."""
    m1 = beta1 * np.asarray(m1, np.float64) + (1 - beta1) * grad
    m2 = beta2 * np.asarray(m2, np.float64) + (1 - beta2) * grad * grad
    mh = m1 / (1 - beta1 ** t)
    vh = m2 / (1 - beta2 ** t)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m1, m2


# --------------------------------------------------------- GA helper
def _bits(mask, m):
    w = np.asarray(mask, np.uint64)
    by = w.view(np.uint8)
    return np.unpackbits(by, bitorder="little")[:m].astype(bool)


def population_after_crossover(d, p, P, NT, seed, X=0):
    """Generation 0 of the GA through its crossover stages: (masks P x W,
    fitness P).  X = 0 means lg NT stages; none when p < 2 or NT = 1."""
    d = np.ascontiguousarray(d, dtype=np.int32)
    n, m = d.shape
    lg = int(math.log2(NT))
    X = X if X > 0 else lg
    pop = np.stack([sample_subset(seed, 0, c, m, p) for c in range(P)])
    fit = objective(d, pop, p)
    if p < 2 or lg == 0:
        return pop, fit
    for k in range(X):
        stride = NT >> (1 + k % lg)
        snap = pop.copy()
        offs, ok = {}, {}
        for c in range(P):
            partner = c ^ stride
            leader = min(c, partner)
            r1, i = stream_draws(seed, ROLE_EVOLVE, 0, leader, 2, k, [m, p // 2])
            good, F = crossover(snap[c], snap[partner], m, int(r1), 1 + int(i))
            if good:
                offs[c] = F
        if offs:
            cs = sorted(offs)
            ofit = objective(d, np.stack([offs[c] for c in cs]), p)
            for c, f in zip(cs, ofit):
                if f < fit[c]:
                    pop[c] = offs[c]
                    fit[c] = f
    return pop, fit
