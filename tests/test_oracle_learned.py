"""Pins of the learned-proposal oracle (oracle/learned.py), CPU only.

Every check compares the oracle with something other than itself: hand-worked
values on the paper's Example 1, a pure-Python brute force of the feature
definitions, exact cost changes from the C objective (Eq. (1)-(3) straight
from d), closed-form networks, finite differences, torch autograd and
torch.optim.Adam, torch's BF16 conversion, and distribution checks.
"""
import json
import os

import numpy as np
import pytest

import oracle
import oracle.learned as OL
import pmp_inputs as gi

HERE = os.path.dirname(os.path.abspath(__file__))


def _bits(masks, m):
    return gi.unpack_masks(np.atleast_2d(masks), m)


def test_example1_feature_sums_by_hand():
    g = json.load(open(os.path.join(HERE, "golden", "example1_features.json")))
    d = gi.example1_matrix()
    bits = np.zeros(4, bool)
    bits[g["open"]] = True
    S = OL.feature_sums(d, bits, 2)
    assert S["f"] == g["f"]
    for k in ("count", "served", "loss", "cnt2", "c2share", "ahead", "gain",
              "bcount", "bgain"):
        assert S[k].tolist() == g[k], k
    colsum, total, near, L = OL.static_sums(d, 2)
    assert colsum.tolist() == g["colsum"] and total == g["total"]
    assert L == g["near_len"] and near.tolist() == g["near"]
    # the swap neighbours' costs are the example's printed ones
    for (j, k), key in (((0, 1), "close_0_open_1"), ((3, 1), "close_3_open_1")):
        b = bits.copy()
        b[j], b[k] = False, True
        cost = oracle.objective(d, gi.pack_masks(b[None], 4), 2)[0]
        assert cost == g["swaps"][key]


def _brute_sums(d, bits, p):
    """The definitions, one client at a time, with Python's sorted()."""
    n, m = d.shape
    K = m - p + 1
    out = {k: [0] * m for k in ("count", "served", "loss", "cnt2", "c2share",
                                "ahead", "gain", "bcount", "bgain")}
    f = 0
    for i in range(n):
        row = sorted(range(m), key=lambda j: (int(d[i, j]), j))
        opens = [s for s, j in enumerate(row) if bits[j]]
        s1 = opens[0]
        a, c1 = row[s1], int(d[i, row[s1]])
        s2 = opens[1] if len(opens) > 1 and opens[1] < K else None
        c2 = int(d[i, row[s2]]) if s2 is not None else int(d[i, row[K - 1]])
        f += c1
        out["count"][a] += 1
        out["served"][a] += c1
        out["loss"][a] += c2 - c1
        if s2 is not None:
            b = row[s2]
            out["cnt2"][b] += 1
            out["c2share"][b] += c2 - c1
        end = s2 if s2 is not None else K
        for s, j in enumerate(row):
            if bits[j]:
                continue
            if s < s1:
                out["ahead"][j] += 1
                out["gain"][j] += c1 - int(d[i, j])
            elif s1 < s < end:
                out["bcount"][j] += 1
                out["bgain"][j] += c2 - int(d[i, j])
    return out, f


@pytest.mark.parametrize("n,m,p,seed", [(7, 9, 1, 0), (7, 9, 2, 1), (9, 7, 3, 2),
                                        (6, 10, 9, 3), (12, 12, 4, 4)])
def test_feature_sums_brute_force(n, m, p, seed):
    rng = np.random.default_rng(seed)
    d = rng.integers(0, 6, size=(n, m)).astype(np.int32)  # many ties
    masks = gi.random_population(5, m, p, seed)
    for bits in _bits(masks, m):
        S = OL.feature_sums(d, bits, p)
        ref, f = _brute_sums(d, bits, p)
        assert S["f"] == f
        for k, v in ref.items():
            assert S[k].tolist() == v, k


@pytest.mark.parametrize("kind,n,p,seed", [("graph", 60, 6, 0), ("euclid", 80, 8, 1),
                                           ("euclid", 50, 2, 2)])
def test_loss_and_gain_are_exact_cost_changes(kind, n, p, seed):
    """Opening closed k changes the cost by -gain_k; closing open j (p - 1
    open) by +loss_j whenever each of j's clients has a second open facility
    inside the truncated row (then c2 is exact)."""
    d = gi.graph_instance(n, 2 * n, seed) if kind == "graph" else gi.euclid_instance(n, seed)
    m = n
    masks = gi.random_population(4, m, p, seed + 10)
    K = m - p + 1
    for bits in _bits(masks, m):
        S = OL.feature_sums(d, bits, p)
        f = int(oracle.objective(d, gi.pack_masks(bits[None], m), p)[0])
        assert S["f"] == f
        plus, minus = [], []
        for j in range(m):
            b = bits.copy()
            b[j] = not b[j]
            (plus if not bits[j] else minus).append((j, b))
        cp = oracle.objective(d, gi.pack_masks(np.stack([b for _, b in plus]), m), 0)
        for (k, _), c in zip(plus, cp):
            assert c - f == -S["gain"][k]
        if p >= 2:
            cm = oracle.objective(d, gi.pack_masks(np.stack([b for _, b in minus]), m), 0)
            order = np.argsort(d, axis=1, kind="stable")
            for (j, _), c in zip(minus, cm):
                # clients of j whose second open facility lies beyond K
                ok = True
                for i in range(n):
                    row = order[i]
                    opens = [s for s in range(m) if bits[row[s]]]
                    if row[opens[0]] == j and opens[1] >= K:
                        ok = False
                if ok:
                    assert c - f == S["loss"][j]


def test_feature_sum_identities():
    d = gi.euclid_instance(120, 3)
    p = 12
    masks = gi.random_population(6, 120, p, 4)
    cost, scan = oracle.objective(d, masks, p, scan=True)
    for bits, f, s in zip(_bits(masks, 120), cost, scan):
        S = OL.feature_sums(d, bits, p)
        assert S["count"].sum() == 120
        assert S["served"].sum() == f
        assert S["ahead"].sum() == s - 120  # entries before the serving one
        assert S["loss"].sum() >= S["c2share"].sum()
        for k in ("count", "served", "loss", "cnt2", "c2share"):
            assert not S[k][~bits].any()
        for k in ("ahead", "gain", "bcount", "bgain"):
            assert not S[k][bits].any()
        F = OL.features(d, bits, p, 0.25)
        assert F.shape == (120, 16) and F.dtype == np.float32
        assert abs(F[:, 1].sum() - p) < 1e-3 and abs(F[:, 2].sum() - p) < 1e-3
        assert np.all(F[:, 15] == 1) and np.all(F[:, 14] == np.float32(0.25))
        assert np.all(F[:, 12] == np.float32(p / 120))


def test_swap_change_bound():
    """For a swap (close j, open k): change <= loss_j - gain_k, with
    equality when no client of j has d_ik below its second cost."""
    d = gi.graph_instance(40, 80, 7)
    p, m = 5, 40
    bits = _bits(gi.random_population(1, m, p, 8), m)[0]
    S = OL.feature_sums(d, bits, p)
    f = S["f"]
    order = np.argsort(d, axis=1, kind="stable")
    K = m - p + 1
    rows = range(40)
    first = [next(order[i][s] for s in range(m) if bits[order[i][s]]) for i in rows]
    opens_pos = [[s for s in range(m) if bits[order[i][s]]] for i in rows]
    if any(op[1] >= K for op in opens_pos):
        pytest.skip("a row without its second open facility inside K")
    c2 = [int(d[i, order[i][opens_pos[i][1]]]) for i in rows]
    for j in np.flatnonzero(bits):
        for k in np.flatnonzero(~bits):
            b = bits.copy()
            b[j], b[k] = False, True
            delta = int(oracle.objective(d, gi.pack_masks(b[None], m), p)[0]) - f
            bound = int(S["loss"][j] - S["gain"][k])
            assert delta <= bound
            if all(d[i, k] >= c2[i] for i in rows if first[i] == j):
                assert delta == bound


# ------------------------------------------------------------- network
def test_bf16_matches_torch_rounding():
    import torch
    rng = np.random.default_rng(0)
    x = (rng.standard_normal(10000) * np.exp(rng.uniform(-20, 20, 10000))).astype(np.float32)
    x[:4] = [0.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8)]  # ties
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(OL.bf16(x), ref)
    np.testing.assert_array_equal(OL.from_bf16_bits(OL.bf16_bits(x)), ref)


def test_forward_closed_form():
    """A network built to compute y = x_0 - x_5 + 3: hidden unit 0 =
    relu(x_0), 1 = relu(-x_0), 2 = relu(x_5), 3 = relu(-x_5), passed on by the
    second layer; exact for BF16-representable inputs."""
    q = np.zeros(OL.N_PARAMS, np.float32)
    W1 = np.zeros((128, 32), np.float32)
    W1[0, 0], W1[1, 0], W1[2, 5], W1[3, 5] = 1, -1, 1, -1
    W2 = np.zeros((128, 128), np.float32)
    for u in range(4):
        W2[u, u] = 1
    w3 = np.zeros(128, np.float32)
    w3[:4] = [1, -1, -1, 1]
    q[OL.OFF_W1:OL.OFF_B1] = W1.ravel()
    q[OL.OFF_W2:OL.OFF_B2] = W2.ravel()
    q[OL.OFF_W3:OL.OFF_B3] = w3
    q[OL.OFF_B3] = 3.0
    rng = np.random.default_rng(1)
    X = OL.bf16(rng.standard_normal((50, 32)).astype(np.float32))
    y, _ = OL.forward(q, X)
    np.testing.assert_array_equal(y, X[:, 0].astype(np.float64) - X[:, 5] + 3.0)


def _random_params(seed, scale=0.2):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(OL.N_PARAMS) * scale).astype(np.float32)


def test_backward_finite_differences():
    q = _random_params(2).astype(np.float64)
    rng = np.random.default_rng(3)
    X = rng.standard_normal((20, 32))
    T = rng.standard_normal(20)
    w = (rng.random(20) < 0.7).astype(np.float64)
    g, _ = OL.backward(q, X, T, w, rounding=False)
    idx = np.concatenate([rng.choice(np.arange(OL.OFF_W1, OL.OFF_B1), 20, replace=False),
                          rng.choice(np.arange(OL.OFF_B1, OL.OFF_W2), 5, replace=False),
                          rng.choice(np.arange(OL.OFF_W2, OL.OFF_B2), 30, replace=False),
                          rng.choice(np.arange(OL.OFF_B2, OL.OFF_W3), 5, replace=False),
                          rng.choice(np.arange(OL.OFF_W3, OL.OFF_B3), 10, replace=False),
                          [OL.OFF_B3]])
    h = 1e-6
    for k in idx:
        a, b = q.copy(), q.copy()
        a[k] += h
        b[k] -= h
        la = OL.backward(a, X, T, w, rounding=False)[1]
        lb = OL.backward(b, X, T, w, rounding=False)[1]
        fd = (la - lb) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 + 1e-5 * abs(g[k]), k


def test_backward_matches_torch_autograd():
    """The BF16-rounded forward in torch float64, roundings passed through as
    identity (x + (round(x) - x).detach()), differentiated by autograd."""
    import torch
    q = _random_params(4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((64, 32)).astype(np.float32)
    T = rng.standard_normal(64)
    w = (rng.random(64) < 0.8).astype(np.float64)
    g, loss = OL.backward(q, X, T, w)

    def rnd(v):
        r = v.to(torch.float32).to(torch.bfloat16).to(torch.float64)
        return v + (r - v).detach()

    P = torch.tensor(q.astype(np.float64), requires_grad=True)
    W1 = P[OL.OFF_W1:OL.OFF_B1].reshape(128, 32)
    b1 = P[OL.OFF_B1:OL.OFF_W2]
    W2 = P[OL.OFF_W2:OL.OFF_B2].reshape(128, 128)
    b2 = P[OL.OFF_B2:OL.OFF_W3]
    w3 = P[OL.OFF_W3:OL.OFF_B3]
    b3 = P[OL.OFF_B3]
    x = rnd(torch.tensor(X, dtype=torch.float64))
    h1 = rnd(torch.relu(x @ rnd(W1).T + b1))
    h2 = torch.relu(h1 @ rnd(W2).T + b2)
    y = h2 @ rnd(w3) + b3
    wt = torch.tensor(w)
    L = (wt * (y - torch.tensor(T)) ** 2).sum() / (2 * wt.sum())
    L.backward()
    np.testing.assert_allclose(loss, L.item(), rtol=1e-12)
    np.testing.assert_allclose(g, P.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_adam_matches_torch():
    import torch
    rng = np.random.default_rng(6)
    q = rng.standard_normal(100)
    P = torch.tensor(q.copy(), requires_grad=True)
    opt = torch.optim.Adam([P], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m1 = np.zeros(100)
    m2 = np.zeros(100)
    for t in range(1, 6):
        g = rng.standard_normal(100)
        P.grad = torch.tensor(g)
        opt.step()
        q, m1, m2 = OL.adam(q, m1, m2, g, 1e-2, t)
    np.testing.assert_allclose(q, P.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_init_distribution():
    q = OL.init_params(7)
    assert q.shape == (OL.N_PARAMS,) and q.dtype == np.float32
    for lo, hi, fan in ((OL.OFF_W1, OL.OFF_B1, 160), (OL.OFF_W2, OL.OFF_B2, 256),
                        (OL.OFF_W3, OL.OFF_B3, 129)):
        a = np.sqrt(6.0 / fan)
        v = q[lo:hi].astype(np.float64)
        assert np.all(np.abs(v) <= a)
        assert abs(v.mean()) < 4 * a / np.sqrt(3 * len(v))
        # sample variance of a uniform: relative spread sqrt(0.8 / count)
        assert abs(v.var() / (a * a / 3) - 1) < 5 * np.sqrt(0.8 / len(v))
    for lo, hi in ((OL.OFF_B1, OL.OFF_W2), (OL.OFF_B2, OL.OFF_W3), (OL.OFF_B3, OL.N_PARAMS)):
        assert not q[lo:hi].any()
    assert not np.array_equal(q, OL.init_params(8))


# ------------------------------------------------------------- proposal
def test_candidates_valid_and_uniform():
    m, p, C = 20, 4, 64
    bits = np.zeros(m, bool)
    bits[[1, 5, 6, 17]] = True
    cj = np.zeros(m, int)
    ck = np.zeros(m, int)
    for chrom in range(60):
        for j, k in OL.candidates(3, 2, chrom, bits, p, C):
            assert bits[j] and not bits[k]
            cj[j] += 1
            ck[k] += 1
    nj, nk = cj[bits], ck[~bits]
    ej, ek = 60 * C / p, 60 * C / (m - p)
    assert ((nj - ej) ** 2 / ej).sum() < 16.3   # chi2, 3 dof, p = 0.001
    assert ((nk - ek) ** 2 / ek).sum() < 39.3   # chi2, 15 dof, p = 0.001
    e, u = zip(*(OL.explore_draws(3, 2, c, a, 7) for c in range(50) for a in range(4)))
    assert 0 <= min(e) and max(e) < 1000 and 0 <= min(u) and max(u) < 7


def test_target_normalisation():
    assert OL.target(-50, 1000, 10) == np.float32(-0.5)
    assert OL.target(10 ** 9, 1000, 10) == np.float32(4.0)
    assert OL.target(-10 ** 9, 1000, 10) == np.float32(-4.0)
    assert OL.target(3, 0, 2) == np.float32(4.0)


def test_population_after_crossover_invariants():
    d = gi.graph_instance(50, 100, 2)
    p, P, NT = 5, 32, 16
    pop, fit = OL.population_after_crossover(d, p, P, NT, seed=4)
    init = np.stack([oracle.sample_subset(4, 0, c, 50, p) for c in range(P)])
    f0 = oracle.objective(d, init, p)
    np.testing.assert_array_equal(fit, oracle.objective(d, pop, p))
    assert np.all(fit <= f0) and np.any(fit < f0)
    pop1, fit1 = OL.population_after_crossover(d, p, P, 1, seed=4)  # no partners
    np.testing.assert_array_equal(pop1, init)
