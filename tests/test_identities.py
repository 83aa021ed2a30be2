"""CPU checks of the identities the device code relies on to run sequential
steps of the method in parallel.  Each test restates the parallel form in
plain Python, the way the kernels organise it, and compares it with the
sequential definition on many random cases.  No GPU and no product code:
these pin the reasoning, the GPU parity tests pin the kernels."""
import itertools
import math
import random

import pytest


# ---------------------------------------------------------------- Floyd
def floyd_sequential(m, p, draws):
    """Floyd's method: for j = m-p .. m-1 take draw t in [0, j], or j when t
    is already taken."""
    chosen = set()
    for e, j in enumerate(range(m - p, m)):
        t = draws[e]
        chosen.add(j if t in chosen else t)
    return chosen


def floyd_in_batches(m, p, draws):
    """The closed form in batches of 64 lanes: a draw is taken already when
    it repeats an earlier draw (an earlier batch, or a lower lane of this
    batch) or equals an earlier j whose own draw was taken; the latter is
    settled lowest lane first.  The subset is every draw plus j for each
    collided step."""
    off = m - p
    earlier = set()          # draws of earlier batches
    collided = [False] * p
    for base in range(0, p, 64):
        lanes = range(base, min(p, base + 64))
        col = {}
        pending = []
        for e in lanes:
            t = draws[e]
            rep = t in earlier or any(draws[x] == t for x in range(base, e))
            if rep:
                col[e] = True
            elif off <= t < off + e:
                tgt = t - off
                if tgt < base:
                    col[e] = collided[tgt]
                else:
                    pending.append((e, tgt))
            else:
                col[e] = False
        while pending:  # the lowest pending lane's target is always settled
            still = []
            for e, tgt in pending:
                if tgt in col:
                    col[e] = col[tgt]
                else:
                    still.append((e, tgt))
            assert len(still) < len(pending)
            pending = still
        for e in lanes:
            collided[e] = col[e]
            earlier.add(draws[e])
    return set(draws[:p]) | {off + e for e in range(p) if collided[e]}


def test_floyd_closed_form_matches_the_loop():
    rng = random.Random(7)
    for _ in range(4000):
        m = rng.choice([1, 2, 3, 7, 64, 65, 100, 129, 200, 300])
        p = rng.randint(1, m)
        # draws skewed towards [m-p, j] make chains through earlier j common
        draws = [rng.randint(0, j) if rng.random() < 0.5 else rng.randint(max(0, m - p), j)
                 for j in range(m - p, m)]
        got = floyd_in_batches(m, p, draws)
        assert got == floyd_sequential(m, p, draws)
        assert len(got) == p and all(0 <= x < m for x in got)


# ------------------------------------------------------- mutation cycle
def cycle_sequential(parent_cost, attempts):
    """Evolve step 5: attempts (differs, cost) in order; an attempt equal to
    the parent is not evaluated; stop at the first strict improvement."""
    evals, taken = 0, -1
    for a, (differs, cost) in enumerate(attempts):
        if not differs:
            continue
        evals += 1
        if cost < parent_cost:
            taken = a
            break
    return taken, evals


def cycle_at_once(parent_cost, attempts):
    """Every attempt evaluated; the first strictly fitter one in attempt
    order is taken; counted evaluations are the evaluated attempts up to it."""
    ok = [d for d, _ in attempts]
    imp = [d and c < parent_cost for d, c in attempts]
    first = next((a for a, v in enumerate(imp) if v), -1)
    upto = len(attempts) if first < 0 else first + 1
    counted = sum(ok[:upto])
    spec = sum(ok) - counted
    return first, counted, spec


def test_mutation_cycle_at_once_matches_the_loop():
    rng = random.Random(11)
    for _ in range(20000):
        Y = rng.randint(1, 20)
        parent = rng.randint(0, 50)
        attempts = [(rng.random() < 0.8, rng.randint(0, 60)) for _ in range(Y)]
        t_seq, e_seq = cycle_sequential(parent, attempts)
        t_all, e_all, spec = cycle_at_once(parent, attempts)
        assert (t_all, e_all) == (t_seq, e_seq)
        assert e_all + spec == sum(d for d, _ in attempts)


# ---------------------------------------------------- lexicographic ranks
def unrank(r, m, p):
    """Subset of lexicographic rank r: for the i-th element skip candidates
    x while the C(m-x-1, p-i-1) subsets starting with x come before r."""
    out, x = [], 0
    for i in range(p):
        while True:
            c = math.comb(m - x - 1, p - i - 1)
            if r < c:
                break
            r -= c
            x += 1
        out.append(x)
        x += 1
    return tuple(out)


@pytest.mark.parametrize("m,p", [(1, 1), (5, 2), (7, 7), (9, 4), (12, 1), (10, 9)])
def test_unranking_follows_lexicographic_order(m, p):
    for r, s in enumerate(itertools.combinations(range(m), p)):
        assert unrank(r, m, p) == s


# ------------------------------------------------ 64 x 64 bit transpose
_U = 0xFFFFFFFF
_M = {16: 0x0000FFFF, 8: 0x00FF00FF, 4: 0x0F0F0F0F, 2: 0x33333333, 1: 0x55555555}


def _rotr(y, s):
    s &= 31
    return ((y >> s) | (y << (32 - s))) & _U


def _byte_perm(own, partner, sel):
    """A byte permute of (own : partner): selector byte 4-7 takes own byte
    0-3, 0-3 takes partner byte 0-3."""
    b = [(partner >> (8 * i)) & 255 for i in range(4)] + [(own >> (8 * i)) & 255 for i in range(4)]
    return sum(b[(sel >> (8 * i)) & 255] << (8 * i) for i in range(4))


def transpose_by_lanes(lo, hi):
    """The evaluation's transpose as the lanes run it: lane l holds row l as
    (hi:lo).  Step 32 swaps the low words of lanes 32-63 with the high words
    of lanes 0-31; steps 16 and 8 merge own and partner (lane ^ J) bytes by
    a byte permute; steps 4, 2, 1 keep the bits whose index has bit J equal
    to the lane's and take the partner's rotated by J the other way."""
    lo, hi = lo[:], hi[:]
    for l in range(32):
        lo[l + 32], hi[l] = hi[l], lo[l + 32]
    sel = {16: (0x01000504, 0x07060302), 8: (0x02060004, 0x07030501)}
    for J in (16, 8, 4, 2, 1):
        ylo = [lo[l ^ J] for l in range(64)]
        yhi = [hi[l ^ J] for l in range(64)]
        for l in range(64):
            up = (l & J) != 0
            if J in sel:
                s = sel[J][1 if up else 0]
                lo[l] = _byte_perm(lo[l], ylo[l], s)
                hi[l] = _byte_perm(hi[l], yhi[l], s)
            else:
                keep = (~_M[J] & _U) if up else _M[J]
                r = J if up else 32 - J
                lo[l] = (lo[l] & keep) | (_rotr(ylo[l], r) & ~keep & _U)
                hi[l] = (hi[l] & keep) | (_rotr(yhi[l], r) & ~keep & _U)
    return lo, hi


def test_lane_transpose_is_the_bit_matrix_transpose():
    rng = random.Random(5)
    for _ in range(60):
        rows = [rng.getrandbits(64) for _ in range(64)]
        lo, hi = transpose_by_lanes([r & _U for r in rows], [r >> 32 for r in rows])
        for c in range(64):
            col = lo[c] | (hi[c] << 32)
            assert col == sum(((rows[k] >> c) & 1) << k for k in range(64))


def test_first_open_positions_from_the_transpose():
    """Row k = the chromosomes in which the facility at position k is open;
    after the transpose, chromosome c's lowest set bit is its first open
    position (and, with two clients in the halves, each half's)."""
    rng = random.Random(6)
    for _ in range(40):
        open_ = [[rng.random() < 0.1 for _ in range(64)] for _ in range(64)]  # [c][k]
        rows = [sum(open_[c][k] << c for c in range(64)) for k in range(64)]
        lo, hi = transpose_by_lanes([r & _U for r in rows], [r >> 32 for r in rows])
        for c in range(64):
            first = next((k for k in range(64) if open_[c][k]), -1)
            col = lo[c] | (hi[c] << 32)
            got = (col & -col).bit_length() - 1 if col else -1
            assert got == first
            first_b = next((k - 32 for k in range(32, 64) if open_[c][k]), -1)
            got_b = (hi[c] & -hi[c]).bit_length() - 1 if hi[c] else -1
            assert got_b == first_b
