"""Worked derivation of GA generations, written out step by step from the
paper's description and kept apart from oracle/ (it imports nothing from it,
nor from the GPU library).  It writes ga_generation.json: every random draw,
every operator's parameters, offspring and accept decision, and the state
after each generation, for two small instances:

* Example 1 of Section 2.1 (5 clients, 4 facilities, p = 2), one generation;
* an 8-cycle (d = cycle distance, many equal costs), p = 4, two generations
  (so migration is exercised too).

Population P = 8 in groups of NT = 4 (NB = 2, lg NT = 2: two crossover
stages with strides 2 and 1, two mutation attempts).

Steps, as the paper gives them (Section 3.1 host steps 7-16, Section 3.2
Evolve steps 1-8, Sections 4.1, 4.3-4.5), with the readings this project
takes where the paper is silent:
  population  every slot a uniform p-subset (Floyd's sampling), except, from
              the second generation on, slot b*NT holds group b's best;
  crossover   stage k pairs slot t with t XOR (NT >> (1 + k mod lg NT)); the
              lower slot of the pair draws r1 in [0, m) and i in [1, p//2];
              each partner walks the positions r1, r1+1, ... (mod m) where the
              parents differ, switching on its first i zeros and off its
              first i ones; fewer than i of either kind: no offspring; the
              offspring replaces its parent only if strictly cheaper; both
              partners read the parents as the stage found them;
  mutation    up to lg NT attempts on the chromosome as crossover left it,
              stopping at its first strict improvement; an attempt draws the
              kind (circular / block), the direction (right = towards higher
              index / left) and either a shift s in [1, m-1], or a block
              [a, b] (a uniform pair of distinct positions) and s in
              [1, b-a]; an offspring equal to its parent is not evaluated;
  bests       least cost, lowest slot on ties, per group; the global best
              only changes on a strict improvement.
Random words: Philox4x64-10 blocks from numpy.random.Philox, key (seed,
role), counter (generation, chromosome, tag << 32 | stage, block); role 1
tag 1 for sampling, role 2 tag 2 for crossover, tag 3 for mutation.  A
bounded draw below r takes a word x and returns floor(x r / 2^64), taking a
fresh word while (x r mod 2^64) < (2^64 - r) mod r (Lemire 2019).

Run from the repository root: python tests/golden/derive_ga_generation.py
"""
from __future__ import annotations

import json
import os

import numpy as np

M64 = (1 << 64) - 1
HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "ga_generation.json")

EXAMPLE1 = [[7, 10, 16, 11], [15, 17, 7, 7], [10, 4, 6, 6], [7, 11, 18, 12],
            [10, 22, 14, 8]]


def cycle8():
    return [[min(abs(i - j), 8 - abs(i - j)) for j in range(8)] for i in range(8)]


def philox_block(seed, role, ctr):
    """One 4-word block for the 256-bit counter ctr (numpy's generator
    increments its counter before producing a block, so it starts one
    below)."""
    c = sum(int(w) << (64 * k) for k, w in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    words = np.array([(c >> (64 * k)) & M64 for k in range(4)], dtype=np.uint64)
    g = np.random.Philox(counter=words, key=np.array([seed, role], dtype=np.uint64))
    return [int(x) for x in g.random_raw(4)]


class Stream:
    def __init__(self, seed, role, gen, chrom, tag, stage):
        self.seed, self.role = seed, role
        self.ctr = [gen, chrom, (tag << 32) | stage, 0]
        self.ctr0 = self.ctr[:3]
        self.words = []
        self.log = []          # (bound, words taken, value)

    def word(self):
        if not self.words:
            self.words = philox_block(self.seed, self.role, self.ctr)
            self.ctr[3] += 1
        return self.words.pop(0)

    def below(self, r):
        taken = [self.word()]
        low = (taken[-1] * r) & M64
        if low < r:
            floor_ = ((1 << 64) - r) % r
            while low < floor_:
                taken.append(self.word())
                low = (taken[-1] * r) & M64
        v = (taken[-1] * r) >> 64
        self.log.append({"bound": r, "words": [f"{w:#018x}" for w in taken], "value": v})
        return v

    def where(self):
        """key and counter words 0-2 of the stream (word 3 = block index)."""
        return {"key": [self.seed, self.role], "counter": self.ctr0}


def cost(d, opened):
    return sum(min(row[j] for j in opened) for row in d)


def floyd(st, m, p):
    chosen = set()
    for j in range(m - p, m):
        t = st.below(j + 1)
        chosen.add(j if t in chosen else t)
    return sorted(chosen)


def crossover(A, B, m, r1, i):
    """A, B sets of open facilities; offspring set or None."""
    F = set(A)
    on = off = 0
    for t in range(m):
        if on == i and off == i:
            break
        j = (r1 + t) % m
        if (j in A) == (j in B):
            continue
        if j not in A and on < i:
            F.add(j)
            on += 1
        elif j in A and off < i:
            F.discard(j)
            off += 1
    return sorted(F) if (on == i and off == i) else None


def mutate(st, A, m):
    bits = [1 if j in A else 0 for j in range(m)]
    kind = st.below(2)
    right = st.below(2) == 0
    if kind == 0:
        s = 1 + st.below(m - 1)
        move = s if right else m - s
        out = [0] * m
        for j in range(m):
            out[(j + move) % m] = bits[j]
        desc = {"kind": "circular", "dir": "right" if right else "left", "s": s}
    else:
        x = st.below(m)
        y = st.below(m - 1)
        if y >= x:
            y += 1
        a, b = min(x, y), max(x, y)
        s = 1 + st.below(b - a)
        block = bits[a:b + 1]
        L = len(block)
        move = s if right else L - s
        rolled = [0] * L
        for q in range(L):
            rolled[(q + move) % L] = block[q]
        out = bits[:a] + rolled + bits[b + 1:]
        desc = {"kind": "block", "dir": "right" if right else "left", "a": a, "b": b, "s": s}
    return sorted(j for j in range(m) if out[j]), desc


def run(d, p, P, NT, seed, generations):
    m = len(d[0])
    NB, lg = P // NT, NT.bit_length() - 1
    X = Y = lg
    gens = []
    pop, fit = [None] * P, [None] * P
    gbest = [None] * NB
    best = None
    counters = {"evals": 0, "xo_fail": 0, "xo_taken": 0, "mut_taken": 0}
    for g in range(generations):
        rec = {"generation": g, "population": [], "crossover": [], "mutation": []}
        for c in range(P):
            if g > 0 and c % NT == 0:
                pop[c] = list(gbest[c // NT][0])
                rec["population"].append({"slot": c, "migrant_of_group": c // NT,
                                          "open": pop[c]})
            else:
                st = Stream(seed, 1, g, c, 1, 0)
                pop[c] = floyd(st, m, p)
                rec["population"].append({"slot": c, "stream": st.where(), "draws": st.log,
                                          "open": pop[c]})
        fit = [cost(d, pop[c]) for c in range(P)]
        counters["evals"] += P
        rec["fitness_after_population"] = list(fit)
        for k in range(X):
            stride = NT >> (1 + k % lg)
            snap = [list(x) for x in pop]
            stage = {"stage": k, "stride": stride, "pairs": []}
            for c in range(P):
                partner = c ^ stride
                leader = min(c, partner)
                st = Stream(seed, 2, g, leader, 2, k)
                r1 = st.below(m)
                i = 1 + st.below(p // 2)
                F = crossover(set(snap[c]), set(snap[partner]), m, r1, i)
                item = {"slot": c, "partner": partner, "draws_of_slot": leader,
                        "stream": st.where(), "draws": st.log, "r1": r1, "i": i, "offspring": F}
                if F is None:
                    counters["xo_fail"] += 1
                else:
                    counters["evals"] += 1
                    fc = cost(d, F)
                    item["offspring_cost"] = fc
                    item["parent_cost"] = fit[c]
                    item["taken"] = fc < fit[c]
                    if fc < fit[c]:
                        pop[c], fit[c] = F, fc
                        counters["xo_taken"] += 1
                stage["pairs"].append(item)
            stage["after"] = {"population": [list(x) for x in pop], "fitness": list(fit)}
            rec["crossover"].append(stage)
        improved = [False] * P
        for a in range(Y):
            att = {"attempt": a, "slots": []}
            for c in range(P):
                if improved[c]:
                    continue
                st = Stream(seed, 2, g, c, 3, a)
                F, desc = mutate(st, pop[c], m)
                item = {"slot": c, "stream": st.where(), "draws": st.log, "move": desc,
                        "offspring": F}
                if F == pop[c]:
                    item["evaluated"] = False
                else:
                    counters["evals"] += 1
                    fc = cost(d, F)
                    item.update(evaluated=True, offspring_cost=fc, parent_cost=fit[c],
                                taken=fc < fit[c])
                    if fc < fit[c]:
                        pop[c], fit[c] = F, fc
                        improved[c] = True
                        counters["mut_taken"] += 1
                att["slots"].append(item)
            rec["mutation"].append(att)
        for b in range(NB):
            slots = range(b * NT, (b + 1) * NT)
            bi = min(slots, key=lambda t: (fit[t], t))
            gbest[b] = (list(pop[bi]), fit[bi])
        bb = min(range(NB), key=lambda b: (gbest[b][1], b))
        if best is None or gbest[bb][1] < best[1]:
            best = gbest[bb]
        rec["end"] = {"population": [list(x) for x in pop], "fitness": list(fit),
                      "group_bests": [{"open": x[0], "cost": x[1]} for x in gbest],
                      "global_best": {"open": best[0], "cost": best[1]},
                      "counters": dict(counters)}
        gens.append(rec)
    return gens


def _flat(x):
    """True when x holds at most one level of containers."""
    if isinstance(x, dict):
        return all(not isinstance(v, (dict, list)) or _scalars(v) for v in x.values())
    if isinstance(x, list):
        return all(not isinstance(v, (dict, list)) or _scalars(v) for v in x)
    return True


def _scalars(x):
    vals = x.values() if isinstance(x, dict) else x
    return all(not isinstance(v, (dict, list)) for v in vals)


def _dump(x, ind=0):
    """JSON with every small record on one line (readable by eye)."""
    if not isinstance(x, (dict, list)) or _flat(x):
        return json.dumps(x)
    pad = " " * (ind + 1)
    if isinstance(x, dict):
        body = (",\n").join(f"{pad}{json.dumps(k)}: {_dump(v, ind + 1)}" for k, v in x.items())
        return "{\n" + body + "\n" + " " * ind + "}"
    body = (",\n").join(pad + _dump(v, ind + 1) for v in x)
    return "[\n" + body + "\n" + " " * ind + "]"


def main():
    cases = [
        {"name": "example1", "source": "Section 2.1, Example 1 (0-based facilities)",
         "d": EXAMPLE1, "p": 2, "P": 8, "NT": 4, "seed": 2024, "generations": 1},
        {"name": "cycle8", "source": "8-cycle, d = cycle distance (many equal costs)",
         "d": cycle8(), "p": 4, "P": 8, "NT": 4, "seed": 7, "generations": 2},
    ]
    for cs in cases:
        cs["trace"] = run(cs["d"], cs["p"], cs["P"], cs["NT"], cs["seed"], cs["generations"])
    doc = {"about": [ln for ln in __doc__.strip().split("\n")],
           "cases": cases}
    with open(OUT, "w") as f:
        f.write(_dump(doc) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
