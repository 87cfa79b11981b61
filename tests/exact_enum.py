"""Exact final-burn distribution of the fire CA on tiny lattices (test helper).

An independent model of the propagation rules (Methods, "Forest Fire Spread
Simulation"), written directly from the process, not from the oracle: at each
step every cell that ignited at the previous step holds one independent coin per
unburnt burnable neighbour, succeeding with that directed edge's probability;
a neighbour ignites when at least one of its coins succeeds. Because the coins
of different targets are disjoint sets of independent events, the chance that
target t ignites is 1 - prod(1 - p_i) over its burning neighbours i (the
paper's per-target rule) and targets ignite independently of each other.
The recursion below sums exactly (Fractions) over every outcome of every step.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

OFFSETS = [(0, -1), (1, -1), (1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1)]


def edge_probabilities_from_thresholds(T, W, H):
    """T[y][x][d] (ints) -> dict {(s, t): Fraction}, s and t as (x, y)."""
    probs = {}
    for y in range(H):
        for x in range(W):
            for d, (dx, dy) in enumerate(OFFSETS):
                tx, ty = x + dx, y + dy
                if 0 <= tx < W and 0 <= ty < H:
                    v = int(T[y][x][d])
                    probs[((x, y), (tx, ty))] = Fraction(1) if v == 0xFFFFFFFF else Fraction(v, 1 << 32)
    return probs


def final_distribution(W, H, burnable, probs, ign):
    """Distribution over final burnt sets {frozenset((x, y)): Fraction}.

    burnable[y][x] is a bool; probs maps (source, target) cells to the
    probability of that directed edge; ign is the ignition cell (x, y).
    """
    if not burnable[ign[1]][ign[0]]:
        return {frozenset(): Fraction(1)}

    def neighbours(c):
        x, y = c
        for dx, dy in OFFSETS:
            tx, ty = x + dx, y + dy
            if 0 <= tx < W and 0 <= ty < H and burnable[ty][tx]:
                yield (tx, ty)

    @lru_cache(maxsize=None)
    def go(burnt: frozenset, active: frozenset):
        if not active:
            return {burnt: Fraction(1)}
        # ignition chance of every unburnt target next to the front
        q = {}
        for s in active:
            for t in neighbours(s):
                if t in burnt:
                    continue
                q[t] = q.get(t, Fraction(1)) * (1 - probs[(s, t)])
        cands = sorted(q)
        out = {}
        for m in range(1 << len(cands)):
            pr = Fraction(1)
            new = []
            for i, t in enumerate(cands):
                p_ign = 1 - q[t]
                if m >> i & 1:
                    pr *= p_ign
                    new.append(t)
                else:
                    pr *= 1 - p_ign
                if pr == 0:
                    break
            if pr == 0:
                continue
            sub = go(burnt | frozenset(new), frozenset(new))
            for k, v in sub.items():
                out[k] = out.get(k, Fraction(0)) + pr * v
        return out

    start = frozenset([tuple(ign)])
    return go(start, start)


def by_count(dist):
    out = {}
    for k, v in dist.items():
        out[len(k)] = out.get(len(k), Fraction(0)) + v
    return dict(sorted(out.items()))


def final_distribution_dur(W, H, burnable, probs, ign, life):
    """As final_distribution, for cells that stay active for life[(x, y)]
    steps after igniting (turn-off time): the state is the burnt set and the
    remaining active steps of every active cell; at each step every active
    cell holds one fresh coin per unburnt burnable neighbour."""
    if not burnable[ign[1]][ign[0]]:
        return {frozenset(): Fraction(1)}

    def neighbours(c):
        x, y = c
        for dx, dy in OFFSETS:
            tx, ty = x + dx, y + dy
            if 0 <= tx < W and 0 <= ty < H and burnable[ty][tx]:
                yield (tx, ty)

    @lru_cache(maxsize=None)
    def go(burnt: frozenset, active: frozenset):
        if not active:
            return {burnt: Fraction(1)}
        q = {}
        for s, _ in active:
            for t in neighbours(s):
                if t in burnt:
                    continue
                q[t] = q.get(t, Fraction(1)) * (1 - probs[(s, t)])
        cands = sorted(q)
        older = frozenset((s, k - 1) for s, k in active if k > 1)
        out = {}
        for m in range(1 << len(cands)):
            pr = Fraction(1)
            new = []
            for i, t in enumerate(cands):
                if m >> i & 1:
                    pr *= 1 - q[t]
                    new.append(t)
                else:
                    pr *= q[t]
                if pr == 0:
                    break
            if pr == 0:
                continue
            nxt = older | frozenset((t, life[t]) for t in new)
            sub = go(burnt | frozenset(new), nxt)
            for k, v in sub.items():
                out[k] = out.get(k, Fraction(0)) + pr * v
        return out

    start = tuple(ign)
    return go(frozenset([start]), frozenset([(start, life[start])]))
