"""Column-count model of carry-save formulas with three-input instructions.

A bitsliced sum is held as bits in weight columns (weights 1, 2, 4 ...).  A full adder takes
three bits of one column to a sum in that column and a carry one column up (two three-input
instructions), a half adder two bits (two instructions).  A carry out of the top column wraps:
for residues modulo 2^c - 1 it re-enters the lowest column as it is (2^c = 1); modulo 5 with
columns of weights 1 and 2 a bit of weight 4 = -1 re-enters weight 1 complemented (4x = ~x - 1,
a constant -1 kept as an offset).  Complements and constant bits cost nothing (they fold into
the truth tables).  A Dijkstra search over column counts (and offset) gives the fewest
instructions for a schedule; it models counts only, so its minimum is a bound for schedules
of adders, not for arbitrary programs.

  accumulate  fewest instructions for one slab step that returns the accumulator to the same
              column counts (the state sizes it can use), for F_3, F_7 and F_5
  f5add       the F_5 table addition / subtraction of 3-bit representatives, result 3 bits
"""
import heapq
import itertools
import sys


def search(start, goal, moves, limit=40):
    best, pq = {start: 0}, [(0, start)]
    while pq:
        c, st = heapq.heappop(pq)
        if st == goal:
            return c
        if c > best.get(st, limit + 1) or c > limit:
            continue
        for nst, cost in moves(st):
            if max(nst[:-1]) > 20:
                continue
            if best.get(nst, limit + 1) > c + cost:
                best[nst] = c + cost
                heapq.heappush(pq, (c + cost, nst))
    return None


def cyclic_moves(ncol):
    """Adders on columns of weights 2^0 .. 2^(ncol-1) modulo 2^ncol - 1 (state: counts, 0)."""
    def moves(st):
        out = []
        for j in range(ncol):
            for take in (3, 2):
                if st[j] >= take:
                    m = list(st)
                    m[j] -= take - 1
                    m[(j + 1) % ncol] += 1
                    out.append((tuple(m), 2))
        return out
    return moves


def f5_moves(st):
    """Columns of weights 1, 2, 4 modulo 5 with an offset: a carry of weight 8 = -2 enters
    weight 2 complemented (offset -2), a bit of weight 4 may move to weight 1 complemented
    (offset -1) and back, and constant bits may be added (offset compensates)."""
    n0, n1, n2, off = st
    n, out = [n0, n1, n2], []
    for j in range(3):
        for take in (3, 2):
            if n[j] >= take:
                m, o = n[:], off
                m[j] -= take - 1
                if j < 2:
                    m[j + 1] += 1
                else:
                    m[1] += 1
                    o = (o - 2) % 5
                out.append((tuple(m) + (o,), 2))
    if n2 >= 1:
        out.append(((n0 + 1, n1, n2 - 1, (off - 1) % 5), 0))
    if n0 >= 1:
        out.append(((n0 - 1, n1, n2 + 1, (off + 1) % 5), 0))
    for j in range(3):
        m = n[:]
        m[j] += 1
        if max(m) <= 6:
            out.append((tuple(m) + ((off - (1, 2, 4)[j]) % 5,), 0))
    return out


def accumulate():
    """Fewest instructions of a slab step, and the smallest state reaching it, per field."""
    fields = {"F_3": (2, (2, 2)), "F_7": (3, (3, 3, 3))}
    res = {}
    for name, (ncol, inputs) in fields.items():
        found = None
        for total in range(ncol, 2 * ncol + 1):
            for state in itertools.product(range(total + 1), repeat=ncol):
                if sum(state) != total:
                    continue
                start = tuple(s + i for s, i in zip(state, inputs)) + (0,)
                mv = cyclic_moves(ncol)
                c = search(start, tuple(state) + (0,), lambda st: [(m + (0,), k) for m, k in mv(st[:-1])])
                if c is not None and (found is None or (c, total) < (found[0], found[1])):
                    found = (c, total, state)
            if found is not None:
                break
        res[name] = found
    return res


def f5_accumulate():
    """F_5 slab step t + 2v + 4w over weights 1, 2, 4 (8 = -2 enters weight 2 complemented,
    16 = 1 weight 1): (2, 4, 3) input bits.  Any fixed offset per slab is allowed (the
    accumulator's starting value cancels it), so the search stops at the first return to the
    state's column counts.  Returns (instructions, state bits, state)."""
    inputs, found = (2, 4, 3), None
    for state in itertools.product(range(4), repeat=3):
        if sum(state) < 3:
            continue
        start = tuple(s + i for s, i in zip(state, inputs)) + (0,)
        best, pq = {start: 0}, [(0, start)]
        while pq:
            c, st = heapq.heappop(pq)
            if st[:3] == state:
                if found is None or (c, sum(state)) < found[:2]:
                    found = (c, sum(state), state)
                break
            if c > best.get(st, 23) or c > 22:
                continue
            for nst, cost in f5_moves(st):
                if best.get(nst, 23) > c + cost:
                    best[nst] = c + cost
                    heapq.heappush(pq, (c + cost, nst))
    return found


def f5add():
    # a + b: weights 1, 2, 4 hold (a0, b0), (a1, b1), (a2, b2); a - b: weight 1 a0, ~b0, b2, ~a2
    # and weight 2 a1, ~b1 with offset -4 = 1; the result is one bit in each column
    return {"add": search((2, 2, 2, 0), (1, 1, 1, 0), f5_moves, 16),
            "sub": search((4, 2, 0, 1), (1, 1, 1, 0), f5_moves, 16)}


if __name__ == "__main__":
    for name, (c, total, state) in accumulate().items():
        print(f"accumulate {name}: {c} instructions, state of {total} bits {state}")
    c, total, state = f5_accumulate()
    print(f"accumulate F_5: {c} instructions, state of {total} bits {state}")
    r = f5add()
    print(f"f5add: add {r['add']} instructions, sub {r['sub']} instructions")
    sys.exit(0)
