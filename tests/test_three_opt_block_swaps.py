"""The GPU 3-opt's way of applying a segment exchange, checked on the CPU.

The kernel swaps whichever two of the tour array's three adjacent blocks
(the two segments and the rest of the tour) moves the fewest nodes; the
cyclic tour and its direction are the same for all three swaps, and the
array differs from the sequential search's by a rotation that an offset
accumulates and the write-back undoes.  This pure-Python model of that
scheme (its block positions computed as the kernel computes them: the
first block from ri = p1 + 1 on the successor side, p1 - end on the
predecessor side) must give the oracle's tour exactly, with each of the
three swaps occurring.
"""

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl
from test_oracle_3opt import _d


def rot_three_opt(d, nl, tour, min_gain):
    t = [int(v) for v in tour]; n = len(t)
    pos = {v: s for s, v in enumerate(t)}
    queue = list(t); inq = set(t); rot = 0; counts = [0, 0, 0]
    def nxt(x, sg): return t[(pos[x] + sg) % n]
    def push(x):
        if x not in inq: queue.append(x); inq.add(x)
    def rev_span(i, ln):
        i %= n
        for s in range(ln // 2):
            x, y = (i + s) % n, (i + ln - 1 - s) % n
            t[x], t[y] = t[y], t[x]; pos[t[x]], pos[t[y]] = x, y
    def swap_blocks(s0, x, y):
        s0 %= n; rev_span(s0, x + y); rev_span(s0, y); rev_span(s0 + y, x)
    def two(a):
        for sg in (1, -1):
            b = nxt(a, sg)
            for c in nl[a]:
                c = int(c)
                if d[a, b] - d[a, c] <= 0.0: break
                e = nxt(c, sg)
                if e == a or c == b: continue
                if (d[a, b] + d[c, e]) - (d[a, c] + d[b, e]) > min_gain:
                    lo, hi = (pos[b], pos[c]) if sg == 1 else (pos[c], pos[b])
                    ln = (hi - lo) % n + 1
                    if 2 * ln > n: lo, hi = (hi + 1) % n, (lo - 1) % n
                    rev_span(lo, (hi - lo) % n + 1); return [a, b, c, e]
        return None
    def exch(a):
        nonlocal rot
        for sg in (1, -1):
            p1 = pos[a]
            steps = lambda x: ((pos[x] - p1) * sg) % n
            t1, t2 = a, nxt(a, sg)
            for t3 in nl[t1]:
                t3 = int(t3); g1 = d[t1, t2] - d[t1, t3]
                if g1 <= 0.0: break
                r3 = steps(t3)
                if r3 < 2: continue
                t4 = nxt(t3, -sg)
                for t5 in nl[t4]:
                    t5 = int(t5); g2 = (g1 + d[t4, t3]) - d[t4, t5]
                    if g2 <= 0.0: break
                    r5 = steps(t5)
                    if not (r5 > r3 or r5 == 0): continue
                    t6 = nxt(t5, -sg)
                    if ((d[t1, t2] + d[t4, t3]) + d[t6, t5]) - ((d[t1, t3] + d[t4, t5]) + d[t6, t2]) > min_gain:
                        end = (n if r5 == 0 else r5) - 1
                        dr = 0 if sg == 1 else 1
                        ri = (p1 + 1) % n if dr == 0 else (p1 - end) % n
                        qb = end - r3 + 1 if dr == 0 else r3 - 1
                        pa = end - qb; zc = n - end
                        if end <= n - pa and end <= n - qb:
                            swap_blocks(ri, pa, qb); counts[0] += 1
                        elif n - pa <= n - qb:
                            swap_blocks(ri + pa, qb, zc); rot = (rot + qb) % n; counts[1] += 1
                        else:
                            swap_blocks(ri + pa + qb, zc, pa); rot = (rot - pa) % n; counts[2] += 1
                        return [t1, t2, t3, t4, t5, t6]
        return None
    moves = 0
    while queue and moves < 64 * n:
        a = queue.pop(0); inq.discard(a)
        while moves < 64 * n:
            r = two(a)
            if r is None: r = exch(a)
            if r is None: break
            moves += 1
            for x in r: push(x)
    out = [t[(s - rot) % n] for s in range(n)]
    return np.array(out, dtype=np.int32), counts



def test_rotated_block_swaps_equal_the_oracle():
    used = [0, 0, 0]
    for n, seed, kk in [(10, 1, 3), (20, 2, 5), (30, 3, 6), (45, 4, 8), (60, 5, 10), (120, 6, 10)]:
        for inst in (wl.random_instance(n, seed=seed, ants=4, iterations=2),
                     wl.random_instance(n, seed=seed + 50, grid=12, ants=4, iterations=2)):
            d = _d(inst)
            nl = oracle.nearest_lists(inst, kk)
            rng = np.random.default_rng(seed)
            for _ in range(3):
                t0 = rng.permutation(n).astype(np.int32)
                got, c = rot_three_opt(d, nl, t0, 1e-9)
                used = [x + y for x, y in zip(used, c)]
                assert np.array_equal(got, oracle.three_opt(inst, nl, t0, 1e-9)), (n, seed)
    assert min(used) > 0, used
