"""Pins of the oracle's 3-opt for symmetric instances (Section III-D).

Reading (the paper names a first-improvement 3-opt on the geometric
neighbour lists with don't-look bits, not its move set): the 2-opt's search
(queue in tour order, FIFO re-queueing of absent end nodes, re-examination
of the node just improved, threshold min_gain) over a larger neighbourhood.
For node a the 2-opt moves come first, exactly as in the 2-opt; if none
improves, the segment exchange: with t2 the next node after t1 = a in the
direction (successor side, then predecessor side), t3 over a's list while
g1 = d(t1,t2) - d(t1,t3) > 0, t4 the node before t3, t5 over t4's list while
g2 = (g1 + d(t4,t3)) - d(t4,t5) > 0, t5 after t3 or t5 = t1, t6 the node
before t5; (t1,t2), (t4,t3), (t6,t5) are replaced by (t1,t3), (t6,t2),
(t4,t5), so the segments t2..t4 and t3..t6 trade places, each keeping its
order; the end nodes t1 .. t6 are re-queued in that order.

Pinned here against eq. (1) and by brute force:
  * with full neighbour lists, once a search leaves the tour unchanged, no
    improving 2-opt move and no improving exchange of two adjacent segments
    is left anywhere in the tour (every position pair and triple
    enumerated).  Don't-look queues alone do not promise that (a node that
    is not re-queued can gain a move from a change elsewhere), but a search
    that starts with every node queued and changes nothing has examined
    every node; a positive-gain exchange has a rotation of its three removed
    edges whose partial gains are all positive, and that rotation is again
    a segment exchange from one of its end nodes, so the list stop rules
    lose nothing.  A move the search misses, or one it applies wrongly,
    shows up as a remaining improvement or as a tour that is no
    permutation;
  * it never lengthens a tour, keeps it a permutation, and reaches shorter
    tours than the 2-opt alone on some instances;
  * with short lists it equals an independent pure-Python version written
    from the reading (move order, stop rules, validity of t5, re-queueing);
  * decodes apply it with local_search 1 and 2; the ATSP refuses it.
"""

import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl


def _d(inst):
    if inst.kind == "coords":
        xy = inst.coords
        dx = xy[:, None, 0] - xy[None, :, 0]
        dy = xy[:, None, 1] - xy[None, :, 1]
        return np.sqrt(dx * dx + dy * dy)
    return np.asarray(inst.dist, dtype=np.float64)


def _len(d, t):
    n = len(t)
    return math.fsum(float(d[t[s], t[(s + 1) % n]]) for s in range(n))


def _best_remaining_gain(d, t):
    """Largest gain of any 2-opt move and of any exchange of two adjacent
    segments, over every position pair and triple."""
    n = len(t)
    best = -math.inf
    for i in range(n):
        a, b = t[i], t[(i + 1) % n]
        for j in range(i + 2, n):
            c, e = t[j], t[(j + 1) % n]
            if e == a:
                continue
            best = max(best, (d[a, b] + d[c, e]) - (d[a, c] + d[b, e]))
    for i in range(n):
        for lj in range(1, n - 1):          # |S1| = lj nodes after position i
            for lk in range(1, n - lj):     # |S2| = lk nodes after S1
                j, k = i + lj, i + lj + lk
                ti, ti1 = t[i], t[(i + 1) % n]
                tj, tj1 = t[j % n], t[(j + 1) % n]
                tk, tk1 = t[k % n], t[(k + 1) % n]
                gain = (d[ti, ti1] + d[tj, tj1] + d[tk, tk1]) - (d[ti, tj1] + d[tk, ti1] + d[tj, tk1])
                best = max(best, gain)
    return best


def _instances():
    out = []
    for n, seed in [(8, 1), (9, 2), (11, 3), (12, 4), (14, 5)]:
        out.append(wl.random_instance(n, seed=seed, ants=4, iterations=2))
    out.append(wl.random_instance(12, seed=6, kind="matrix", symmetric=True, ants=4, iterations=2))
    out.append(wl.random_instance(13, seed=7, grid=4, ants=4, iterations=2))  # equal distances
    return out


@pytest.mark.parametrize("x", range(7))
def test_full_lists_leave_no_improving_move(x):
    inst = _instances()[x]
    n = inst.n
    d = _d(inst)
    nl = oracle.nearest_lists(inst, n - 1)
    rng = np.random.default_rng(100 + x)
    mg = 1e-9
    for _ in range(4):
        t0 = rng.permutation(n).astype(np.int32)
        t = oracle.three_opt(inst, nl, t0, mg)
        for _ in range(50):  # until a whole search changes nothing
            t1 = oracle.three_opt(inst, nl, t, mg)
            if np.array_equal(t1, t):
                break
            assert _len(d, t1) < _len(d, t)
            t = t1
        else:
            raise AssertionError("no fixed point")
        assert sorted(t.tolist()) == list(range(n))
        L0, L = _len(d, t0), _len(d, t)
        assert L <= L0 + 1e-12 * L0
        assert _best_remaining_gain(d, t) <= mg + 1e-12 * L, "an improving move is left"


def test_three_opt_goes_beyond_two_opt():
    shorter = 0
    for seed in range(12):
        inst = wl.random_instance(40, seed=200 + seed, ants=4, iterations=2)
        d = _d(inst)
        nl = oracle.nearest_lists(inst, 10)
        t0 = np.random.default_rng(seed).permutation(40).astype(np.int32)
        L2 = _len(d, oracle.two_opt(inst, nl, t0, 1e-9))
        L3 = _len(d, oracle.three_opt(inst, nl, t0, 1e-9))
        shorter += L3 < L2 - 1e-9
    assert shorter >= 6, shorter


# ---- an independent version written from the reading ----------------------

def _py_three_opt(d, nl, tour, min_gain):
    t = [int(v) for v in tour]
    n = len(t)
    pos = {v: s for s, v in enumerate(t)}
    queue = list(t)
    inq = set(t)
    kk = nl.shape[1]

    def nxt(x, sign):
        return t[(pos[x] + sign) % n]

    def push(x):
        if x not in inq:
            queue.append(x)
            inq.add(x)

    def reverse(i, j):  # positions i..j, cyclic
        ln = (j - i) % n + 1
        for s in range(ln // 2):
            x, y = (i + s) % n, (j - s) % n
            t[x], t[y] = t[y], t[x]
            pos[t[x]], pos[t[y]] = x, y

    def two_opt_move(a):
        for sign in (1, -1):
            b = nxt(a, sign)
            for c in nl[a]:
                c = int(c)
                if d[a, b] - d[a, c] <= 0.0:
                    break
                e = nxt(c, sign)
                if e == a or c == b:
                    continue
                if (d[a, b] + d[c, e]) - (d[a, c] + d[b, e]) > min_gain:
                    lo, hi = (pos[b], pos[c]) if sign == 1 else (pos[c], pos[b])
                    ln = (hi - lo) % n + 1
                    if 2 * ln > n:  # the shorter side
                        lo, hi = (hi + 1) % n, (lo - 1) % n
                    reverse(lo, hi)
                    return [a, b, c, e]
        return None

    def exchange_move(a):
        for sign in (1, -1):
            p1 = pos[a]

            def steps(x):
                return ((pos[x] - p1) * sign) % n

            t1, t2 = a, nxt(a, sign)
            for t3 in nl[t1]:
                t3 = int(t3)
                g1 = d[t1, t2] - d[t1, t3]
                if g1 <= 0.0:
                    break
                r3 = steps(t3)
                if r3 < 2:
                    continue
                t4 = nxt(t3, -sign)
                for t5 in nl[t4]:
                    t5 = int(t5)
                    g2 = (g1 + d[t4, t3]) - d[t4, t5]
                    if g2 <= 0.0:
                        break
                    r5 = steps(t5)
                    if not (r5 > r3 or r5 == 0):
                        continue
                    t6 = nxt(t5, -sign)
                    gain = ((d[t1, t2] + d[t4, t3]) + d[t6, t5]) - ((d[t1, t3] + d[t4, t5]) + d[t6, t2])
                    if gain > min_gain:
                        r6 = (r5 - 1) % n
                        seg1 = [t[(p1 + sign * s) % n] for s in range(1, r3)]
                        seg2 = [t[(p1 + sign * s) % n] for s in range(r3, r6 + 1)]
                        for s, v in enumerate(seg2 + seg1, start=1):
                            at = (p1 + sign * s) % n
                            t[at] = v
                            pos[v] = at
                        return [t1, t2, t3, t4, t5, t6]
        return None

    while queue:
        a = queue.pop(0)
        inq.discard(a)
        while True:
            ends = two_opt_move(a)
            if ends is None:
                ends = exchange_move(a)
            if ends is None:
                break
            for x in ends:
                push(x)
    return np.array(t, dtype=np.int32)


@pytest.mark.parametrize("n,seed,kk", [(10, 1, 3), (20, 2, 5), (30, 3, 6), (45, 4, 8), (60, 5, 10)])
def test_equals_an_independent_version(n, seed, kk):
    for inst in (wl.random_instance(n, seed=seed, ants=4, iterations=2),
                 wl.random_instance(n, seed=seed + 50, grid=8, ants=4, iterations=2)):
        d = _d(inst)
        nl = oracle.nearest_lists(inst, kk)
        rng = np.random.default_rng(seed)
        for _ in range(3):
            t0 = rng.permutation(n).astype(np.int32)
            got = oracle.three_opt(inst, nl, t0, 1e-9)
            ref = _py_three_opt(d, nl, t0, 1e-9)
            assert np.array_equal(got, ref), (n, seed, kk)


@pytest.mark.parametrize("ls", [1, 2])
def test_decodes_with_three_opt(ls):
    inst = dataclasses.replace(wl.random_instance(60, seed=31, ants=6, iterations=8, local_search=ls, k_ls=10),
                               ls_op=3)
    st, tour, L, _ = oracle.decode(inst)
    assert st == 0 and sorted(tour.tolist()) == list(range(60))
    st2, tour2, L2, _ = oracle.decode(dataclasses.replace(inst, ls_op=2))
    assert st2 == 0 and not np.array_equal(tour, tour2)


def test_atsp_refuses_three_opt():
    inst = dataclasses.replace(wl.random_instance(20, seed=9, kind="matrix", symmetric=False, ants=4,
                                                  iterations=2, local_search=1), ls_op=3)
    st, _, _, _ = oracle.decode(inst)
    assert st != 0
