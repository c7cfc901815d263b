"""CPU pins of the oracle against what the paper and mathematics fix.

Each test names the passage it pins.  None of them retypes the oracle's own
formula: they use published known answers, hand-worked rows, brute force,
closed forms reached by a different route, library routines, and
invariants the paper states.
"""

import json
import math
import os
from decimal import Decimal, getcontext

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Random numbers: Philox4x32-10 known answers (SC'11 reference vectors)
# --------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        ctr = [int(x, 16) for x in r[0:4]]
        key = [int(x, 16) for x in r[4:6]]
        want = [int(x, 16) for x in r[6:10]]
        assert list(oracle.philox(ctr, key)) == want


def test_draw_layout_and_uniformity():
    # the 32-bit draw is word 0 of the block at counter (s, a, t, 0)
    seed = 0x0123456789ABCDEF
    out = oracle.philox([7, 3, 5, 0], [seed & 0xFFFFFFFF, seed >> 32])
    assert oracle.draw(seed, 5, 3, 7) == int(out[0])
    # chi-square on the top 6 bits of 40k draws
    bins = np.zeros(64)
    for s in range(40000):
        bins[oracle.draw(11, 1 + s % 7, s % 13, s) >> 26] += 1
    exp = 40000 / 64
    chi2 = ((bins - exp) ** 2 / exp).sum()
    # 63 dof: P(chi2 > 120) ~ 1e-5
    assert chi2 < 120


# --------------------------------------------------------------------------
# Section III-A, eq. (3): candidate lists, against brute force
# --------------------------------------------------------------------------
def brute_candidates(inst, k, theta=1e-4):
    n = inst.n
    ke = min(k, n - 1)
    H = inst.heat
    out = np.zeros((n, ke), dtype=np.int64)
    for i in range(n):
        if inst.kind == "coords":
            # exact squared distances as Python floats, same expression
            keys = [float((inst.coords[i, 0] - inst.coords[j, 0]) * (inst.coords[i, 0] - inst.coords[j, 0])
                          + (inst.coords[i, 1] - inst.coords[j, 1]) * (inst.coords[i, 1] - inst.coords[j, 1]))
                    for j in range(n)]
        else:
            keys = [float(inst.dist[i, j]) for j in range(n)]
        a, b = H.row_ptr[i], H.row_ptr[i + 1]
        P = {int(j) for j, v in zip(H.col[a:b], H.val[a:b]) if j != i and float(v) > theta}
        sup = sorted(P, key=lambda j: (keys[j], j))
        if len(sup) >= ke:
            chosen = sup[:ke]
        else:
            rest = sorted((j for j in range(n) if j != i and j not in P), key=lambda j: (keys[j], j))
            chosen = sup + rest[: ke - len(sup)]
        chosen.sort(key=lambda j: (keys[j], j))
        out[i] = chosen
    return out


@pytest.mark.parametrize("n,topk,k,grid", [(40, 10, 8, None), (40, 4, 10, None), (60, 10, 10, None),
                                          (50, 10, 12, 9), (30, 6, 29, 6), (12, 3, 20, None)])
def test_candidates_match_brute_force(n, topk, k, grid):
    inst = wl.random_instance(n, seed=n + topk + k, topk=topk, k=k, grid=grid)
    got = oracle.candidates(inst)
    want = brute_candidates(inst, k)
    assert got.shape == want.shape
    assert np.array_equal(got, want)
    ke = min(k, n - 1)
    for i in range(n):
        assert i not in got[i]
        assert len(set(got[i])) == ke


def test_candidates_support_larger_smaller_equal_k():
    # row sizes of |P_i| above, below and equal to k all occur in this instance
    inst = wl.tsp500(iterations=1)
    H = inst.heat
    P = np.array([(H.val[H.row_ptr[i]:H.row_ptr[i + 1]] > 1e-4).sum() for i in range(inst.n)])
    assert (P > 20).any() and (P < 20).any() and (P == 20).any()
    sub_ok = brute_candidates(inst, 20)
    assert np.array_equal(oracle.candidates(inst), sub_ok)


def test_candidates_matrix_and_empty_heatmap():
    inst = wl.random_instance(35, seed=3, kind="matrix", symmetric=False, k=7)
    assert np.array_equal(oracle.candidates(inst), brute_candidates(inst, 7))
    inst = wl.random_instance(35, seed=4, heat="empty", k=7)
    cand = oracle.candidates(inst)
    # with no support the list is the 7 geometric nearest neighbours
    assert np.array_equal(cand, oracle.nearest_lists(inst, 7))


# --------------------------------------------------------------------------
# Section III-C, eq. (9)-(11): worked rows
# --------------------------------------------------------------------------
def _row_instance(confs):
    """Node 0 at the origin, node j at (0.1 j, 0); heatmap row 0 = confs."""
    k = len(confs)
    n = k + 1
    xy = np.zeros((n, 2))
    xy[1:, 0] = 0.1 * np.arange(1, n)
    cols = [j + 1 for j, c in enumerate(confs) if c > 0]
    vals = [c for c in confs if c > 0]
    rp = np.array([0, len(cols)] + [len(cols)] * (n - 1), dtype=np.int32)
    heat = wl.Heatmap(n, rp, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.float32))
    return wl.Instance(n, "coords", True, xy, None, heat, ants=2, iterations=1, k=k)


def test_evidence_worked_rows():
    rows = [l for l in open(os.path.join(GOLDEN, "evidence_examples.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 4
    for line in rows:
        lhs, rhs = line.split("->")
        lhs = lhs.split()
        dstar = int(lhs[0])
        confs = [float(x) for x in lhs[1:]]
        rhs = [float(x) for x in rhs.split()]
        inst = _row_instance(confs)
        cand = oracle.candidates(inst)
        assert list(cand[0]) == list(range(1, len(confs) + 1))
        ev = oracle.evidence(inst, cand, degree_target=dstar)
        # values pass through FP32 storage: compare at FP32 resolution
        assert ev["base"][0] == pytest.approx(rhs[0], rel=1e-6)
        assert ev["evid"][0] == pytest.approx(rhs[1:], rel=1e-6)


def test_evidence_threshold_worked_row():
    # eq. (9): confidences at or below theta_h count as 0, so with
    # theta_h = 0.02 the row 0.5, 0.01, 0.009 has one positive confidence;
    # eq. (10) then misses the third order statistic (d* = 2) and b = eps
    inst = _row_instance([0.5, 0.01, 0.009])
    cand = oracle.candidates(inst, theta_h=0.02)
    # eq. (3): node 1 is supported, the list is filled with the nearest others
    assert list(cand[0]) == [1, 2, 3]
    ev = oracle.evidence(inst, cand, theta_h=0.02, degree_target=2)
    assert list(ev["conf"][0]) == [0.5, 0.0, 0.0]
    assert ev["base"][0] == 1e-9
    assert ev["evid"][0] == pytest.approx([0.5 / 1e-9, 1.0, 1.0], rel=1e-6)


def test_evidence_full_row_ignores_the_diagonal():
    # eq. (10) over the full heatmap row (baseline_scope = 1) takes j in
    # V \ {i}: a diagonal entry of 0.9 beside 0.5, 0.3, 0.2, 0.1 leaves the
    # third largest at 0.2, so e = 2.5, 1.5, 1, 1
    n = 5
    xy = np.zeros((n, 2))
    xy[1:, 0] = 0.1 * np.arange(1, n)
    rp = np.array([0, 5, 5, 5, 5, 5], dtype=np.int32)
    heat = wl.Heatmap(n, rp, np.arange(5, dtype=np.int32), np.array([0.9, 0.5, 0.3, 0.2, 0.1], dtype=np.float32))
    inst = wl.Instance(n, "coords", True, xy, None, heat, ants=2, iterations=1, k=4)
    cand = oracle.candidates(inst)
    assert list(cand[0]) == [1, 2, 3, 4]
    ev = oracle.evidence(inst, cand, baseline_scope=1, degree_target=2)
    assert ev["base"][0] == pytest.approx(0.2, rel=1e-6)
    assert ev["evid"][0] == pytest.approx([2.5, 1.5, 1.0, 1.0], rel=1e-6)


def test_evidence_at_most_dstar_above_one_per_row():
    for inst, dstar in [(wl.tsp500(iterations=1), 2), (wl.serve_request("atsp1000", 1), 1),
                        (wl.random_instance(80, seed=5, topk=12, k=10), 2)]:
        cand = oracle.candidates(inst)
        ev = oracle.evidence(inst, cand)
        per_row = (ev["evid"] > 1.0).sum(axis=1)
        assert per_row.max() <= dstar
        # e > 1 exactly when the confidence exceeds the row baseline
        c = np.maximum(ev["conf"], 1e-9)
        assert np.array_equal(ev["evid"] > 1.0, c > ev["base"][:, None])


def test_baseline_scope_full_row():
    # with the full heatmap row as scope, b_i is the (d*+1)-th largest
    # thresholded entry of the whole row
    inst = wl.tsp500(iterations=1)
    cand = oracle.candidates(inst)
    ev = oracle.evidence(inst, cand, baseline_scope=1)
    H = inst.heat
    for i in range(0, 500, 37):
        a, b = H.row_ptr[i], H.row_ptr[i + 1]
        v = sorted((float(x) for j, x in zip(H.col[a:b], H.val[a:b]) if j != i and float(x) > 1e-4),
                   reverse=True)
        want = max(v[2] if len(v) >= 3 else 0.0, 1e-9)
        assert ev["base"][i] == want


# --------------------------------------------------------------------------
# eq. (12)-(14): quantile, dynamic range and kappa
# --------------------------------------------------------------------------
def test_q90_is_linear_quantile():
    for inst in [wl.tsp100(), wl.tsp500(iterations=1), wl.serve_request("atsp1000", 2)]:
        cand = oracle.candidates(inst)
        ev = oracle.evidence(inst, cand)
        logs = np.log(ev["evid"][ev["evid"] > 1.0])
        assert ev["q90"] == pytest.approx(float(np.quantile(logs, 0.9, method="linear")), rel=1e-12)


def _ratio_of_bounds(n, k, p_best, rho, L, ls):
    """eq. (5)/(6) evaluated literally at 60 digits, then tau_max / tau_min."""
    getcontext().prec = 60
    n_, k_ = Decimal(n), Decimal(min(k, n - 1))
    tmax = 1 / (Decimal(rho) * Decimal(L))
    if ls:
        tmin = tmax / (2 * n_)
    else:
        px = Decimal(p_best) ** (1 / n_)
        tmin = tmax * (1 - px) / (((k_ - 1) / 2) * px)
    return tmax / tmin


@pytest.mark.parametrize("n,k,ls", [(100, 10, 0), (500, 20, 0), (750, 10, 0), (1000, 20, 0), (10000, 20, 0),
                                    (10000, 20, 1), (60, 10, 1)])
def test_r_hat_is_bound_ratio_for_any_length(n, k, ls):
    # R = tau_max / tau_min does not depend on L (both bounds scale as 1/L):
    # the oracle's value must equal the literal ratio at two unrelated L.
    inst = wl.random_instance(n, seed=1, k=k, heat="empty", local_search=ls)
    cand = oracle.candidates(inst)
    ev = oracle.evidence(inst, cand)
    for L in (0.37, 123.0):
        want = _ratio_of_bounds(n, k, 0.05, 0.2, L, ls)
        assert ev["r_hat"] == pytest.approx(float(want), rel=1e-12)


def test_kappa_caps_the_90th_percentile_margin():
    # Section III-C: kappa * q90 = c_cap * alpha * log R (half the log range)
    for inst in [wl.tsp100(), wl.tsp500(iterations=1), wl.serve_request("atsp1000", 3)]:
        cand = oracle.candidates(inst)
        for c_cap in (0.5, 0.125, 2.0):
            ev = oracle.evidence(inst, cand, c_cap=c_cap)
            assert ev["kappa"] * ev["q90"] == pytest.approx(c_cap * math.log(ev["r_hat"]), rel=1e-12)


def test_kappa_zero_without_evidence():
    # "If the heatmap provides no edge with e > 1, then kappa = 0"
    inst = wl.random_instance(40, seed=9, heat="empty", k=8)
    cand = oracle.candidates(inst)
    ev = oracle.evidence(inst, cand)
    assert ev["kappa"] == 0.0 and ev["q90"] == 0.0
    assert np.all(ev["evid"] == 1.0)


def test_fold_matches_power_law():
    # S = eta^beta e^kappa (clipped log-weight); with e = 1 it is exactly fl32(eta^2)
    inst = wl.tsp100()
    cand = oracle.candidates(inst)
    ev = oracle.evidence(inst, cand)
    xy = inst.coords
    d = np.sqrt(((xy[:, None, :] - xy[cand]) ** 2).sum(-1))
    eta2 = (1.0 / d) ** 2
    one = ev["evid"] == 1.0
    assert one.any() and (~one).any()
    assert np.array_equal(ev["heur"][one], eta2[one].astype(np.float32))
    full = eta2 * np.power(ev["evid"], ev["kappa"])
    np.testing.assert_allclose(ev["heur"][~one], full[~one], rtol=2e-7)
    # the clip bounds the evidence multiplier at e^clip
    ev2 = oracle.evidence(inst, cand, clip=0.5)
    mult = ev2["heur"].astype(np.float64) / eta2
    assert mult.max() <= math.exp(0.5) * (1 + 1e-6)


def test_fixed_kappa_ablation():
    # Section IV-E "fixed kappa = 1": the scale of eq. (14) is replaced by a
    # constant, so S = eta^2 e on every candidate edge; e itself is unchanged.
    # Checked on the worked rows, whose e values are written out by hand.
    rows = [l for l in open(os.path.join(GOLDEN, "evidence_examples.txt")) if l.strip() and not l.startswith("#")]
    for line in rows:
        lhs, rhs = line.split("->")
        lhs = lhs.split()
        dstar = int(lhs[0])
        confs = [float(x) for x in lhs[1:]]
        want_e = np.array([float(x) for x in rhs.split()][1:])
        inst = _row_instance(confs)
        cand = oracle.candidates(inst)
        for kap in (1.0, 0.25):
            ev = oracle.evidence(inst, cand, degree_target=dstar, kappa_fixed=kap)
            assert ev["kappa"] == kap
            eta2 = (1.0 / (0.1 * np.arange(1, len(confs) + 1))) ** 2
            np.testing.assert_allclose(ev["heur"][0].astype(np.float64), eta2 * want_e ** kap, rtol=1e-6)
    # on a real heatmap the fixed scale leaves e and q90 alone and ignores c_cap
    inst = wl.tsp100()
    cand = oracle.candidates(inst)
    a = oracle.evidence(inst, cand)
    b = oracle.evidence(inst, cand, kappa_fixed=1.0, c_cap=7.0)
    assert np.array_equal(a["evid"], b["evid"]) and a["q90"] == b["q90"] and b["kappa"] == 1.0
    assert a["kappa"] != 1.0 and not np.array_equal(a["heur"], b["heur"])


def test_parameters_match_paper():
    prm = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    d = oracle.DEFAULTS
    for key in ("alpha", "beta", "p_best", "c_cap", "theta_h", "eps", "xi_bf", "bf_period", "restart_stall"):
        assert d[key] == prm[key], key
    assert d["lambda_bf"] == pytest.approx(prm["lambda_bf"], rel=0, abs=1e-15)
    assert d["ugb_max"] == prm["ugb_start"]


# --------------------------------------------------------------------------
# eq. (4): the roulette reproduces the transition probabilities
# --------------------------------------------------------------------------
def _chi2_select(w, visited_mask, draws, seed):
    k = len(w)
    cand = np.arange(1, k + 1, dtype=np.int32)
    vis = np.zeros(k + 1, dtype=np.uint8)
    vis[1:][visited_mask] = 1
    counts = np.zeros(k)
    for s in range(draws):
        slot = oracle.select(cand, w, vis, oracle.draw(seed, 1 + s // 4096, s % 4096, 7))
        counts[slot] += 1
    open_ = ~visited_mask
    p = np.where(open_, w.astype(np.float64), 0.0)
    p /= p.sum()
    assert counts[visited_mask].sum() == 0
    e = p[open_] * draws
    o = counts[open_]
    return ((o - e) ** 2 / e).sum(), open_.sum() - 1


@pytest.mark.parametrize("case", ["spread", "equal", "evidence"])
def test_select_frequencies_follow_eq4(case):
    rng = np.random.default_rng(17)
    if case == "spread":
        w = rng.uniform(0.05, 1.0, size=10).astype(np.float32)
        vis = np.zeros(10, dtype=bool); vis[[2, 7]] = True
    elif case == "equal":
        w = np.full(7, 0.3, dtype=np.float32)
        vis = np.zeros(7, dtype=bool); vis[0] = True
    else:
        # one edge with a large evidence multiplier among ordinary ones
        w = rng.uniform(0.5, 1.0, size=12).astype(np.float32)
        w[3] *= 40.0
        w[9] *= 1e-3
        vis = np.zeros(12, dtype=bool); vis[5] = True
    chi2, dof = _chi2_select(w, vis, 60000, seed=5)
    # P(chi2 > dof + 6 sqrt(2 dof)) < 1e-4 for these dof
    assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


def test_select_edge_cases():
    cand = np.array([4, 9, 2], dtype=np.int32)
    w = np.array([1.0, 2.0, 3.0], dtype=np.float32)
    vis = np.zeros(10, dtype=np.uint8)
    vis[[4, 2]] = 1
    # one unvisited candidate: always chosen
    for s in range(50):
        assert oracle.select(cand, w, vis, oracle.draw(3, 1, 0, s)) == 1
    vis[9] = 1
    assert oracle.select(cand, w, vis, 12345) == -1
    # extreme draws hit the first and the last open slot
    vis[:] = 0
    assert oracle.select(cand, w, vis, 0) == 0
    assert oracle.select(cand, w, vis, 2 ** 32 - 1) == 2


def _select_mass(cand, w, vis):
    """Exact probability of each slot under the roulette: the chosen slot is
    non-decreasing in the draw u, so the boundaries between slots are found
    by bisection over u in [0, 2^32) and each slot's share of the draws is
    counted exactly."""
    k = len(cand)
    first = []  # first draw that picks a slot > s
    for s in range(k):
        lo, hi = 0, 2 ** 32  # select(hi - 1) may still be <= s: hi = 2^32 means never
        while lo < hi:
            mid = (lo + hi) // 2
            if oracle.select(cand, w, vis, mid) > s:
                hi = mid
            else:
                lo = mid + 1
        first.append(lo)
    mass, prev = [], 0
    for s in range(k):
        mass.append((first[s] - prev) / 2 ** 32)
        prev = first[s]
    return np.array(mass)


def test_select_intervals_are_half_open():
    # Eq. (4) sampled by inverse CDF: slot s owns the draws whose scaled
    # value lies in [prefix before s, prefix through s).  Two open slots of
    # equal weight split the 2^32 draws into equal halves, the lower half
    # to the first slot and the point 2^31 itself to the second.
    cand = np.array([1, 2], dtype=np.int32)
    w = np.array([3.0, 3.0], dtype=np.float32)
    vis = np.zeros(3, dtype=np.uint8)
    assert oracle.select(cand, w, vis, 2 ** 31 - 1) == 0
    assert oracle.select(cand, w, vis, 2 ** 31) == 1


@pytest.mark.parametrize("light", [3, 5, 1000])
def test_select_exact_for_weights_on_the_24_bit_grid(light):
    # With the largest open weight 1 (exponent 0), whole multiples of 2^-23
    # are on the grid the roulette works at, so it adds no error of its own:
    # the share of the 2^32 draws that pick the light slot equals eq. (4)'s
    # w1 / (w0 + w1) to within the draw granularity 2^-32.
    w1 = light * 2.0 ** -23
    cand = np.array([1, 2], dtype=np.int32)
    w = np.array([1.0, w1], dtype=np.float32)
    vis = np.zeros(3, dtype=np.uint8)
    mass = _select_mass(cand, w, vis)
    assert abs(mass[1] - w1 / (1.0 + w1)) <= 2.0 ** -32


@pytest.mark.parametrize("seed", range(6))
def test_select_probabilities_within_the_discretisation_bound(seed):
    """Each slot's probability under the fixed-point roulette is within
    (k+1) 2^-23 + 2^-32 of eq. (4), also for weights spread over many
    binades (the light slots are floored to q = 1)."""
    rng = np.random.default_rng(100 + seed)
    k = int(rng.integers(2, 65))
    w = np.exp(rng.uniform(-30.0, 0.0, size=k) if seed % 2 else rng.uniform(-2.0, 0.0, size=k))
    w = w.astype(np.float32)
    cand = np.arange(k, dtype=np.int32)
    vis = (rng.random(k) < 0.3).astype(np.uint8)
    vis[int(rng.integers(k))] = 0
    mass = _select_mass(cand, w, vis)
    p = np.where(vis == 0, w.astype(np.float64), 0.0)
    p /= p.sum()
    assert mass[vis == 1].sum() == 0
    assert abs(mass.sum() - 1.0) < 1e-15
    assert np.max(np.abs(mass - p)) <= (k + 1) * 2.0 ** -23 + 2.0 ** -32


# --------------------------------------------------------------------------
# Alg. 1 preparation: NN tour; eq. (1): tour length
# --------------------------------------------------------------------------
def brute_nn_tour(inst):
    n = inst.n
    vis = [False] * n
    t = [0]
    vis[0] = True
    for _ in range(n - 1):
        i = t[-1]
        best = None
        for j in range(n):
            if vis[j]:
                continue
            if inst.kind == "coords":
                dx = inst.coords[i, 0] - inst.coords[j, 0]
                dy = inst.coords[i, 1] - inst.coords[j, 1]
                key = float(dx * dx + dy * dy)
            else:
                key = float(inst.dist[i, j])
            if best is None or (key, j) < best:
                best = (key, j)
        t.append(best[1])
        vis[best[1]] = True
    return np.array(t)


def test_nn_tour_brute_force_with_ties():
    for inst in [wl.random_instance(60, seed=2), wl.random_instance(60, seed=3, grid=8),
                 wl.random_instance(45, seed=4, kind="matrix", symmetric=False)]:
        t, L = oracle.nn_tour(inst)
        assert np.array_equal(t, brute_nn_tour(inst))
        assert L == pytest.approx(math.fsum(_edge_lengths(inst, t)), rel=1e-12)


def _edge_lengths(inst, t):
    n = len(t)
    out = []
    for s in range(n):
        i, j = int(t[s]), int(t[(s + 1) % n])
        if inst.kind == "coords":
            out.append(math.dist(inst.coords[i], inst.coords[j]))
        else:
            out.append(float(inst.dist[i, j]))
    return out


def test_tour_length_is_eq1():
    inst = wl.random_instance(200, seed=8)
    t = np.random.default_rng(0).permutation(200)
    assert oracle.tour_length(inst, t) == pytest.approx(math.fsum(_edge_lengths(inst, t)), rel=1e-13)


# --------------------------------------------------------------------------
# Section III-D: 2-opt on neighbour lists
# --------------------------------------------------------------------------
def _two_opt_gain_left(inst, nl, t, min_gain):
    """largest gain of any succ/pred neighbour-list 2-opt move (brute force)"""
    n = len(t)
    pos = np.empty(n, dtype=np.int64)
    pos[t] = np.arange(n)
    d = lambda i, j: math.dist(inst.coords[i], inst.coords[j])
    best = -1.0
    for a in range(n):
        for step in (1, -1):
            b = t[(pos[a] + step) % n]
            for c in nl[a]:
                if d(a, c) >= d(a, b):
                    break
                e = t[(pos[c] + step) % n]
                if e == a or c == b:
                    continue
                best = max(best, d(a, b) + d(c, e) - d(a, c) - d(b, e))
    return best


def test_two_opt_local_optimum():
    inst = wl.random_instance(150, seed=21)
    nl = oracle.nearest_lists(inst, 10)
    rng = np.random.default_rng(1)
    for trial in range(3):
        t0 = rng.permutation(150).astype(np.int32)
        L0 = oracle.tour_length(inst, t0)
        t1 = oracle.two_opt(inst, nl, t0, 1e-12)
        assert sorted(t1) == list(range(150))
        L1 = oracle.tour_length(inst, t1)
        assert L1 < L0
        assert _two_opt_gain_left(inst, nl, t1, 1e-12) <= 1e-12
    # an optimal tour of a convex polygon is left unchanged
    ang = np.linspace(0, 2 * np.pi, 40, endpoint=False)
    xy = np.stack([np.cos(ang), np.sin(ang)], 1)
    poly = wl.Instance(40, "coords", True, xy, None, wl.empty_heatmap(40), 2, 1, 5)
    nlp = oracle.nearest_lists(poly, 6)
    t = np.arange(40, dtype=np.int32)
    assert np.array_equal(oracle.two_opt(poly, nlp, t, 1e-12), t)


# --------------------------------------------------------------------------
# Exact small instances: the decoder reaches the optimum
# --------------------------------------------------------------------------
def held_karp(D):
    n = len(D)
    full = 1 << (n - 1)
    INF = float("inf")
    dp = np.full((full, n - 1), INF)
    for j in range(n - 1):
        dp[1 << j, j] = D[0][j + 1]
    for S in range(1, full):
        for j in range(n - 1):
            if not (S >> j) & 1 or dp[S, j] == INF:
                continue
            base = dp[S, j]
            for q in range(n - 1):
                if (S >> q) & 1:
                    continue
                T = S | (1 << q)
                v = base + D[j + 1][q + 1]
                if v < dp[T, q]:
                    dp[T, q] = v
    return min(dp[full - 1, j] + D[j + 1][0] for j in range(n - 1))


def brute_force(D):
    import itertools
    n = len(D)
    best = float("inf")
    for perm in itertools.permutations(range(1, n)):
        t = (0,) + perm
        best = min(best, sum(D[t[s]][t[(s + 1) % n]] for s in range(n)))
    return best


def _dense(inst):
    if inst.kind == "coords":
        xy = inst.coords
        return [[math.dist(xy[i], xy[j]) for j in range(inst.n)] for i in range(inst.n)]
    return inst.dist.tolist()


# The ATSP runs with rho = 0.2 (Section IV-C), which evaporates slowly, so it
# gets a longer budget; plain MMAS (empty heatmap) needs the same.
@pytest.mark.parametrize("n,kind,sym,exact,iters", [(7, "coords", True, "bf", 100), (9, "coords", True, "bf", 100),
                                                    (11, "coords", True, "hk", 100),
                                                    (10, "matrix", False, "hk", 400)])
def test_decoder_reaches_optimum(n, kind, sym, exact, iters):
    hits = 0
    seeds = 100
    for seed in range(seeds):
        inst = wl.random_instance(n, seed=1000 + seed, topk=3, k=n - 1, ants=20, iterations=iters,
                                  kind=kind, symmetric=sym)
        D = _dense(inst)
        opt = brute_force(D) if exact == "bf" else held_karp(D)
        st, tour, L, _ = oracle.decode(inst)
        assert st == 0
        assert sorted(tour) == list(range(n))
        assert L >= opt * (1 - 1e-12)
        hits += L <= opt * (1 + 1e-12)
    if n <= 7:
        assert hits == seeds
    else:
        assert hits >= 95


# --------------------------------------------------------------------------
# Invariants of the whole loop (eq. (7), Section III-B)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["tsp100", "sym_matrix", "atsp", "ls"])
def test_decode_invariants(which):
    if which == "tsp100":
        inst = wl.tsp100(iterations=60)
    elif which == "sym_matrix":
        inst = wl.random_instance(70, seed=5, kind="matrix", symmetric=True, ants=10, iterations=40)
    elif which == "atsp":
        inst = wl.random_instance(70, seed=6, kind="matrix", symmetric=False, ants=10, iterations=40)
    else:
        inst = wl.random_instance(120, seed=7, ants=10, iterations=30, local_search=1, k_ls=10)
    st, tour, L, info = oracle.decode(inst, trace=True, state=True)
    assert st == 0
    n = inst.n
    assert sorted(tour) == list(range(n)) and tour[0] == 0
    for t in info["ant_tours"]:
        assert sorted(t) == list(range(n))
    assert L == pytest.approx(math.fsum(_edge_lengths(inst, tour)), rel=1e-12)
    lg = info["l_gb"]
    assert np.all(np.diff(lg) <= 0) and lg[0] <= info["l_nn"]
    assert L == lg[-1]
    tau = info["tau"]
    cand = info["cand"]
    # all trails inside [tau_min, tau_max] of the final bounds
    lo, hi = tau.min(), tau.max()
    assert lo > 0 and hi / lo <= info["r_hat"] * (1 + 1e-5)
    # weights are tau * S in FP32
    assert np.array_equal(info["weight"], (tau * info["heur"]).astype(np.float32))
    if inst.symmetric:
        # the same pheromone on both slots of an undirected candidate edge
        slot = {(i, int(j)): tau[i, u] for i in range(n) for u, j in enumerate(cand[i])}
        for (i, j), v in slot.items():
            if (j, i) in slot:
                assert slot[(j, i)] == v


def test_heatmap_never_enters_pheromone():
    # Section III-B: the heatmap acts only through construction, so with no
    # iterations the pheromone is uniformly tau_max whatever the heatmap
    a = wl.tsp100(iterations=0)
    b = wl.tsp100(iterations=0)
    b.heat = wl.empty_heatmap(100)
    _, _, _, ia = oracle.decode(a, state=True)
    _, _, _, ib = oracle.decode(b, state=True)
    assert np.all(ia["tau"] == ia["tau"][0, 0])
    assert ia["tau"][0, 0] == ib["tau"][0, 0]


def test_invalid_inputs_rejected():
    inst = wl.random_instance(20, seed=1)
    bad = wl.random_instance(20, seed=1)
    bad.heat = wl.Heatmap(20, inst.heat.row_ptr.copy(), inst.heat.col.copy(), inst.heat.val.copy())
    bad.heat.col[1] = bad.heat.col[0]  # duplicate column in row 0
    assert oracle.decode(bad)[0] != 0
    assert oracle.decode(inst, rho=1.5)[0] != 0
    assert oracle.decode(inst, alpha=2.0)[0] != 0
    assert oracle.decode(inst)[0] == 0


# --------------------------------------------------------------------------
# Section V: heatmap diagnostics against a known tour
# --------------------------------------------------------------------------
def _hexagon(entries, kind="coords"):
    n = 6
    xy = np.array([[math.cos(2 * math.pi * i / n), math.sin(2 * math.pi * i / n)] for i in range(n)])
    keys = sorted(entries)
    rp = np.zeros(n + 1, dtype=np.int32)
    for i, _ in keys:
        rp[i + 1] += 1
    heat = wl.Heatmap(n, np.cumsum(rp).astype(np.int32), np.array([j for _, j in keys], dtype=np.int32),
                      np.array([entries[x] for x in keys], dtype=np.float32))
    if kind == "coords":
        return wl.Instance(n, "coords", True, xy, None, heat, ants=2, iterations=1, k=3)
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    return wl.Instance(n, "matrix", False, None, d, heat, ants=2, iterations=1, k=3)


def _hexagon_entries():
    # tour 0-1-2-3-4-5 with both directions at 1.0, except {2,3} at 0.1; a
    # chord {0,3} at 1.0; a directed chord (2,5) at 1.0; (1,4) below theta_h
    e = {}
    for i in range(6):
        e[(i, (i + 1) % 6)] = 1.0
        e[((i + 1) % 6, i)] = 1.0
    e[(2, 3)] = e[(3, 2)] = 0.1
    e[(0, 3)] = e[(3, 0)] = 1.0
    e[(2, 5)] = 1.0
    e[(1, 4)] = 5e-5
    return e


def test_diagnostics_worked_example():
    # Worked by hand (d* = 2, k = 3):
    #  entries above theta_h: 12 tour directions + (0,3), (3,0), (2,5) = 15,
    #  so Edges/n = 15 / 12; every tour edge is present: coverage 1, Miss 0.
    #  Row 0: three equal confidences, b = 1, no e > 1.  Rows 1, 4, 5: two
    #  supported candidates, b = eps, both tour neighbours get e > 1.  Row 2:
    #  {1: 1, 3: 0.1, 5: 1}, b = 0.1, e > 1 on 1 (tour) and 5 (chord).  Row 3:
    #  {2: 0.1, 4: 1, 0: 1}, e > 1 on 4 (tour) and 0 (chord).  10 slots, 8 on
    #  the tour: P(e>1) = 0.8.
    d = oracle.diagnostics(_hexagon(_hexagon_entries()), np.arange(6))
    assert d["entries"] == 15 and d["edges_per_node"] == 15 / 12
    assert d["coverage"] == 1.0 and d["miss_pct"] == 0.0
    assert d["evidence_slots"] == 10 and d["evidence_on_tour"] == 8 and d["p_evidence"] == 0.8
    # the same tour read backwards covers the same undirected edges
    d2 = oracle.diagnostics(_hexagon(_hexagon_entries()), np.arange(6)[::-1])
    assert d2["coverage"] == 1.0 and d2["p_evidence"] == 0.8


def test_diagnostics_directed_coverage():
    # Drop the direction (2,3): a symmetric instance still covers tour edge
    # {2,3} through (3,2); on the ATSP the directed edge 2 -> 3 is missing.
    e = _hexagon_entries()
    del e[(2, 3)]
    sym = oracle.diagnostics(_hexagon(e), np.arange(6))
    asym = oracle.diagnostics(_hexagon(e, kind="matrix"), np.arange(6))
    assert sym["coverage"] == 1.0
    assert asym["coverage"] == 5 / 6 and asym["miss_pct"] == pytest.approx(100 / 6, rel=1e-12)
    # an entry below the threshold does not count
    e2 = _hexagon_entries()
    e2[(4, 5)] = e2[(5, 4)] = 5e-5
    assert oracle.diagnostics(_hexagon(e2), np.arange(6))["coverage"] == 5 / 6


def test_diagnostics_invalid_tour():
    assert oracle.diagnostics(_hexagon(_hexagon_entries()), [0, 1, 2, 3, 4, 4]) is None
    assert oracle.diagnostics(_hexagon(_hexagon_entries()), [0, 1, 2, 3, 4, 6]) is None
