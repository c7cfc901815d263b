"""The FP32 error bounds the GPU 2-opt and 3-opt use to decide their tests
without FP64 (distances from an FP32 copy of the coordinates).

A test decided in FP32 must agree with the FP64 decision whenever the FP32
value is farther from the threshold than the bound:
  d(a,b) - d(a,c) > 0                            bound E1 = 2^-18 M
  (ab + ce) - (ac + be) > g_min                  bound E2 = 2^-17 M
  (g1 + d43) - d45 > 0, g1 = d12 - d13           bound E2 = 2^-17 M
  ((d12 + d43) + d65) - ((d13 + d45) + d62) > g_min  bound E3 = 2^-16 M
with M the largest coordinate magnitude.  numpy's float32 arithmetic rounds
each operation to nearest, in the kernel's order (no fused multiply-add);
the square root is additionally perturbed by up to 4 ulp, so the bounds
hold for a square root that is not correctly rounded.  Near-ties are
planted on purpose so that both sides of each bound are exercised.
"""

import numpy as np
import pytest

F = np.float32


def d64(p, q):
    dx, dy = p[..., 0] - q[..., 0], p[..., 1] - q[..., 1]
    return np.sqrt(dx * dx + dy * dy)


def d32(p, q, rng):
    dx = p[..., 0].astype(F) - q[..., 0].astype(F)
    dy = p[..., 1].astype(F) - q[..., 1].astype(F)
    r = np.sqrt(dx * dx + dy * dy).astype(F)
    # a square root off by up to 4 ulp
    return _perturb(r, rng.integers(-4, 5, size=r.shape))


def _perturb(r, k):
    out = r.copy()
    for _ in range(4):
        up = k > 0
        dn = k < 0
        out = np.where(up, np.nextafter(out, F(np.inf)), out)
        out = np.where(dn, np.nextafter(out, F(-np.inf)), out)
        k = k - np.sign(k)
    return out.astype(F)


def _points(kind, rng, m):
    if kind == "unit":
        return rng.random((m, 2))
    if kind == "far":
        return rng.random((m, 2)) * 1e5 + 3e6
    if kind == "negative":
        return (rng.random((m, 2)) - 0.5) * 2e3
    return rng.integers(0, 40, size=(m, 2)).astype(np.float64) / 7.0  # lattice: exact ties


@pytest.mark.parametrize("kind", ["unit", "far", "negative", "lattice"])
def test_fp32_decisions_outside_the_bound_match_fp64(kind):
    rng = np.random.default_rng({"unit": 1, "far": 2, "negative": 3, "lattice": 4}[kind])
    m = 200_000
    a, b, c, e = (_points(kind, rng, m) for _ in range(4))
    # plant near-ties: c on (or next to) the circle through b around a
    t = rng.random(m) < 0.5
    ang = rng.random(m) * 2 * np.pi
    r = d64(a, b) * (1 + rng.normal(0, 1e-7, m))
    c[t] = a[t] + np.stack([r[t] * np.cos(ang[t]), r[t] * np.sin(ang[t])], axis=1)
    pts = np.concatenate([a, b, c, e])
    M = np.abs(pts).max()
    e1, e2 = M * 2.0 ** -18, M * 2.0 ** -17
    gmin = 1e-9 * 0.7

    dab, dac, dce, dbe = d64(a, b), d64(a, c), d64(c, e), d64(b, e)
    g1_64 = dab - dac > 0.0
    gain_64 = (dab + dce) - (dac + dbe) > gmin

    fab, fac, fce, fbe = (d32(p, q, rng) for p, q in ((a, b), (a, c), (c, e), (b, e)))
    g1f = (fab - fac).astype(F).astype(np.float64)
    gf = ((fab + fce).astype(F) - (fac + fbe).astype(F)).astype(F).astype(np.float64)

    sure_pos, sure_neg = g1f > e1, g1f < -e1
    assert not np.any(sure_pos & ~g1_64)
    assert not np.any(sure_neg & g1_64)
    sure_imp, sure_not = gf > gmin + e2, gf < gmin - e2
    assert not np.any(sure_imp & ~gain_64)
    assert not np.any(sure_not & gain_64)
    # both outcomes and the uncertain band all occur
    assert sure_pos.any() and sure_neg.any() and (~sure_pos & ~sure_neg).any()
    assert sure_imp.any() and sure_not.any()


@pytest.mark.parametrize("kind", ["unit", "far", "negative", "lattice"])
def test_fp32_exchange_decisions_outside_the_bound_match_fp64(kind):
    """The 3-opt's segment exchange: g2 (four distances) and the gain (six)."""
    rng = np.random.default_rng({"unit": 11, "far": 12, "negative": 13, "lattice": 14}[kind])
    m = 200_000
    p1, p2, p3, p4, p5, p6 = (_points(kind, rng, m) for _ in range(6))
    # plant near-ties of g2: t5 on (or next to) the circle around t4 whose
    # radius makes g2 zero, where that radius is positive
    g1 = d64(p1, p2) - d64(p1, p3)
    rad = (g1 + d64(p4, p3)) * (1 + rng.normal(0, 1e-7, m))
    t = (rng.random(m) < 0.5) & (rad > 0)
    ang = rng.random(m) * 2 * np.pi
    p5[t] = p4[t] + np.stack([rad[t] * np.cos(ang[t]), rad[t] * np.sin(ang[t])], axis=1)
    # and of the gain: t6 moved along the line t5-t2 until d65 - d62 takes the
    # value that makes the gain zero (where one exists on the segment)
    d12, d13, d43, d45 = d64(p1, p2), d64(p1, p3), d64(p4, p3), d64(p4, p5)
    want = (d13 + d45) - (d12 + d43)  # d65 - d62 at a zero gain
    L = d64(p5, p2)
    u = rng.random(m) < 0.5
    ok = u & (np.abs(want) < L) & (L > 0)
    s_ = np.where(ok, (L + want) / (2 * np.where(L > 0, L, 1)), 0.5)  # point at distance L*s_ from t5
    s_ = s_ * (1 + rng.normal(0, 1e-7, m))
    p6[ok] = p5[ok] + (p2[ok] - p5[ok]) * s_[ok, None]
    pts = np.concatenate([p1, p2, p3, p4, p5, p6])
    M = np.abs(pts).max()
    e2, e3 = M * 2.0 ** -17, M * 2.0 ** -16
    gmin = 1e-9 * 0.7

    d12, d13, d43, d45, d65, d62 = (d64(a, b) for a, b in ((p1, p2), (p1, p3), (p4, p3), (p4, p5),
                                                          (p6, p5), (p6, p2)))
    g2_64 = ((d12 - d13) + d43) - d45 > 0.0
    gain_64 = ((d12 + d43) + d65) - ((d13 + d45) + d62) > gmin

    f12, f13, f43, f45, f65, f62 = (d32(a, b, rng) for a, b in ((p1, p2), (p1, p3), (p4, p3), (p4, p5),
                                                               (p6, p5), (p6, p2)))
    g2f = (((f12 - f13).astype(F) + f43).astype(F) - f45).astype(F).astype(np.float64)
    gf = (((f12 + f43).astype(F) + f65).astype(F)
          - ((f13 + f45).astype(F) + f62).astype(F)).astype(F).astype(np.float64)

    sure_pos, sure_neg = g2f > e2, g2f < -e2
    assert not np.any(sure_pos & ~g2_64)
    assert not np.any(sure_neg & g2_64)
    sure_imp, sure_not = gf > gmin + e3, gf < gmin - e3
    assert not np.any(sure_imp & ~gain_64)
    assert not np.any(sure_not & gain_64)
    assert sure_pos.any() and sure_neg.any() and (~sure_pos & ~sure_neg).any()
    assert sure_imp.any() and sure_not.any() and (~sure_imp & ~sure_not).any()


def test_exchange_bounds_are_needed():
    """Shrunk 2^8-fold, the exchange bounds admit wrong FP32 decisions."""
    rng = np.random.default_rng(21)
    m = 200_000
    p1, p2, p3, p4, p5 = (_points("far", rng, m) for _ in range(5))
    g1 = d64(p1, p2) - d64(p1, p3)
    rad = (g1 + d64(p4, p3)) * (1 + rng.normal(0, 1e-9, m))
    t = rad > 0
    ang = rng.random(m) * 2 * np.pi
    p5[t] = p4[t] + np.stack([rad[t] * np.cos(ang[t]), rad[t] * np.sin(ang[t])], axis=1)
    M = np.abs(np.concatenate([p1, p2, p3, p4, p5])).max()
    g2_64 = ((d64(p1, p2) - d64(p1, p3)) + d64(p4, p3)) - d64(p4, p5) > 0.0
    f12, f13, f43, f45 = (d32(a, b, rng) for a, b in ((p1, p2), (p1, p3), (p4, p3), (p4, p5)))
    g2f = (((f12 - f13).astype(F) + f43).astype(F) - f45).astype(F).astype(np.float64)
    e = M * 2.0 ** -17 / 256
    wrong = np.sum((g2f > e) & ~g2_64) + np.sum((g2f < -e) & g2_64)
    assert wrong > 0
