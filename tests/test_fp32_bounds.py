"""The FP32 error bounds the GPU 2-opt uses to decide its tests without
FP64 (distances from an FP32 copy of the coordinates).

A test decided in FP32 must agree with the FP64 decision whenever the FP32
value is farther from the threshold than the bound:
  d(a,b) - d(a,c) > 0            bound E1 = 2^-18 M
  (ab + ce) - (ac + be) > g_min  bound E2 = 2^-17 M
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
