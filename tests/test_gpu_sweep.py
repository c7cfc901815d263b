"""GPU parity over the random sweep cases: one mixed batch, each case alone,
and all cases through the request server.  Every tour equals the oracle's
and every length agrees within 1e-12 relative."""

import numpy as np
import pytest

import oracle
from _sweep import sweep_cases

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def hac():
    import paper_2601_19041_amd as hac
    return hac


@pytest.fixture(scope="module")
def ctx(hac):
    c = hac.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def cases():
    out = []
    for inst, over in sweep_cases():
        st, tour, L, _ = oracle.decode(inst, **over)
        assert st == 0, inst.name
        out.append((inst, over, tour, L))
    return out


def _same(got, ref_tour, ref_len, what):
    tour, L = got[0], got[1]
    assert np.array_equal(tour, ref_tour), f"{what}: tours differ at {np.flatnonzero(tour != ref_tour)[:5]}"
    assert abs(L - ref_len) <= REL * max(ref_len, 1.0), (what, L, ref_len)


def test_sweep_batch_and_alone(ctx, cases):
    print(f"case sweep batch of {len(cases)}", flush=True)
    got = ctx.decode_batch([c[0] for c in cases], [c[1] for c in cases])
    for (inst, over, tour, L), g in zip(cases, got):
        _same(g, tour, L, "batch " + inst.name)
    for inst, over, tour, L in cases:
        print(f"case sweep alone {inst.name}", flush=True)
        _same(ctx.decode(inst, **over), tour, L, "alone " + inst.name)


def test_sweep_served(hac, ctx, cases):
    print(f"case sweep served {len(cases)}", flush=True)
    srv = hac.Server(ctx, budget=1 << 30, max_slots=5)
    try:
        tickets = [srv.submit(inst, **over) for inst, over, _, _ in cases]
        for t, (inst, over, tour, L) in zip(tickets, cases):
            got = srv.wait(t)
            _same(got, tour, L, "served " + inst.name)
    finally:
        srv.close()


def test_sweep_device_inputs(hac, ctx, cases):
    """hac_decode_batch_dev: inputs and outputs in device memory."""
    print(f"case sweep device inputs {len(cases)}", flush=True)
    b = hac.DeviceBatch([c[0] for c in cases], [c[1] for c in cases])
    ctx.decode_batch_dev(b)
    lens = b.lengths.cpu().numpy()
    for x, (inst, over, tour, L) in enumerate(cases):
        _same((b.tours[x].cpu().numpy(), float(lens[x])), tour, L, "device " + inst.name)


@pytest.mark.parametrize("shape", ["2,0,1", "7,1,2", "12,2,4", "5,3,3", "16,1,4", "3,2,1"])
def test_sweep_pinned_shapes(ctx, cases, shape, monkeypatch):
    """The cases below the grid size in one batch at pinned launch shapes
    (ants per block, LDS staging form, ants per wave)."""
    small = [c for c in cases if c[0].n < 2048]
    monkeypatch.setenv("HAC_SHAPE", shape)
    print(f"case sweep shape {shape} ({len(small)} cases)", flush=True)
    got = ctx.decode_batch([c[0] for c in small], [c[1] for c in small])
    st = ctx.stats()
    assert (st["ants_per_block"], st["lds_staged"], st["ants_per_wave"]) == tuple(map(int, shape.split(",")))
    for (inst, over, tour, L), g in zip(small, got):
        _same(g, tour, L, f"shape {shape} " + inst.name)


@pytest.mark.parametrize("env", [(("HAC_LS_MODE", "0"),), (("HAC_LS_MODE", "1"),), (("HAC_LS_WAVES", "3"),),
                                 (("HAC_BIT_MARKS", "1"), ("HAC_SHAPE", "8,0,4"))],
                         ids=["ls_global", "ls_lds_int32", "ls_3_waves", "bit_marks"])
def test_sweep_pinned_variants(ctx, cases, env, monkeypatch):
    """2-opt working arrays in global memory or as int32 in LDS, 2-opt blocks
    of three waves, and bit visited marks: the tours do not change."""
    use = [c for c in cases if c[0].n < 2048] if dict(env).get("HAC_SHAPE") else cases
    for name, value in env:
        monkeypatch.setenv(name, value)
    print(f"case sweep {env} ({len(use)} cases)", flush=True)
    got = ctx.decode_batch([c[0] for c in use], [c[1] for c in use])
    if dict(env).get("HAC_BIT_MARKS"):
        assert ctx.stats()["byte_marks"] == 0
    for (inst, over, tour, L), g in zip(use, got):
        _same(g, tour, L, f"{env} " + inst.name)
