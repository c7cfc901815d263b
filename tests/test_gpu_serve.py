"""GPU tests of the batched device-input path and the continuous-batching
request loop: every result equals the plain path's and the oracle's, the
admission never exceeds the memory budget or slot count, arrival order does
not change any result, and cancellation / oversize requests are reported."""

import time

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hac():
    import paper_2601_19041_amd as hac
    return hac


@pytest.fixture(scope="module")
def ctx(hac):
    c = hac.Context(0)
    yield c
    c.close()


def _mix():
    out = []
    for x in range(5):
        out.append(wl.random_instance(60 + 37 * x, seed=200 + x, k=8 + x, ants=6 + x, iterations=10 + 3 * x))
    out.append(wl.random_instance(80, seed=300, kind="matrix", symmetric=False, k=9, ants=7, iterations=14))
    out.append(wl.random_instance(120, seed=301, k=10, ants=8, iterations=9, local_search=1, k_ls=10))
    # 2-opt on every ant's tour (its work area is per ant)
    out.append(wl.random_instance(140, seed=303, k=10, ants=6, iterations=8, local_search=2, k_ls=10))
    # the next size class: another lane, running concurrently
    out.append(wl.random_instance(800, seed=304, k=8, ants=6, iterations=6))
    out.append(wl.random_instance(1, seed=302))
    return out


def test_batch_dev_equals_plain(ctx, hac):
    insts = _mix()[:-1]
    print("case batch_dev", flush=True)
    db = hac.DeviceBatch(insts)
    ctx.decode_batch_dev(db)
    got = db.results()
    for x, inst in enumerate(insts):
        st, ot, ol, _ = oracle.decode(inst)
        assert np.array_equal(got[x][0], ot), x
        assert got[x][1] == ol


def test_served_equals_alone_under_budget(ctx, hac):
    insts = _mix()
    alone = [ctx.decode(x) for x in insts]
    fps = [hac.footprint(x) for x in insts]
    budget = int(sum(sorted(fps)[-3:]) * 1.05)  # about three requests at a time
    print("case serve budget", budget, flush=True)
    srv = hac.Server(ctx, budget=budget, max_slots=3)
    tickets = [srv.submit(x) for x in insts]
    res = [srv.wait(t) for t in tickets]
    cnt = srv.counters()
    srv_lanes = srv.lane_stats()
    srv.close()
    for x in range(len(insts)):
        assert np.array_equal(res[x][0], alone[x][0]), x
        assert res[x][1] == alone[x][1]
        assert res[x][2] >= 0.0
    assert cnt["completed"] == len(insts)
    assert cnt["peak_slots"] <= 3
    assert 0 < cnt["peak_bytes"] <= budget
    # every request with n > 1 ran in the lane of its size class
    lanes = srv_lanes
    for ln in lanes:
        want = sum(1 for x in insts if x.n > 1 and x.n >= ln["min_n"] and (ln["max_n"] == 0 or x.n < ln["max_n"]))
        assert ln["admitted"] == want and ln["completed"] == want, ln
        assert ln["peak_active"] <= 3
        if want:
            assert ln["rounds"] > 0 and ln["instance_iterations"] >= ln["iterations"] > 0


@pytest.mark.parametrize("order_seed", [0, 1])
def test_arrival_order_does_not_matter(ctx, hac, order_seed):
    insts = _mix()
    alone = [ctx.decode(x) for x in insts]
    rng = np.random.default_rng(order_seed)
    order = rng.permutation(len(insts))
    print("case serve order", order_seed, flush=True)
    srv = hac.Server(ctx, budget=1 << 30, max_slots=4)
    tickets = {}
    for i in order:
        tickets[int(i)] = srv.submit(insts[int(i)])
        time.sleep(float(rng.uniform(0, 0.01)))
    for i, t in tickets.items():
        tour, L, lat = srv.wait(t)
        assert np.array_equal(tour, alone[i][0]) and L == alone[i][1]
    srv.close()


def test_cancel_and_oversize(ctx, hac):
    big = wl.random_instance(300, seed=400, k=10, ants=20, iterations=100000)
    small = wl.random_instance(50, seed=401, k=8, ants=5, iterations=5)
    print("case serve cancel", flush=True)
    srv = hac.Server(ctx, budget=hac.footprint(big) + hac.footprint(small) + 4096, max_slots=2)
    t_big = srv.submit(big)
    t_small = srv.submit(small)
    time.sleep(0.2)
    assert srv.cancel(t_big) == hac.HAC_OK
    assert srv.wait_status(t_big) == hac.HAC_ECANCELLED
    tour, L, lat = srv.wait(t_small)
    assert np.array_equal(tour, ctx.decode(small)[0])
    huge = wl.random_instance(1500, seed=402, k=10, ants=600, iterations=5)
    assert hac.footprint(huge) > hac.footprint(big) + hac.footprint(small) + 4096
    with pytest.raises(hac.HacError) as e:
        srv.submit(huge)
    assert e.value.status == hac.HAC_ENOMEM
    srv.close()


def test_served_ablation_settings_equal_alone(ctx, hac):
    """Requests with the fixed-kappa ablation and a c_cap of the sweep are
    served with their own parameters, beside default ones."""
    inst = wl.random_instance(110, seed=310, k=8, ants=6, iterations=10)
    overs = [{}, dict(kappa_fixed=1.0), dict(c_cap=0.125), dict(kappa_fixed=0.0)]
    alone = [ctx.decode(inst, **o) for o in overs]
    print("case serve ablation", flush=True)
    srv = hac.Server(ctx, budget=1 << 30, max_slots=4)
    tickets = [srv.submit(inst, **o) for o in overs]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for x, o in enumerate(overs):
        assert np.array_equal(res[x][0], alone[x][0]) and res[x][1] == alone[x][1], o
        st, ot, ol, _ = oracle.decode(inst, **o)
        assert np.array_equal(res[x][0], ot), o
