"""GPU parity of the directed 2-opt (the ATSP with local search): tours,
lengths, the last iteration's ant tours and the per-iteration trace equal
the oracle's, with the 2-opt on the iteration best and on every ant, with
the work area in LDS and in global memory, inside mixed batches and among
served requests."""

import dataclasses

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl

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


def _same(gpu, ref, what=""):
    gt, gl = gpu
    st, ot, ol, _ = ref
    assert st == 0
    assert np.array_equal(gt, ot), f"{what}: tours differ at {np.flatnonzero(gt != ot)[:5]}"
    assert abs(gl - ol) <= REL * ol, (what, gl, ol)


def _state(ctx, inst):
    g = ctx.debug_state(0, inst.n, inst.k, inst.ants)
    st, tour, L, info = oracle.decode(inst, trace=True, state=True)
    assert st == 0
    for name in ("cand", "tau", "weight", "ant_tours", "nn_tour"):
        assert np.array_equal(g[name], info[name]), f"{name} differs"
    assert np.array_equal(g["ant_len"], info["ant_len"])
    tr = ctx.debug_trace(0, inst.iterations)
    assert np.array_equal(tr["l_ib"], info["l_ib"])
    assert np.array_equal(tr["l_gb"], info["l_gb"])


def _atsp(n, seed, ls, **kw):
    kw.setdefault("k", 8)
    kw.setdefault("ants", 10)
    kw.setdefault("iterations", 15)
    kw.setdefault("k_ls", 10)
    return wl.random_instance(n, seed=seed, kind="matrix", symmetric=False, local_search=ls, **kw)


@pytest.mark.parametrize("ls", [1, 2])
@pytest.mark.parametrize("mode", ["lds", "lds_work_only", "global"])
def test_directed_small(ctx, ls, mode, monkeypatch):
    """Work arrays and neighbour lists in LDS (the default here), work
    arrays only in LDS, and everything in global memory."""
    inst = _atsp(90, 50 + ls, ls)
    if mode == "global":
        monkeypatch.setenv("HAC_LS_MODE", "0")
    elif mode == "lds_work_only":
        monkeypatch.setenv("HAC_LS_MODE", "1")
    print(f"case directed n=90 local_search {ls} {mode}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"ls{ls} {mode}")
    _state(ctx, inst)


@pytest.mark.parametrize("n", [3, 4, 5, 8, 17])
def test_directed_tiny(ctx, n):
    inst = _atsp(n, 60 + n, 2, k=min(8, n - 1), ants=4, iterations=6, k_ls=min(10, n - 1))
    print(f"case directed tiny n={n}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"n{n}")


def test_directed_atsp1000(ctx):
    """The served ATSP request kind (n = 1000, k = 20, 50 ants) with the
    2-opt on the iteration best."""
    inst = dataclasses.replace(wl.serve_request("atsp1000", 3, iterations=12), local_search=1, k_ls=20)
    print("case directed atsp1000", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), "atsp1000")
    _state(ctx, inst)


def test_directed_past_lds(ctx):
    """n large enough that the work area does not fit in LDS."""
    inst = _atsp(3700, 70, 1, k=10, ants=6, iterations=3, k_ls=10)
    print("case directed n=3700 (global work area)", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), "n3700")


def test_directed_in_mixed_batch(ctx):
    """ATSP instances with and without local search beside symmetric ones
    with the 2-opt: each result equals the oracle's and the instance decoded
    alone."""
    insts = [_atsp(70, 80, 1), _atsp(110, 81, 2, ants=7),
             wl.random_instance(100, seed=82, k=8, ants=8, iterations=10, local_search=1, k_ls=10),
             _atsp(60, 83, 0),
             wl.random_instance(120, seed=84, k=8, ants=6, iterations=10, local_search=2, k_ls=10)]
    print("case directed mixed batch", flush=True)
    got = ctx.decode_batch(insts)
    for x, inst in enumerate(insts):
        _same(got[x], oracle.decode(inst), f"mixed{x}")
        alone = ctx.decode(inst)
        assert np.array_equal(alone[0], got[x][0]) and alone[1] == got[x][1]


def test_directed_served(ctx, hac):
    """Served ATSP requests with local search, beside other kinds, equal the
    same requests decoded alone and the oracle."""
    insts = [_atsp(80, 90, 1), wl.random_instance(90, seed=91, k=8, ants=6, iterations=10),
             _atsp(130, 92, 2, ants=6, iterations=9),
             wl.random_instance(100, seed=93, k=8, ants=6, iterations=8, local_search=1, k_ls=10),
             _atsp(70, 94, 0)]
    alone = [ctx.decode(x) for x in insts]
    print("case directed served", flush=True)
    srv = hac.Server(ctx, budget=1 << 30, max_slots=3)
    tickets = [srv.submit(x) for x in insts]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for x, inst in enumerate(insts):
        assert np.array_equal(res[x][0], alone[x][0]) and res[x][1] == alone[x][1], x
        _same(alone[x], oracle.decode(inst), f"served{x}")
