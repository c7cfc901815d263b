"""GPU parity of the 3-opt (symmetric instances): tours, lengths, the last
iteration's ant tours and the per-iteration trace equal the oracle's, with
the 3-opt on the iteration best and on every ant, with the working arrays
in LDS (uint16 with FP32-filtered tests on tour-ordered coordinates, or
int32 with FP64 tests) and in global memory, on coordinates (near the
origin, far from it, on a lattice) and on a symmetric matrix, inside mixed
batches beside the 2-opt and the directed 2-opt, and among served
requests."""

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
    for name in ("tau", "ant_tours", "nn_tour"):
        assert np.array_equal(g[name], info[name]), f"{name} differs"
    assert np.array_equal(g["ant_len"], info["ant_len"])
    tr = ctx.debug_trace(0, inst.iterations)
    assert np.array_equal(tr["l_ib"], info["l_ib"])
    assert np.array_equal(tr["l_gb"], info["l_gb"])


def _three(inst):
    return dataclasses.replace(inst, ls_op=3)


# working arrays (HAC_LS_MODE) and waves per block (HAC_LS_WAVES): FP32 mode
# blocks of four or more waves stop waves whose result will be dropped,
# narrower ones do not
MODES = {"lds_fp32": (None, None), "lds_fp32_2_waves": (None, "2"), "lds_int32": ("1", None),
         "global": ("0", None)}


@pytest.mark.parametrize("ls", [1, 2])
@pytest.mark.parametrize("mode", list(MODES))
def test_three_opt_small(ctx, ls, mode, monkeypatch):
    inst = _three(wl.random_instance(120, seed=60 + ls, k=8, ants=8, iterations=15, local_search=ls, k_ls=10))
    ls_mode, waves = MODES[mode]
    if ls_mode is not None:
        monkeypatch.setenv("HAC_LS_MODE", ls_mode)
    if waves is not None:
        monkeypatch.setenv("HAC_LS_WAVES", waves)
    print(f"case 3-opt n=120 local_search {ls} {mode}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"ls{ls} {mode}")
    _state(ctx, inst)


@pytest.mark.parametrize("where", ["offset", "lattice"])
def test_three_opt_fp32_filters(ctx, where):
    """Far from the origin (the FP32 error bounds scale with the largest
    coordinate) and on a lattice (exact ties, decided in FP64 inside the
    bounds), with the 3-opt on every ant."""
    if where == "offset":
        inst = _three(wl.random_instance(300, seed=66, k=10, ants=8, iterations=12, local_search=2, k_ls=16))
        inst.coords = inst.coords * 1e5 + 3e6
    else:
        inst = _three(wl.random_instance(196, seed=67, grid=14, k=10, ants=8, iterations=12, local_search=2,
                                         k_ls=16))
    print(f"case 3-opt FP32 filters {where}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), where)
    _state(ctx, inst)


def test_three_opt_symmetric_matrix(ctx):
    inst = _three(wl.random_instance(90, seed=64, kind="matrix", symmetric=True, k=8, ants=8, iterations=12,
                                     local_search=2, k_ls=12))
    print("case 3-opt symmetric matrix n=90", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), "symmatrix")


@pytest.mark.parametrize("n", [5, 6, 8, 13])
def test_three_opt_tiny(ctx, n):
    inst = _three(wl.random_instance(n, seed=70 + n, k=min(8, n - 1), ants=4, iterations=6, local_search=2,
                                     k_ls=min(10, n - 1)))
    print(f"case 3-opt tiny n={n}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"n{n}")


def test_three_opt_ties(ctx):
    """Coordinates on a lattice: many equal distances and gains."""
    inst = _three(wl.random_instance(100, seed=75, grid=11, k=8, ants=6, iterations=10, local_search=2, k_ls=10))
    print("case 3-opt lattice n=100", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), "ties")


@pytest.mark.parametrize("waves", [None, "1"])
def test_three_opt_paper_setting(ctx, waves, monkeypatch):
    """n = 1000 with the paper's k = 20, k_ls = 20, 32 ants, rho = 0.8, the
    3-opt on every ant's tour (16-wave blocks, and one wave per tour)."""
    if waves is not None:
        monkeypatch.setenv("HAC_LS_WAVES", waves)
    inst = _three(wl.paper_budget(1000, count=1, local_search=2, iterations=6)[0])
    print(f"case 3-opt paper setting n=1000 waves {waves}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), "paper1000")
    _state(ctx, inst)


def test_three_opt_in_mixed_batch(ctx):
    """3-opt instances beside 2-opt ones, an ATSP with the directed 2-opt and
    one without local search: each result equals the oracle's and the
    instance decoded alone."""
    insts = [_three(wl.random_instance(80, seed=80, k=8, ants=6, iterations=10, local_search=1, k_ls=10)),
             wl.random_instance(100, seed=81, k=8, ants=6, iterations=10, local_search=2, k_ls=10),
             _three(wl.random_instance(110, seed=82, k=8, ants=7, iterations=9, local_search=2, k_ls=10)),
             wl.random_instance(70, seed=83, kind="matrix", symmetric=False, k=8, ants=6, iterations=8,
                                local_search=1, k_ls=10),
             wl.random_instance(60, seed=84, k=8, ants=6, iterations=8)]
    print("case 3-opt mixed batch", flush=True)
    got = ctx.decode_batch(insts)
    for x, inst in enumerate(insts):
        _same(got[x], oracle.decode(inst), f"mixed{x}")
        alone = ctx.decode(inst)
        assert np.array_equal(alone[0], got[x][0]) and alone[1] == got[x][1]


def test_three_opt_served(ctx, hac):
    """Served 3-opt requests, beside other kinds, equal the same requests
    decoded alone and the oracle."""
    insts = [_three(wl.random_instance(90, seed=90, k=8, ants=6, iterations=9, local_search=1, k_ls=10)),
             wl.random_instance(80, seed=91, k=8, ants=6, iterations=8),
             _three(wl.random_instance(120, seed=92, k=8, ants=6, iterations=8, local_search=2, k_ls=10)),
             wl.random_instance(100, seed=93, k=8, ants=6, iterations=8, local_search=1, k_ls=10)]
    alone = [ctx.decode(x) for x in insts]
    print("case 3-opt served", flush=True)
    srv = hac.Server(ctx, budget=1 << 30, max_slots=3)
    tickets = [srv.submit(x) for x in insts]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for x, inst in enumerate(insts):
        assert np.array_equal(res[x][0], alone[x][0]) and res[x][1] == alone[x][1], x
        _same(alone[x], oracle.decode(inst), f"served{x}")


def test_three_opt_tsp10k_sampled(ctx):
    """n = 10 000 (the tour-ordered arrays take 150 KB of LDS): the 3-opt on
    the NN tour and on the iteration best of two instances decoded in one
    batch, the first two iterations of one compared with the oracle."""
    insts = [_three(x) for x in wl.tsp10k(2, iterations=2)]
    print("case 3-opt tsp10k sampled", flush=True)
    got = ctx.decode_batch(insts)
    _same(got[1], oracle.decode(insts[1]), "tsp10k")
    t, L = got[0]
    assert sorted(t.tolist()) == list(range(insts[0].n))
