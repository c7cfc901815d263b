"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Tours must be identical and lengths equal within 1e-12 relative (they are
summed in the same order, so in practice they are bit-identical).  Small
cases also compare the internal state (candidate lists, folded weights,
pheromone, choice weights, the last iteration's ant tours) bit for bit and
the per-iteration trace.
"""

import os

import numpy as np
import pytest

import oracle
from paper_2601_19041_amd import workloads as wl

pytestmark = pytest.mark.gpu

REL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    import paper_2601_19041_amd as hac
    c = hac.Context(0)
    yield c
    c.close()


def _same(gpu, ref, what=""):
    gt, gl = gpu
    st, ot, ol, _ = ref
    assert st == 0
    assert np.array_equal(gt, ot), f"{what}: tours differ at {np.flatnonzero(gt != ot)[:5]}"
    assert abs(gl - ol) <= REL * ol, (what, gl, ol)


def _state_parity(ctx, inst, which=0, **over):
    n, ants = inst.n, over.get("ants", inst.ants)
    k = over.get("k", inst.k)
    g = ctx.debug_state(which, n, k, ants)
    st, tour, L, info = oracle.decode(inst, trace=True, state=True, **over)
    assert st == 0
    for name in ("cand", "heur", "tau", "weight", "ant_tours", "nn_tour"):
        assert np.array_equal(g[name], info[name]), f"{name} differs"
    assert np.array_equal(g["ant_len"], info["ant_len"]), "ant lengths differ"
    tr = ctx.debug_trace(which, over.get("iterations", inst.iterations))
    assert np.array_equal(tr["l_ib"], info["l_ib"])
    assert np.array_equal(tr["l_gb"], info["l_gb"])
    assert np.array_equal(tr["elite_rb"], info["elite_rb"])
    return info


def test_tsp100_full(ctx):
    """The n=100 workload at its full size (k=10, 20 ants, 100 iterations)."""
    inst = wl.tsp100()
    print("case tsp100 full", flush=True)
    gpu = ctx.decode(inst)
    ref = oracle.decode(inst, trace=True)
    _same(gpu, ref, "tsp100")
    info = _state_parity(ctx, inst)
    assert ctx.stats()["fallback_steps"] == info["fallback_steps"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tsp100_seeds(ctx, seed):
    inst = wl.tsp100(instance=seed, seed=seed, iterations=40)
    print(f"case tsp100 seed {seed}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"seed{seed}")


@pytest.mark.parametrize("name", ["atsp", "symmatrix", "ls", "symmatrix_ls", "ls_grid", "ls_offset", "empty",
                                  "grid_ties", "k_full", "scope1", "ugb_restart", "ls_every",
                                  "symmatrix_ls_every", "ls_every_grid"])
def test_small_variants(ctx, name):
    over = {}
    if name == "symmatrix_ls":
        # 2-opt on a distance matrix: int32 working arrays, no FP32 filter
        inst = wl.random_instance(120, seed=13, kind="matrix", symmetric=True, k=8, ants=10, iterations=20,
                                  local_search=1, k_ls=10)
    elif name == "ls_every":
        # 2-opt on every ant's tour (Alg. 1): the ant tours compared below are the improved ones
        inst = wl.random_instance(150, seed=7, k=10, ants=12, iterations=25, local_search=2, k_ls=12)
    elif name == "symmatrix_ls_every":
        inst = wl.random_instance(110, seed=17, kind="matrix", symmetric=True, k=8, ants=9, iterations=15,
                                  local_search=2, k_ls=10)
    elif name == "ls_every_grid":
        inst = wl.random_instance(130, seed=18, grid=12, k=10, ants=7, iterations=15, local_search=2, k_ls=12)
    elif name == "ls_grid":
        # lattice points: many equal distances, so the FP32 2-opt tests fall
        # inside their error bound and are decided in FP64
        inst = wl.random_instance(140, seed=14, grid=13, k=10, ants=10, iterations=20, local_search=1, k_ls=12)
    elif name == "ls_offset":
        # far from the origin: the FP32 error bounds scale with the largest coordinate
        inst = wl.random_instance(150, seed=15, k=10, ants=10, iterations=20, local_search=1, k_ls=12)
        inst.coords = inst.coords * 1e5 + 3e6
    elif name == "atsp":
        inst = wl.random_instance(60, seed=5, kind="matrix", symmetric=False, k=8, ants=12, iterations=30)
    elif name == "symmatrix":
        inst = wl.random_instance(60, seed=6, kind="matrix", symmetric=True, k=8, ants=12, iterations=30)
    elif name == "ls":
        inst = wl.random_instance(150, seed=7, k=10, ants=12, iterations=25, local_search=1, k_ls=12)
    elif name == "empty":
        inst = wl.random_instance(80, seed=8, heat="empty", k=8, ants=10, iterations=30)
    elif name == "grid_ties":
        inst = wl.random_instance(90, seed=9, grid=12, k=10, ants=10, iterations=30)
    elif name == "k_full":
        inst = wl.random_instance(12, seed=10, k=11, ants=20, iterations=40)
    elif name == "scope1":
        inst = wl.random_instance(70, seed=11, k=6, ants=10, iterations=20)
        over = dict(baseline_scope=1)
    else:
        inst = wl.random_instance(40, seed=12, k=5, ants=6, iterations=60)
        over = dict(ugb_max=3, bf_period=7, restart_stall=2, lambda_bf=1e9)
    print(f"case {name}", flush=True)
    gpu = ctx.decode(inst, **over)
    ref = oracle.decode(inst, **over)
    _same(gpu, ref, name)
    _state_parity(ctx, inst, **over)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7])
def test_tiny_instances(ctx, n):
    inst = wl.random_instance(n, seed=20 + n, k=10, ants=3, iterations=5)
    print(f"case tiny n={n}", flush=True)
    gpu = ctx.decode(inst)
    ref = oracle.decode(inst)
    _same(gpu, ref, f"n{n}")


def test_batch_equals_alone(ctx):
    insts = [wl.random_instance(40 + 17 * x, seed=30 + x, k=8 + x % 3, ants=6 + x, iterations=15 + x)
             for x in range(6)]
    insts.append(wl.random_instance(50, seed=99, kind="matrix", symmetric=False, k=7, ants=5, iterations=12))
    print("case batch", flush=True)
    got = ctx.decode_batch(insts)
    for x, inst in enumerate(insts):
        _same(got[x], oracle.decode(inst), f"batch{x}")
        alone = ctx.decode(inst)
        assert np.array_equal(alone[0], got[x][0]) and alone[1] == got[x][1]


@pytest.mark.parametrize("shape", ["1,0", "4,0", "16,0", "1,1", "8,1", "4,0,1", "3,1,2", "4,1,1", "8,2", "3,2,2",
                                   "3,2,1", "8,3", "3,3,2"])
def test_launch_shape_independence(ctx, shape, monkeypatch):
    """Ants per block, LDS staging and ants per wave change nothing."""
    inst = wl.tsp100(instance=4, seed=4, iterations=25)
    monkeypatch.setenv("HAC_SHAPE", shape)
    print(f"case shape {shape}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), shape)


@pytest.mark.parametrize("shape", ["4,0", "8,1", "3,0,1", "8,2", "2,2,2", "8,3"])
def test_bit_marks(ctx, shape, monkeypatch):
    """Visited marks as bits instead of bytes (the form used when bytes do
    not fit in LDS) give the same tours."""
    inst = wl.tsp100(instance=5, seed=6, iterations=25)
    monkeypatch.setenv("HAC_SHAPE", shape)
    monkeypatch.setenv("HAC_BIT_MARKS", "1")
    print(f"case bit marks {shape}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), shape)
    assert ctx.stats()["byte_marks"] == 0


@pytest.mark.parametrize("geo", ["0", "1", "2"])
@pytest.mark.parametrize("shape", ["4,0", "8,1", "3,2,1", "4,3,2"])
def test_geo_list_modes(ctx, shape, geo, monkeypatch):
    """Each way an exhausted row consults its geometric list (not at all,
    int32 lists, uint16 lists a step ahead; a kernel per mode) with the table
    in global memory and in each LDS form.  k = 5 makes exhausted rows, list
    hits and scans frequent."""
    inst = wl.random_instance(160, seed=33, k=5, ants=8, iterations=12)
    monkeypatch.setenv("HAC_SHAPE", shape)
    monkeypatch.setenv("HAC_GEO_MODE", geo)
    print(f"case list mode {geo} shape {shape}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"{shape}/{geo}")
    assert ctx.stats()["geo_mode"] == int(geo)


@pytest.mark.parametrize("k,shape", [(24, "8,0"), (24, "4,1,1"), (40, "8,1"), (40, "2,0,2"), (64, "4,0"),
                                     (24, "8,2"), (40, "3,2,1"), (64, "4,2,2"), (24, "3,3,1")])
def test_wide_candidate_rows(ctx, k, shape, monkeypatch):
    """k > 16: each lane of an ant's row holds 2 or 4 slots; a batch with
    rows of different widths uses the widest."""
    insts = [wl.random_instance(150, seed=70 + k, k=k, ants=9, iterations=12),
             wl.random_instance(90, seed=71 + k, k=7, ants=5, iterations=12)]
    monkeypatch.setenv("HAC_SHAPE", shape)
    print(f"case wide k={k} shape {shape}", flush=True)
    got = ctx.decode_batch(insts)
    for x, inst in enumerate(insts):
        _same(got[x], oracle.decode(inst), f"k{k}/{x}")


def test_invalid_inputs_leave_outputs(ctx):
    import paper_2601_19041_amd as hac
    inst = wl.random_instance(30, seed=3)
    bad = wl.random_instance(30, seed=3)
    bad.heat = wl.Heatmap(30, inst.heat.row_ptr.copy(), inst.heat.col.copy(), inst.heat.val.copy())
    bad.heat.col[1] = bad.heat.col[0]
    assert ctx.decode_status(bad) == hac.HAC_EINVAL
    assert ctx.decode_status(inst, rho=0.0) == hac.HAC_EINVAL
    assert ctx.decode_status(inst, alpha=2.0) == hac.HAC_EUNSUPPORTED
    assert ctx.decode_status(inst, k=65) == hac.HAC_EUNSUPPORTED
    assert ctx.decode_status(inst) == hac.HAC_OK


def _grid_case(name):
    """Coordinate instances large enough for the uniform-grid search."""
    rng = np.random.default_rng(40)
    if name == "clusters":
        # tight clusters: the geometric lists run out whenever an ant leaves
        # one, so most fallbacks reach the grid search
        centres = rng.random((40, 2))
        xy = (centres[:, None, :] + 0.004 * rng.random((40, 60, 2))).reshape(-1, 2)
    elif name == "lattice":
        # distinct lattice points: equal keys across cells and rings
        cells = rng.permutation(50 * 50)[:2100]
        xy = np.stack([cells % 50, cells // 50], 1).astype(np.float64) / 50
    else:
        # every x equal: a bounding box of zero width
        xy = np.stack([np.full(2048, 0.5), rng.permutation(2048) / 2048.0], 1)
    xy = np.ascontiguousarray(xy)
    hm = wl.softdist_heatmap(xy, 6)
    return wl.Instance(len(xy), "coords", True, xy, None, hm, ants=8, iterations=3, k=6, seed=41,
                       name=f"grid-{name}")


@pytest.mark.parametrize("name", ["clusters", "lattice", "line"])
def test_grid_search(ctx, name):
    """n >= 2048 coordinates: nearest-unvisited searches go through the
    uniform grid and must return the (key, index) minimum of a full scan."""
    inst = _grid_case(name)
    print(f"case grid {name} n={inst.n}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), name)
    info = _state_parity(ctx, inst)
    assert info["fallback_steps"] > 0
    assert ctx.stats()["fallback_steps"] == info["fallback_steps"]


@pytest.mark.parametrize("ls", [1, 2])
@pytest.mark.parametrize("mode", ["0", "1", "2"])
def test_two_opt_modes(ctx, mode, ls, monkeypatch):
    """The 2-opt working-array modes (global memory; int32 arrays in LDS;
    uint16 arrays with FP32 coordinates in LDS and FP64 rechecks inside the
    error bound) give the same tours, on the iteration best and on every ant."""
    inst = wl.random_instance(600, seed=21, k=10, ants=8, iterations=6, local_search=ls, k_ls=16)
    monkeypatch.setenv("HAC_LS_MODE", mode)
    print(f"case 2-opt mode {mode} local_search {ls}", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"ls mode {mode}")
    if ls == 2:
        _state_parity(ctx, inst)


def test_batch_mixed_local_search(ctx):
    """One batch holding instances without local search, with 2-opt on the
    iteration best and with 2-opt on every ant (different ant counts): each
    result equals the oracle's and the instance decoded alone."""
    insts = [wl.random_instance(80, seed=41, k=8, ants=6, iterations=12),
             wl.random_instance(100, seed=42, k=8, ants=8, iterations=10, local_search=1, k_ls=10),
             wl.random_instance(120, seed=43, k=10, ants=10, iterations=12, local_search=2, k_ls=10),
             wl.random_instance(90, seed=44, k=6, ants=4, iterations=14, local_search=2, k_ls=8)]
    print("case batch mixed local search", flush=True)
    got = ctx.decode_batch(insts)
    for x, inst in enumerate(insts):
        _same(got[x], oracle.decode(inst), f"mixed{x}")
        alone = ctx.decode(inst)
        assert np.array_equal(alone[0], got[x][0]) and alone[1] == got[x][1]


@pytest.mark.parametrize("over", [dict(kappa_fixed=1.0), dict(kappa_fixed=0.0), dict(c_cap=0.0625), dict(c_cap=0.125),
                                  dict(c_cap=0.25), dict(c_cap=1.0), dict(c_cap=2.0)])
def test_ablation_settings(ctx, over):
    """Section IV-E: the fixed-scale ablation and the c_cap sweep."""
    inst = wl.tsp100(instance=3, seed=4, iterations=30)
    print(f"case ablation {over}", flush=True)
    gpu = ctx.decode(inst, **over)
    ref = oracle.decode(inst, **over)
    _same(gpu, ref, str(over))
    assert ctx.stats()["kappa"] == ref[3]["kappa"]


@pytest.mark.parametrize("waves", ["1", "3", "16"])
def test_every_ant_block_waves(ctx, waves, monkeypatch):
    """The waves of a 2-opt block set how many queue entries are evaluated
    at once; the outcome stays the sequential one."""
    inst = wl.random_instance(300, seed=23, k=10, ants=12, iterations=5, local_search=2, k_ls=12)
    monkeypatch.setenv("HAC_LS_WAVES", waves)
    print(f"case every-ant 2-opt, {waves} waves per block", flush=True)
    _same(ctx.decode(inst), oracle.decode(inst), f"waves {waves}")
    _state_parity(ctx, inst)


@pytest.mark.parametrize("which", ["tsp500", "atsp1000", "empty", "scope1"])
def test_heatmap_diagnostics(ctx, which):
    """Section V diagnostics through the C ABI equal the oracle's, against
    the oracle's NN tour and against a decoded tour."""
    over = {}
    if which == "tsp500":
        inst = wl.tsp500(iterations=5)
    elif which == "atsp1000":
        inst = wl.serve_request("atsp1000", 4, iterations=5)
    elif which == "empty":
        inst = wl.random_instance(60, seed=8, heat="empty", k=8, ants=6, iterations=5)
    else:
        inst = wl.random_instance(90, seed=11, k=6, ants=6, iterations=5)
        over = dict(baseline_scope=1)
    print(f"case diagnostics {which}", flush=True)
    st, t, L, info = oracle.decode(inst, state=True, **over)
    for tour in (info["nn_tour"], t):
        got = ctx.diagnostics(inst, tour, **over)
        want = oracle.diagnostics(inst, tour, **over)
        assert got == want, (got, want)
    if which == "empty":
        assert want["entries"] == 0 and want["coverage"] == 0.0 and want["evidence_slots"] == 0


def test_heatmap_diagnostics_rejects_bad_tours(ctx):
    import paper_2601_19041_amd as hac
    inst = wl.random_instance(30, seed=3)
    for bad in ([0] * 30, list(range(29)) + [30]):
        with pytest.raises(hac.HacError) as e:
            ctx.diagnostics(inst, bad)
        assert e.value.status == hac.HAC_EINVAL


def test_device_error_word_reported(ctx, monkeypatch):
    """When a kernel's own check flags an instance (forced here from the
    host through the error word, so no kernel misbehaves), every kernel of
    that instance stops, the call returns HAC_EDEVICE and the outputs stay
    untouched; the context then decodes normally again."""
    import paper_2601_19041_amd as hac
    inst = wl.tsp100(iterations=6)
    other = wl.random_instance(60, seed=3, ants=6, iterations=6)
    print("case forced device error word", flush=True)
    monkeypatch.setenv("HAC_FORCE_DEVICE_ERROR", "0")
    tour, L = ctx.decode(inst, raise_on_error=False)
    assert ctx.status == hac.HAC_EDEVICE and "pick contract" in ctx.last_error()
    assert not tour.any() and L == 0.0
    with pytest.raises(hac.HacError) as e:
        ctx.decode_batch([other, inst])
    assert e.value.status == hac.HAC_EDEVICE
    monkeypatch.delenv("HAC_FORCE_DEVICE_ERROR")
    _same(ctx.decode(inst), oracle.decode(inst), "after the error")
