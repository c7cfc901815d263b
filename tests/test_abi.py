"""CPU checks of the C-ABI library: it loads, exports every declared symbol,
and its host-only validation and defaults behave as documented."""

import json
import os
import re

import numpy as np
import pytest

from paper_2601_19041_amd import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hac():
    import paper_2601_19041_amd as hac
    if not os.path.exists(hac.LIB_PATH):
        from paper_2601_19041_amd import build
        build.build()
    hac.lib()
    return hac


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hac.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hac_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(hac):
    names = declared_functions()
    assert len(names) >= 20
    L = hac.lib()
    for name in names:
        assert hasattr(L, name), name
    assert sorted(hac.EXPORTS) == names


def test_server_lane_count_matches_the_header(hac):
    text = open(os.path.join(ROOT, "include", "hac.h")).read()
    assert int(re.search(r"#define HAC_SERVER_LANES (\d+)", text).group(1)) == hac.SERVER_LANES


def test_defaults_are_the_papers(hac):
    prm = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_parameters.json")))
    p = hac.params_default()
    assert p.k == prm["k"] and p.k_ls == prm["k_ls"]
    assert p.alpha == prm["alpha"] and p.beta == prm["beta"]
    assert p.theta_h == prm["theta_h"] and p.eps == prm["eps"] and p.c_cap == prm["c_cap"]
    assert p.bf_period == prm["bf_period"] and p.xi_bf == prm["xi_bf"]
    assert p.restart_stall == prm["restart_stall"] and p.p_best == prm["p_best"]
    assert p.ugb_max == prm["ugb_start"]
    assert abs(p.lambda_bf - prm["lambda_bf"]) < 1e-15


def test_validate_host_only(hac):
    inst = wl.random_instance(30, seed=3)
    assert hac.validate(inst) == hac.HAC_OK
    bad = wl.random_instance(30, seed=3)
    bad.heat = wl.Heatmap(30, inst.heat.row_ptr.copy(), inst.heat.col.copy(), inst.heat.val.copy())
    bad.heat.col[1] = bad.heat.col[0]
    assert hac.validate(bad) == hac.HAC_EINVAL
    bad2 = wl.random_instance(30, seed=3)
    bad2.heat = wl.Heatmap(30, inst.heat.row_ptr.copy(), inst.heat.col.copy(), inst.heat.val.copy())
    bad2.heat.val[0] = -1.0
    assert hac.validate(bad2) == hac.HAC_EINVAL
    bad3 = wl.random_instance(30, seed=3)
    bad3.heat = wl.Heatmap(30, inst.heat.row_ptr.copy(), inst.heat.col.copy(), inst.heat.val.copy())
    bad3.heat.col[0] = 30
    assert hac.validate(bad3) == hac.HAC_EINVAL
    assert hac.validate(inst, rho=1.0) == hac.HAC_EINVAL
    assert hac.validate(inst, p_best=0.0) == hac.HAC_EINVAL
    assert hac.validate(inst, ants=0) == hac.HAC_EINVAL
    assert hac.validate(inst, alpha=2.0) == hac.HAC_EUNSUPPORTED
    assert hac.validate(inst, k=65) == hac.HAC_EUNSUPPORTED
    assert hac.validate(inst, local_search=1, k_ls=40) == hac.HAC_EUNSUPPORTED
    at = wl.random_instance(20, seed=4, kind="matrix", symmetric=False)
    assert hac.validate(at) == hac.HAC_OK
    assert hac.validate(at, local_search=1) == hac.HAC_OK  # the directed 2-opt
    # the 3-opt is for symmetric instances; other operators are invalid
    assert hac.validate(at, local_search=1, ls_op=3) == hac.HAC_EUNSUPPORTED
    assert hac.validate(at, ls_op=3) == hac.HAC_OK  # no local search, nothing to refuse
    assert hac.validate(inst, local_search=2, ls_op=3) == hac.HAC_OK
    assert hac.validate(inst, local_search=1, ls_op=4) == hac.HAC_EINVAL
    sm = wl.random_instance(20, seed=4, kind="matrix", symmetric=True)
    sm.dist = sm.dist.copy()
    sm.dist[1, 2] += 1e-3
    assert hac.validate(sm) == hac.HAC_EINVAL
    xy = wl.random_instance(20, seed=5)
    xy.coords = xy.coords.copy()
    xy.coords[3, 0] = np.nan
    assert hac.validate(xy) == hac.HAC_EINVAL


def test_strerror(hac):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert hac.strerror(code)
    assert hac.strerror(-99) == "unknown status"
