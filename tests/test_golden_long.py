"""The stored full-length oracle results (tests/golden/long/) describe the
current oracle and these inputs.

The files are written by tests/golden/make_long_goldens.py, which calls only
the oracle and the input generators.  Checked here without a GPU: the
oracle source has not changed since (its SHA-256), every stored tour is a
Hamiltonian cycle in canonical form whose length, recomputed independently,
is the stored one, the global-best trace is monotone and ends at that
length, and the oracle's first two iterations of two cases reproduce the
stored traces (so the files belong to these seeded inputs).
"""

import hashlib
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden", "long")
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
import make_long_goldens as mk  # noqa: E402


@pytest.fixture(scope="module")
def index():
    return json.load(open(os.path.join(GOLD, "index.json")))


def test_goldens_describe_the_current_oracle(index):
    src = hashlib.sha256(open(os.path.join(ROOT, "oracle", "hac_oracle.c"), "rb").read()).hexdigest()
    assert index["oracle_source_sha256"] == src, \
        "the oracle changed since tests/golden/long was written: run python tests/golden/make_long_goldens.py"
    assert sorted(index["cases"]) == sorted(name for name, _ in mk.cases())


def test_stored_tours_are_canonical_cycles_of_their_length(index):
    for name, meta in index["cases"].items():
        g = np.load(os.path.join(GOLD, name + ".npz"))
        inst = mk.build_instance(tuple(meta["spec"]))
        t = g["tour"]
        n = inst.n
        assert sorted(t.tolist()) == list(range(n)) and t[0] == 0 and t[1] < t[-1]
        xy = inst.coords
        L = math.fsum(math.dist(xy[t[s]], xy[t[(s + 1) % n]]) for s in range(n))
        assert float(g["length"]) == pytest.approx(L, rel=1e-12)
        assert np.all(np.diff(g["l_gb"]) <= 0) and g["l_gb"][-1] == float(g["length"])
        assert len(g["l_ib"]) == inst.iterations


@pytest.mark.parametrize("name", ["tsp10k_3", "serve_tsp10000_12"])
def test_first_iterations_reproduce(index, name):
    meta = index["cases"][name]
    inst = mk.build_instance(tuple(meta["spec"]))
    st, _, _, info = oracle.decode(inst, trace=True, iterations=2)
    g = np.load(os.path.join(GOLD, name + ".npz"))
    assert st == 0
    assert np.array_equal(info["l_ib"], g["l_ib"][:2]) and np.array_equal(info["l_gb"], g["l_gb"][:2])
