"""Writes the full-length expected results of the two largest workloads.

Run from the repository root:  python tests/golden/make_long_goldens.py

It calls only the CPU oracle (oracle/) and the seeded input generators
(paper_2601_19041_amd/workloads.py, which holds none of the method's
arithmetic), one process per case:
  * tsp10k_<x>: the eight 10 000-node instances of the batched workload
    (instance x, seed 1 + x), 200 iterations of 100 ants with k = 20 and
    the neighbour-list 2-opt (20 neighbours) on every iteration-best tour;
  * serve_tsp10000_<r>: the first 10 000-node request of the serving mix
    the benchmark submits (request r, seed 1 + r), 100 iterations of 100
    ants with k = 20, no local search.
Each case is stored as <name>.npz: the canonical tour (int32), its length,
and the per-iteration iteration-best length, global-best length and
restart-best deposit flags.  index.json records the oracle source's
SHA-256, so tests can tell when the files no longer describe the oracle.
An oracle decode of one case takes about 2-4 minutes on one core.
"""

import hashlib
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

OUT = os.path.join(HERE, "long")
ORACLE_SRC = os.path.join(ROOT, "oracle", "hac_oracle.c")


def serve_tsp10000_request() -> int:
    """Index of the first 10 000-node request in the benchmark's serving mix
    (240 requests, mix seed 1)."""
    from paper_2601_19041_amd import workloads as wl
    mix, _ = wl.serve_mix(240, 1.0, seed=1)
    return mix.index("tsp10000")


def cases():
    out = [("tsp10k_%d" % x, ("tsp10k", x)) for x in range(8)]
    r = serve_tsp10000_request()
    out.append(("serve_tsp10000_%d" % r, ("serve", r)))
    return out


def build_instance(spec):
    from paper_2601_19041_amd import workloads as wl
    kind, x = spec
    if kind == "tsp10k":
        return wl.tsp10k_instance(x, iterations=200)
    return wl.serve_request("tsp10000", x)


def _one(item):
    name, spec = item
    import oracle
    inst = build_instance(spec)
    st, tour, length, info = oracle.decode(inst, trace=True)
    assert st == 0, (name, st)
    np.savez_compressed(os.path.join(OUT, name + ".npz"), tour=tour.astype(np.int32),
                        length=np.float64(length), l_ib=info["l_ib"], l_gb=info["l_gb"],
                        elite_rb=info["elite_rb"].astype(np.int32))
    return name, float(length), int(info["fallback_steps"])


def oracle_sha256() -> str:
    return hashlib.sha256(open(ORACLE_SRC, "rb").read()).hexdigest()


def main():
    import oracle
    oracle.build(force=False)
    os.makedirs(OUT, exist_ok=True)
    todo = cases()
    with ProcessPoolExecutor(max_workers=min(len(todo), os.cpu_count() or 1)) as ex:
        done = list(ex.map(_one, todo))
    index = {"oracle_source_sha256": oracle_sha256(),
             "command": "python tests/golden/make_long_goldens.py",
             "cases": {name: {"length": length, "fallback_steps": fb, "spec": list(spec)}
                       for (name, length, fb), (_, spec) in zip(done, todo)}}
    with open(os.path.join(OUT, "index.json"), "w") as f:
        json.dump(index, f, indent=1)
    print(json.dumps(index["cases"], indent=1))


if __name__ == "__main__":
    main()
