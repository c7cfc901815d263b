"""Seeded random decode configurations for the sweep tests.

Each case is an instance (kind, size, heatmap density, ties) with its own
MMAS settings. Together they cross the settings the fixed parity cases take
one at a time:
* candidate width from 1 to 32 (one or two slots per lane);
* evaporation, p_best (both bound formulas), beta (integral and not);
* evidence threshold and scale, baseline scope, degree target;
* 2-opt on none, the iteration best, or every ant;
* short restart and elite schedules;
* tiny instances, and coordinate instances large enough for the grid
  search.
"""

import numpy as np

from paper_2601_19041_amd import workloads as wl


def sweep_cases(count: int = 96, seed: int = 2601):
    rng = np.random.default_rng(seed)
    cases = []
    for x in range(count):
        r = rng.random()
        kind = "coords" if r < 0.55 else ("symmatrix" if r < 0.75 else "atsp")
        size = rng.random()
        large = kind == "coords" and size > 0.9
        if size < 0.15:
            n = int(rng.choice([1, 2, 3, 5, 9, 17]))
        elif large:  # the grid search for nearest unvisited nodes
            n = int(rng.integers(2048, 3201))
        else:
            n = int(rng.integers(20, 401))
        k = int(rng.integers(1, 33))
        topk = int(rng.integers(2, 16))
        ants = int(rng.integers(1, 7 if large else 25))
        iterations = int(rng.integers(1, 4 if large else 26))
        ls = int(rng.choice([0, 0, 1, 2]))  # the ATSP takes the directed 2-opt
        k_ls = int(rng.integers(1, 25))
        heat = "empty" if rng.random() < 0.1 else "softdist"
        grid = None
        if kind == "coords" and n >= 4 and rng.random() < 0.25:
            grid = int(np.ceil(np.sqrt(n))) + int(rng.integers(0, 4))
        over = dict(
            beta=float(rng.choice([1.0, 2.0, 3.0, 2.5])),
            rho=float(np.round(rng.uniform(0.05, 0.95), 3)),
            p_best=float(rng.choice([0.05, 0.005, 0.3])),
            c_cap=float(rng.choice([0.0625, 0.5, 2.0])),
            theta_h=float(rng.choice([1e-4, 0.02])),
            baseline_scope=int(rng.integers(0, 2)),
            kappa_fixed=float(rng.choice([-1.0, -1.0, 0.0, 1.0])),
            degree_target=int(rng.integers(0, 3)),
        )
        if rng.random() < 0.3:
            over.update(ugb_max=int(rng.integers(1, 6)), bf_period=int(rng.integers(1, 10)),
                        restart_stall=int(rng.integers(0, 5)),
                        lambda_bf=float(rng.choice([1.0 + 1e-5, 1e9])))
        inst = wl.random_instance(n, seed=5000 + x, topk=topk, k=k, ants=ants, iterations=iterations,
                                  kind="coords" if kind == "coords" else "matrix",
                                  symmetric=kind != "atsp", local_search=ls, k_ls=k_ls, heat=heat,
                                  grid=grid)
        # the 3-opt on a third of the symmetric cases with local search (a
        # draw of its own, so the other draws stay as they were)
        if ls and kind != "atsp" and np.random.default_rng(7000 + x).random() < 0.35:
            inst.ls_op = 3
        inst.name = f"sweep{x}:{kind} n={n} k={k} ants={ants} it={iterations} ls={ls} op={inst.ls_op}"
        cases.append((inst, over))
    return cases
