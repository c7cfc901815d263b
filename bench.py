#!/usr/bin/env python3
"""Benchmark of the heatmap-guided MMAS decoder on one MI355X.

Default workload (the batched configuration the metric is quoted on): 64
TSP instances with n uniform on [500, 1000], top-10 SoftDist heatmaps,
k = 10, 50 ants, 500 iterations each.  One step = one hac_decode_batch_dev
call over all 64 instances with their inputs already in HBM: candidate
lists, evidence fold, NN tours, 500 iterations of construction + update
for every instance, results.

Reported on one JSON line:
  value             ant-steps/s of the batched path (whole job)
  decodes_per_s     instances decoded per second, batched
  plain             the plain one-instance-per-call path on the same GPU
                    (a sample of the instances, decoded one after another)
  batched_vs_plain  decodes/s ratio; both paths return bit-identical tours,
                    so the mean gap is equal by construction (asserted)
  latency_ms        p50/p99 per-decode latency of both paths
  roofline          construction kernel: algorithmic bytes per launch over
                    its mean launch time (HIP events on the library's
                    stream), against 8 TB/s HBM
  cpu_baseline      the CPU oracle on the host cores, on a bounded sample
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def construct_bytes_per_step(k: int, kind: str) -> int:
    """Algorithmic bytes of one ant step: k candidate ids (int32) + k choice
    weights (FP32) of the current row, the tour entry written (int32), and
    the coordinates of the chosen node (2 x FP64) or one FP64 matrix entry."""
    return 8 * k + 4 + (16 if kind == "coords" else 8)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    pos = (len(xs) - 1) * q
    lo = int(math.floor(pos))
    hi = min(lo + 1, len(xs) - 1)
    return xs[lo] + (pos - lo) * (xs[hi] - xs[lo])


def _oracle_job(args):
    inst, iters = args
    import oracle
    from time import perf_counter
    t = perf_counter()
    st, tour, L, info = oracle.decode(inst, iterations=iters)
    return info["ant_steps"], perf_counter() - t


def cpu_baseline(insts, sample: int, iters: int):
    """The oracle as it stands, one process per instance on the host cores."""
    from concurrent.futures import ProcessPoolExecutor
    import oracle
    oracle.build(force=False)
    jobs = [(insts[x], iters) for x in range(min(sample, len(insts)))]
    cores = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=cores) as ex:
        res = list(ex.map(_oracle_job, jobs))
    wall = time.perf_counter() - t0
    steps = sum(r[0] for r in res)
    cpu = sum(r[1] for r in res)
    return {"value": steps / wall, "unit": "ant-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(jobs)} of the {len(insts)} instances at {iters} iterations each "
                      f"(one process per instance), {cpu:.1f} s of CPU work, {wall:.1f} s wall"}


def traffic_from_profile(kernel_src_hash: str, launches_key: str):
    path = os.path.join(ROOT, "profiles", "construct_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        entry = d.get(launches_key)
        if not entry or entry.get("kernel_source_sha256") != kernel_src_hash:
            return None
        return entry["hbm_bytes_per_launch"]
    except Exception:
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="batch64", choices=["batch64"])
    ap.add_argument("--iterations", type=int, default=500)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--cpu-sample", type=int, default=16)
    ap.add_argument("--cpu-iterations", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the decoder runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2601_19041_amd import workloads as wl

    insts = wl.batch64(64, iterations=args.iterations)
    count = len(insts)
    # the CPU leg runs first, before this process initialises the GPU
    cpu = None if args.no_cpu else cpu_baseline(insts, args.cpu_sample, args.cpu_iterations)

    import torch
    import paper_2601_19041_amd as hac

    ant_steps = sum(x.ants * (x.n - 1) * x.iterations for x in insts)
    ctx = hac.Context(0)
    db = hac.DeviceBatch(insts)

    # warmup (also runs the launch-shape autotuner once)
    for _ in range(args.warmup):
        ctx.decode_batch_dev(db)
    ctx.set_timing(True)
    torch.cuda.synchronize()
    times, cms, launches = [], 0.0, 0
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        ctx.decode_batch_dev(db)
        times.append(time.perf_counter() - t0)
        st = ctx.stats()
        cms += st["construct_ms"]
        launches += st["construct_launches"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_all
    ctx.set_timing(False)
    batched = db.results()
    ms_per_step = 1000.0 * wall / args.steps
    value = ant_steps * args.steps / wall
    decodes_per_s = count * args.steps / wall

    # roofline of the construction kernel: one launch = one iteration of
    # every instance's ants
    bytes_per_launch = sum(x.ants * (x.n - 1) * construct_bytes_per_step(x.k, x.kind) for x in insts)
    avg_launch_s = (cms / 1000.0) / max(launches, 1)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    src = open(os.path.join(ROOT, "paper_2601_19041_amd", "csrc", "hac_kernels.hip"), "rb").read()
    traffic = traffic_from_profile(hashlib.sha256(src).hexdigest(), "batch64")

    # plain path: the same instances, one decode per call
    plain_lat = []
    gap_equal = True
    for x in range(min(args.plain_sample, count)):
        t0 = time.perf_counter()
        tour, L = ctx.decode(insts[x])
        plain_lat.append(time.perf_counter() - t0)
        gap_equal &= bool(np.array_equal(tour, batched[x][0]) and L == batched[x][1])
    assert gap_equal, "plain and batched tours differ"
    plain_dps = len(plain_lat) / sum(plain_lat)
    plain_steps = sum(insts[x].ants * (insts[x].n - 1) * insts[x].iterations for x in range(len(plain_lat)))

    out = {
        "metric": "ant-steps/s, batched decode of 64 TSP instances (n 500-1000)",
        "value": value,
        "unit": "ant-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batch64: 64 TSP instances, n uniform on [500,1000], top-10 SoftDist "
                               "heatmaps, k=10, 50 ants, 500 iterations, no local search",
                   "instances": count, "iterations": args.iterations, "ants": 50, "k": 10,
                   "inputs": "resident in HBM (hac_decode_batch_dev)"},
        "decodes_per_s": decodes_per_s,
        "plain": {"decodes_per_s": plain_dps, "ant_steps_per_s": plain_steps / sum(plain_lat),
                  "sample": len(plain_lat)},
        "batched_vs_plain": decodes_per_s / plain_dps,
        "equal_gap": gap_equal,
        "latency_ms": {"batched_p50": 1000 * percentile(times, 0.5), "batched_p99": 1000 * percentile(times, 0.99),
                       "plain_p50": 1000 * percentile(plain_lat, 0.5), "plain_p99": 1000 * percentile(plain_lat, 0.99)},
        "roofline": {"bound": "hbm", "kernel": "construct_kernel", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "avg_launch_us": avg_launch_s * 1e6, "launches": launches,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
    }
    out["cpu_baseline"] = cpu
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
