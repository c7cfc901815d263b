"""Seeded synthetic inputs for the heatmap-guided MMAS decoder.

This module only *makes inputs*: Euclidean and asymmetric instances and
SoftDist-style edge-confidence heatmaps in CSR form.  It holds none of the
decoder's arithmetic (no candidate lists, no evidence factor, no pheromone,
no sampling), so the HIP library and the CPU oracle can both be fed from it
without sharing code.

The paper evaluates on uniform Euclidean TSP500/TSP1K/TSP10K suites with
heatmaps from pretrained predictors (Section IV-A); neither the instance
files nor the heatmaps exist here.  These generators stand in for them:

* coordinates are FP64 uniform on [0,1)^2, the distribution of those suites;
* the heatmap is the "SoftDist" construction of Table VII (a softmax over
  negative distances restricted to each node's nearest neighbours, i.e. a
  proximity-only heatmap), plus a planted nearest-neighbour tour, so that
  rows have a few clearly separated entries as learned heatmaps do
  (Table IX reports 2.5-11.4 undirected edges per node above the
  threshold);
* the ATSP recipe perturbs Euclidean distances per ordered pair and keeps
  the directed heatmap unsymmetrised (Section II-B: for the ATSP the
  directed matrix is consumed as is).

All randomness comes from numpy's Philox bit generator keyed by
(workload id, instance id), so every input is reproducible on any host.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

# workload ids used to key the generators
WL_TSP100 = 1
WL_TSP500 = 2
WL_BATCH64 = 3
WL_TSP10K = 4
WL_SERVE = 5
WL_PAPER = 6


def _rng(workload: int, instance: int, stream: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[workload, instance * 16 + stream]))


@dataclasses.dataclass
class Heatmap:
    """Edge confidences h as the decoder consumes them, in CSR form.

    row_ptr int32[n+1], col int32[nnz] (ascending within a row), val float32[nnz].
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def dense(self) -> np.ndarray:
        h = np.zeros((self.n, self.n), dtype=np.float32)
        for i in range(self.n):
            a, b = self.row_ptr[i], self.row_ptr[i + 1]
            h[i, self.col[a:b]] = self.val[a:b]
        return h


@dataclasses.dataclass
class Instance:
    """One decode request: the instance, its heatmap and its MMAS settings."""

    n: int
    kind: str  # "coords" (Euclidean, symmetric) or "matrix"
    symmetric: bool
    coords: Optional[np.ndarray]  # float64 [n,2]
    dist: Optional[np.ndarray]  # float64 [n,n], row-major
    heat: Heatmap
    ants: int
    iterations: int
    k: int
    local_search: int = 0
    k_ls: int = 20
    rho: float = 0.2
    seed: int = 1
    name: str = ""
    ls_op: int = 2  # local-search operator: 2 the 2-opt, 3 the 3-opt (symmetric instances)


def uniform_coords(n: int, rng: np.random.Generator) -> np.ndarray:
    return rng.random((n, 2), dtype=np.float64)


def _pairwise(coords: np.ndarray, rows: np.ndarray) -> np.ndarray:
    # sqrt(dx*dx + dy*dy), the same FP64 operations as a sum over the axis
    dx = coords[rows, 0][:, None] - coords[None, :, 0]
    dy = coords[rows, 1][:, None] - coords[None, :, 1]
    return np.sqrt(dx * dx + dy * dy)


def _topk_rows(dist_rows: np.ndarray, rows: np.ndarray, topk: int) -> np.ndarray:
    """Indices of the `topk` nearest other nodes per row, ordered by
    (distance, index).  A partial selection finds them; rows where the
    selection boundary is tied fall back to a full stable sort, so the
    result is always that of the stable sort."""
    d = dist_rows.copy()
    d[np.arange(len(rows)), rows] = np.inf
    n = d.shape[1]
    if topk + 1 >= n:
        return np.argsort(d, axis=1, kind="stable")[:, :topk]
    part = np.argpartition(d, topk, axis=1)[:, : topk + 1]
    pv = np.take_along_axis(d, part, axis=1)
    order = np.lexsort((part, pv), axis=1)
    part = np.take_along_axis(part, order, axis=1)
    pv = np.take_along_axis(pv, order, axis=1)
    idx = part[:, :topk].copy()
    # the k-th and (k+1)-th smallest equal: other nodes may share that
    # distance, and the lowest indices among them must win
    tied = pv[:, topk - 1] == pv[:, topk]
    if tied.any():
        t = np.flatnonzero(tied)
        idx[t] = np.argsort(d[t], axis=1, kind="stable")[:, :topk]
    return idx


def _nn_tour_from_dist_fn(n: int, row_fn, near: Optional[np.ndarray] = None) -> np.ndarray:
    """Greedy nearest-neighbour tour from node 0 (only used to plant edges).
    `near[i]`, if given, lists i's nearest nodes in (distance, index) order:
    its first unvisited entry is the nearest unvisited node, and only when
    the list is exhausted is the whole row scanned."""
    visited = np.zeros(n, dtype=bool)
    tour = np.empty(n, dtype=np.int64)
    cur = 0
    for s in range(n):
        tour[s] = cur
        visited[cur] = True
        if s == n - 1:
            break
        if near is not None:
            free = near[cur][~visited[near[cur]]]
            if free.size:
                cur = int(free[0])
                continue
        row = row_fn(cur).copy()
        row[visited] = np.inf
        cur = int(np.argmin(row))
    return tour


def _to_csr(n: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray) -> Heatmap:
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Heatmap(n, row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float32))


def softdist_heatmap(
    coords: np.ndarray,
    topk: int,
    rng: Optional[np.random.Generator] = None,
    temp: float = 0.05,
    plant: float = 0.5,
    noise_sigma: float = 0.0,
    row_sum: float = 2.0,
    chunk: int = 512,
) -> Heatmap:
    """Symmetric-TSP heatmap: softmax(-d/temp) over each node's `topk` nearest,
    +`plant` on both directions of a nearest-neighbour tour, optional
    N(0, sigma^2) noise clipped at 0, symmetrised by max, rows rescaled to
    `row_sum`, stored as FP32 CSR."""
    n = coords.shape[0]
    topk = min(topk, n - 1)
    if topk < 1:
        return empty_heatmap(n)
    rows_l, cols_l, vals_l = [], [], []
    kn = min(n - 1, max(topk, 32))  # nearest lists for the planted NN tour
    near = np.empty((n, kn), dtype=np.int64)
    for a in range(0, n, chunk):
        rows = np.arange(a, min(n, a + chunk))
        dr = _pairwise(coords, rows)
        idxk = _topk_rows(dr, rows, kn)
        near[rows] = idxk
        idx = idxk[:, :topk]
        dsel = np.take_along_axis(dr, idx, axis=1)
        z = -dsel / temp
        z -= z.max(axis=1, keepdims=True)
        w = np.exp(z)
        w /= w.sum(axis=1, keepdims=True)
        rows_l.append(np.repeat(rows, topk))
        cols_l.append(idx.reshape(-1))
        vals_l.append(w.reshape(-1))
    r = np.concatenate(rows_l)
    c = np.concatenate(cols_l)
    v = np.concatenate(vals_l)
    # plant a nearest-neighbour tour in both directions
    tour = _nn_tour_from_dist_fn(n, lambda i: _pairwise(coords, np.array([i]))[0], near)
    nxt = np.roll(tour, -1)
    r = np.concatenate([r, tour, nxt])
    c = np.concatenate([c, nxt, tour])
    v = np.concatenate([v, np.full(n, plant), np.full(n, plant)])
    # accumulate duplicates (a planted edge may already be a top-k entry)
    key = r.astype(np.int64) * n + c
    uk, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(len(uk))
    np.add.at(acc, inv, v)
    r, c, v = uk // n, uk % n, acc
    if noise_sigma > 0:
        assert rng is not None
        v = np.maximum(v + rng.normal(0.0, noise_sigma, size=v.shape), 0.0)
    # symmetrise by max on the union pattern
    allk = np.concatenate([r * n + c, c * n + r])
    allv = np.concatenate([v, v])
    uk, inv = np.unique(allk, return_inverse=True)
    mx = np.zeros(len(uk))
    np.maximum.at(mx, inv, allv)
    r, c, v = uk // n, uk % n, mx
    keep = r != c
    r, c, v = r[keep], c[keep], v[keep]
    rs = np.bincount(r, weights=v, minlength=n)
    scale = np.where(rs > 0, row_sum / np.where(rs > 0, rs, 1.0), 0.0)
    v = v * scale[r]
    return _to_csr(n, r, c, v)


def atsp_instance(n: int, rng: np.random.Generator) -> np.ndarray:
    """d_ij = ||x_i - x_j||_2 + U[0, 0.5) per ordered pair, d_ii = 0."""
    xy = uniform_coords(n, rng)
    d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
    d = d + rng.random((n, n)) * 0.5
    np.fill_diagonal(d, 0.0)
    return np.ascontiguousarray(d)


def atsp_heatmap(dist: np.ndarray, topk: int = 20, temp: float = 0.05, plant: float = 0.5,
                 row_sum: float = 1.0) -> Heatmap:
    """Directed heatmap: softmax over each row's `topk` nearest outgoing
    entries, +`plant` on the directed nearest-neighbour tour, not symmetrised,
    rows rescaled to `row_sum`."""
    n = dist.shape[0]
    topk = min(topk, n - 1)
    if topk < 1:
        return empty_heatmap(n)
    rows = np.arange(n)
    idx = _topk_rows(dist, rows, topk)
    dsel = np.take_along_axis(dist, idx, axis=1)
    z = -dsel / temp
    z -= z.max(axis=1, keepdims=True)
    w = np.exp(z)
    w /= w.sum(axis=1, keepdims=True)
    r = np.repeat(rows, topk)
    c = idx.reshape(-1)
    v = w.reshape(-1)
    tour = _nn_tour_from_dist_fn(n, lambda i: dist[i])
    nxt = np.roll(tour, -1)
    r = np.concatenate([r, tour])
    c = np.concatenate([c, nxt])
    v = np.concatenate([v, np.full(n, plant)])
    key = r.astype(np.int64) * n + c
    uk, inv = np.unique(key, return_inverse=True)
    acc = np.zeros(len(uk))
    np.add.at(acc, inv, v)
    r, c, v = uk // n, uk % n, acc
    rs = np.bincount(r, weights=v, minlength=n)
    v = v * (row_sum / rs)[r]
    return _to_csr(n, r, c, v)


def empty_heatmap(n: int) -> Heatmap:
    return Heatmap(n, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32),
                   np.zeros(0, dtype=np.float32))


# ---------------------------------------------------------------------------
# The five workloads.  Sizes follow the decode settings stated with each one.
# ---------------------------------------------------------------------------

def tsp100(instance: int = 0, seed: Optional[int] = None, iterations: int = 100) -> Instance:
    """n=100, top-10 heatmap, k=10, 20 ants, 100 iterations, no local search."""
    rng = _rng(WL_TSP100, instance)
    xy = uniform_coords(100, rng)
    heat = softdist_heatmap(xy, 10)
    return Instance(100, "coords", True, xy, None, heat, ants=20, iterations=iterations, k=10,
                    seed=seed if seed is not None else 1 + instance, name=f"tsp100#{instance}")


def tsp500(instance: int = 0, seed: Optional[int] = None, iterations: int = 1000) -> Instance:
    """n=500, top-20 heatmap with N(0,0.05^2) noise, k=20, 50 ants, 1000 iterations."""
    rng = _rng(WL_TSP500, instance)
    xy = uniform_coords(500, rng)
    heat = softdist_heatmap(xy, 20, rng=_rng(WL_TSP500, instance, 1), noise_sigma=0.05)
    return Instance(500, "coords", True, xy, None, heat, ants=50, iterations=iterations, k=20,
                    seed=seed if seed is not None else 1 + instance, name=f"tsp500#{instance}")


def batch64_instance(x: int, iterations: int = 500) -> Instance:
    """Instance x of the 64-instance batch (see batch64)."""
    rng = _rng(WL_BATCH64, x)
    n = 500 + int(rng.integers(0, 501))
    xy = uniform_coords(n, rng)
    heat = softdist_heatmap(xy, 10)
    return Instance(n, "coords", True, xy, None, heat, ants=50, iterations=iterations,
                    k=10, seed=1 + x, name=f"batch64#{x}")


def batch64(count: int = 64, iterations: int = 500) -> List[Instance]:
    """64 instances, n uniform on [500, 1000], top-10 heatmap, k=10, 50 ants, 500 iterations."""
    return [batch64_instance(x, iterations) for x in range(count)]


def tsp10k_instance(x: int, iterations: int = 200, n: int = 10000) -> Instance:
    """Instance x of the 10 000-node batch (see tsp10k)."""
    rng = _rng(WL_TSP10K, x)
    xy = uniform_coords(n, rng)
    heat = softdist_heatmap(xy, 20)
    return Instance(n, "coords", True, xy, None, heat, ants=100, iterations=iterations,
                    k=20, local_search=1, k_ls=20, seed=1 + x, name=f"tsp10k#{x}")


def tsp10k(count: int = 8, iterations: int = 200, n: int = 10000) -> List[Instance]:
    """8 instances of n=10000, top-20 heatmap, k=20, 100 ants, 200 iterations,
    neighbour-list 2-opt (20 neighbours) on each iteration-best tour."""
    return [tsp10k_instance(x, iterations, n) for x in range(count)]


def paper_budget(n: int, count: int = 1, local_search: int = 0, iterations: int = 5000,
                 first: int = 0) -> List[Instance]:
    """The paper's own decode setting (Section IV-C) on synthetic uniform
    instances standing in for its TSP500/1K/10K test sets: 32 ants, 5000
    iterations, k = 20, rho = 0.8 for the symmetric TSP, and with local
    search the 2-opt on every ant's tour (local_search = 2, 20 neighbours).
    The heatmap is the top-20 generator without noise."""
    out = []
    for x in range(first, first + count):
        rng = _rng(WL_PAPER, n * 1000 + x)
        xy = uniform_coords(n, rng)
        heat = softdist_heatmap(xy, 20)
        out.append(Instance(n, "coords", True, xy, None, heat, ants=32, iterations=iterations, k=20,
                            local_search=local_search, k_ls=20, rho=0.8, seed=1 + x,
                            name=f"paper{n}#{x}"))
    return out


def serve_request(kind: str, r: int, iterations: int = 100) -> Instance:
    """One request of the serving mix: 'tsp500', 'tsp1000', 'tsp10000' or 'atsp1000'."""
    rng = _rng(WL_SERVE, r)
    if kind in ("tsp500", "tsp1000"):
        n = 500 if kind == "tsp500" else 1000
        xy = uniform_coords(n, rng)
        heat = softdist_heatmap(xy, 20, rng=_rng(WL_SERVE, r, 1), noise_sigma=0.05)
        return Instance(n, "coords", True, xy, None, heat, ants=50, iterations=iterations, k=20,
                        seed=1 + r, name=f"{kind}#{r}")
    if kind == "tsp10000":
        xy = uniform_coords(10000, rng)
        heat = softdist_heatmap(xy, 20)
        return Instance(10000, "coords", True, xy, None, heat, ants=100, iterations=iterations,
                        k=20, seed=1 + r, name=f"{kind}#{r}")
    if kind == "atsp1000":
        d = atsp_instance(1000, rng)
        heat = atsp_heatmap(d, 20)
        return Instance(1000, "matrix", False, None, d, heat, ants=50, iterations=iterations,
                        k=20, seed=1 + r, name=f"{kind}#{r}")
    raise ValueError(kind)


def serve_mix(count: int, rate_hz: float, seed: int = 0):
    """Request kinds in a 40/40/10/10 mix and Poisson arrival times (seconds)."""
    rng = _rng(WL_SERVE, 1 << 20, seed)
    kinds = rng.choice(["tsp500", "tsp1000", "tsp10000", "atsp1000"], size=count,
                       p=[0.4, 0.4, 0.1, 0.1])
    gaps = rng.exponential(1.0 / rate_hz, size=count)
    return list(kinds), np.cumsum(gaps)


def random_instance(n: int, seed: int, topk: int = 10, k: int = 10, ants: int = 8,
                    iterations: int = 20, kind: str = "coords", symmetric: bool = True,
                    local_search: int = 0, k_ls: int = 20, heat: str = "softdist",
                    grid: Optional[int] = None) -> Instance:
    """Small instances for tests.  `grid` snaps coordinates to a grid so that
    equal distances (ties) occur; heat='empty' gives a heatmap with no entries."""
    rng = _rng(99, seed)
    if kind == "coords":
        xy = uniform_coords(n, rng)
        if grid:
            # distinct points of a grid x grid lattice: many equal distances
            assert n <= grid * grid
            cells = rng.permutation(grid * grid)[:n]
            xy = np.stack([cells % grid, cells // grid], 1).astype(np.float64) / grid
        hm = softdist_heatmap(xy, topk) if heat == "softdist" else empty_heatmap(n)
        return Instance(n, "coords", True, xy, None, hm, ants=ants, iterations=iterations, k=k,
                        local_search=local_search, k_ls=k_ls, seed=seed, name=f"rand{n}#{seed}")
    if symmetric:
        xy = uniform_coords(n, rng)
        d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1))
        d = np.ascontiguousarray(np.minimum(d, d.T))
        hm = softdist_heatmap(xy, topk) if heat == "softdist" else empty_heatmap(n)
    else:
        d = atsp_instance(n, rng)
        hm = atsp_heatmap(d, topk) if heat == "softdist" else empty_heatmap(n)
    return Instance(n, "matrix", symmetric, None, d, hm, ants=ants, iterations=iterations, k=k,
                    local_search=local_search, k_ls=k_ls, seed=seed, name=f"mat{n}#{seed}")
