"""ctypes binding of the plain CPU oracle (hac_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it to produce expected results.  The product library
never imports it.  The C source is compiled with gcc, FP64, without
contraction or fast-math.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hac_oracle.c")
_SO_BUILT = os.path.join(_HERE, "liboracle.so")
# HAC_ORACLE_LIB loads another build of the same source instead (the
# mutation tests point it at copies with one planted mistake each)
_SO = os.environ.get("HAC_ORACLE_LIB") or _SO_BUILT

GCC_FLAGS = ["-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
             "-Wall", "-Wno-unused-function"]


def build(force: bool = True) -> str:
    """Compile the oracle into oracle/liboracle.so."""
    if force or not os.path.exists(_SO_BUILT):
        tmp = _SO_BUILT + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _SO_BUILT)
    return _SO_BUILT


class Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("kind", ctypes.c_int32), ("symmetric", ctypes.c_int32),
        ("coords", ctypes.c_void_p), ("dist", ctypes.c_void_p),
        ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
        ("ants", ctypes.c_int32), ("iterations", ctypes.c_int32), ("k", ctypes.c_int32),
        ("k_ls", ctypes.c_int32), ("local_search", ctypes.c_int32),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("rho", ctypes.c_double),
        ("p_best", ctypes.c_double), ("c_cap", ctypes.c_double), ("theta_h", ctypes.c_double),
        ("eps", ctypes.c_double), ("xi_bf", ctypes.c_double), ("lambda_bf", ctypes.c_double),
        ("clip", ctypes.c_double),
        ("degree_target", ctypes.c_int32), ("bf_period", ctypes.c_int32),
        ("restart_stall", ctypes.c_int32), ("ugb_max", ctypes.c_int32),
        ("baseline_scope", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("kappa_fixed", ctypes.c_double),
        ("ls_op", ctypes.c_int32),
    ]


class Trace(ctypes.Structure):
    _fields_ = [
        ("k_eff", ctypes.c_int32),
        ("q90", ctypes.c_double), ("r_hat", ctypes.c_double), ("kappa", ctypes.c_double),
        ("l_nn", ctypes.c_double), ("l_nn_raw", ctypes.c_double),
        ("ant_steps", ctypes.c_int64), ("fallback_steps", ctypes.c_int64),
        ("restarts", ctypes.c_int32),
        ("l_ib", ctypes.c_void_p), ("l_gb", ctypes.c_void_p), ("elite_rb", ctypes.c_void_p),
        ("cand", ctypes.c_void_p), ("heur", ctypes.c_void_p), ("tau", ctypes.c_void_p),
        ("weight", ctypes.c_void_p), ("ant_tours", ctypes.c_void_p), ("ant_len", ctypes.c_void_p),
        ("nn_tour", ctypes.c_void_p), ("ugb", ctypes.c_void_p), ("restart", ctypes.c_void_p),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _SO == _SO_BUILT and (not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_SO)
        P = ctypes.POINTER(Problem)
        vp = ctypes.c_void_p
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.orc_draw.restype = ctypes.c_uint32
        L.orc_candidates.argtypes = [P, vp]
        L.orc_candidates.restype = ctypes.c_int32
        L.orc_nearest_lists.argtypes = [P, ctypes.c_int32, vp]
        L.orc_nearest_lists.restype = ctypes.c_int32
        L.orc_evidence.argtypes = [P, vp, ctypes.c_int32, vp, vp, vp, vp, vp, vp]
        L.orc_evidence.restype = ctypes.c_double
        L.orc_select.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_uint32]
        L.orc_select.restype = ctypes.c_int32
        L.orc_nn_tour.argtypes = [P, vp]
        L.orc_nn_tour.restype = ctypes.c_double
        L.orc_tour_length.argtypes = [P, vp]
        L.orc_tour_length.restype = ctypes.c_double
        L.orc_two_opt.argtypes = [P, vp, ctypes.c_int32, ctypes.c_double, vp]
        L.orc_three_opt.argtypes = [P, vp, ctypes.c_int32, ctypes.c_double, vp]
        L.orc_nearest_in_lists.argtypes = [P, ctypes.c_int32, vp]
        L.orc_nearest_in_lists.restype = ctypes.c_int32
        L.orc_two_opt_directed.argtypes = [P, vp, vp, ctypes.c_int32, ctypes.c_double, vp]
        L.orc_directed_move.argtypes = [P, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp]
        L.orc_directed_move.restype = ctypes.c_double
        L.orc_decode.argtypes = [P, vp, vp, ctypes.POINTER(Trace)]
        L.orc_decode.restype = ctypes.c_int32
        L.orc_diagnostics.argtypes = [P, vp, vp, vp]
        L.orc_diagnostics.restype = ctypes.c_int32
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


DEFAULTS = dict(alpha=1.0, beta=2.0, rho=0.2, p_best=0.05, c_cap=0.5, theta_h=1e-4, eps=1e-9,
                xi_bf=0.05, lambda_bf=1.0 + 1e-5, clip=40.0, degree_target=0, bf_period=100,
                restart_stall=250, ugb_max=25, baseline_scope=0, kappa_fixed=-1.0)


class OracleProblem:
    """Holds numpy buffers alive and the ctypes struct that points at them."""

    def __init__(self, inst, **over):
        self.inst = inst
        self.n = inst.n
        if inst.kind == "coords":
            self.coords = np.ascontiguousarray(inst.coords, dtype=np.float64)
            self.dist = None
            kind, sym = 0, 1
        else:
            self.coords = None
            self.dist = np.ascontiguousarray(inst.dist, dtype=np.float64)
            kind, sym = 1, int(inst.symmetric)
        self.row_ptr = np.ascontiguousarray(inst.heat.row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(inst.heat.col, dtype=np.int32)
        self.val = np.ascontiguousarray(inst.heat.val, dtype=np.float32)
        prm = dict(DEFAULTS)
        prm.update(ants=inst.ants, iterations=inst.iterations, k=inst.k, k_ls=inst.k_ls,
                   local_search=inst.local_search, rho=inst.rho, seed=inst.seed,
                   ls_op=getattr(inst, "ls_op", 2))
        prm.update(over)
        self.params = prm
        self.s = Problem(n=inst.n, kind=kind, symmetric=sym, coords=_ptr(self.coords),
                         dist=_ptr(self.dist), row_ptr=_ptr(self.row_ptr), col=_ptr(self.col),
                         val=_ptr(self.val), **prm)

    @property
    def ref(self):
        return ctypes.byref(self.s)

    @property
    def k_eff(self) -> int:
        return min(self.params["k"], self.n - 1)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def draw(seed: int, t: int, a: int, s: int) -> int:
    return int(lib().orc_draw(seed, t, a, s))


def candidates(inst, **over) -> np.ndarray:
    p = OracleProblem(inst, **over)
    ke = p.k_eff
    out = np.zeros((p.n, max(ke, 1)), dtype=np.int32)
    lib().orc_candidates(p.ref, _ptr(out))
    return out[:, :ke]


def nearest_lists(inst, kk: int) -> np.ndarray:
    p = OracleProblem(inst)
    kk = min(kk, p.n - 1)
    out = np.zeros((p.n, kk), dtype=np.int32)
    lib().orc_nearest_lists(p.ref, kk, _ptr(out))
    return out


def evidence(inst, cand: np.ndarray, **over) -> dict:
    p = OracleProblem(inst, **over)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    ke = cand.shape[1]
    conf = np.zeros(cand.shape)
    evid = np.zeros(cand.shape)
    base = np.zeros(p.n)
    heur = np.zeros(cand.shape, dtype=np.float32)
    q90 = ctypes.c_double()
    rh = ctypes.c_double()
    kappa = lib().orc_evidence(p.ref, _ptr(cand), ke, _ptr(conf), _ptr(base), _ptr(evid),
                               _ptr(heur), ctypes.byref(q90), ctypes.byref(rh))
    return dict(conf=conf, base=base, evid=evid, heur=heur, kappa=kappa, q90=q90.value,
                r_hat=rh.value)


def select(cand_row, w_row, visited, u: int) -> int:
    c = np.ascontiguousarray(cand_row, dtype=np.int32)
    w = np.ascontiguousarray(w_row, dtype=np.float32)
    v = np.ascontiguousarray(visited, dtype=np.uint8)
    return int(lib().orc_select(len(c), _ptr(c), _ptr(w), _ptr(v), u))


def nn_tour(inst):
    p = OracleProblem(inst)
    t = np.zeros(p.n, dtype=np.int32)
    L = lib().orc_nn_tour(p.ref, _ptr(t))
    return t, L


def tour_length(inst, tour) -> float:
    p = OracleProblem(inst)
    t = np.ascontiguousarray(tour, dtype=np.int32)
    return float(lib().orc_tour_length(p.ref, _ptr(t)))


def two_opt(inst, nl: np.ndarray, tour, min_gain: float) -> np.ndarray:
    p = OracleProblem(inst)
    nl = np.ascontiguousarray(nl, dtype=np.int32)
    t = np.array(tour, dtype=np.int32)
    lib().orc_two_opt(p.ref, _ptr(nl), nl.shape[1], min_gain, _ptr(t))
    return t


def three_opt(inst, nl: np.ndarray, tour, min_gain: float) -> np.ndarray:
    p = OracleProblem(inst)
    nl = np.ascontiguousarray(nl, dtype=np.int32)
    t = np.array(tour, dtype=np.int32)
    lib().orc_three_opt(p.ref, _ptr(nl), nl.shape[1], min_gain, _ptr(t))
    return t


def nearest_in_lists(inst, kk: int) -> np.ndarray:
    p = OracleProblem(inst)
    kk = min(kk, p.n - 1)
    out = np.zeros((p.n, kk), dtype=np.int32)
    lib().orc_nearest_in_lists(p.ref, kk, _ptr(out))
    return out


def two_opt_directed(inst, nl_out: np.ndarray, nl_in: np.ndarray, tour, min_gain: float) -> np.ndarray:
    p = OracleProblem(inst)
    a = np.ascontiguousarray(nl_out, dtype=np.int32)
    b = np.ascontiguousarray(nl_in, dtype=np.int32)
    t = np.array(tour, dtype=np.int32)
    lib().orc_two_opt_directed(p.ref, _ptr(a), _ptr(b), a.shape[1], min_gain, _ptr(t))
    return t


def directed_move(inst, tour, a: int, c: int, direction: int):
    """(gain, tour after the move) of one directed 2-opt move; gain is NaN
    for a degenerate move."""
    p = OracleProblem(inst)
    t = np.ascontiguousarray(tour, dtype=np.int32)
    out = np.zeros_like(t)
    g = lib().orc_directed_move(p.ref, _ptr(t), a, c, direction, _ptr(out))
    return g, out


def decode(inst, trace: bool = False, state: bool = False, **over):
    """Run Alg. 1.  Returns (status, tour, length, info)."""
    p = OracleProblem(inst, **over)
    n = p.n
    tour = np.zeros(n, dtype=np.int32)
    L = ctypes.c_double()
    tr = Trace()
    bufs = {}
    iters = p.params["iterations"]
    ants = p.params["ants"]
    ke = max(p.k_eff, 1)
    if trace:
        bufs["l_ib"] = np.zeros(max(iters, 1))
        bufs["l_gb"] = np.zeros(max(iters, 1))
        bufs["elite_rb"] = np.zeros(max(iters, 1), dtype=np.int32)
        bufs["ugb"] = np.zeros(max(iters, 1), dtype=np.int32)
        bufs["restart"] = np.zeros(max(iters, 1), dtype=np.int32)
    if state:
        bufs["cand"] = np.zeros((n, ke), dtype=np.int32)
        bufs["heur"] = np.zeros((n, ke), dtype=np.float32)
        bufs["tau"] = np.zeros((n, ke), dtype=np.float32)
        bufs["weight"] = np.zeros((n, ke), dtype=np.float32)
        bufs["ant_tours"] = np.zeros((ants, n), dtype=np.int32)
        bufs["ant_len"] = np.zeros(ants)
        bufs["nn_tour"] = np.zeros(n, dtype=np.int32)
    for name, arr in bufs.items():
        setattr(tr, name, arr.ctypes.data)
    st = lib().orc_decode(p.ref, _ptr(tour), ctypes.byref(L), ctypes.byref(tr))
    info = dict(k_eff=tr.k_eff, q90=tr.q90, r_hat=tr.r_hat, kappa=tr.kappa, l_nn=tr.l_nn,
                l_nn_raw=tr.l_nn_raw, ant_steps=tr.ant_steps, fallback_steps=tr.fallback_steps,
                restarts=tr.restarts)
    for name, arr in bufs.items():
        info[name] = arr[:iters] if name in ("l_ib", "l_gb", "elite_rb", "ugb", "restart") else arr
    return st, tour, L.value, info


def diagnostics(inst, tour, **over) -> dict:
    """Heatmap diagnostics against a known tour (Section V): Edges/n,
    coverage, Miss% and P(e>1).  Returns None on invalid input."""
    p = OracleProblem(inst, **over)
    t = np.ascontiguousarray(tour, dtype=np.int32)
    out = np.zeros(4)
    cnt = np.zeros(3, dtype=np.int64)
    st = lib().orc_diagnostics(p.ref, _ptr(t), _ptr(out), _ptr(cnt))
    if st != 0:
        return None
    return dict(edges_per_node=float(out[0]), coverage=float(out[1]), miss_pct=float(out[2]),
                p_evidence=float(out[3]), entries=int(cnt[0]), evidence_slots=int(cnt[1]),
                evidence_on_tour=int(cnt[2]))
