"""Python binding of libhac, the MI355X heatmap-guided MMAS decoder.

Argument marshalling only: every step of a decode runs in the HIP library
(include/hac.h).  PyTorch is used, where it is used at all, for device
memory and streams.  Importing the binding does not need a GPU; creating a
Context does.  There is no CPU fallback: without the built library every
entry point raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhac.so")

HAC_OK = 0
HAC_EINVAL = -1
HAC_ENOMEM = -2
HAC_EDEVICE = -3
HAC_EUNSUPPORTED = -4
HAC_EBUSY = -5
HAC_ECANCELLED = -6
HAC_ERANGE = -7
HAC_COORDS_EUC2D = 0
HAC_MATRIX = 1


class HacError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class hac_instance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("kind", ctypes.c_int32), ("symmetric", ctypes.c_int32),
                ("coords", ctypes.c_void_p), ("dist", ctypes.c_void_p)]


class hac_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class hac_params(ctypes.Structure):
    _fields_ = [
        ("ants", ctypes.c_int32), ("iterations", ctypes.c_int32), ("k", ctypes.c_int32),
        ("k_ls", ctypes.c_int32), ("local_search", ctypes.c_int32),
        ("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("rho", ctypes.c_double),
        ("p_best", ctypes.c_double), ("c_cap", ctypes.c_double), ("theta_h", ctypes.c_double),
        ("eps", ctypes.c_double), ("xi_bf", ctypes.c_double), ("lambda_bf", ctypes.c_double),
        ("clip", ctypes.c_double),
        ("degree_target", ctypes.c_int32), ("bf_period", ctypes.c_int32),
        ("restart_stall", ctypes.c_int32), ("ugb_max", ctypes.c_int32),
        ("baseline_scope", ctypes.c_int32),
        ("kappa_fixed", ctypes.c_double),
        ("ls_op", ctypes.c_int32),
    ]


class hac_diagnostics(ctypes.Structure):
    _fields_ = [("edges_per_node", ctypes.c_double), ("coverage", ctypes.c_double),
                ("miss_pct", ctypes.c_double), ("p_evidence", ctypes.c_double),
                ("heatmap_edges", ctypes.c_int64), ("evidence_slots", ctypes.c_int64),
                ("evidence_on_tour", ctypes.c_int64)]


class hac_lane_stats(ctypes.Structure):
    _fields_ = [("min_n", ctypes.c_int32), ("max_n", ctypes.c_int32), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("rounds", ctypes.c_int64), ("iterations", ctypes.c_int64),
                ("instance_iterations", ctypes.c_int64), ("peak_active", ctypes.c_int32),
                ("prep_ms", ctypes.c_double), ("round_ms", ctypes.c_double), ("idle_ms", ctypes.c_double)]


SERVER_LANES = 3


class hac_stats(ctypes.Structure):
    _fields_ = [("total_ms", ctypes.c_double), ("prep_ms", ctypes.c_double),
                ("search_ms", ctypes.c_double), ("construct_ms", ctypes.c_double),
                ("construct_launches", ctypes.c_int64), ("ant_steps", ctypes.c_int64),
                ("fallback_steps", ctypes.c_int64), ("restarts", ctypes.c_int32),
                ("instances", ctypes.c_int32), ("kappa", ctypes.c_double), ("q90", ctypes.c_double),
                ("r_hat", ctypes.c_double), ("l_nn", ctypes.c_double),
                ("ants_per_block", ctypes.c_int32), ("lds_staged", ctypes.c_int32),
                ("ants_per_wave", ctypes.c_int32),
                ("byte_marks", ctypes.c_int32),
                ("local_search_ms", ctypes.c_double), ("local_search_launches", ctypes.c_int64),
                ("update_ms", ctypes.c_double), ("update_launches", ctypes.c_int64),
                ("geo_mode", ctypes.c_int32)]


# every symbol include/hac.h declares
EXPORTS = ["hac_params_default", "hac_strerror", "hac_validate", "hac_create", "hac_destroy",
           "hac_last_error", "hac_set_timing", "hac_decode", "hac_decode_noalloc", "hac_decode_dev", "hac_decode_batch",
           "hac_decode_batch_dev",
           "hac_last_stats", "hac_debug_state", "hac_debug_trace", "hac_footprint",
           "hac_server_create", "hac_server_submit", "hac_server_poll", "hac_server_wait",
           "hac_server_cancel", "hac_server_counters", "hac_server_lane_stats", "hac_server_destroy",
           "hac_heatmap_diagnostics"]

_lib = None


def lib():
    """The loaded libhac.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "(there is no fallback implementation)")
        # One HIP runtime per process: torch ships its own libamdhip64 with
        # the same soname, so load it first and libhac binds to that copy
        # (otherwise torch would later load a second runtime that cannot
        # see the GPU).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, u64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
        PI, PC, PP = ctypes.POINTER(hac_instance), ctypes.POINTER(hac_csr), ctypes.POINTER(hac_params)
        L.hac_params_default.argtypes = [PP]
        L.hac_strerror.argtypes = [i32]
        L.hac_strerror.restype = ctypes.c_char_p
        L.hac_validate.argtypes = [PI, PC, PP]
        L.hac_validate.restype = i32
        L.hac_create.argtypes = [ctypes.POINTER(vp), i32, vp, u64]
        L.hac_create.restype = i32
        L.hac_destroy.argtypes = [vp]
        L.hac_last_error.argtypes = [vp]
        L.hac_last_error.restype = ctypes.c_char_p
        L.hac_set_timing.argtypes = [vp, i32]
        L.hac_set_timing.restype = i32
        L.hac_decode.argtypes = [vp, PI, PC, PP, u64, vp, vp]
        L.hac_decode.restype = i32
        L.hac_decode_noalloc.argtypes = [vp, PI, PC, PP, u64, vp, vp]
        L.hac_decode_noalloc.restype = i32
        L.hac_decode_dev.argtypes = [vp, PI, PC, PP, u64, vp, vp]
        L.hac_decode_dev.restype = i32
        L.hac_decode_batch.argtypes = [vp, i32, PI, PC, PP, vp, vp, vp]
        L.hac_decode_batch.restype = i32
        L.hac_decode_batch_dev.argtypes = [vp, i32, PI, PC, PP, vp, vp, vp]
        L.hac_decode_batch_dev.restype = i32
        L.hac_last_stats.argtypes = [vp, ctypes.POINTER(hac_stats)]
        L.hac_last_stats.restype = i32
        L.hac_debug_state.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.hac_debug_state.restype = i32
        L.hac_debug_trace.argtypes = [vp, i32, vp, vp, vp]
        L.hac_debug_trace.restype = i32
        L.hac_heatmap_diagnostics.argtypes = [vp, PI, PC, PP, vp, ctypes.POINTER(hac_diagnostics)]
        L.hac_heatmap_diagnostics.restype = i32
        if hasattr(L, "hac_footprint"):
            L.hac_footprint.argtypes = [PI, PC, PP]
            L.hac_footprint.restype = u64
            L.hac_server_create.argtypes = [vp, u64, i32, ctypes.POINTER(vp)]
            L.hac_server_create.restype = i32
            L.hac_server_submit.argtypes = [vp, PI, PC, PP, u64, ctypes.POINTER(u64)]
            L.hac_server_submit.restype = i32
            for name in ("hac_server_poll", "hac_server_wait"):
                getattr(L, name).argtypes = [vp, u64, vp, vp, vp]
                getattr(L, name).restype = i32
            L.hac_server_cancel.argtypes = [vp, u64]
            L.hac_server_cancel.restype = i32
            L.hac_server_counters.argtypes = [vp, vp, vp, vp, vp]
            L.hac_server_counters.restype = i32
            L.hac_server_lane_stats.argtypes = [vp, i32, ctypes.POINTER(hac_lane_stats)]
            L.hac_server_lane_stats.restype = i32
            L.hac_server_destroy.argtypes = [vp]
        _lib = L
    return _lib


def strerror(status: int) -> str:
    return lib().hac_strerror(status).decode()


def params_default(**over) -> hac_params:
    p = hac_params()
    lib().hac_params_default(ctypes.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


class Marshalled:
    """ctypes views of one instance's host arrays (kept alive here)."""

    def __init__(self, inst, **param_over):
        self.inst = inst
        n = inst.n
        if inst.kind == "coords":
            self.coords = np.ascontiguousarray(inst.coords, dtype=np.float64)
            self.dist = None
            self.s_inst = hac_instance(n, HAC_COORDS_EUC2D, 1, self.coords.ctypes.data, None)
        else:
            self.coords = None
            self.dist = np.ascontiguousarray(inst.dist, dtype=np.float64)
            self.s_inst = hac_instance(n, HAC_MATRIX, int(inst.symmetric), None, self.dist.ctypes.data)
        self.row_ptr = np.ascontiguousarray(inst.heat.row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(inst.heat.col, dtype=np.int32)
        self.val = np.ascontiguousarray(inst.heat.val, dtype=np.float32)
        self.s_csr = hac_csr(n, int(self.row_ptr[-1]), self.row_ptr.ctypes.data,
                             self.col.ctypes.data if len(self.col) else None,
                             self.val.ctypes.data if len(self.val) else None)
        over = dict(ants=inst.ants, iterations=inst.iterations, k=inst.k, k_ls=inst.k_ls,
                    local_search=inst.local_search, rho=inst.rho, ls_op=getattr(inst, "ls_op", 2))
        over.update(param_over)
        self.s_params = params_default(**over)
        self.seed = int(param_over.get("seed", inst.seed))


def validate(inst, **over) -> int:
    m = Marshalled(inst, **over)
    return int(lib().hac_validate(ctypes.byref(m.s_inst), ctypes.byref(m.s_csr), ctypes.byref(m.s_params)))


def footprint(inst, **over) -> int:
    m = Marshalled(inst, **over)
    return int(lib().hac_footprint(ctypes.byref(m.s_inst), ctypes.byref(m.s_csr), ctypes.byref(m.s_params)))


class Context:
    """A decoder context on one GPU (hac_create / hac_destroy)."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, budget: int = 0):
        self._h = ctypes.c_void_p()
        st = lib().hac_create(ctypes.byref(self._h), device, stream, budget)
        if st != HAC_OK:
            raise HacError(st, f"hac_create: {strerror(st)}")

    def close(self):
        if self._h:
            lib().hac_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def last_error(self) -> str:
        return lib().hac_last_error(self._h).decode()

    def _check(self, st: int, what: str):
        if st != HAC_OK:
            raise HacError(st, f"{what}: {strerror(st)}: {self.last_error()}")

    def set_timing(self, on: bool):
        self._check(lib().hac_set_timing(self._h, int(on)), "hac_set_timing")

    def decode(self, inst, raise_on_error: bool = True, **over) -> Tuple[np.ndarray, float]:
        """Plain path: one instance.  Returns (tour int32[n], length)."""
        m = Marshalled(inst, **over)
        tour = np.zeros(inst.n, dtype=np.int32)
        L = ctypes.c_double()
        st = lib().hac_decode(self._h, ctypes.byref(m.s_inst), ctypes.byref(m.s_csr),
                              ctypes.byref(m.s_params), m.seed, tour.ctypes.data, ctypes.byref(L))
        if raise_on_error:
            self._check(st, "hac_decode")
        else:
            self.status = st
        return tour, L.value

    def decode_noalloc(self, inst, raise_on_error: bool = True, **over) -> Tuple[np.ndarray, float]:
        """The allocation-free variant of decode (hac_decode_noalloc)."""
        m = Marshalled(inst, **over)
        tour = np.zeros(inst.n, dtype=np.int32)
        L = ctypes.c_double()
        st = lib().hac_decode_noalloc(self._h, ctypes.byref(m.s_inst), ctypes.byref(m.s_csr),
                                      ctypes.byref(m.s_params), m.seed, tour.ctypes.data, ctypes.byref(L))
        if raise_on_error:
            self._check(st, "hac_decode_noalloc")
        else:
            self.status = st
        return tour, L.value

    def decode_status(self, inst, **over) -> int:
        self.decode(inst, raise_on_error=False, **over)
        return self.status

    def decode_batch(self, insts: Sequence, over: Optional[Sequence[dict]] = None
                     ) -> List[Tuple[np.ndarray, float]]:
        """Batched path: all instances share launches.  Returns [(tour, length)]."""
        count = len(insts)
        ms = [Marshalled(x, **((over[i] if over else {}) or {})) for i, x in enumerate(insts)]
        A_inst = (hac_instance * count)(*[m.s_inst for m in ms])
        A_csr = (hac_csr * count)(*[m.s_csr for m in ms])
        A_par = (hac_params * count)(*[m.s_params for m in ms])
        seeds = np.array([m.seed for m in ms], dtype=np.uint64)
        tours = [np.zeros(x.n, dtype=np.int32) for x in insts]
        ptrs = (ctypes.c_void_p * count)(*[t.ctypes.data for t in tours])
        lens = np.zeros(count)
        st = lib().hac_decode_batch(self._h, count, A_inst, A_csr, A_par, seeds.ctypes.data, ptrs,
                                    lens.ctypes.data)
        self._check(st, "hac_decode_batch")
        return [(tours[i], float(lens[i])) for i in range(count)]

    def decode_batch_dev(self, dev_batch: "DeviceBatch"):
        """Batched path on device-resident inputs (see DeviceBatch).  Results
        land in dev_batch.tours / dev_batch.lengths (torch tensors)."""
        b = dev_batch
        st = lib().hac_decode_batch_dev(self._h, b.count, b.s_inst, b.s_csr, b.s_par,
                                        b.seeds.ctypes.data, b.out_ptrs, b.lengths.data_ptr())
        self._check(st, "hac_decode_batch_dev")

    def decode_dev(self, inst, **over):
        """Device-memory variant: inputs and outputs as torch tensors on the GPU."""
        import torch
        dev = torch.device("cuda")
        m = Marshalled(inst, **over)
        keep = []
        if inst.kind == "coords":
            xy = torch.from_numpy(m.coords).to(dev)
            keep.append(xy)
            s_inst = hac_instance(inst.n, HAC_COORDS_EUC2D, 1, xy.data_ptr(), None)
        else:
            dm = torch.from_numpy(m.dist).to(dev)
            keep.append(dm)
            s_inst = hac_instance(inst.n, HAC_MATRIX, int(inst.symmetric), None, dm.data_ptr())
        rp = torch.from_numpy(m.row_ptr).to(dev)
        col = torch.from_numpy(m.col.copy() if len(m.col) else np.zeros(1, np.int32)).to(dev)
        val = torch.from_numpy(m.val.copy() if len(m.val) else np.zeros(1, np.float32)).to(dev)
        keep += [rp, col, val]
        s_csr = hac_csr(inst.n, int(m.row_ptr[-1]), rp.data_ptr(), col.data_ptr(), val.data_ptr())
        tour = torch.zeros(inst.n, dtype=torch.int32, device=dev)
        length = torch.zeros(1, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        st = lib().hac_decode_dev(self._h, ctypes.byref(s_inst), ctypes.byref(s_csr),
                                  ctypes.byref(m.s_params), m.seed, tour.data_ptr(), length.data_ptr())
        self._check(st, "hac_decode_dev")
        return tour, length

    def stats(self) -> dict:
        s = hac_stats()
        self._check(lib().hac_last_stats(self._h, ctypes.byref(s)), "hac_last_stats")
        return {name: getattr(s, name) for name, _ in hac_stats._fields_}

    def debug_state(self, which: int, n: int, k: int, ants: int) -> dict:
        k = min(k, n - 1)
        out = dict(cand=np.zeros((n, k), np.int32), heur=np.zeros((n, k), np.float32),
                   tau=np.zeros((n, k), np.float32), weight=np.zeros((n, k), np.float32),
                   ant_tours=np.zeros((ants, n), np.int32), ant_len=np.zeros(ants),
                   nn_tour=np.zeros(n, np.int32))
        st = lib().hac_debug_state(self._h, which, *[out[x].ctypes.data for x in
                                                     ("cand", "heur", "tau", "weight", "ant_tours",
                                                      "ant_len", "nn_tour")])
        self._check(st, "hac_debug_state")
        return out

    def diagnostics(self, inst, known_tour, **over) -> dict:
        """Heatmap diagnostics against a known tour (hac_heatmap_diagnostics)."""
        m = Marshalled(inst, **over)
        t = np.ascontiguousarray(known_tour, dtype=np.int32)
        d = hac_diagnostics()
        st = lib().hac_heatmap_diagnostics(self._h, ctypes.byref(m.s_inst), ctypes.byref(m.s_csr),
                                           ctypes.byref(m.s_params), t.ctypes.data, ctypes.byref(d))
        self._check(st, "hac_heatmap_diagnostics")
        return dict(edges_per_node=d.edges_per_node, coverage=d.coverage, miss_pct=d.miss_pct,
                    p_evidence=d.p_evidence, entries=d.heatmap_edges, evidence_slots=d.evidence_slots,
                    evidence_on_tour=d.evidence_on_tour)

    def debug_trace(self, which: int, iterations: int) -> dict:
        out = dict(l_ib=np.zeros(iterations), l_gb=np.zeros(iterations),
                   elite_rb=np.zeros(iterations, np.int32))
        st = lib().hac_debug_trace(self._h, which, out["l_ib"].ctypes.data, out["l_gb"].ctypes.data,
                                   out["elite_rb"].ctypes.data)
        self._check(st, "hac_debug_trace")
        return out


class DeviceBatch:
    """Instances uploaded once into torch device tensors, for repeated
    hac_decode_batch_dev calls (inputs resident in HBM)."""

    def __init__(self, insts: Sequence, over: Optional[Sequence[dict]] = None):
        import torch
        dev = torch.device("cuda")
        self.count = count = len(insts)
        self.keep = []
        ms = [Marshalled(x, **((over[i] if over else {}) or {})) for i, x in enumerate(insts)]
        s_inst, s_csr = [], []
        for m, inst in zip(ms, insts):
            if inst.kind == "coords":
                xy = torch.from_numpy(m.coords).to(dev)
                self.keep.append(xy)
                s_inst.append(hac_instance(inst.n, HAC_COORDS_EUC2D, 1, xy.data_ptr(), None))
            else:
                dm = torch.from_numpy(m.dist).to(dev)
                self.keep.append(dm)
                s_inst.append(hac_instance(inst.n, HAC_MATRIX, int(inst.symmetric), None, dm.data_ptr()))
            rp = torch.from_numpy(m.row_ptr).to(dev)
            col = torch.from_numpy(m.col.copy() if len(m.col) else np.zeros(1, np.int32)).to(dev)
            val = torch.from_numpy(m.val.copy() if len(m.val) else np.zeros(1, np.float32)).to(dev)
            self.keep += [rp, col, val]
            s_csr.append(hac_csr(inst.n, int(m.row_ptr[-1]), rp.data_ptr(), col.data_ptr(), val.data_ptr()))
        self.s_inst = (hac_instance * count)(*s_inst)
        self.s_csr = (hac_csr * count)(*s_csr)
        self.s_par = (hac_params * count)(*[m.s_params for m in ms])
        self.seeds = np.array([m.seed for m in ms], dtype=np.uint64)
        self.tours = [torch.zeros(x.n, dtype=torch.int32, device=dev) for x in insts]
        self.lengths = torch.zeros(count, dtype=torch.float64, device=dev)
        self.out_ptrs = (ctypes.c_void_p * count)(*[t.data_ptr() for t in self.tours])
        torch.cuda.synchronize()

    def results(self):
        return [(t.cpu().numpy(), float(l)) for t, l in zip(self.tours, self.lengths.cpu().numpy())]


class Server:
    """Continuous-batching request loop (hac_server_*)."""

    def __init__(self, ctx: Context, budget: int, max_slots: int):
        self.ctx = ctx
        self._h = ctypes.c_void_p()
        self._keep = {}
        st = lib().hac_server_create(ctx.handle, budget, max_slots, ctypes.byref(self._h))
        if st != HAC_OK:
            raise HacError(st, f"hac_server_create: {strerror(st)}")

    def submit(self, inst, **over) -> int:
        m = Marshalled(inst, **over)
        t = ctypes.c_uint64()
        st = lib().hac_server_submit(self._h, ctypes.byref(m.s_inst), ctypes.byref(m.s_csr),
                                     ctypes.byref(m.s_params), m.seed, ctypes.byref(t))
        if st != HAC_OK:
            raise HacError(st, f"hac_server_submit: {strerror(st)}")
        self._keep[t.value] = inst.n
        return t.value

    def _result(self, fn, ticket: int):
        n = self._keep[ticket]
        tour = np.zeros(n, dtype=np.int32)
        L = ctypes.c_double()
        lat = ctypes.c_double()
        st = fn(self._h, ticket, tour.ctypes.data, ctypes.byref(L), ctypes.byref(lat))
        return st, tour, L.value, lat.value

    def poll(self, ticket: int):
        st, tour, L, lat = self._result(lib().hac_server_poll, ticket)
        if st == HAC_EBUSY:
            return None
        if st != HAC_OK:
            raise HacError(st, f"hac_server_poll: {strerror(st)}")
        self._keep.pop(ticket, None)
        return tour, L, lat

    def wait(self, ticket: int):
        st, tour, L, lat = self._result(lib().hac_server_wait, ticket)
        if st != HAC_OK:
            raise HacError(st, f"hac_server_wait: {strerror(st)}")
        self._keep.pop(ticket, None)
        return tour, L, lat

    def wait_status(self, ticket: int) -> int:
        st, _, _, _ = self._result(lib().hac_server_wait, ticket)
        return st

    def cancel(self, ticket: int) -> int:
        return int(lib().hac_server_cancel(self._h, ticket))

    def counters(self) -> dict:
        a, c = ctypes.c_int64(), ctypes.c_int64()
        ps, pb = ctypes.c_int32(), ctypes.c_uint64()
        lib().hac_server_counters(self._h, ctypes.byref(a), ctypes.byref(c), ctypes.byref(ps),
                                  ctypes.byref(pb))
        return dict(admitted=a.value, completed=c.value, peak_slots=ps.value, peak_bytes=pb.value)

    def lane_stats(self) -> list:
        """Per-lane counters (hac_server_lane_stats), one dict per size class."""
        out = []
        for lane in range(SERVER_LANES):
            st = hac_lane_stats()
            code = lib().hac_server_lane_stats(self._h, lane, ctypes.byref(st))
            if code != HAC_OK:
                raise HacError(code, f"hac_server_lane_stats: {strerror(code)}")
            out.append({name: getattr(st, name) for name, _ in hac_lane_stats._fields_})
        return out

    def close(self):
        if self._h:
            lib().hac_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
