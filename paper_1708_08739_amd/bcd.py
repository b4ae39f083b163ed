"""ctypes binding for ``libbcd.so`` (include/bcd.h).

Argument marshalling only: every step of the computation runs in the
library's HIP kernels.  The binding refuses to work without the built
library -- there is no fallback of any kind.

Low-level functions keep the C names (``bcd_bc_exact`` ...).  ``Graph`` is a
small convenience wrapper that owns a handle.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbcd.so")

BCD_OK = 0
BCD_ERR_INVALID_ARG = 1
BCD_ERR_BAD_GRAPH = 2
BCD_ERR_SIGMA_OVERFLOW = 3
BCD_ERR_OUT_OF_MEMORY = 4
BCD_ERR_DEVICE = 5
BCD_ERR_BUFFER_TOO_SMALL = 6
BCD_ERR_UNSUPPORTED = 7
BCD_ERR_AGAIN = 8
BCD_ERR_CANCELLED = 9

BCD_ENGINE_BATCHED = 0
BCD_ENGINE_PLAIN = 1
BCD_ENGINE_LDS = 2

BCD_EPS_ABSOLUTE = 1
BCD_K_TRIVIAL = 2
BCD_NO_EXACT_FALLBACK = 4
BCD_SAMPLE_ALL_VERTICES = 8

U64_MAX = np.uint64(0xFFFFFFFFFFFFFFFF)


class Stats(C.Structure):
    _fields_ = [("rv_size", C.c_int64), ("fr_size", C.c_int64), ("samples", C.c_int64),
                ("distinct_sources", C.c_int64), ("traversed_edges", C.c_uint64),
                ("reached", C.c_uint64), ("dag_arcs", C.c_uint64), ("t_rv_s", C.c_double),
                ("t_bc_s", C.c_double), ("batch_width", C.c_int32), ("ran_exact", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class Config(C.Structure):
    _fields_ = [("engine", C.c_int32), ("groups", C.c_int32), ("block", C.c_int32),
                ("grid_mult", C.c_int32), ("items", C.c_int32), ("bottom_up", C.c_int32),
                ("compress", C.c_int32), ("push", C.c_int32)]


class SampleParams(C.Structure):
    _fields_ = [("eps", C.c_double), ("delta", C.c_double), ("seed", C.c_uint64),
                ("flags", C.c_uint32), ("T_override", C.c_int64)]


class KernelProfile(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double), ("alg_bytes", C.c_double),
                ("vertex_pairs", C.c_uint64), ("arc_pairs", C.c_uint64), ("dag_pairs", C.c_uint64),
                ("items", C.c_uint64), ("union_ms", C.c_double), ("item_arcs", C.c_uint64),
                ("sched_bytes", C.c_double)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("workers", C.c_int32), ("groups", C.c_int32),
                ("queue_capacity", C.c_int32), ("reserved", C.c_int32)]


class Query(C.Structure):
    _fields_ = [("kind", C.c_int32), ("r", C.c_int32), ("rs", C.c_void_p), ("l", C.c_int64),
                ("params", SampleParams), ("bc_out", C.c_void_p), ("tag", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("tag", C.c_uint64), ("status", C.c_int32), ("kind", C.c_int32),
                ("bc", C.c_double), ("stats", Stats), ("t_arrive_s", C.c_double), ("t_admit_s", C.c_double),
                ("t_done_s", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("queries_done", C.c_uint64), ("batches", C.c_uint64), ("lanes_used", C.c_uint64),
                ("lane_slots", C.c_uint64), ("traversed_edges", C.c_uint64), ("shared_lanes", C.c_uint64)]


BCD_QUERY_EXACT = 0
BCD_QUERY_SAMPLED = 1
BCD_QUERY_SET = 2


class BcdError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({detail})")
        self.code = code


STATUS_NAMES = {
    0: "BCD_OK", 1: "BCD_ERR_INVALID_ARG", 2: "BCD_ERR_BAD_GRAPH", 3: "BCD_ERR_SIGMA_OVERFLOW",
    4: "BCD_ERR_OUT_OF_MEMORY", 5: "BCD_ERR_DEVICE", 6: "BCD_ERR_BUFFER_TOO_SMALL",
    7: "BCD_ERR_UNSUPPORTED", 8: "BCD_ERR_AGAIN", 9: "BCD_ERR_CANCELLED",
}

# name -> (argtypes, restype); restype None means bcd_status (int)
_p = C.c_void_p
_i64, _i32, _u64, _d = C.c_int64, C.c_int32, C.c_uint64, C.c_double
SIGNATURES = {
    "bcd_graph_load_csr": [_i64, _i64, _p, _p, _p, C.POINTER(_p)],
    "bcd_graph_free": [_p],
    "bcd_graph_info": [_p, _p, _p, _p],
    "bcd_set_config": [_p, C.POINTER(Config)],
    "bcd_get_config": [_p, C.POINTER(Config)],
    "bcd_rv": [_p, _i32, _p, _i64, C.POINTER(_i64)],
    "bcd_rv_noalloc": [_p, _i32, _p, _i64, C.POINTER(_i64)],
    "bcd_bc_exact": [_p, _i32, C.POINTER(_d), C.POINTER(Stats)],
    "bcd_bc_sampled": [_p, _i32, C.POINTER(SampleParams), C.POINTER(_d), C.POINTER(Stats)],
    "bcd_bc_set": [_p, _p, _i64, _p, C.POINTER(Stats)],
    "bcd_bc_bcd": [_p, _i32, _i64, _u64, C.POINTER(_d), C.POINTER(Stats)],
    "bcd_source_pass": [_p, _i32, _p, _p, _p],
    "bcd_multi_source_pass": [_p, _p, _i64, _p, _p, _p],
    "bcd_dependencies": [_p, _i32, _p, _i64, _p, _p],
    "bcd_sample_count": [_d, _d, _d, _i64, C.POINTER(_i64)],
    "bcd_profile_enable": [_p, _i32],
    "bcd_profile_get": [_p, _i32, C.POINTER(KernelProfile)],
    "bcd_profile_reset": [_p],
    "bcd_bandwidth_probe": [_i64, _i32, C.POINTER(_d)],
    "bcd_read_bandwidth_probe": [_i64, _i32, C.POINTER(_d)],
    "bcd_autotune": [_p, _i32, _i32, _i64, C.POINTER(Config), C.POINTER(_d)],
    "bcd_server_create": [_p, C.POINTER(ServerConfig), C.POINTER(_p)],
    "bcd_server_submit": [_p, C.POINTER(Query), C.POINTER(_u64)],
    "bcd_server_poll": [_p, _p, _i32, C.POINTER(_i32), _i64],
    "bcd_server_shutdown": [_p],
    "bcd_server_destroy": [_p],
    "bcd_server_get_stats": [_p, C.POINTER(ServerStats)],
    "bcd_server_workspace_bytes": [_p, _i32, _i32, C.POINTER(_u64)],
}
OPTIONAL_SIGNATURES: dict = {}

_lib = None


def load(path: str | None = None):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1708_08739_amd.build`")
    L = C.CDLL(path)
    for name, args in {**SIGNATURES, **OPTIONAL_SIGNATURES}.items():
        fn = getattr(L, name, None)
        if fn is None:
            if name in SIGNATURES:
                raise RuntimeError(f"{path} does not export {name}")
            continue
        fn.argtypes = args
        fn.restype = C.c_int
    L.bcd_status_string.argtypes = [C.c_int]
    L.bcd_status_string.restype = C.c_char_p
    L.bcd_server_now.argtypes = []
    L.bcd_server_now.restype = C.c_double
    L.bcd_last_error.argtypes = []
    L.bcd_last_error.restype = C.c_char_p
    _lib = L
    return L


def last_error() -> str:
    return load().bcd_last_error().decode()


def check(rc: int, where: str) -> None:
    if rc != BCD_OK:
        raise BcdError(rc, where, last_error())


def _ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def bcd_sample_count(eps_abs: float, delta: float, K: float, rv_size: int) -> int:
    T = C.c_int64()
    check(load().bcd_sample_count(eps_abs, delta, K, rv_size, C.byref(T)), "bcd_sample_count")
    return T.value


def bcd_bandwidth_probe(nbytes: int = 1 << 30, reps: int = 5) -> float:
    g = C.c_double()
    check(load().bcd_bandwidth_probe(nbytes, reps, C.byref(g)), "bcd_bandwidth_probe")
    return g.value


def bcd_read_bandwidth_probe(nbytes: int = 1 << 30, reps: int = 5) -> float:
    g = C.c_double()
    check(load().bcd_read_bandwidth_probe(nbytes, reps, C.byref(g)), "bcd_read_bandwidth_probe")
    return g.value


class Graph:
    """A digraph resident on the GPU (``bcd_graph_load_csr``)."""

    def __init__(self, n, row_ptr, col, weight=None):
        L = load()
        self.n = int(n)
        self._rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self._col = np.ascontiguousarray(col, dtype=np.int32)
        self._w = None if weight is None else np.ascontiguousarray(weight, dtype=np.uint32)
        self.m = int(self._rp[-1]) if self._rp.size else 0
        h = C.c_void_p()
        check(L.bcd_graph_load_csr(self.n, self._col.size, _ptr(self._rp), _ptr(self._col),
                                   _ptr(self._w), C.byref(h)), "bcd_graph_load_csr")
        self.h = h

    @classmethod
    def from_digraph(cls, g):
        return cls(g.n, g.row_ptr, g.col, g.weight)

    def info(self) -> tuple[int, int, bool]:
        """(n, m, weighted) as the library holds them (``bcd_graph_info``)."""
        n, m, w = C.c_int64(), C.c_int64(), C.c_int32()
        check(load().bcd_graph_info(self.h, C.byref(n), C.byref(m), C.byref(w)), "bcd_graph_info")
        return n.value, m.value, bool(w.value)

    def close(self):
        if getattr(self, "h", None):
            load().bcd_graph_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- configuration
    def config(self) -> Config:
        c = Config()
        check(load().bcd_get_config(self.h, C.byref(c)), "bcd_get_config")
        return c

    def set_config(self, engine=None, groups=None, block=None, grid_mult=None, items=None,
                   bottom_up=None, compress=None, push=None) -> Config:
        c = self.config()
        if compress is not None:
            c.compress = int(compress)
        if push is not None:
            c.push = int(push)
        if items is not None:
            c.items = items
        if bottom_up is not None:
            c.bottom_up = bottom_up
        if engine is not None:
            c.engine = engine
        if groups is not None:
            c.groups = groups
        if block is not None:
            c.block = block
        if grid_mult is not None:
            c.grid_mult = grid_mult
        check(load().bcd_set_config(self.h, C.byref(c)), "bcd_set_config")
        return c

    # -- queries
    def rv(self, r: int) -> np.ndarray:
        cnt = C.c_int64()
        check(load().bcd_rv(self.h, r, None, 0, C.byref(cnt)), "bcd_rv")
        out = np.empty(max(cnt.value, 1), dtype=np.int32)
        check(load().bcd_rv(self.h, r, _ptr(out), out.size, C.byref(cnt)), "bcd_rv")
        return out[: cnt.value].copy()

    def bc_exact(self, r: int):
        bc = C.c_double()
        st = Stats()
        check(load().bcd_bc_exact(self.h, r, C.byref(bc), C.byref(st)), "bcd_bc_exact")
        return bc.value, st.as_dict()

    def bc_sampled(self, r: int, eps: float = 0.01, delta: float = 0.1, seed: int = 0, flags: int = 0,
                   T: int = 0):
        p = SampleParams(eps, delta, seed & 0xFFFFFFFFFFFFFFFF, flags, T)
        bc = C.c_double()
        st = Stats()
        check(load().bcd_bc_sampled(self.h, r, C.byref(p), C.byref(bc), C.byref(st)), "bcd_bc_sampled")
        return bc.value, st.as_dict()

    def bc_bcd(self, r: int, tau: int = 1000, seed: int = 0):
        """The BCD procedure (exact if |RV(r)| <= tau, else tau draws)."""
        bc = C.c_double()
        st = Stats()
        check(load().bcd_bc_bcd(self.h, r, tau, seed & 0xFFFFFFFFFFFFFFFF, C.byref(bc), C.byref(st)), "bcd_bc_bcd")
        return bc.value, st.as_dict()

    def bc_set(self, rs):
        r = np.ascontiguousarray(rs, dtype=np.int32)
        bc = np.empty(r.size, dtype=np.float64)
        st = Stats()
        check(load().bcd_bc_set(self.h, _ptr(r), r.size, _ptr(bc), C.byref(st)), "bcd_bc_set")
        return bc, st.as_dict()

    def source_pass(self, s: int):
        dist = np.empty(self.n, dtype=np.uint64)
        sig = np.empty(self.n, dtype=np.uint64)
        dl = np.empty(self.n, dtype=np.float64)
        check(load().bcd_source_pass(self.h, s, _ptr(dist), _ptr(sig), _ptr(dl)), "bcd_source_pass")
        return dist, sig, dl

    def multi_source_pass(self, sources):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        k = src.size
        dist = np.empty((k, self.n), dtype=np.uint64)
        sig = np.empty((k, self.n), dtype=np.uint64)
        dl = np.empty((k, self.n), dtype=np.float64)
        check(load().bcd_multi_source_pass(self.h, _ptr(src), k, _ptr(dist), _ptr(sig), _ptr(dl)),
              "bcd_multi_source_pass")
        return dist, sig, dl

    def dependencies(self, r: int, sources, counters: bool = False):
        src = np.ascontiguousarray(sources, dtype=np.int32)
        dep = np.empty(src.size, dtype=np.float64)
        cnt = np.empty((src.size, 3), dtype=np.uint64) if counters else None
        check(load().bcd_dependencies(self.h, r, _ptr(src), src.size, _ptr(dep), _ptr(cnt)),
              "bcd_dependencies")
        return (dep, cnt) if counters else dep

    def autotune(self, r: int, max_groups: int = 16, max_sources: int = 4096):
        c = Config()
        rate = C.c_double()
        check(load().bcd_autotune(self.h, r, max_groups, max_sources, C.byref(c), C.byref(rate)), "bcd_autotune")
        return c, rate.value

    # -- profiling
    def profile_enable(self, on: bool = True):
        check(load().bcd_profile_enable(self.h, 1 if on else 0), "bcd_profile_enable")

    def profile_reset(self):
        check(load().bcd_profile_reset(self.h), "bcd_profile_reset")

    def profile(self, kind: int) -> dict:
        p = KernelProfile()
        check(load().bcd_profile_get(self.h, kind, C.byref(p)), "bcd_profile_get")
        return {k: getattr(p, k) for k, _ in p._fields_}


class Server:
    """Serving loop on a loaded ``Graph`` (``bcd_server_*``)."""

    def __init__(self, graph: Graph, hbm_budget_bytes: int = 0, workers: int = 0, groups: int = 0,
                 queue_capacity: int = 0):
        self.graph = graph
        cfg = ServerConfig(hbm_budget_bytes, workers, groups, queue_capacity, 0)
        h = C.c_void_p()
        check(load().bcd_server_create(graph.h, C.byref(cfg), C.byref(h)), "bcd_server_create")
        self.h = h
        self._keep: dict[int, tuple] = {}

    @staticmethod
    def workspace_bytes(graph: Graph, groups: int = 0, workers: int = 0) -> int:
        """Device bytes of the batch workspaces a server with these settings
        reserves out of its HBM budget."""
        b = C.c_uint64()
        check(load().bcd_server_workspace_bytes(graph.h, groups, workers, C.byref(b)), "bcd_server_workspace_bytes")
        return int(b.value)

    def submit(self, kind: int, r: int = 0, rs=None, eps: float = 0.01, delta: float = 0.1, seed: int = 0,
               flags: int = 0, T: int = 0, tag: int = 0) -> int:
        q = Query()
        q.kind = kind
        q.r = r
        keep = ()
        if kind == BCD_QUERY_SET:
            arr = np.ascontiguousarray(rs, dtype=np.int32)
            out = np.zeros(arr.size, dtype=np.float64)
            q.rs = arr.ctypes.data
            q.l = arr.size
            q.bc_out = out.ctypes.data
            keep = (arr, out)
        q.params = SampleParams(eps, delta, seed & 0xFFFFFFFFFFFFFFFF, flags, T)
        q.tag = tag
        t = C.c_uint64()
        check(load().bcd_server_submit(self.h, C.byref(q), C.byref(t)), "bcd_server_submit")
        self._keep[t.value] = keep
        return t.value

    def poll(self, cap: int = 64, timeout_s: float = -1.0) -> list[dict]:
        buf = (Result * cap)()
        n = C.c_int32()
        ns = -1 if timeout_s < 0 else int(timeout_s * 1e9)
        rc = load().bcd_server_poll(self.h, buf, cap, C.byref(n), ns)
        if rc == BCD_ERR_AGAIN:
            return []
        check(rc, "bcd_server_poll")
        out = []
        for i in range(n.value):
            r = buf[i]
            d = {k: getattr(r, k) for k, _ in Result._fields_ if k != "stats"}
            d["stats"] = r.stats.as_dict()
            keep = self._keep.pop(r.ticket, ())
            if keep:
                d["bcs"] = keep[1].copy()
            out.append(d)
        return out

    def stats(self) -> dict:
        st = ServerStats()
        check(load().bcd_server_get_stats(self.h, C.byref(st)), "bcd_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    @staticmethod
    def now() -> float:
        return load().bcd_server_now()

    def shutdown(self):
        """Cancel queries not yet admitted, let admitted ones finish; results
        stay pollable."""
        check(load().bcd_server_shutdown(self.h), "bcd_server_shutdown")

    def close(self):
        if getattr(self, "h", None):
            load().bcd_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
