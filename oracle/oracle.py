"""ctypes front-end for the CPU oracle (``bcd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
bench's CPU-baseline leg, never by the library or its binding.  The C file
is compiled with gcc (``-O3 -ffp-contract=off``) into ``libbcd_oracle.so``
next to this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "bcd_oracle.c")
LIB = os.path.join(HERE, "libbcd_oracle.so")

OK, INVALID, BAD_GRAPH, OVERFLOW, NOMEM, TOO_SMALL = 0, 1, 2, 3, 4, 6
INF = np.uint64(0xFFFFFFFFFFFFFFFF)


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O3", "-ffp-contract=off", "-fPIC", "-shared",
               "-std=gnu11", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm", "-lpthread"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OStats(C.Structure):
    _fields_ = [("rv_size", C.c_int64), ("fr_size", C.c_int64), ("samples", C.c_int64),
                ("distinct_sources", C.c_int64), ("te", C.c_uint64), ("reached", C.c_uint64),
                ("dag_arcs", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        p = C.c_void_p
        i64, i32, u64 = C.c_int64, C.c_int32, C.c_uint64
        L.oracle_check_graph.argtypes = [i64, i64, p, p, p]
        L.oracle_rv.argtypes = [i64, i64, p, p, i32, p, i64, p]
        L.oracle_fr_count.argtypes = [i64, i64, p, p, i32, p]
        L.oracle_source_pass.argtypes = [i64, i64, p, p, p, i32, p, p, p, p, p]
        L.oracle_bc_exact.argtypes = [i64, i64, p, p, p, i32, C.c_int, C.c_int, p, p]
        L.oracle_dependencies.argtypes = [i64, i64, p, p, p, i32, p, i64, C.c_int, p, p]
        L.oracle_bc_set.argtypes = [i64, i64, p, p, p, p, i64, C.c_int, p, p]
        L.oracle_bc_sampled.argtypes = [i64, i64, p, p, p, i32, i64, u64, C.c_int, p, p]
        L.oracle_sample_count.argtypes = [C.c_double, C.c_double, C.c_double, i64, p]
        L.oracle_draw_index.argtypes = [u64, i64, i64]
        L.oracle_draw_index.restype = i64
        L.oracle_pair_dependency.argtypes = [i64, i64, p, p, p, i32, i32, p]
        L.oracle_bc_sampled_all.argtypes = [i64, i64, p, p, p, i32, i64, u64, C.c_int, p]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def _ptr(a):
    return None if a is None else a.ctypes.data


def _g(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.weight is None else np.ascontiguousarray(g.weight, dtype=np.uint32)
    return rp, col, w


def _check(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


def default_threads() -> int:
    return max(1, min(os.cpu_count() or 1, 16))


def check_graph(g) -> int:
    rp, col, w = _g(g)
    return lib().oracle_check_graph(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w))


def rv(g, r: int) -> np.ndarray:
    """RV(r) ascending (Def.3 / Prop.2)."""
    rp, col, _ = _g(g)
    out = np.empty(g.n, dtype=np.int32)
    cnt = C.c_int64()
    _check(lib().oracle_rv(g.n, g.m, _ptr(rp), _ptr(col), r, _ptr(out), g.n, C.byref(cnt)), "rv")
    return out[: cnt.value].copy()


def fr_count(g, r: int) -> int:
    rp, col, _ = _g(g)
    cnt = C.c_int64()
    _check(lib().oracle_fr_count(g.n, g.m, _ptr(rp), _ptr(col), r, C.byref(cnt)), "fr")
    return cnt.value


def source_pass(g, s: int):
    """(dist uint64[n] with INF for unreached, sigma uint64[n], delta f64[n],
    overflow flag, (n_s, m_s, a_s))."""
    rp, col, w = _g(g)
    dist = np.empty(g.n, dtype=np.uint64)
    sig = np.empty(g.n, dtype=np.uint64)
    dl = np.empty(g.n, dtype=np.float64)
    ovf = C.c_int()
    cnt = np.zeros(3, dtype=np.uint64)
    _check(lib().oracle_source_pass(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), s, _ptr(dist),
                                    _ptr(sig), _ptr(dl), C.byref(ovf), _ptr(cnt)), "source_pass")
    return dist, sig, dl, bool(ovf.value), tuple(int(x) for x in cnt)


def bc_exact(g, r: int, pruned: bool = True, threads: int | None = None):
    """(BC(r), stats dict); raises OracleError(OVERFLOW) on sigma overflow."""
    rp, col, w = _g(g)
    bc = C.c_double()
    st = OStats()
    _check(lib().oracle_bc_exact(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), r, int(pruned),
                                 threads or default_threads(), C.byref(bc), C.byref(st)),
           "bc_exact")
    return bc.value, _stats(st)


def dependencies(g, r: int, sources, threads: int | None = None):
    """delta_s.(r) for each s in ``sources`` and per-source (n_s, m_s, a_s)."""
    rp, col, w = _g(g)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    dep = np.empty(src.size, dtype=np.float64)
    cnt = np.empty((src.size, 3), dtype=np.uint64)
    _check(lib().oracle_dependencies(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), r, _ptr(src),
                                     src.size, threads or default_threads(), _ptr(dep),
                                     _ptr(cnt)), "dependencies")
    return dep, cnt


def bc_set(g, rs, threads: int | None = None):
    rp, col, w = _g(g)
    r = np.ascontiguousarray(rs, dtype=np.int32)
    bc = np.empty(r.size, dtype=np.float64)
    st = OStats()
    _check(lib().oracle_bc_set(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), _ptr(r), r.size,
                               threads or default_threads(), _ptr(bc), C.byref(st)), "bc_set")
    return bc, _stats(st)


def bc_sampled(g, r: int, T: int, seed: int, threads: int | None = None):
    rp, col, w = _g(g)
    bc = C.c_double()
    st = OStats()
    _check(lib().oracle_bc_sampled(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), r, T,
                                   seed & 0xFFFFFFFFFFFFFFFF, threads or default_threads(),
                                   C.byref(bc), C.byref(st)), "bc_sampled")
    return bc.value, _stats(st)


def bc_sampled_all(g, r: int, T: int, seed: int, threads: int | None = None) -> float:
    """Uniform source sampling over V minus r (the unpruned baseline)."""
    rp, col, w = _g(g)
    bc = C.c_double()
    _check(lib().oracle_bc_sampled_all(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), r, T,
                                       seed & 0xFFFFFFFFFFFFFFFF, threads or default_threads(),
                                       C.byref(bc)), "bc_sampled_all")
    return bc.value


def bc_bcd(g, r: int, tau: int, seed: int, threads: int | None = None):
    """The procedure of Section 5: exact when |RV(r)| <= tau, else tau draws."""
    k = len(rv(g, r))
    if k <= tau:
        return bc_exact(g, r, threads=threads)[0], True
    return bc_sampled(g, r, tau, seed, threads=threads)[0], False


def sample_count(eps_abs: float, delta: float, K: float, rv_size: int) -> int:
    T = C.c_int64()
    _check(lib().oracle_sample_count(eps_abs, delta, K, rv_size, C.byref(T)), "sample_count")
    return T.value


def draw_index(seed: int, t: int, rv_size: int) -> int:
    return lib().oracle_draw_index(seed & 0xFFFFFFFFFFFFFFFF, t, rv_size)


def pair_dependency(g, s: int, r: int) -> float:
    rp, col, w = _g(g)
    d = C.c_double()
    _check(lib().oracle_pair_dependency(g.n, g.m, _ptr(rp), _ptr(col), _ptr(w), s, r,
                                        C.byref(d)), "pair_dependency")
    return d.value


def _stats(st: OStats) -> dict:
    return {k: getattr(st, k) for k, _ in OStats._fields_}
