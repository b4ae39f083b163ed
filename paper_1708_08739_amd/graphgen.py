"""Seeded synthetic digraphs and query vertices.

This module only draws inputs: it holds none of the method's arithmetic
(no shortest paths, no path counting, no dependency scores).  Both the CPU
oracle and the GPU library are fed from here, so every test and the bench
see the same bytes.

Randomness: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) used as a
counter-based generator.  Value ``i`` of the stream with seed ``S`` is
``mix64(S + (i + 1) * GAMMA)``, i.e. the ``i``-th output of a SplitMix64
generator started at state ``S``.  Integers in ``[0, k)`` are the high 64
bits of ``x * k``; doubles in ``[0, 1)`` are ``(x >> 11) * 2**-53``.

Graph model (paper, Section 2): directed, no self-loops, no multi-arcs.
Rows of the CSR are sorted ascending.  Arc weights, when present, are
positive integers (the paper assumes positive weights).
"""
from __future__ import annotations

import ctypes
import dataclasses
import functools
import os

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK32 = np.uint64(0xFFFFFFFF)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream(seed: int, start: int, count: int) -> np.ndarray:
    """Values ``start .. start+count-1`` of the SplitMix64 stream ``seed``."""
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GAMMA
    return mix64(state)


def below(x: np.ndarray, k: int) -> np.ndarray:
    """``floor(x * k / 2**64)`` for uint64 ``x`` and ``0 < k < 2**32``."""
    if not (0 < k < (1 << 32)):
        raise ValueError("k must be in (0, 2**32)")
    kk = np.uint64(k)
    x = np.asarray(x, dtype=np.uint64)
    hi = x >> np.uint64(32)
    lo = x & _MASK32
    with np.errstate(over="ignore"):
        return (hi * kk + ((lo * kk) >> np.uint64(32))) >> np.uint64(32)


def unit(x: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (np.asarray(x, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclasses.dataclass
class Digraph:
    """A CSR digraph: ``row_ptr`` int64[n+1], ``col`` int32[m], optional
    ``weight`` uint32[m] (arc ``e`` goes from its row to ``col[e]``)."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    weight: np.ndarray | None = None
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1])

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int64)

    def arcs(self) -> tuple[np.ndarray, np.ndarray]:
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.out_degree())
        return src, self.col.astype(np.int64)


def from_arcs(n: int, src, dst, weight=None, name: str = "") -> Digraph:
    """CSR from an arc list.  Self-loops and repeated arcs are rejected (the
    paper's graphs have neither); callers dedupe before calling."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("endpoint out of range")
    if np.any(src == dst):
        raise ValueError("self-loop")
    key = src * n + dst
    order = np.argsort(key, kind="stable")
    key = key[order]
    if key.size and np.any(key[1:] == key[:-1]):
        raise ValueError("repeated arc")
    s = key // n
    d = key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=row_ptr[1:])
    w = None
    if weight is not None:
        w = np.asarray(weight, dtype=np.uint32)[order].copy()
    return Digraph(n, row_ptr, d.astype(np.int32), w, name)


def _dedupe_sorted(n: int, src: np.ndarray, dst: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    keep = src != dst
    key = np.unique(src[keep] * np.int64(n) + dst[keep])
    return key // n, key % n


def erdos_renyi(n: int, m: int, seed: int) -> Digraph:
    """G(n, m): arcs (u, v) with u, v uniform; self-loops and repeats are
    rejected in draw order until exactly ``m`` distinct arcs remain."""
    if m > n * (n - 1):
        raise ValueError("too many arcs")
    seen: dict[int, None] = {}
    pos = 0
    chunk = max(2 * m, 1024)
    while len(seen) < m:
        x = stream(seed, pos, 2 * chunk)
        pos += 2 * chunk
        u = below(x[0::2], n).astype(np.int64)
        v = below(x[1::2], n).astype(np.int64)
        for a, b in zip(u.tolist(), v.tolist()):
            if a == b:
                continue
            k = a * n + b
            if k not in seen:
                seen[k] = None
                if len(seen) == m:
                    break
    keys = np.fromiter(seen.keys(), dtype=np.int64, count=m)
    return from_arcs(n, keys // n, keys % n, name=f"er_n{n}_m{m}_s{seed}")


RMAT_ABCD = (0.57, 0.19, 0.19, 0.05)

_NATIVE_DRAWS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "gen", "librmat_draws.so")
_native = None


def _native_draws():
    """The C form of the quadrant draws (gen/rmat_draws.c, built next to the
    library), or None when it has not been built."""
    global _native
    if _native is None:
        _native = False
        if os.path.exists(_NATIVE_DRAWS):
            lib = ctypes.CDLL(_NATIVE_DRAWS)
            lib.rmat_draws.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
            lib.rmat_draws.restype = None
            _native = lib
    return _native or None


def rmat_draws(scale: int, ne: int, seed: int, abcd=RMAT_ABCD, chunk: int = 1 << 21,
               native: bool | None = None) -> tuple[np.ndarray, np.ndarray]:
    """The ``ne`` R-MAT draws before relabelling: at each of ``scale`` bit
    levels (most significant first) value ``e * scale + level`` of stream
    ``seed``, as a uniform double, picks quadrant a:(0,0) b:(0,1) c:(1,0)
    d:(1,1) as (source bit, destination bit).  ``native`` None uses the C
    form when built (same values), False forces NumPy."""
    a, b, c, _ = abcd
    t1, t2, t3 = a, a + b, a + b + c
    lib = _native_draws() if native is not False else None
    if lib is not None:
        src = np.empty(ne, dtype=np.int64)
        dst = np.empty(ne, dtype=np.int64)
        lib.rmat_draws(seed & 0xFFFFFFFFFFFFFFFF, scale, ne, t1, t2, t3, src.ctypes.data, dst.ctypes.data)
        return src, dst
    if native:
        raise RuntimeError("gen/librmat_draws.so is not built")
    srcs = []
    dsts = []
    for e0 in range(0, ne, chunk):
        ce = min(chunk, ne - e0)
        u = unit(stream(seed, e0 * scale, ce * scale)).reshape(ce, scale)
        sbit = (u >= t2).astype(np.int64)
        dbit = (((u >= t1) & (u < t2)) | (u >= t3)).astype(np.int64)
        wts = (np.int64(1) << np.arange(scale - 1, -1, -1, dtype=np.int64))
        srcs.append(sbit @ wts)
        dsts.append(dbit @ wts)
        del u, sbit, dbit
    if not srcs:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    return np.concatenate(srcs), np.concatenate(dsts)


def rmat(scale: int, edge_factor: int, seed: int, abcd=RMAT_ABCD,
         weighted: bool = False, max_weight: int = 100, chunk: int = 1 << 21,
         orient_seed: int | None = None) -> Digraph:
    """R-MAT (Chakrabarti, Zhan and Faloutsos): ``edge_factor * 2**scale``
    draws; at each of ``scale`` bit levels a uniform double picks quadrant
    a:(0,0) b:(0,1) c:(1,0) d:(1,1) as (source bit, destination bit), most
    significant bit first.  Vertex ids are then relabelled by a seeded
    permutation; self-loops and repeated arcs are dropped; rows sorted.
    Weighted: arc ``e`` of the final CSR gets ``1 + floor(x_e * W / 2**64)``
    from stream ``seed + 2``, so weights are uniform in ``[1, W]``.
    ``orient_seed``: after the relabelling every arc is turned to point from
    the endpoint of lower to the one of higher rank, vertex ``v`` having key
    ``x_v`` of stream ``orient_seed`` (ties by id), so the graph is acyclic;
    repeats are dropped after turning."""
    n = 1 << scale
    ne = edge_factor * n
    src, dst = rmat_draws(scale, ne, seed, abcd, chunk=chunk)
    perm = np.argsort(stream(seed + 1, 0, n), kind="stable").astype(np.int64)
    src = perm[src]
    dst = perm[dst]
    if orient_seed is not None:
        key = stream(orient_seed, 0, n)
        rank = np.empty(n, dtype=np.int64)
        rank[np.lexsort((np.arange(n), key))] = np.arange(n, dtype=np.int64)
        flip = rank[src] > rank[dst]
        src, dst = np.where(flip, dst, src), np.where(flip, src, dst)
    s, d = _dedupe_sorted(n, src, dst)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=row_ptr[1:])
    w = None
    if weighted:
        w = (below(stream(seed + 2, 0, s.size), max_weight) + np.uint64(1)).astype(np.uint32)
    name = f"rmat_s{scale}_ef{edge_factor}_seed{seed}" + ("_w" if weighted else "")
    if orient_seed is not None:
        name += f"_dag{orient_seed}"
    return Digraph(n, row_ptr, d.astype(np.int32), w, name)


def with_unit_weights(g: Digraph) -> Digraph:
    return Digraph(g.n, g.row_ptr, g.col, np.ones(g.m, dtype=np.uint32), g.name + "_w1")


def with_weights(g: Digraph, seed: int, max_weight: int) -> Digraph:
    w = (below(stream(seed, 0, g.m), max_weight) + np.uint64(1)).astype(np.uint32)
    return Digraph(g.n, g.row_ptr, g.col, w, g.name + f"_w{max_weight}")


# ---------------------------------------------------------------- queries

def top_out_degree(g: Digraph, k: int) -> list[int]:
    """The ``k`` vertices of largest out-degree, ties to the smaller id."""
    deg = g.out_degree()
    order = np.lexsort((np.arange(g.n), -deg))
    return [int(v) for v in order[:k]]


def max_in_degree(g: Digraph) -> int:
    deg = g.in_degree()
    return int(np.lexsort((np.arange(g.n), -deg))[0])


def uniform_vertices(n: int, k: int, seed: int, exclude=()) -> list[int]:
    """``k`` distinct vertices, uniform over ``[0, n)`` minus ``exclude``,
    drawn in stream order."""
    out: list[int] = []
    taken = set(int(v) for v in exclude)
    pos = 0
    while len(out) < k:
        x = stream(seed, pos, 64)
        pos += 64
        for v in below(x, n).tolist():
            if v not in taken:
                taken.add(v)
                out.append(int(v))
                if len(out) == k:
                    break
    return out


def queries_top_and_random(g: Digraph, seed: int, top: int = 4, rnd: int = 4) -> list[int]:
    """Top-``top`` out-degree vertices followed by ``rnd`` uniform others."""
    t = top_out_degree(g, top)
    return t + uniform_vertices(g.n, rnd, seed, exclude=t)


# ------------------------------------------------------- named workloads

def er_2000() -> tuple[Digraph, list[int]]:
    """Directed Erdos-Renyi, n = 2,000, m = 10,000, unweighted; the query is
    the vertex of largest in-degree."""
    g = erdos_renyi(2000, 10000, seed=1)
    return g, [max_in_degree(g)]


def rmat16() -> tuple[Digraph, list[int]]:
    """R-MAT scale 16, edge factor 8, unweighted; top-4 out-degree plus four
    seeded uniform vertices."""
    g = rmat(16, 8, seed=2)
    return g, queries_top_and_random(g, seed=102)


def rmat18_weighted() -> tuple[Digraph, list[int]]:
    """R-MAT scale 18, edge factor 16, weights uniform in [1, 100]."""
    g = rmat(18, 16, seed=3, weighted=True, max_weight=100)
    return g, queries_top_and_random(g, seed=103)


@functools.lru_cache(maxsize=1)
def rmat20() -> Digraph:
    return rmat(20, 16, seed=4)


@functools.lru_cache(maxsize=1)
def rmat22() -> Digraph:
    return rmat(22, 16, seed=5)


def rmat20_dag() -> Digraph:
    """The R-MAT scale 20 draws of ``rmat20`` turned into a DAG by a second
    seeded ranking: ancestor sets (and so RV(r)) then range from a handful
    of vertices to a large fraction of the graph."""
    return rmat(20, 16, seed=4, orient_seed=14)


# ----------------------------------------------- small structured graphs

def directed_path(n: int) -> Digraph:
    i = np.arange(n - 1)
    return from_arcs(n, i, i + 1, name=f"path{n}")


def bidirected_path(n: int) -> Digraph:
    i = np.arange(n - 1)
    return from_arcs(n, np.concatenate([i, i + 1]), np.concatenate([i + 1, i]), name=f"bipath{n}")


def directed_cycle(n: int) -> Digraph:
    i = np.arange(n)
    return from_arcs(n, i, (i + 1) % n, name=f"cycle{n}")


def in_out_star(a: int, b: int) -> tuple[Digraph, int]:
    """``a`` leaves pointing to a centre ``c``, which points to ``b`` leaves."""
    c = 0
    ins = np.arange(1, a + 1)
    outs = np.arange(a + 1, a + b + 1)
    g = from_arcs(a + b + 1, np.concatenate([ins, np.full(b, c)]),
                  np.concatenate([np.full(a, c), outs]), name=f"star{a}_{b}")
    return g, c


def transitive_tournament(n: int) -> Digraph:
    s, d = np.triu_indices(n, 1)
    return from_arcs(n, s, d, name=f"tt{n}")


def complete_digraph(n: int) -> Digraph:
    s, d = np.nonzero(~np.eye(n, dtype=bool))
    return from_arcs(n, s, d, name=f"k{n}")


def diamond_chain(k: int) -> tuple[Digraph, dict]:
    """x_0 -> {a_i, b_i} -> x_i for i = 1..k.  Ids: x_i = 3i, a_i = 3i-2,
    b_i = 3i-1."""
    src, dst = [], []
    for i in range(1, k + 1):
        xp, a, b, x = 3 * (i - 1), 3 * i - 2, 3 * i - 1, 3 * i
        src += [xp, xp, a, b]
        dst += [a, b, x, x]
    ids = {"x": [3 * i for i in range(k + 1)], "a": [None] + [3 * i - 2 for i in range(1, k + 1)],
           "b": [None] + [3 * i - 1 for i in range(1, k + 1)]}
    return from_arcs(3 * k + 1, src, dst, name=f"diamond{k}"), ids


def diamond_chain_weighted(k: int, mixed: bool) -> tuple[Digraph, dict, int]:
    """``diamond_chain(k)`` with arc weights that keep both branches of every
    diamond equally long: all 3 (``mixed`` False), or x -> a 1, x -> b 2,
    a -> x' 2, b -> x' 1 (``mixed`` True: the two middle vertices of a
    diamond at different distances).  Returns (graph, ids, length of one
    diamond)."""
    g, ids = diamond_chain(k)
    w = np.empty(g.m, dtype=np.uint32)
    for u in range(g.n):
        a, b = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
        if not mixed:
            w[a:b] = 3
        elif u % 3 == 0:  # a joint x_{i-1}: its arcs to a_i then b_i
            w[a:b] = [1, 2][: b - a]
        else:  # a_i (id 3i-2) or b_i (id 3i-1): its one arc to x_i
            w[a:b] = 2 if u % 3 == 1 else 1
    name = g.name + ("_mixed" if mixed else "_w3")
    return Digraph(g.n, g.row_ptr, g.col, w, name), ids, (3 if mixed else 6)


def grid_right_down(rows: int, cols: int) -> Digraph:
    """Directed grid: (i, j) -> (i, j+1) and (i, j) -> (i+1, j); id = i*cols + j."""
    src, dst = [], []
    for i in range(rows):
        for j in range(cols):
            v = i * cols + j
            if j + 1 < cols:
                src.append(v)
                dst.append(v + 1)
            if i + 1 < rows:
                src.append(v)
                dst.append(v + cols)
    return from_arcs(rows * cols, src, dst, name=f"grid{rows}x{cols}")


def random_small(n: int, p_arc: float, seed: int, max_weight: int = 0) -> Digraph:
    """Small random digraph: each ordered pair is an arc with probability
    ``p_arc``; optional weights uniform in ``[1, max_weight]``."""
    x = unit(stream(seed, 0, n * n)).reshape(n, n)
    adj = (x < p_arc) & ~np.eye(n, dtype=bool)
    s, d = np.nonzero(adj)
    w = None
    if max_weight:
        w = (below(stream(seed + 7, 0, s.size), max_weight) + np.uint64(1)).astype(np.uint32)
    return from_arcs(n, s, d, w, name=f"rand{n}_{seed}")


def digraph_from_code(n: int, code: int) -> Digraph:
    """Digraph number ``code`` on ``n`` vertices: bit ``k`` of ``code`` is the
    ``k``-th off-diagonal ordered pair in row-major order."""
    src, dst = [], []
    k = 0
    for u in range(n):
        for v in range(n):
            if u == v:
                continue
            if code >> k & 1:
                src.append(u)
                dst.append(v)
            k += 1
    return from_arcs(n, src, dst, name=f"code{n}_{code}")


def superseded_tie_chain(k: int, final_paths: int) -> tuple[Digraph, dict]:
    """A weighted trap for path counting: the diamond chain of ``k`` (every
    arc length 1, so x_k has 2^k shortest paths from x_0), then x_k -> p and
    x_k -> q (length 1), p -> t and q -> t (length 10), and ``final_paths``
    vertices z_j with x_k -> z_j (length 2) and z_j -> t (length 1).  Before
    any z_j is settled, t holds the tentative distance d(x_k) + 11 with the
    counts of p and q added together; every z_j then gives t the shorter
    distance d(x_k) + 3, reached only through the z_j.  Ids: the chain's
    (``x``, ``a``, ``b``), then p, q, t and the z_j."""
    g, ids = diamond_chain(k)
    x = ids["x"][k]
    p, q, t = g.n, g.n + 1, g.n + 2
    zs = [g.n + 3 + j for j in range(final_paths)]
    src, dst = [list(a) for a in g.arcs()]
    w = [1] * g.m
    for a, b, ln in [(x, p, 1), (x, q, 1), (p, t, 10), (q, t, 10)]:
        src.append(a), dst.append(b), w.append(ln)
    for z in zs:
        for a, b, ln in [(x, z, 2), (z, t, 1)]:
            src.append(a), dst.append(b), w.append(ln)
    out = from_arcs(g.n + 3 + final_paths, src, dst, w, name=f"supersede{k}_{final_paths}")
    return out, dict(ids, p=p, q=q, t=t, z=zs)


def seeded_subset(count: int, k: int, seed: int, skip: int = 0) -> np.ndarray:
    """Positions ``skip .. skip+k-1`` of a seeded shuffle of ``range(count)``
    (the order of stream ``seed``'s values), ascending: ``k`` distinct
    positions, disjoint from those of any other ``skip`` window."""
    order = np.argsort(stream(seed, 0, count), kind="stable")
    return np.sort(order[skip: skip + k]).astype(np.int64)


def headed_random(n_core: int, heads: int, seed: int, max_weight: int = 0, p_core: float = 0.25) -> Digraph:
    """A small random core (each ordered pair an arc with probability
    ``p_core``) with ``heads`` acyclic pieces hanging off it.  Piece j has
    2-4 vertices h_1.. h_k and an exit core vertex a_j: each h_i has arcs to
    a seeded nonempty subset of {h_i+1 .. h_k, a_j} (h_k always to a_j), so
    every path out of the piece passes a_j; nothing points into a piece
    from outside it.  One extra vertex per piece points to two different
    core vertices (a vertex on no cycle whose paths do not funnel).
    Optional weights uniform in [1, max_weight]."""
    x = unit(stream(seed, 0, n_core * n_core + 32 * heads + 64))
    pos = 0

    def nxt():
        nonlocal pos
        v = float(x[pos])
        pos += 1
        return v

    src, dst = [], []
    for u in range(n_core):
        for v in range(n_core):
            if u != v and nxt() < p_core:
                src.append(u)
                dst.append(v)
    n = n_core
    for _ in range(heads):
        a = int(nxt() * n_core)
        k = 2 + int(nxt() * 3)
        ids = list(range(n, n + k))
        n += k
        for i, h in enumerate(ids):
            later = ids[i + 1:] + [a]
            chosen = [w for w in later if nxt() < 0.5]
            if not chosen or h == ids[-1]:
                chosen = sorted(set(chosen + [later[-1]]))
            for w in chosen:
                src.append(h)
                dst.append(w)
        b = int(nxt() * n_core)
        c = (b + 1 + int(nxt() * (n_core - 1))) % n_core
        src += [n, n]
        dst += [b, c]
        n += 1
    w = None
    if max_weight:
        w = (below(stream(seed + 7, 0, len(src)), max_weight) + np.uint64(1)).astype(np.uint32)
    return from_arcs(n, src, dst, w, name=f"headed{n_core}_{heads}_{seed}")
