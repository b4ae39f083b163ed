"""Seeded inputs: the acyclic R-MAT variant and the stored query set of the
acyclic R-MAT 20 workload (CPU only)."""
import os

import numpy as np

from paper_1708_08739_amd import graphgen as gg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_rmat_orientation_is_acyclic_and_keeps_pairs():
    n = 1 << 10
    g = gg.rmat(10, 16, seed=4, orient_seed=14)
    h = gg.rmat(10, 16, seed=4)
    src, dst = g.arcs()
    key = gg.stream(14, 0, n)
    # every arc climbs the ranking (key, then id): no cycle is possible
    up = (key[src] < key[dst]) | ((key[src] == key[dst]) & (src < dst))
    assert up.all()
    # the same unordered vertex pairs as the unturned graph
    a, b = h.arcs()
    pairs = lambda u, v: np.unique(np.minimum(u, v) * n + np.maximum(u, v))
    assert np.array_equal(pairs(src, dst), pairs(a, b))
    assert g.m == pairs(a, b).size


def test_dag_set_list(oracle):
    rows = [ln.split() for ln in open(os.path.join(GOLD, "rmat20_dag_set64.txt"))
            if ln.strip() and not ln.startswith("#")]
    qs = [int(x[0]) for x in rows]
    sizes = [int(x[1]) for x in rows]
    assert len(qs) == 64 and len(set(qs)) == 64
    assert min(sizes) <= 20 and max(sizes) >= 90000
    g = gg.rmat20_dag()
    for i in (0, 31, 63):
        assert oracle.rv(g, qs[i]).size == sizes[i]


def test_native_rmat_draws_equal_numpy():
    """The C form of the R-MAT quadrant draws gives the NumPy form's values
    bit for bit (scales and seeds of several workloads, other thresholds)."""
    from paper_1708_08739_amd import build
    if not os.path.exists(build.GEN_LIB):
        build.build_gen()
    for scale, ef, seed, abcd in ((10, 8, 3, gg.RMAT_ABCD), (13, 16, 4, gg.RMAT_ABCD), (12, 8, 2, (0.45, 0.15, 0.15, 0.25))):
        a = gg.rmat_draws(scale, ef << scale, seed, abcd, native=True)
        b = gg.rmat_draws(scale, ef << scale, seed, abcd, native=False)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]), (scale, seed)
