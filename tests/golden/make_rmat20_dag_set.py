"""Writes rmat20_dag_set64.txt: the 64-vertex query set of the R-MAT 20 DAG
workload, chosen so that |RV(r)| spans 10 .. 1e5.

Only the CPU oracle computes here.  A seeded pool of vertices with in- and
out-arcs is drawn (stream 114); RV(r) of each is computed with the oracle;
for each of 64 targets spaced evenly in log10 over [1, 5], in order, the
unused pool vertex whose |RV| is nearest to the target in log scale is taken
(ties to the smaller id).  Run from the repository root:

    python3 tests/golden/make_rmat20_dag_set.py
"""
import math
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_1708_08739_amd import graphgen as gg  # noqa: E402
from oracle import oracle as O  # noqa: E402

POOL = 4000
_G = None


def _init():
    global _G
    _G = gg.rmat20_dag()


def _rv_size(r):
    return int(O.rv(_G, int(r)).size)


def main():
    g = gg.rmat20_dag()
    indeg = np.bincount(g.col, minlength=g.n)
    outdeg = np.diff(g.row_ptr)
    ok = np.flatnonzero((indeg > 0) & (outdeg > 0))
    pool = np.unique(ok[gg.below(gg.stream(114, 0, POOL), ok.size).astype(np.int64)])
    with Pool(8, initializer=_init) as p:
        sizes = np.array(p.map(_rv_size, pool.tolist(), chunksize=16), dtype=np.int64)
    used = np.zeros(pool.size, dtype=bool)
    logs = np.log10(np.maximum(sizes, 1).astype(np.float64))
    rows = []
    for t in np.linspace(1.0, 5.0, 64):
        d = np.where(used | (sizes == 0), np.inf, np.abs(logs - t))
        i = int(np.lexsort((pool, d))[0])
        used[i] = True
        rows.append((int(pool[i]), int(sizes[i]), float(10 ** t)))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmat20_dag_set64.txt")
    with open(out, "w") as f:
        f.write("# Query set of the R-MAT 20 DAG workload (graphgen.rmat20_dag: R-MAT scale 20,\n"
                "# edge factor 16, seed 4, arcs turned by the ranking of stream 14).\n"
                f"# Pool: {pool.size} distinct vertices with in- and out-arcs (stream 114); |RV(r)| by the\n"
                "# CPU oracle (RV as the set of vertices with a path to r, r excluded);\n"
                "# written by make_rmat20_dag_set.py.\n"
                "# Format: r  |RV(r)|  target\n")
        for r, sz, t in rows:
            f.write(f"{r} {sz} {t:.1f}\n")
    print(out, [s for _, s, _ in rows])


if __name__ == "__main__":
    main()
