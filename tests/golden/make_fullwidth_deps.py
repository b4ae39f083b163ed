"""Writes the expected per-source dependencies of the full-width parity
tests: 1,024 seeded sources of RV(r) for the vertex r of largest out-degree
on the R-MAT scale 20 and scale 22 workloads (edge factor 16), each with
delta_s.(r) as a hexadecimal double and the pass counters (n_s, m_s, a_s).

Calls only the CPU oracle and the input generator.  Run from the repository
root:  python tests/golden/make_fullwidth_deps.py [scale ...]
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1708_08739_amd import graphgen as gg  # noqa: E402

TRACKED = 1024
SEEDS = {20: 2020, 22: 2022}


def graph(scale):
    return gg.rmat20() if scale == 20 else gg.rmat22()


def main(scales):
    for scale in scales:
        g = graph(scale)
        r = gg.top_out_degree(g, 1)[0]
        rv = O.rv(g, r)
        src = rv[gg.seeded_subset(rv.size, TRACKED, SEEDS[scale])]
        t0 = time.time()
        dep, cnt = O.dependencies(g, r, src, threads=os.cpu_count())
        path = os.path.join(HERE, f"rmat{scale}_fullwidth_deps.txt")
        with open(path, "w") as f:
            f.write(f"# R-MAT scale {scale}, edge factor 16 ({g.name}): r = {r} (largest out-degree), "
                    f"|RV(r)| = {rv.size}\n")
            f.write(f"# {TRACKED} sources of RV(r) at positions gg.seeded_subset(|RV|, {TRACKED}, {SEEDS[scale]})\n")
            f.write("# source  delta_s.(r) as float.hex  n_s  m_s  a_s   (CPU oracle)\n")
            for s, d, c in zip(src.tolist(), dep.tolist(), cnt.tolist()):
                f.write(f"{s} {float(d).hex()} {c[0]} {c[1]} {c[2]}\n")
        print(f"scale {scale}: r={r} |RV|={rv.size} {TRACKED} sources in {time.time() - t0:.1f} s -> {path}",
              flush=True)


if __name__ == "__main__":
    main([int(x) for x in sys.argv[1:]] or [20, 22])
