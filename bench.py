#!/usr/bin/env python3
"""Benchmark: RV(r)-pruned betweenness of single vertices on one MI355X.

Default workload: serving sampled BC(r) queries (Alg.2, T from Eq.(8) with
eps = 0.01 normalised, delta = 0.1, K = the vertices r reaches, seeded
draws) on a directed R-MAT scale 22 graph (4,194,304 vertices, edge factor
16, a,b,c,d = .57,.19,.19,.05, seeded relabelling, repeats and self-loops
dropped, unweighted), CSR and transpose resident in HBM, through the
library's server with a 64 GB HBM budget.  Query vertices are seeded
uniform vertices with in- and out-arcs.  One step = 25 queries: the K
steps' queries (500 at K = 20) are all submitted at once to a warm server
and the timed region ends when the last one is reduced on the host, so
the region is the saturation run; step i ends when 25 * i queries are
done.  Then the same queries arrive as a Poisson process at 0.5x and 0.9x
the measured saturation rate (p50/p99 latency from arrival to result).

value = whole-job GTEPS = traversed arcs (sum of m_s over every source pass
the server ran) / wall time of the timed region.

Other workloads (--workload): rmat16 (R-MAT 16, edge factor 8, 8 exact
queries, one step = the 8 queries), er2000 (ER n=2,000, m=10,000, one
exact query; LDS engine), rmat18w (weighted R-MAT 18), rmat20set (set of
64 vertices on R-MAT 20), rmat20dagset (set of 64 vertices with |RV(r)|
spread from 15 to 1e5 on an acyclic R-MAT 20), rmat16bcd (the paper's BCD
procedure and the unpruned sampling baseline on R-MAT 16, per query),
oracle (the CPU oracle alone on the host cores: the ER 2,000 and R-MAT 16
queries in full, seeded samples of R-MAT 18 weighted, 20 and 22 queries
with extrapolated full-query times, and one-thread rates).

The JSON line also carries the forward kernels' HBM roofline figures, the
plain one-source-per-launch engine on a sample of sources, and the CPU
oracle timed on a bounded sample of the same work.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, each scaled by what it reads for a copy kernel of known size),
# valid only while the sources of the kernels hash to the recorded value.
TRAFFIC_FILES = {"k_fwd_level": ["profiles/k_fwd_level_rmat16_ef8.md"],
                 "k_fwd_level+k_bu_level": ["profiles/k_fwd_level_rmat22_serving.md",
                                            "profiles/k_fwd_level_rmat20_set.md"],
                 "k_w_relax+k_w_count+k_w_sigma": ["profiles/k_w_kernels_rmat18w.md"]}
_CSRC = "paper_1708_08739_amd/csrc/"
_UNWEIGHTED_SOURCES = [_CSRC + "bcd_kernels.hip", _CSRC + "bcd_device.h", _CSRC + "bcd_internal.h"]
_WEIGHTED_SOURCES = [_CSRC + "bcd_weighted.hip", _CSRC + "bcd_device.h", _CSRC + "bcd_internal.h"]


def kernel_sources(kernel: str) -> list[str]:
    return _WEIGHTED_SOURCES if kernel.startswith("k_w_") else _UNWEIGHTED_SOURCES


def kernel_sources_sha256(kernel: str = "k_fwd_level") -> str:
    import hashlib
    h = hashlib.sha256()
    for f in kernel_sources(kernel):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload_name: str, batch_width: int):
    """Counter-measured HBM bytes per launch of `kernel` on `workload_name` at
    `batch_width` sources per batch, or None when none were taken at that
    width or the kernel sources changed since."""
    rec = {}
    for path in TRAFFIC_FILES.get(kernel, []):
        if not os.path.exists(os.path.join(ROOT, path)):
            continue
        with open(os.path.join(ROOT, path)) as fh:
            for line in fh:
                if line.startswith("traffic:"):
                    parts = dict(kv.split("=", 1) for kv in line[len("traffic:"):].split())
                    if (parts.get("kernel") == kernel and parts.get("workload") == workload_name
                            and parts.get("batch_width") == str(batch_width)):
                        rec = parts
    if not rec or rec.get("sources_sha256") != kernel_sources_sha256(kernel):
        return None
    return float(rec["bytes_per_launch"])


def roofline_from_profile(G, fwd: dict, bwd: dict, ename: str, wname: str, batch_width: int | None = None,
                          probe_gbs: float | None = None, bottom_up: bool = False,
                          probe_copy_gbs: float | None = None):
    """HBM roofline of the dominant pass from the library's kernel profile.

    Bytes: the per-source model (32 per (source, vertex) + 8 per (source,
    arc) + 8 per (source, DAG arc) in each pass), and the schedule-aware
    model that counts the graph structure once per work item (64 sources of
    a column group at one vertex and level).  Time: launches of concurrent
    batches overlap on their streams, so `achieved` and `frac` divide by the
    union of the launch intervals (each instant counted once); the
    per-launch figures divide by the summed durations.  `traffic` is the
    counter-measured HBM bytes per launch recorded in profiles/ for this
    workload and width, or None.  `probe_gbs` is the measured streaming-read
    bandwidth (the traversal kernels' traffic is mostly reads), the
    achievable reference for the probe-relative fractions."""
    if fwd["launches"] == 0:
        return None
    dom, kind = (fwd, "forward") if fwd["total_ms"] >= bwd["total_ms"] else (bwd, "backward")
    busy_ms = dom["union_ms"] if dom["union_ms"] > 0 else dom["total_ms"]
    achieved = dom["alg_bytes"] / (busy_ms * 1e-3) / 1e9
    per_launch = dom["alg_bytes"] / (dom["total_ms"] * 1e-3) / 1e9
    sched = dom.get("sched_bytes", 0.0) or 0.0
    if G.info()[2]:
        # weighted engine: the forward is three kernels (relaxation rounds, DAG
        # in-degrees, topological rounds), profiled together
        kname = "k_w_relax+k_w_count+k_w_sigma" if kind == "forward" else "k_w_bwd"
    elif ename == "lds":
        kname = "k_lds_pass"  # both passes in one kernel, timed as the forward
    elif kind == "forward" and bottom_up:
        kname = "k_fwd_level+k_bu_level"  # a level found bottom-up runs both, timed as two launches
    else:
        kname = f"k_{'fwd' if kind == 'forward' else 'bwd'}_level"
    if batch_width is None:
        batch_width = 64 * G.config().groups if ename == "batched" else 1
    traffic = measured_traffic(kname, wname, batch_width)
    per_launch_s = dom["total_ms"] * 1e-3 / dom["launches"]
    out = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4),
           "traffic": None if traffic is None else round(traffic, 1),
           "kernel": kname,
           "launches": dom["launches"], "avg_launch_us": round(per_launch_s * 1e6, 2),
           "alg_bytes_per_launch": round(dom["alg_bytes"] / dom["launches"], 1),
           "launch_union_ms": round(busy_ms, 3), "launch_sum_ms": round(dom["total_ms"], 3),
           "per_launch_achieved": round(per_launch, 2),
           "per_launch_frac": round(per_launch / HBM_PEAK_GBS, 4),
           "lanes_per_item": round(dom["vertex_pairs"] / dom["items"], 2) if dom["items"] else None}
    if sched > 0:
        out["sched_bytes_per_launch"] = round(sched / dom["launches"], 1)
        out["sched_achieved"] = round(sched / (busy_ms * 1e-3) / 1e9, 2)
        out["sched_frac"] = round(out["sched_achieved"] / HBM_PEAK_GBS, 4)
    if traffic is not None:
        # counter bytes per launch over the per-launch time, and over the busy
        # time (the launches of one timed region, overlapping)
        out["traffic_achieved"] = round(traffic * dom["launches"] / (busy_ms * 1e-3) / 1e9, 2)
        out["traffic_frac"] = round(out["traffic_achieved"] / HBM_PEAK_GBS, 4)
    if probe_gbs:
        out["probe_read_gbs"] = round(probe_gbs, 1)
        out["probe_frac"] = round(achieved / probe_gbs, 4)
        if sched > 0:
            out["sched_probe_frac"] = round(out["sched_achieved"] / probe_gbs, 4)
        if traffic is not None:
            out["traffic_probe_frac"] = round(out["traffic_achieved"] / probe_gbs, 4)
    if probe_copy_gbs:
        out["probe_copy_gbs"] = round(probe_copy_gbs, 1)
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    from paper_1708_08739_amd import graphgen as gg
    if name == "rmat16":
        g, q = gg.rmat16()
        return g, q, "rmat16_ef8_8queries_exact"
    if name == "er2000":
        g, q = gg.er_2000()
        return g, q, "er_n2000_m10000_maxindeg_exact"
    if name == "rmat18w":
        g, q = gg.rmat18_weighted()
        return g, q, "rmat18_ef16_w1-100_8queries_exact"
    if name == "rmat20set":
        return gg.rmat20(), None, "rmat20_ef16_set64_exact"
    if name == "rmat20dagset":
        return gg.rmat20_dag(), dag_set_queries(), "rmat20_ef16_dag_set64_uneven_exact"
    if name == "rmat22serve":
        return gg.rmat22(), None, "rmat22_ef16_serving_sampled"
    if name == "rmat16bcd":
        g, _ = gg.rmat16()
        return g, None, "rmat16_ef8_bcd_procedure_64queries"
    raise SystemExit(f"unknown workload {name}")


def dag_set_queries() -> list[int]:
    """The 64 query vertices of the acyclic R-MAT 20 set: |RV(r)| log-spaced
    over 15 .. 1e5 (chosen once on the CPU, list stored with its sizes)."""
    path = os.path.join(ROOT, "tests", "golden", "rmat20_dag_set64.txt")
    with open(path) as fh:
        return [int(line.split()[0]) for line in fh if line.strip() and not line.startswith("#")]


def run_weighted(G, g, queries, args):
    """R-MAT scale 18, edge factor 16, weights in [1,100]: the four top
    out-degree vertices through one set call (they share RV), the others
    one exact call each."""
    if not args.no_autotune:
        # batch width from {32, 64, 128, 256} column groups (and launch shape),
        # timed on 16,384 sources of the first query, before the timed region
        cfg, rate = G.autotune(queries[0], max_groups=256, max_sources=16384)
        log(f"[bench] autotune: groups={cfg.groups} block={cfg.block} grid_mult={cfg.grid_mult} ({rate:.2f} GTEPS)")
        G.profile_reset()
    t0 = time.perf_counter()
    bcs, st = G.bc_set(queries[:4])
    te = st["traversed_edges"]
    lat = [time.perf_counter() - t0]
    for r in queries[4:]:
        t = time.perf_counter()
        bc, s2 = G.bc_exact(r)
        lat.append(time.perf_counter() - t)
        te += s2["traversed_edges"]
    wall = time.perf_counter() - t0
    return te, wall, lat


def select_uneven(G, g, k: int, seed: int, lo=10, hi=100000):
    """k query vertices whose |RV(r)| is closest to k log-spaced targets in
    [lo, hi], from a seeded pool of vertices with in- and out-degree > 0."""
    from paper_1708_08739_amd import graphgen as gg
    ind, outd = g.in_degree(), g.out_degree()
    cand = [v for v in gg.uniform_vertices(g.n, 4000, seed=seed) if ind[v] > 0 and outd[v] > 0][:1500]
    sizes = {}
    for v in cand:
        sizes[v] = len(G.rv(v))
    targets = np.logspace(np.log10(lo), np.log10(hi), k)
    chosen = []
    for t in targets:
        best = min((v for v in cand if v not in chosen), key=lambda v: (abs(np.log(max(sizes[v], 1)) - np.log(t)), v))
        chosen.append(best)
    return chosen, [sizes[v] for v in chosen]


def serving_queries(g, count: int, seed: int) -> list[int]:
    """`count` seeded uniform vertices with in- and out-arcs."""
    from paper_1708_08739_amd import graphgen as gg
    ind, outd = g.in_degree(), g.out_degree()
    pool = [v for v in gg.uniform_vertices(g.n, 20 * count + 100, seed=seed) if ind[v] > 0 and outd[v] > 0]
    if len(pool) < count:
        raise SystemExit("not enough query vertices")
    return pool[:count]


def hbm_free_bytes() -> int:
    import torch
    free, _ = torch.cuda.mem_get_info()
    return int(free)


def serve_bench(args):
    """The serving workload: see the module docstring.  Prints the JSON line."""
    import torch
    from paper_1708_08739_amd import bcd, graphgen as gg
    t_start = time.perf_counter()
    g = gg.rmat22()
    log(f"[bench] R-MAT 22 generated: n={g.n} m={g.m} ({time.perf_counter() - t_start:.1f} s)")
    G = bcd.Graph.from_digraph(g)
    kw = config_overrides(args)
    if kw:
        G.set_config(**kw)
    cfg = G.config()
    K, W, Q = args.steps, args.warmup, args.queries_per_step
    qs = serving_queries(g, K * Q, seed=105)
    warm = serving_queries(g, max(W * Q, 1), seed=106)[: W * Q]
    if args.hbm_budget_gb > 0:
        budget = int(args.hbm_budget_gb * 1e9)
    else:  # all free HBM but 8 GB
        budget = hbm_free_bytes() - (8 << 30)
    groups = args.groups or serving_width(lambda gr: bcd.Server.workspace_bytes(G, gr, args.workers), 96, budget)
    log(f"[bench] serving: {args.workers} workers x {groups} groups, HBM budget {budget / 1e9:.1f} GB, "
        f"{K} steps x {Q} queries, {W} warm-up steps")
    S = bcd.Server(G, workers=args.workers, groups=groups, hbm_budget_bytes=budget)

    def submit_all(vertices, seed0, gaps=None):
        """Submit every query (at the given arrival gaps), return the results."""
        t0 = time.perf_counter()
        arrive = 0.0
        tickets = {}
        for i, r in enumerate(vertices):
            if gaps is not None:
                arrive += gaps[i]
                while True:
                    rem = arrive - (time.perf_counter() - t0)
                    if rem <= 0:
                        break
                    time.sleep(min(0.001, rem))
            tickets[S.submit(bcd.BCD_QUERY_SAMPLED, r=r, eps=0.01, delta=0.1, seed=seed0 + i)] = i
        return t0, tickets

    def drain(tickets, step_every=0):
        res = []
        done_steps = 0
        while len(res) < len(tickets):
            res += S.poll(timeout_s=1.0)
            while step_every and len(res) >= (done_steps + 1) * step_every:
                done_steps += 1
                log(f"[bench] step {done_steps}/{len(tickets) // step_every} done")
        bad = [x for x in res if x["status"] != bcd.BCD_OK]
        if bad:
            raise SystemExit(f"serving: {len(bad)} queries failed: {bad[0]}")
        return res

    if W > 0:
        _, tk = submit_all(warm, 905)
        drain(tk)
        log(f"[bench] warm-up: {W} steps ({len(warm)} queries) done")
    probe = probe_copy = None
    if not args.no_probe:
        probe_copy = bcd.bcd_bandwidth_probe(4 << 30, 5)
        probe = bcd.bcd_read_bandwidth_probe(4 << 30, 5)
        log(f"[bench] probes: copy {probe_copy:.1f} GB/s (4 GiB read + 4 GiB written per launch), "
            f"read {probe:.1f} GB/s (4 GiB per launch)")
    if not args.no_profile:
        G.profile_reset()
        G.profile_enable(True)
    st0 = S.stats()
    torch.cuda.synchronize()
    t0, tk = submit_all(qs, 305)
    res = drain(tk, step_every=Q)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    G.profile_enable(False)
    st1 = S.stats()
    te = st1["traversed_edges"] - st0["traversed_edges"]
    lat = np.array([x["t_done_s"] - x["t_arrive_s"] for x in res]) * 1e3
    qps = len(qs) / wall
    sat = {"queries": len(qs), "wall_s": round(wall, 3), "qps": round(qps, 3), "gteps": round(te / wall / 1e9, 3),
           "p50_ms": round(float(np.percentile(lat, 50)), 2), "p99_ms": round(float(np.percentile(lat, 99)), 2),
           "samples_mean": float(np.mean([x["stats"]["samples"] for x in res])),
           "distinct_sources_mean": float(np.mean([x["stats"]["distinct_sources"] for x in res])),
           "exact_fallbacks": int(sum(x["stats"]["ran_exact"] for x in res)),
           "batches": st1["batches"] - st0["batches"],
           "lane_occupancy": round((st1["lanes_used"] - st0["lanes_used"]) /
                                   max(st1["lane_slots"] - st0["lane_slots"], 1), 3),
           "shared_lanes": st1["shared_lanes"] - st0["shared_lanes"]}
    log(f"[bench] saturation: {sat}")
    roof = None
    if not args.no_profile:
        roof = roofline_from_profile(G, G.profile(0), G.profile(1), "batched", traffic_key_serving(args),
                                     batch_width=64 * groups, probe_gbs=probe, bottom_up=cfg.bottom_up > 0,
                                     probe_copy_gbs=probe_copy)
        log(f"[bench] roofline: {roof}")
    poisson = {}
    if not args.no_poisson:
        for frac in (0.5, 0.9):
            rate = frac * qps
            u = gg.unit(gg.stream(205, 0, len(qs)))
            gaps = list(-np.log1p(-u) / rate)
            a = S.stats()
            tp0, tk = submit_all(qs, 305, gaps)
            r2 = drain(tk)
            w2 = time.perf_counter() - tp0
            b = S.stats()
            l2 = np.array([x["t_done_s"] - x["t_arrive_s"] for x in r2]) * 1e3
            poisson[f"poisson_{frac}"] = {
                "rate_qps": round(rate, 3), "wall_s": round(w2, 3), "qps": round(len(qs) / w2, 3),
                "gteps": round((b["traversed_edges"] - a["traversed_edges"]) / w2 / 1e9, 3),
                "p50_ms": round(float(np.percentile(l2, 50)), 2), "p99_ms": round(float(np.percentile(l2, 99)), 2)}
            log(f"[bench] Poisson arrivals at {frac} x saturation: {poisson[f'poisson_{frac}']}")
    S.close()
    plain = None
    if args.plain_sources > 0:
        plain = plain_form(G, g, qs[0], min(args.plain_sources, 16))
        log(f"[bench] plain engine: {plain}")
    cpu = None
    if not args.no_cpu:
        from oracle import oracle as O
        rv = O.rv(g, qs[0])
        idx = [int(gg.below(np.array([x], dtype=np.uint64), rv.size)[0]) for x in gg.stream(305, 0, 1024)]
        src = rv[np.unique(np.array(idx, dtype=np.int64))] if rv.size else rv
        cpu = cpu_baseline(g, qs[0], src, args.cpu_budget, args.cpu_threads,
                           f"distinct drawn sources of the first query (r = {qs[0]}, |RV| = {rv.size}, "
                           f"seed 305 draws)")
        log(f"[bench] cpu baseline: {cpu}")
    out = {
        "metric": "GTEPS for RV(r)-pruned BC(r) on one MI355X; p50/p99 query latency",
        "value": round(te / wall / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(wall * 1e3 / K, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64+f64",
        "data": "synthetic",
        "config": {"workload": wname_serving(args), "graph": g.name, "n": g.n, "m": g.m,
                   "queries": len(qs), "queries_per_step": Q, "query": "sampled eps=0.01 (normalised) delta=0.1",
                   "hbm_budget_gb": round(budget / 1e9, 1), "workers": args.workers, "groups": groups,
                   "batch_width": 64 * groups, "block": cfg.block, "grid_mult": cfg.grid_mult, "items": cfg.items,
                   "bottom_up": cfg.bottom_up, "push": cfg.push},
        "qps": sat["qps"],
        "p50_query_ms": sat["p50_ms"],
        "p99_query_ms": sat["p99_ms"],
        "traversed_edges": int(te),
        "saturation": sat,
        **poisson,
        "plain_form": plain,
        "roofline": roof,
        "cpu_baseline": cpu,
        "bench_wall_s": round(time.perf_counter() - t_start, 1),
    }
    print(json.dumps(out), flush=True)


def wname_serving(args) -> str:
    budget = f"{args.hbm_budget_gb:g}GB" if args.hbm_budget_gb > 0 else "freeHBM"
    return f"rmat22_ef16_serving_sampled_{args.steps * args.queries_per_step}q_{budget}"


def traffic_key_serving(args) -> str:
    """Workload key of counter-measured traffic: the batches do not depend on
    how many queries a run serves, only on the graph, the query kind and the
    width (which the lookup also matches)."""
    budget = f"{args.hbm_budget_gb:g}GB" if args.hbm_budget_gb > 0 else "freeHBM"
    return f"rmat22_ef16_serving_sampled_{budget}"


def plain_form(G, g, r, nsrc):
    """The plain engine (one source per launch, one launch per BFS level) on
    the first sources of RV(r)."""
    from paper_1708_08739_amd import bcd
    rv = G.rv(r)
    src = rv[:nsrc]
    if src.size == 0:
        return None
    old = G.config().engine
    G.set_config(engine=bcd.BCD_ENGINE_PLAIN)
    G.dependencies(r, src[:2])
    t = time.perf_counter()
    G.dependencies(r, src)
    dt = time.perf_counter() - t
    G.set_config(engine=old)
    _, cnt = G.dependencies(r, src, counters=True)
    te_p = int(cnt[:, 1].sum())
    return {"gteps": round(te_p / dt / 1e9, 3), "sources": int(src.size), "query": int(r)}


def bcd_procedure(G, g, args):
    """The paper's experimental procedure (Section 5) on R-MAT 16: for 64
    seeded query vertices with in- and out-arcs, BCD with tau = 1000 (exact
    when |RV(r)| <= tau, else A-BCD with T = tau), reporting t_RV, t, exact or
    not, and Error% = |BCD - BC| / BC x 100 against the exact value (Eq.(9));
    then, at equal eps = 0.01 (normalised) and delta = 0.1, A-BCD drawing
    from RV(r) against the unpruned baseline drawing from V (sample count
    from Eq.(8) with n - 1 in place of |RV(r)|)."""
    from paper_1708_08739_amd import bcd, graphgen as gg
    ind, outd = g.in_degree(), g.out_degree()
    nq = args.max_queries or 64
    pool = [v for v in gg.uniform_vertices(g.n, 40 * nq, seed=106) if ind[v] > 0 and outd[v] > 0]
    qs = pool[:nq]
    rows = []
    te_bcd = 0
    t_bcd = 0.0
    for i, r in enumerate(qs):
        exact, _ = G.bc_exact(r)
        t0 = time.perf_counter()
        v, st = G.bc_bcd(r, tau=1000, seed=1000 + i)
        dt = time.perf_counter() - t0
        te_bcd += st["traversed_edges"]
        t_bcd += dt
        err = abs(v - exact) / exact * 100.0 if exact != 0 else (0.0 if v == 0 else float("inf"))
        row = {"r": int(r), "rv": int(st["rv_size"]), "exact": bool(st["ran_exact"]), "t_rv_ms": round(st["t_rv_s"] * 1e3, 3),
               "t_ms": round(st["t_bc_s"] * 1e3, 3), "error_pct": round(err, 4)}
        if st["rv_size"] > 1000:
            # equal eps, delta: pruned draws from RV(r), unpruned from V
            a, sa = G.bc_sampled(r, eps=0.01, delta=0.1, seed=2000 + i, flags=bcd.BCD_NO_EXACT_FALLBACK)
            b, sb = G.bc_sampled(r, eps=0.01, delta=0.1, seed=2000 + i, flags=bcd.BCD_SAMPLE_ALL_VERTICES)
            row["pruned"] = {"T": int(sa["samples"]), "t_ms": round(sa["t_bc_s"] * 1e3, 3),
                             "error_pct": round(abs(a - exact) / exact * 100.0, 4) if exact else None}
            row["unpruned"] = {"T": int(sb["samples"]), "t_ms": round(sb["t_bc_s"] * 1e3, 3),
                               "error_pct": round(abs(b - exact) / exact * 100.0, 4) if exact else None}
        rows.append(row)
        log(f"[bench] bcd query {i + 1}/{len(qs)}: {row}")
    ex = [x for x in rows if x["exact"]]
    ap_ = [x for x in rows if not x["exact"]]
    big = [x for x in rows if "pruned" in x]
    summary = {
        "queries": len(rows), "pct_exact": round(100.0 * len(ex) / max(len(rows), 1), 2),
        "mean_error_pct_sampled": round(float(np.mean([x["error_pct"] for x in ap_])), 4) if ap_ else None,
        "max_error_pct_sampled": round(float(np.max([x["error_pct"] for x in ap_])), 4) if ap_ else None,
        "mean_t_rv_ms": round(float(np.mean([x["t_rv_ms"] for x in rows])), 3),
        "mean_t_ms": round(float(np.mean([x["t_ms"] for x in rows])), 3),
        "pruned_vs_unpruned": {
            "mean_T": [round(float(np.mean([x["pruned"]["T"] for x in big])), 1),
                       round(float(np.mean([x["unpruned"]["T"] for x in big])), 1)] if big else None,
            "mean_t_ms": [round(float(np.mean([x["pruned"]["t_ms"] for x in big])), 3),
                          round(float(np.mean([x["unpruned"]["t_ms"] for x in big])), 3)] if big else None,
            "mean_error_pct": [round(float(np.mean([x["pruned"]["error_pct"] for x in big])), 4),
                               round(float(np.mean([x["unpruned"]["error_pct"] for x in big])), 4)] if big else None,
        },
    }
    return te_bcd, t_bcd, summary, rows


def cpu_info() -> dict:
    """Model, cores, hardware threads and clock of the host CPU (lscpu)."""
    import subprocess
    info = {"threads": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {a.strip(): b.strip() for a, b in (ln.split(":", 1) for ln in out.splitlines() if ":" in ln)}
        info["model"] = kv.get("Model name")
        sockets = int(kv.get("Socket(s)", "1") or 1)
        cores = int(kv.get("Core(s) per socket", "0") or 0)
        info["cores"] = sockets * cores if cores else None
        info["threads_per_core"] = kv.get("Thread(s) per core")
        info["max_mhz"] = kv.get("CPU max MHz")
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    try:
        # the clock the kernel reports for the first CPU (when lscpu gives no maximum)
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("cpu MHz"):
                    info["mhz"] = float(ln.split(":", 1)[1])
                    break
    except (OSError, ValueError):
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except OSError:
        pass
    return info


def cpu_baseline(g, r, src, budget_s: float, threads: int, what: str):
    """The oracle as it stands, on a bounded sample of the same work: the
    per-source passes of `src` (sources of one query of the workload), in
    chunks until about `budget_s` seconds have been spent, on `threads` host
    threads (0: every thread this process may use, at most 64), then again on
    one thread for a fifth of the budget."""
    from oracle import oracle as O
    info = cpu_info()
    if threads <= 0:
        threads = max(1, min(info.get("affinity") or os.cpu_count() or 1, 64))

    def rate(nthreads, budget):
        te = 0
        done = 0
        t0 = time.perf_counter()
        chunk = max(1, 2 * nthreads)
        while time.perf_counter() - t0 < budget and done < src.size:
            part = src[done:done + chunk]
            _, cnt = O.dependencies(g, r, part, threads=nthreads)
            te += int(cnt[:, 1].sum())
            done += part.size
            chunk = min(chunk * 2, 8192)
        return te, done, time.perf_counter() - t0

    te, done, dt = rate(threads, budget_s)
    te1, done1, dt1 = rate(1, max(5.0, budget_s / 4))
    return {"value": te / dt / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{done} {what}, per-source passes, {te} traversed arcs in {dt:.1f} s on {threads} threads",
            "one_thread_gteps": te1 / dt1 / 1e9,
            "one_thread_sample": f"{done1} of the same sources, {te1} traversed arcs in {dt1:.1f} s",
            "cpu": info}


def seeded_rv_sources(g, r):
    """RV(r) in a seeded order (the CPU baseline's sample of a query)."""
    from oracle import oracle as O
    from paper_1708_08739_amd import graphgen as gg
    rv = O.rv(g, r)
    return rv[np.argsort(gg.stream(12345, 0, rv.size), kind="stable")]


def config_overrides(args) -> dict:
    kw = {}
    if args.groups and args.workload != "rmat22serve":
        kw["groups"] = args.groups
    if args.block:
        kw["block"] = args.block
    if args.grid_mult:
        kw["grid_mult"] = args.grid_mult
    if args.items:
        kw["items"] = args.items
    if args.bottom_up >= 0:
        kw["bottom_up"] = args.bottom_up
    if args.compress:
        kw["compress"] = 1
    if args.push >= 0:
        kw["push"] = args.push
    return kw


def oracle_timing(args):
    """The CPU oracle on the host cores alone (no GPU), per workload: the
    ER 2,000 query and the 8 R-MAT 16 queries run in full on every thread;
    for R-MAT 18 weighted, 20 and 22 a seeded sample of sources of the
    largest-out-degree vertex's RV(r) is timed and the full query's time is
    extrapolated from the sample's traversed-arc rate (labelled as such).
    Every workload also gets a one-thread rate on a sample.  The RV(r)
    search is outside the timed window (as t_BC excludes t_RV)."""
    from oracle import oracle as O
    from paper_1708_08739_amd import graphgen as gg
    info = cpu_info()
    threads = args.cpu_threads or max(1, min(info.get("affinity") or os.cpu_count() or 1, 64))
    out = {"kind": "oracle_timing", "cpu": info, "threads": threads, "workloads": {}}

    def timed(g, r, src, nthreads):
        t0 = time.perf_counter()
        _, cnt = O.dependencies(g, r, src, threads=nthreads)
        dt = time.perf_counter() - t0
        return int(cnt[:, 1].sum()), dt

    def one_thread(g, r, rv, budget):
        te = 0
        done = 0
        t0 = time.perf_counter()
        order = rv[np.argsort(gg.stream(777, 0, rv.size), kind="stable")]
        while time.perf_counter() - t0 < budget and done < order.size:
            part = order[done:done + 4]
            a, _ = timed(g, r, part, 1)
            te += a
            done += part.size
        dt = time.perf_counter() - t0
        return {"gteps": te / dt / 1e9, "sources": done, "traversed_edges": te, "seconds": round(dt, 2)}

    full = [("er2000", *gg.er_2000()), ("rmat16", *gg.rmat16())]
    for name, g, qs in full:
        te = 0
        dt = 0.0
        for r in qs:
            rv = O.rv(g, r)
            if rv.size == 0:
                continue
            a, b = timed(g, r, rv, threads)
            te += a
            dt += b
            log(f"[oracle] {name} r={r} |RV|={rv.size} {a} arcs in {b:.1f} s")
        big = max(qs, key=lambda r: O.rv(g, r).size)
        out["workloads"][name] = {"queries": len(qs), "full_run": True, "traversed_edges": te,
                                  "seconds": round(dt, 3), "gteps": te / dt / 1e9 if dt else None,
                                  "one_thread": one_thread(g, big, O.rv(g, big), args.cpu_budget / 4)}
    samp = [("rmat18w", gg.rmat18_weighted()[0]), ("rmat20", gg.rmat20()), ("rmat22", gg.rmat22())]
    for name, g in samp:
        r = gg.top_out_degree(g, 1)[0]
        rv = O.rv(g, r)
        src = rv[gg.seeded_subset(rv.size, min(args.oracle_sample, rv.size), 4242)]
        a, b = timed(g, r, src, threads)
        rate = a / b
        per_source = a / src.size
        est_s = per_source * rv.size / rate
        log(f"[oracle] {name} r={r} |RV|={rv.size}: {src.size} sources, {a} arcs in {b:.1f} s")
        out["workloads"][name] = {"query": int(r), "rv_size": int(rv.size), "sample_sources": int(src.size),
                                  "sample_traversed_edges": a, "sample_seconds": round(b, 3),
                                  "gteps": rate / 1e9,
                                  "extrapolated_full_query_seconds": round(est_s, 1),
                                  "extrapolated": "full-query time = |RV| x mean arcs per sampled source / sample rate",
                                  "one_thread": one_thread(g, r, rv, args.cpu_budget / 4)}
    if args.oracle_full:
        # full runs where a query finishes within minutes: the top R-MAT 18
        # weighted query (every source of RV(r)) and the first serving queries
        # of R-MAT 22 with the server's draws (the same seeds, T from Eq.(8))
        g = gg.rmat18_weighted()[0]
        r = gg.top_out_degree(g, 1)[0]
        rv = O.rv(g, r)
        # in 16 slices of RV(r), so that progress shows while it runs
        a = 0
        b = 0.0
        for k, part in enumerate(np.array_split(rv, 16)):
            x, y = timed(g, r, part, threads)
            a += x
            b += y
            log(f"[oracle] rmat18w full query r={r}: slice {k + 1}/16 done, {a} arcs in {b:.1f} s")
        out["workloads"]["rmat18w"]["full_query"] = {"traversed_edges": a, "seconds": round(b, 3),
                                                     "gteps": a / b / 1e9}
        g = gg.rmat22()
        qs = serving_queries(g, args.oracle_full_queries, seed=105)
        rows = []
        for i, r in enumerate(qs):
            rvr = O.rv(g, r)
            T = O.sample_count(0.01 * g.n * (g.n - 1), 0.1, O.fr_count(g, r), rvr.size)
            t0 = time.perf_counter()
            bc, st = O.bc_sampled(g, r, T, 305 + i, threads=threads)
            dt = time.perf_counter() - t0
            te = int(st["te"])
            rows.append({"r": int(r), "rv_size": int(rvr.size), "T": int(T), "traversed_edges": te,
                         "seconds": round(dt, 3), "gteps": te / dt / 1e9})
            log(f"[oracle] rmat22 serving query {i} r={r} T={T}: {te} arcs in {dt:.1f} s")
        out["workloads"]["rmat22"]["serving_queries_full"] = rows
    print(json.dumps(out), flush=True)


def serving_width(workspace_bytes, start: int, budget: int) -> int:
    """Largest group count <= start whose workspaces (workspace_bytes(groups),
    all workers) fit in 85 % of the budget (the rest holds the queries'
    result buffers) and that splits evenly over the 8 XCD partitions (at most
    8 groups, or a multiple of 8): group g goes to partition g % 8, so 9
    groups would leave one partition twice the work.  At least 1."""
    groups = max(1, start)
    while groups > 1 and (workspace_bytes(groups) > budget * 85 // 100 or (groups > 8 and groups % 8 != 0)):
        groups -= 1
    return groups


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="rmat22serve",
                    choices=["rmat22serve", "rmat16", "er2000", "rmat18w", "rmat20set", "rmat20dagset", "rmat16bcd",
                             "oracle"])
    ap.add_argument("--groups", type=int, default=0, help="64-source column groups per batch (0 = library default)")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--grid-mult", type=int, default=0)
    ap.add_argument("--items", type=int, default=0, help="frontier items per wavefront step (0 = library default)")
    ap.add_argument("--bottom-up", type=int, default=-1,
                    help="bottom-up threshold denominator for the unweighted forward (0 = off, -1 = library default)")
    ap.add_argument("--push", type=int, default=-1,
                    help="unweighted forward: 1 = add path counts along DAG arcs, 0 = pull them over in-arcs, "
                         "-1 = library default")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (0 = every thread this process may use, at most 64)")
    ap.add_argument("--compress", action="store_true",
                    help="exact and set calls fold sources with no in-arcs and one out-arc into their successor")
    ap.add_argument("--engine", choices=["auto", "batched", "lds", "plain"], default="auto",
                    help="per-source engine (auto: the LDS engine for the ER 2k workload, else batched)")
    ap.add_argument("--plain-sources", type=int, default=256)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="rmat20set: autotune the configuration first")
    ap.add_argument("--no-autotune", action="store_true",
                    help="rmat18w: keep the library's default width instead of autotuning it")
    ap.add_argument("--queries-per-step", type=int, default=25, help="serving: sampled queries per step")
    ap.add_argument("--workers", type=int, default=3, help="serving: concurrent batches")
    ap.add_argument("--hbm-budget-gb", type=float, default=64.0,
                    help="serving: HBM budget in GB (1e9 bytes) for workspaces and query buffers; 0 = all free HBM but 8 GiB")
    ap.add_argument("--no-poisson", action="store_true", help="serving: skip the Poisson-arrival runs")
    ap.add_argument("--no-probe", action="store_true", help="serving: skip the streaming-copy probe")
    ap.add_argument("--set-size", type=int, default=64)
    ap.add_argument("--max-queries", type=int, default=0,
                    help="rmat16, rmat18w, er2000: run only the first N query vertices (profiling runs)")
    ap.add_argument("--oracle-sample", type=int, default=512,
                    help="oracle workload: sources timed per large query (extrapolated to the full query)")
    ap.add_argument("--oracle-full", action="store_true",
                    help="oracle workload: also run the top R-MAT 18 weighted query and the first serving "
                         "queries of R-MAT 22 in full")
    ap.add_argument("--oracle-full-queries", type=int, default=4,
                    help="oracle workload with --oracle-full: R-MAT 22 serving queries run in full")
    ap.add_argument("--probe-bw", action="store_true",
                    help="also run the library's streaming-copy probe (4 GiB copied, known traffic)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the whole path on a single MI355X "
              "(multi-GPU source sharding is designed but not built); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload == "rmat22serve":
        serve_bench(args)
        return
    if args.workload == "oracle":
        oracle_timing(args)
        return

    import torch
    from paper_1708_08739_amd import bcd

    g, queries, wname = workload(args.workload)
    if args.max_queries > 0 and queries is not None and len(queries) > args.max_queries:
        queries = queries[: args.max_queries]
        wname += f"_first{args.max_queries}"
    log(f"[bench] workload {wname}: n={g.n} m={g.m} queries={queries}")
    G = bcd.Graph.from_digraph(g)
    kw = config_overrides(args)
    engines = {"batched": bcd.BCD_ENGINE_BATCHED, "lds": bcd.BCD_ENGINE_LDS, "plain": bcd.BCD_ENGINE_PLAIN}
    ename = args.engine if args.engine != "auto" else ("lds" if args.workload == "er2000" else "batched")
    cfg = G.set_config(engine=engines[ename], **kw)
    log(f"[bench] config groups={cfg.groups} block={cfg.block} grid_mult={cfg.grid_mult}")

    if args.workload in ("rmat18w", "rmat20set", "rmat20dagset", "rmat16bcd"):
        extra = {}
        if not args.no_profile:
            G.profile_reset()
            G.profile_enable(True)
        if args.workload == "rmat18w":
            te, wall, lat = run_weighted(G, g, queries, args)
        elif args.workload == "rmat20set":
            qs, sizes = select_uneven(G, g, args.set_size, seed=104)
            log(f"[bench] set of {len(qs)}: |RV| from {min(sizes)} to {max(sizes)}")
            if args.autotune:
                c2, rate = G.autotune(qs[int(np.argmax(sizes))], max_groups=8, max_sources=2048)
                log(f"[bench] autotune: groups={c2.groups} ({rate:.2f} GTEPS)")
                G.profile_reset()
            t0 = time.perf_counter()
            bcs, st = G.bc_set(qs)
            wall = time.perf_counter() - t0
            te, lat = st["traversed_edges"], [wall]
            extra = {"set_size": len(qs), "rv_sizes": sizes, "distinct_sources": st["distinct_sources"]}
        elif args.workload == "rmat20dagset":
            qs = queries
            sizes = [len(G.rv(r)) for r in qs]
            log(f"[bench] set of {len(qs)}: |RV| from {min(sizes)} to {max(sizes)}")
            G.bc_set(qs[:8])  # warm-up: workspace and hub signatures
            G.profile_reset()
            lat = []
            te = 0
            t0 = time.perf_counter()
            for i in range(args.steps):
                t = time.perf_counter()
                bcs, st = G.bc_set(qs)
                lat.append(time.perf_counter() - t)
                te += st["traversed_edges"]
                log(f"[bench] step {i + 1}/{args.steps} done")
            wall = time.perf_counter() - t0
            extra = {"set_size": len(qs), "rv_sizes": sizes, "distinct_sources": st["distinct_sources"],
                     "steps": args.steps, "bc_first": [float(x) for x in bcs[:4]]}
        else:
            te, wall, summary, rows = bcd_procedure(G, g, args)
            lat = [x["t_ms"] / 1e3 for x in rows]
            extra = {"bcd_procedure": summary, "per_query": rows}
        bw = bwr = None
        if not args.no_profile:
            G.profile_enable(False)
        if args.probe_bw:
            bw = round(bcd.bcd_bandwidth_probe(4 << 30, 5), 1)
            bwr = round(bcd.bcd_read_bandwidth_probe(4 << 30, 5), 1)
            log(f"[bench] probes: copy {bw} GB/s (4 GiB read + 4 GiB written per launch), read {bwr} GB/s")
        if not args.no_profile:
            extra["roofline"] = roofline_from_profile(G, G.profile(0), G.profile(1), ename, wname,
                                                      bottom_up=G.config().bottom_up > 0, probe_gbs=bwr,
                                                      probe_copy_gbs=bw)
            log(f"[bench] roofline: {extra['roofline']}")
        if not args.no_cpu:
            # the oracle on a bounded sample of one query's sources: for the set,
            # its largest RV; for serving, the first query vertex
            if args.workload == "rmat18w":
                rq = queries[0]
            elif args.workload in ("rmat20set", "rmat20dagset"):
                rq = qs[int(np.argmax(sizes))]
            else:
                rq = max(rows, key=lambda x: x["rv"])["r"]
            extra["cpu_baseline"] = cpu_baseline(g, rq, seeded_rv_sources(g, rq), args.cpu_budget,
                                                 args.cpu_threads, f"seeded sources of RV({rq})")
            log(f"[bench] cpu baseline: {extra['cpu_baseline']}")
        cfg = G.config()
        # one timed step is the whole workload (rmat20dagset: --steps calls)
        nsteps = args.steps if args.workload == "rmat20dagset" else 1
        conf = {"workload": wname, "graph": g.name, "n": g.n, "m": g.m, "engine": ename,
                "batch_width": 64 * cfg.groups, "groups": cfg.groups, "block": cfg.block,
                "grid_mult": cfg.grid_mult, "items": cfg.items, "bottom_up": cfg.bottom_up, "compress": cfg.compress}
        if args.workload == "rmat18w":
            conf["autotuned"] = not args.no_autotune
        extra.pop("steps", None)
        print(json.dumps({"metric": "GTEPS for RV(r)-pruned BC(r) on one MI355X; p50/p99 query latency",
                          "value": round(te / wall / 1e9, 3), "unit": "GTEPS", "n_gpus": 1,
                          "steps": nsteps, "warmup": 0, "ms_per_step": round(wall * 1e3 / nsteps, 3),
                          "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64+f64",
                          "data": "synthetic", "workload": wname, "wall_s": round(wall, 3),
                          "traversed_edges": int(te), "latencies_s": [round(x, 4) for x in lat][:16],
                          "config": conf, **extra}), flush=True)
        return

    def step(lat=None):
        te = 0
        for r in queries:
            t = time.perf_counter()
            bc, st = G.bc_exact(r)
            if lat is not None:
                lat.append(time.perf_counter() - t)
            te += st["traversed_edges"]
        return te

    for i in range(args.warmup):
        step()
        log(f"[bench] warmup {i + 1}/{args.warmup} done")
    if not args.no_profile:
        G.profile_reset()
        G.profile_enable(True)
    torch.cuda.synchronize()
    lat: list[float] = []
    te_total = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        te_total += step(lat)
        log(f"[bench] step {i + 1}/{args.steps} done")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    G.profile_enable(False)
    fwd = G.profile(0)
    bwd = G.profile(1)

    bw = bwr = None
    if args.probe_bw:
        bw = round(bcd.bcd_bandwidth_probe(4 << 30, 5), 1)
        bwr = round(bcd.bcd_read_bandwidth_probe(4 << 30, 5), 1)
        log(f"[bench] probes: copy {bw} GB/s (4 GiB read + 4 GiB written per launch), read {bwr} GB/s")
    roofline = None if args.no_profile else roofline_from_profile(G, fwd, bwd, ename, wname, probe_gbs=bwr,
                                                                  bottom_up=G.config().bottom_up > 0,
                                                                  probe_copy_gbs=bw)

    # plain one-source-per-launch form on a sample of the same sources
    plain = None
    if args.plain_sources > 0:
        plain = plain_form(G, g, queries[0], args.plain_sources)
        log(f"[bench] plain engine: {plain}")

    cpu = None
    if not args.no_cpu:
        r = queries[0]
        cpu = cpu_baseline(g, r, seeded_rv_sources(g, r), args.cpu_budget, args.cpu_threads,
                           f"seeded sources of RV({r})")
        log(f"[bench] cpu baseline: {cpu}")

    lat_ms = np.array(lat) * 1e3
    value = te_total / wall / 1e9
    out = {
        "metric": "GTEPS for RV(r)-pruned BC(r) on one MI355X; p50/p99 query latency",
        "value": round(value, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64+f64",
        "data": "synthetic",
        "config": {"workload": wname, "graph": g.name, "n": g.n, "m": g.m, "queries": [int(q) for q in queries],
                   "engine": ename, "batch_width": 64 * cfg.groups if ename == "batched" else 1, "block": cfg.block,
                   "grid_mult": cfg.grid_mult, "items": cfg.items, "bottom_up": cfg.bottom_up, "compress": cfg.compress},
        "p50_query_ms": round(float(np.percentile(lat_ms, 50)), 3),
        "p99_query_ms": round(float(np.percentile(lat_ms, 99)), 3),
        "traversed_edges_per_step": te_total // args.steps,
        "plain_form": plain,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if bw is not None:
        out["copy_probe_gbs"] = bw
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
