"""GPU path vs the CPU oracle, through the C ABI.

Bars: distances and path counts bit-exact; dependencies and BC within
1e-10 relative of the oracle (exactly 0.0 where the oracle gives 0.0);
RV(r) as a set (and ascending list) bit-exact.  Sizes span several
64-source column groups and ragged last groups; the largest cases use the
launch configuration the bench times, compared on sampled sources.
"""
import numpy as np
import pytest

from paper_1708_08739_amd import graphgen as gg

pytestmark = pytest.mark.gpu

REL = 1e-10


def close(a, b, rel=REL):
    """|a - b| <= rel |b| elementwise, and a == 0 exactly where b == 0."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return bool(np.array_equal(a == 0, b == 0) and np.all(np.abs(a - b) <= rel * np.abs(b)))


@pytest.fixture(scope="module")
def B():
    from paper_1708_08739_amd import bcd
    bcd.load()
    return bcd


def dev(B, g, **cfg):
    G = B.Graph.from_digraph(g)
    if cfg:
        G.set_config(**cfg)
    return G


# ------------------------------------------------------------ RV(r)

def test_rv_matches_oracle(B, oracle):
    g, q = gg.rmat16()
    G = dev(B, g)
    for r in q + gg.uniform_vertices(g.n, 6, seed=11, exclude=q):
        print("rv r", r, flush=True)
        got = G.rv(r)
        want = oracle.rv(g, r)
        assert np.array_equal(got, want), r


def test_reach_bottom_up_levels_match_oracle(B, oracle):
    """RV(r) and the forward reach behind K of Eq.(8) on graphs whose large
    levels go bottom-up (frontiers of at least m/64 arcs), both directions,
    against the oracle's plain BFS: R-MAT 18 (weights ignored) and a graph of
    long chains hanging off a dense core, where the frontier shrinks again
    after the bottom-up levels and the traversal switches back."""
    g18, q18 = gg.rmat18_weighted()
    cases = [(g18, q18[:4] + gg.uniform_vertices(g18.n, 4, seed=12, exclude=q18))]
    core = gg.rmat(16, 8, seed=41)
    n0 = core.n
    tails = 8
    src, dst = [], []
    for u in range(n0):
        for e in range(core.row_ptr[u], core.row_ptr[u + 1]):
            src.append(u)
            dst.append(int(core.col[e]))
    # chains of 200 vertices into and out of the core
    nxt = n0
    for t in range(tails):
        prev = t * 97 % n0
        for _ in range(200):
            src.append(nxt)
            dst.append(prev)
            src.append(prev if t % 2 else nxt)
            dst.append(nxt if t % 2 else prev)
            prev = nxt
            nxt += 1
    pairs = sorted(set(zip(src, dst)) - {(a, a) for a in range(nxt)})
    chained = gg.from_arcs(nxt, [a for a, _ in pairs], [b for _, b in pairs], name="core_chains")
    cases.append((chained, gg.top_out_degree(core, 2) + [n0 + 300, n0 + 199, n0 + 200 * 7 + 3]))
    for g, rs in cases:
        G = dev(B, g)
        for r in rs:
            print("reach", g.name, r, flush=True)
            assert np.array_equal(G.rv(r), oracle.rv(g, r)), (g.name, r)
            _, st = G.bc_sampled(r, eps=0.5, seed=3)
            if st["rv_size"] > 0:
                assert st["fr_size"] == oracle.fr_count(g, r), (g.name, r)


def test_rv_small_graphs_one_workgroup(B, oracle):
    """Graphs below 2^16 vertices take the single-workgroup reachability
    kernel; RV(r) and the sampled bound's forward reach (through K) match."""
    cases = [(gg.er_2000()[0], None), (gg.rmat(12, 8, seed=31), None), (gg.directed_path(7), None),
             (gg.Digraph(1, np.array([0, 0]), np.zeros(0, dtype=np.int32)), None)]
    for g, _ in cases:
        G = dev(B, g)
        for r in sorted(set([0, g.n - 1] + gg.uniform_vertices(g.n, min(5, g.n), seed=2))):
            assert np.array_equal(G.rv(r), oracle.rv(g, r)), (g.name, r)
            # the reverse pass of RV and the forward pass of #FR both feed the sampled call
            got, st = G.bc_sampled(r, eps=0.2, seed=5)
            if st["rv_size"] > 0:  # #FR is only computed when there are sources to draw
                assert st["fr_size"] == oracle.fr_count(g, r), (g.name, r)


def test_rv_buffer_too_small(B):
    import ctypes as C
    g = gg.directed_path(10)
    G = dev(B, g)
    out = np.empty(3, dtype=np.int32)
    cnt = C.c_int64()
    rc = B.load().bcd_rv(G.h, 9, out.ctypes.data, 3, C.byref(cnt))
    assert rc == B.BCD_ERR_BUFFER_TOO_SMALL and cnt.value == 9


# ------------------------------------------------- per-source passes

SMALL = [
    ("diamond9", lambda: gg.diamond_chain(9)[0]),
    ("grid12", lambda: gg.grid_right_down(12, 12)),
    ("cycle9", lambda: gg.directed_cycle(9)),
    ("rand40", lambda: gg.random_small(40, 0.08, seed=3)),
    ("er300", lambda: gg.erdos_renyi(300, 1500, seed=9)),
    ("rmat10", lambda: gg.rmat(10, 8, seed=21)),
]


@pytest.mark.parametrize("name,make", SMALL)
@pytest.mark.parametrize("engine", ["batched", "plain", "lds"])
def test_source_pass_bitexact(B, oracle, name, make, engine):
    g = make()
    G = dev(B, g, engine={"plain": B.BCD_ENGINE_PLAIN, "lds": B.BCD_ENGINE_LDS}.get(engine, B.BCD_ENGINE_BATCHED))
    for s in sorted(set([0, g.n - 1] + gg.uniform_vertices(g.n, min(6, g.n - 2), seed=4, exclude=[0, g.n - 1]))):
        print(name, engine, "s", s, flush=True)
        d, sg, dl = G.source_pass(s)
        od, osg, odl, ovf, _ = oracle.source_pass(g, s)
        assert not ovf
        assert np.array_equal(d, od), (name, s)
        assert np.array_equal(sg, osg), (name, s)
        assert close(dl, odl), (name, s, np.max(np.abs(dl - odl)))


@pytest.mark.parametrize("k", [1, 63, 64, 65, 130])
def test_multi_source_pass_groups(B, oracle, k):
    """k sources in one batch: spans 1..3 column groups with a ragged last one."""
    g = gg.rmat(11, 8, seed=5)
    src = gg.uniform_vertices(g.n, k, seed=k)
    want = [oracle.source_pass(g, s) for s in src]
    for items, bu, push in ((1, 0, 0), (2, -1, 0), (4, 0, 0), (1, 4096, 0), (2, 4096, 0), (4, 4096, 0),
                            (1, 0, 1), (2, 0, 1), (4, 0, 1), (2, 4096, 1), (4, 2, 1)):
        G = dev(B, g, groups=3, items=items, bottom_up=bu, push=push)
        print("multi k", k, "items", items, "bottom_up", bu, "push", push, flush=True)
        d, sg, dl = G.multi_source_pass(src)
        for i, s in enumerate(src):
            od, osg, odl, ovf, _ = want[i]
            assert np.array_equal(d[i], od) and np.array_equal(sg[i], osg), (k, items, i, s)
            assert close(dl[i], odl), (k, items, i, s)
    d, sg, dl = dev(B, g, engine=B.BCD_ENGINE_LDS).multi_source_pass(src)
    for i, s in enumerate(src):
        od, osg, odl, ovf, _ = want[i]
        assert np.array_equal(d[i], od) and np.array_equal(sg[i], osg), ("lds", k, i, s)
        assert close(dl[i], odl), ("lds", k, i, s)


def test_push_and_pull_alternate_on_one_workspace(B, oracle):
    """Pulled path counts leave values in the count rows, pushed ones add
    into them: switching the form between calls on one graph (one pooled
    workspace) gives the same bits every time, and the oracle's values."""
    g = gg.rmat(12, 8, seed=19)
    r = gg.top_out_degree(g, 1)[0]
    src = oracle.rv(g, r)[:300]
    want, _ = oracle.dependencies(g, r, src)
    G = dev(B, g, groups=2, bottom_up=0)
    first = G.dependencies(r, src)
    assert close(first, want)
    for push, bu in ((1, 0), (0, 0), (1, 4096), (1, 0), (0, 4096), (1, 2)):
        G.set_config(push=push, bottom_up=bu)
        print("alternate push", push, "bottom_up", bu, flush=True)
        assert np.array_equal(G.dependencies(r, src), first), (push, bu)


def test_partition_count_changes_between_batches(B, oracle):
    """Batches of 1, 2, 8 and 3 groups on one workspace (groups=8): each uses
    min(8, groups used) partitions, so the item-list layout changes from one
    batch to the next, unweighted and weighted."""
    for weighted in (False, True):
        g = gg.rmat(12, 8, seed=21, weighted=weighted, max_weight=20)
        r = gg.top_out_degree(g, 1)[0]
        rv = oracle.rv(g, r)
        G = dev(B, g, groups=8)
        for k in (30, 100, 512, 150, 1):
            src = rv[gg.uniform_vertices(rv.size, min(k, rv.size), seed=k)]
            print("parts weighted", weighted, "k", src.size, flush=True)
            dep = G.dependencies(r, src)
            assert close(dep, oracle.dependencies(g, r, src)[0]), (weighted, k)


def test_counters_match_oracle(B, oracle):
    g = gg.rmat(10, 8, seed=3)
    r = gg.top_out_degree(g, 1)[0]
    src = oracle.rv(g, r)[:20]
    for engine in (B.BCD_ENGINE_BATCHED, B.BCD_ENGINE_PLAIN, B.BCD_ENGINE_LDS):
        G = dev(B, g, engine=engine)
        dep, cnt = G.dependencies(r, src, counters=True)
        odep, ocnt = oracle.dependencies(g, r, src)
        assert np.array_equal(cnt, ocnt)
        assert close(dep, odep)


# -------------------------------------------------------------- BC(r)

def test_bc_exact_er2000_both_engines(B, oracle):
    g, (r,) = gg.er_2000()
    want, ost = oracle.bc_exact(g, r)
    vals = []
    for cfg in [dict(engine=B.BCD_ENGINE_BATCHED, groups=1), dict(engine=B.BCD_ENGINE_BATCHED, groups=5),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=16, block=512),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=2, block=64, grid_mult=1),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=5, items=1),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=5, items=2, block=128),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=3, items=4, grid_mult=1),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=5, bottom_up=0),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=5, bottom_up=4096, items=1),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=7, bottom_up=4096, items=4, block=512),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=2, bottom_up=2, items=2),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=5, push=1),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=3, push=1, items=4, bottom_up=4096),
                dict(engine=B.BCD_ENGINE_BATCHED, groups=16, push=1, block=512, items=1),
                dict(engine=B.BCD_ENGINE_LDS),
                dict(engine=B.BCD_ENGINE_PLAIN)]:
        print("er2000", cfg, flush=True)
        G = dev(B, g, **cfg)
        got, st = G.bc_exact(r)
        assert close(got, want), (cfg, got, want)
        assert st["rv_size"] == ost["rv_size"]
        assert st["traversed_edges"] == ost["te"]
        assert st["reached"] == ost["reached"] and st["dag_arcs"] == ost["dag_arcs"]
        vals.append(got)
    # batched results do not depend on the batch width, the items per step or
    # the direction of the level scans, and the LDS engine gives the same bits
    assert all(v == vals[0] for v in vals[:-1])


def test_autotune_installs_choice_and_keeps_values(B, oracle):
    """The autotuner times engines and settings on a sample of RV(r), installs
    the fastest, and no choice changes a value: BC before and after are equal
    bit for bit (unweighted, where the LDS engine competes, and weighted)."""
    cases = [(gg.er_2000()[0], gg.er_2000()[1][0]),
             (gg.rmat(11, 8, seed=41, weighted=True, max_weight=9), None)]
    for g, r in cases:
        if r is None:
            r = gg.top_out_degree(g, 1)[0]
        G = dev(B, g)
        before, _ = G.bc_exact(r)
        cfg, rate = G.autotune(r, max_groups=4, max_sources=512)
        print("autotune", g.name, cfg.engine, cfg.groups, cfg.block, cfg.grid_mult, cfg.items, cfg.bottom_up, rate,
              flush=True)
        assert rate > 0
        now = G.config()
        assert (now.engine, now.groups, now.block, now.grid_mult, now.items, now.bottom_up) == \
            (cfg.engine, cfg.groups, cfg.block, cfg.grid_mult, cfg.items, cfg.bottom_up)
        after, _ = G.bc_exact(r)
        assert after == before
        assert close(after, oracle.bc_exact(g, r)[0])


def test_bc_exact_repeatable(B):
    g = gg.rmat(12, 8, seed=8)
    G = dev(B, g)
    r = gg.top_out_degree(g, 1)[0]
    a = G.bc_exact(r)[0]
    b = G.bc_exact(r)[0]
    assert a == b


def test_closed_forms(B):
    n = 40
    G = dev(B, gg.directed_path(n))
    for i in range(0, n, 7):
        assert G.bc_exact(i)[0] == i * (n - 1 - i)
    G = dev(B, gg.directed_cycle(17))
    assert G.bc_exact(5)[0] == 16 * 15 / 2
    g, c = gg.in_out_star(7, 5)
    assert dev(B, g).bc_exact(c)[0] == 35.0
    k = 9
    g, ids = gg.diamond_chain(k)
    G = dev(B, g)
    for i in range(1, k):
        assert G.bc_exact(ids["x"][i])[0] == 9 * i * (k - i)
        assert G.bc_exact(ids["a"][i])[0] == (3 * i - 2) * (3 * k - 3 * i + 1) / 2
    G = dev(B, gg.complete_digraph(9))
    v, st = G.bc_exact(3)
    assert v == 0.0 and st["rv_size"] == 8
    G = dev(B, gg.transitive_tournament(12))
    v, st = G.bc_exact(11)
    assert v == 0.0 and st["rv_size"] == -1


def test_degenerate_graphs(B):
    one = gg.Digraph(1, np.array([0, 0]), np.zeros(0, dtype=np.int32))
    G = dev(B, one)
    assert G.bc_exact(0)[0] == 0.0
    assert G.rv(0).size == 0
    empty = gg.Digraph(5, np.zeros(6, dtype=np.int64), np.zeros(0, dtype=np.int32))
    G = dev(B, empty)
    assert G.bc_exact(2)[0] == 0.0 and G.bc_exact(2)[1]["rv_size"] == -1
    # in-degree 0 but out-degree > 0: RV empty
    g = gg.directed_path(6)
    v, st = dev(B, g).bc_exact(0)
    assert v == 0.0 and st["rv_size"] == 0


def test_sigma_overflow(B, oracle):
    g, ids = gg.diamond_chain(63)
    G = dev(B, g)
    assert G.bc_exact(ids["x"][31])[0] == 9 * 31 * 32
    d, sg, _ = G.source_pass(0)
    assert int(sg[ids["x"][63]]) == 1 << 63
    g64, ids64 = gg.diamond_chain(64)
    for cfg in (dict(engine=B.BCD_ENGINE_BATCHED, items=1), dict(engine=B.BCD_ENGINE_BATCHED, items=2),
                dict(engine=B.BCD_ENGINE_BATCHED, items=4), dict(engine=B.BCD_ENGINE_BATCHED, bottom_up=4096),
                dict(engine=B.BCD_ENGINE_BATCHED, push=1, items=1), dict(engine=B.BCD_ENGINE_BATCHED, push=1),
                dict(engine=B.BCD_ENGINE_BATCHED, push=1, items=4, bottom_up=4096),
                dict(engine=B.BCD_ENGINE_PLAIN), dict(engine=B.BCD_ENGINE_LDS)):
        G = dev(B, g64, **cfg)
        with pytest.raises(B.BcdError) as e:
            G.bc_exact(ids64["x"][40])
        assert e.value.code == B.BCD_ERR_SIGMA_OVERFLOW
    # counts on both sides of 2^32 in one batch, and in one (group, vertex)
    # row on different levels (sources at different depths of the chain)
    g40, ids40 = gg.diamond_chain(40)
    src = [ids40["x"][i] for i in (0, 3, 9, 20, 30)] + [ids40["a"][2], ids40["b"][7]]
    want = [oracle.source_pass(g40, s) for s in src]
    for items, bu, push in ((1, 0, 0), (4, 0, 0), (2, 4096, 0), (4, 4096, 0), (2, 0, 1), (4, 4096, 1)):
        d, sg, dl = dev(B, g40, groups=1, items=items, bottom_up=bu, push=push).multi_source_pass(src)
        for i, s in enumerate(src):
            od, osg, odl, ovf, _ = want[i]
            assert np.array_equal(d[i], od) and np.array_equal(sg[i], osg), (items, s)
            assert close(dl[i], odl), (items, s)
    assert int(want[0][1][ids40["x"][40]]) == 1 << 40
    import math
    for engine in (B.BCD_ENGINE_BATCHED, B.BCD_ENGINE_LDS):
        G = dev(B, gg.grid_right_down(35, 35), engine=engine)
        with pytest.raises(B.BcdError) as e:
            G.source_pass(0)
        assert e.value.code == B.BCD_ERR_SIGMA_OVERFLOW
        G = dev(B, gg.grid_right_down(34, 34), engine=engine)
        d, sg, _ = G.source_pass(0)
        assert int(sg[33 * 34 + 33]) == math.comb(66, 33)
    assert dev(B, g, engine=B.BCD_ENGINE_LDS).bc_exact(ids["x"][31])[0] == 9 * 31 * 32


def test_bc_set_and_identity(B, oracle):
    g = gg.rmat(10, 8, seed=23)
    rs = gg.queries_top_and_random(g, seed=9, top=3, rnd=4)
    rs = rs + [rs[1]]
    G = dev(B, g)
    got, st = G.bc_set(rs)
    want, ost = oracle.bc_set(g, rs)
    assert close(got, want)
    assert st["distinct_sources"] == ost["distinct_sources"] and st["traversed_edges"] == ost["te"]
    # sum of BC over all vertices = sum over reachable pairs of (d - 1)
    g2 = gg.erdos_renyi(120, 400, seed=12)
    G2 = dev(B, g2, groups=1)
    allbc, _ = G2.bc_set(list(range(g2.n)))
    obc, _ = oracle.bc_set(g2, list(range(g2.n)))
    assert close(allbc, obc)


def test_lds_engine_queries_and_limits(B, oracle):
    """The LDS engine through the query calls (exact, set, sampled) gives the
    batched engine's values bit for bit; graphs it cannot hold are refused."""
    g = gg.rmat(10, 8, seed=23)
    rs = gg.queries_top_and_random(g, seed=9, top=3, rnd=4)
    Gb = dev(B, g)
    Gl = dev(B, g, engine=B.BCD_ENGINE_LDS)
    sb, stb = Gb.bc_set(rs)
    sl, stl = Gl.bc_set(rs)
    assert np.array_equal(sl, sb) and stl["traversed_edges"] == stb["traversed_edges"]
    assert close(sl, oracle.bc_set(g, rs)[0])
    for r in rs[:3]:
        assert Gl.bc_exact(r)[0] == Gb.bc_exact(r)[0]
        assert Gl.bc_sampled(r, eps=0.05, seed=3)[0] == Gb.bc_sampled(r, eps=0.05, seed=3)[0]

    # 8,000 vertices fit only because sigma and psi share their LDS words
    # (16 n bytes per workgroup rather than 24 n)
    g8 = gg.erdos_renyi(8000, 40000, seed=31)
    r8 = gg.max_in_degree(g8)
    got8, st8 = dev(B, g8, engine=B.BCD_ENGINE_LDS).bc_exact(r8)
    want8, stw8 = dev(B, g8).bc_exact(r8)
    print("lds n=8000", st8["rv_size"], got8, flush=True)
    assert got8 == want8 and st8["traversed_edges"] == stw8["traversed_edges"]

    def with_rv(gx):
        ind, outd = gx.in_degree(), gx.out_degree()
        return next(v for v in gg.top_out_degree(gx, 50) if ind[v] > 0 and outd[v] > 0)

    for gx in (gg.with_weights(gg.erdos_renyi(300, 1500, seed=9), seed=19, max_weight=7), gg.rmat16()[0]):
        Gx = dev(B, gx, engine=B.BCD_ENGINE_LDS)
        with pytest.raises(B.BcdError) as e:
            Gx.bc_exact(with_rv(gx))
        assert e.value.code == B.BCD_ERR_UNSUPPORTED


def test_bc_sampled_matches_oracle(B, oracle):
    g = gg.rmat(12, 8, seed=7)
    r = gg.top_out_degree(g, 1)[0]
    G = dev(B, g)
    for T, seed in [(50, 1), (333, 77), (1, 5)]:
        got, st = G.bc_sampled(r, T=T, seed=seed, flags=B.BCD_NO_EXACT_FALLBACK)
        want, ost = oracle.bc_sampled(g, r, T, seed)
        assert close(got, want), (T, seed)
        assert st["samples"] == T and st["distinct_sources"] == ost["distinct_sources"]
    # Eq.(8) with K = #FR, normalised eps; T >= |RV| falls back to the exact sum
    got, st = G.bc_sampled(r, eps=0.01, delta=0.1, seed=3)
    K = oracle.fr_count(g, r)
    T = oracle.sample_count(0.01 * g.n * (g.n - 1), 0.1, K, st["rv_size"])
    assert st["samples"] == T and st["fr_size"] == K
    if T >= st["rv_size"]:
        assert st["ran_exact"] == 1 and close(got, oracle.bc_exact(g, r)[0])


# ------------------------------------------- full-size R-MAT scale 16

def test_rmat16_sampled_sources_bench_config(B, oracle):
    """R-MAT scale 16, edge factor 8, in the bench's launch configuration:
    per-source dependencies on 96 seeded sources of each query's RV(r)
    (spanning two column groups), and one whole query end to end."""
    g, q = gg.rmat16()
    G = dev(B, g)
    for r in q:
        rv = oracle.rv(g, r)
        if rv.size == 0:
            got, st = G.bc_exact(r)
            assert got == 0.0
            continue
        pick = rv[np.sort(np.unique(gg.below(gg.stream(r, 0, 96), rv.size).astype(np.int64)))]
        print("rmat16 r", r, "sources", pick.size, flush=True)
        dep = G.dependencies(r, pick)
        odep, _ = oracle.dependencies(g, r, pick)
        assert close(dep, odep), r
    r = q[0]
    got, st = G.bc_exact(r)
    want, ost = oracle.bc_exact(g, r)
    assert close(got, want) and st["traversed_edges"] == ost["te"]
    # heavy levels found bottom-up: the same value bit for bit, and the same counters
    got0, st0 = dev(B, g, bottom_up=16).bc_exact(r)
    assert got0 == got and st0["traversed_edges"] == st["traversed_edges"] and st0["dag_arcs"] == st["dag_arcs"]


def test_profile_union_of_launch_intervals(B, oracle):
    """Kernel profile on a query split into many batches (run two at a time on
    two streams when HBM has room): the busy time (union of the launch
    intervals) is positive and never above the summed launch durations, the
    per-kind pair counts match the query's own counters, and profiling leaves
    the value unchanged."""
    g, q = gg.rmat16()
    r = q[0]
    G = dev(B, g, groups=2)
    want, _ = G.bc_exact(r)
    G.profile_reset()
    G.profile_enable(True)
    got, st = G.bc_exact(r)
    G.profile_enable(False)
    assert got == want
    f, b = G.profile(0), G.profile(1)
    print("profile fwd", f, "bwd", b, flush=True)
    for p in (f, b):
        assert p["launches"] > 0 and p["total_ms"] > 0
        assert 0 < p["union_ms"] <= p["total_ms"] * (1 + 1e-9) + 1e-6
    assert f["arc_pairs"] == st["traversed_edges"]
    G.profile_reset()
    z = G.profile(0)
    assert z["launches"] == 0 and z["union_ms"] == 0.0 and z["total_ms"] == 0.0


# ------------------------------------------------------------ weighted

WSMALL = [
    ("rand40w", lambda: gg.random_small(40, 0.1, seed=5, max_weight=3)),
    ("er300w", lambda: gg.with_weights(gg.erdos_renyi(300, 1500, seed=9), seed=19, max_weight=7)),
    ("rmat10w", lambda: gg.with_weights(gg.rmat(10, 8, seed=21), seed=4, max_weight=100)),
    ("grid10w1", lambda: gg.with_unit_weights(gg.grid_right_down(10, 10))),
]


@pytest.mark.parametrize("name,make", WSMALL)
def test_weighted_source_pass_bitexact(B, oracle, name, make):
    g = make()
    G = dev(B, g, groups=2)
    src = sorted(set([0, g.n - 1] + gg.uniform_vertices(g.n, min(70, g.n - 2), seed=6, exclude=[0, g.n - 1])))
    print("weighted", name, len(src), flush=True)
    d, sg, dl = G.multi_source_pass(src)
    for i, s in enumerate(src):
        od, osg, odl, ovf, _ = oracle.source_pass(g, s)
        assert np.array_equal(d[i], od), (name, s)
        assert np.array_equal(sg[i], osg), (name, s)
        assert close(dl[i], odl), (name, s)


def test_weighted_bc_and_counters(B, oracle):
    g = gg.with_weights(gg.rmat(11, 8, seed=13), seed=5, max_weight=100)
    G = dev(B, g)
    for r in gg.queries_top_and_random(g, seed=2, top=2, rnd=3):
        print("weighted bc r", r, flush=True)
        got, st = G.bc_exact(r)
        want, ost = oracle.bc_exact(g, r)
        assert close(got, want), (r, got, want)
        assert st["traversed_edges"] == ost["te"] and st["dag_arcs"] == ost["dag_arcs"]
    rs = gg.top_out_degree(g, 3)
    got, _ = G.bc_set(rs)
    want, _ = oracle.bc_set(g, rs)
    assert close(got, want)
    # unit weights reproduce the unweighted engine exactly
    g1 = gg.with_unit_weights(gg.rmat(10, 8, seed=3))
    g0 = gg.rmat(10, 8, seed=3)
    r = gg.top_out_degree(g0, 1)[0]
    assert dev(B, g1).bc_exact(r)[0] == dev(B, g0).bc_exact(r)[0]


def test_weighted_many_batches_two_streams(B, oracle):
    """A weighted query split into many one-group batches (run two at a time
    on two workspaces and streams when HBM has room): the same value and
    counters as one wide batch, bit for bit, and the oracle's value; the
    kernel profile's busy time stays within the summed launch times."""
    g = gg.with_weights(gg.rmat(11, 8, seed=13), seed=5, max_weight=100)
    r = gg.top_out_degree(g, 1)[0]
    wide, stw = dev(B, g).bc_exact(r)
    G = dev(B, g, groups=1)
    G.profile_reset()
    G.profile_enable(True)
    got, st = G.bc_exact(r)
    G.profile_enable(False)
    want, ost = oracle.bc_exact(g, r)
    print("weighted batches", st["rv_size"], got, want, flush=True)
    assert got == wide and close(got, want)
    assert st["traversed_edges"] == stw["traversed_edges"] == ost["te"]
    rs = gg.top_out_degree(g, 3)
    assert np.array_equal(G.bc_set(rs)[0], dev(B, g).bc_set(rs)[0])
    for p in (G.profile(0), G.profile(1)):
        assert p["launches"] > 0 and 0 < p["union_ms"] <= p["total_ms"] * (1 + 1e-9) + 1e-6


@pytest.mark.parametrize("weighted,bottom_up,push", [(False, 0, 0), (False, 4, 0), (True, 0, 0), (False, 0, 1),
                                                     (False, 4, 1)])
def test_every_source_of_a_many_batch_query(B, oracle, weighted, bottom_up, push):
    """Every source of RV(r) on R-MAT 14 (edge factor 16), elementwise against
    the oracle, in batches of 4 groups (dozens of batches, two at a time on
    two streams), top-down and with bottom-up levels: catches a wrong value on
    any lane of any batch, not only in the sum."""
    g = gg.rmat(14, 16, seed=41, weighted=weighted, max_weight=100)
    r = gg.top_out_degree(g, 1)[0]
    rv = oracle.rv(g, r)
    print("every source weighted", weighted, "bottom_up", bottom_up, "push", push, "sources", rv.size, flush=True)
    dep = dev(B, g, groups=4, bottom_up=bottom_up, push=push).dependencies(r, rv)
    odep, _ = oracle.dependencies(g, r, rv)
    assert close(dep, odep)
    again = dev(B, g, groups=4, bottom_up=bottom_up, push=1 - push).dependencies(r, rv)
    assert np.array_equal(dep, again)


@pytest.mark.parametrize("weighted", [False, True])
def test_concurrent_queries_on_one_graph(B, weighted):
    """Several host threads query one graph at once (every call leases its
    own workspace and stream; ctypes drops the GIL during the call): each
    value equals the one-at-a-time value bit for bit."""
    import threading
    g = gg.rmat(12, 8, seed=21, weighted=weighted, max_weight=20)
    G = dev(B, g, groups=2)  # 128 sources per batch: every query takes several
    rs = gg.top_out_degree(g, 8)
    want = {("e", r): G.bc_exact(r)[0] for r in rs}
    want.update({("s", r): G.bc_sampled(r, T=300, seed=r)[0] for r in rs})
    assert sum(G.bc_exact(r)[1]["rv_size"] > 128 for r in rs) >= 4
    got, errs = {}, []

    def work(part):
        try:
            for r in part:
                got[("e", r)] = G.bc_exact(r)[0]
                got[("s", r)] = G.bc_sampled(r, T=300, seed=r)[0]
        except Exception as e:  # reported by the assertion below
            errs.append(e)

    ts = [threading.Thread(target=work, args=(rs[i::4],)) for i in range(4)]
    for t in ts:
        t.start()
    for t in ts:
        t.join(timeout=100)
    assert not errs, errs
    assert not any(t.is_alive() for t in ts)
    assert got == want


def test_recovers_from_device_allocation_failure(B):
    """A batch width whose path counts fit in HBM but whose psi rows do not
    fails with BCD_ERR_OUT_OF_MEMORY, and what it had allocated is released:
    a width needing most of HBM then succeeds on the same graph and gives the
    right value."""
    import ctypes as C
    # free HBM from the HIP runtime the library itself loaded
    hip_path = next(ln.split()[-1] for ln in open("/proc/self/maps") if "libamdhip64" in ln)
    hip = C.CDLL(hip_path)
    free_b, total_b = C.c_size_t(), C.c_size_t()
    assert hip.hipMemGetInfo(C.byref(free_b), C.byref(total_b)) == 0
    free = free_b.value
    n = 1 << 22
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = 2
    rp[1] = 1  # arcs 0 -> 1 -> 2: BC(1) = 1, RV(1) = {0}
    g = gg.Digraph(n, rp, np.array([1, 2], dtype=np.int32))
    G = dev(B, g, groups=1)
    assert G.bc_exact(1)[0] == 1.0
    row = n * 64 * 8  # one group's path counts (and as much again for psi)
    g_fail = int(0.55 * free) // row  # sigma fits, sigma + psi does not
    g_ok = int(0.60 * free) // (n * 1312)  # every array of the width: fits only if nothing leaked
    assert g_fail * row * 2 > free and g_ok > 8
    G.set_config(groups=g_fail)
    with pytest.raises(B.BcdError) as e:
        G.bc_exact(1)
    assert e.value.code == B.BCD_ERR_OUT_OF_MEMORY
    G.set_config(groups=g_ok)
    assert G.bc_exact(1)[0] == 1.0
    G.set_config(groups=1)
    assert G.bc_exact(1)[0] == 1.0
    G.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_weighted_sigma_overflow(B, oracle, mixed):
    """Exact uint64 path counts and the overflow error of the weighted
    engine.  The weighted diamond chains keep both branches of every diamond
    equally long (all arcs 3, or 1+2 against 2+1 with the two middle
    vertices at different distances): 2^i shortest paths from x_0 to x_i, so
    63 diamonds reach 2^63 exactly and 64 overflow."""
    g63, ids63, span = gg.diamond_chain_weighted(63, mixed)
    G = dev(B, g63)
    d, sg, _ = G.source_pass(0)
    assert int(sg[ids63["x"][63]]) == 1 << 63 and int(d[ids63["x"][63]]) == span * 63
    assert G.bc_exact(ids63["x"][31])[0] == 9 * 31 * 32
    # the plain engine runs a weighted query one source per batch
    assert dev(B, g63, engine=B.BCD_ENGINE_PLAIN).bc_exact(ids63["x"][31])[0] == 9 * 31 * 32
    g64, ids64, _ = gg.diamond_chain_weighted(64, mixed)
    for cfg in (dict(), dict(engine=B.BCD_ENGINE_PLAIN)):
        G = dev(B, g64, **cfg)
        with pytest.raises(B.BcdError) as e:
            G.bc_exact(ids64["x"][40])
        assert e.value.code == B.BCD_ERR_SIGMA_OVERFLOW, cfg
    with pytest.raises(B.BcdError) as e:
        G.source_pass(0)
    assert e.value.code == B.BCD_ERR_SIGMA_OVERFLOW
    # counts on both sides of 2^32 in one batch, sources at different depths
    g40, ids40, _ = gg.diamond_chain_weighted(40, mixed)
    src = [ids40["x"][i] for i in (0, 3, 9, 20, 30)] + [ids40["a"][2], ids40["b"][7]]
    want = [oracle.source_pass(g40, s) for s in src]
    for cfg in (dict(groups=1), dict(engine=B.BCD_ENGINE_PLAIN)):
        d, sg, dl = dev(B, g40, **cfg).multi_source_pass(src)
        for i, s in enumerate(src):
            od, osg, odl, ovf, _ = want[i]
            assert not ovf
            assert np.array_equal(d[i], od) and np.array_equal(sg[i], osg), (cfg, s)
            assert close(dl[i], odl), (cfg, s)
        assert int(sg[0][ids40["x"][40]]) == 1 << 40


def test_weighted_superseded_tie_is_not_overflow(B, oracle):
    """The weighted trap graph: t first gets a tentative distance from p and q
    whose path counts (2^63 each) would wrap, then a shorter distance through
    z with 2^63 paths.  Only final counts matter: the weighted engine, batched
    and one source per batch, returns the oracle's distances and counts bit
    for bit and BC(z) = 190; with a second z the 2^64 final paths of t are an
    overflow on both engines."""
    g, ids = gg.superseded_tie_chain(63, 1)
    od, osg, odl, ovf, _ = oracle.source_pass(g, 0)
    assert not ovf
    src = [0, ids["a"][1], ids["x"][40], ids["p"], ids["z"][0]]
    want = [oracle.source_pass(g, s) for s in src]
    for cfg in (dict(groups=1), dict(groups=2, block=256), dict(engine=B.BCD_ENGINE_PLAIN)):
        print("supersede", cfg, flush=True)
        G = dev(B, g, **cfg)
        d, sg, dl = G.source_pass(0)
        assert np.array_equal(d, od) and np.array_equal(sg, osg), cfg
        assert int(sg[ids["t"]]) == 1 << 63 and close(dl, odl), cfg
        md, msg, mdl = G.multi_source_pass(src)
        for i, s in enumerate(src):
            assert np.array_equal(md[i], want[i][0]) and np.array_equal(msg[i], want[i][1]), (cfg, s)
            assert close(mdl[i], want[i][2]), (cfg, s)
        assert G.bc_exact(ids["z"][0])[0] == 190.0 == oracle.bc_exact(g, ids["z"][0])[0]
    g2, ids2 = gg.superseded_tie_chain(63, 2)
    for cfg in (dict(groups=1), dict(engine=B.BCD_ENGINE_PLAIN)):
        G = dev(B, g2, **cfg)
        with pytest.raises(B.BcdError) as e:
            G.bc_exact(ids2["z"][0])
        assert e.value.code == B.BCD_ERR_SIGMA_OVERFLOW, cfg


@pytest.mark.parametrize("weighted", [False, True])
def test_compression_folds_leaf_sources(B, oracle, weighted):
    """Compression on (sources with no in-arcs and one out-arc take their
    successor's dependency, or its reach count when the successor is the
    target): exact and set values match the oracle and the uncompressed run,
    with fewer sources run; queries include successors of such sources."""
    g = gg.rmat(12, 8, seed=8, weighted=weighted, max_weight=50)
    ind, outd = g.in_degree(), g.out_degree()
    leaves = np.flatnonzero((ind == 0) & (outd == 1))
    succ = sorted(set(int(g.col[g.row_ptr[s]]) for s in leaves))
    qs = gg.queries_top_and_random(g, seed=4, top=4, rnd=4) + [v for v in succ if outd[v] > 0][:4]
    G0, G1 = dev(B, g), dev(B, g, compress=1)
    fewer = 0
    for r in qs:
        a, sa = G0.bc_exact(r)
        b, sb = G1.bc_exact(r)
        want, _ = oracle.bc_exact(g, r)
        print("compress r", r, sa["distinct_sources"], sb["distinct_sources"], a, b, flush=True)
        assert close(b, want) and close(b, a), (r, a, b, want)
        assert sb["distinct_sources"] <= sa["distinct_sources"]
        fewer += sb["distinct_sources"] < sa["distinct_sources"]
    assert fewer > 0
    assert close(G1.bc_set(qs)[0], oracle.bc_set(g, qs)[0])
    # in-out star: every in-leaf is folded, BC(c) = a * b exactly
    gs, c = gg.in_out_star(5, 7)
    got, st = dev(B, gs, compress=1).bc_exact(c)
    assert got == 35.0 and st["distinct_sources"] == 0


@pytest.mark.parametrize("weighted", [False, True])
def test_compression_gates_of_acyclic_pieces(B, oracle, weighted):
    """Sources in acyclic pieces that funnel into one vertex (gated sources
    with several out-arcs, chains) fold into that vertex: exact and set
    values equal the oracle's and the uncompressed run's, targets include
    the pieces' exits and vertices inside pieces (whose pieces then run)."""
    g = gg.headed_random(300, 60, seed=17, max_weight=20 if weighted else 0, p_core=0.012)
    n_core = 300
    outd = g.out_degree()
    exits = sorted({int(g.col[e]) for v in range(n_core, g.n) for e in range(g.row_ptr[v], g.row_ptr[v + 1])
                    if g.col[e] < n_core})
    inside = [v for v in range(n_core, g.n) if outd[v] > 0][:3]
    qs = exits[:6] + gg.uniform_vertices(n_core, 4, seed=5) + inside
    G0, G1 = dev(B, g, groups=2), dev(B, g, groups=2, compress=1)
    folded = 0
    for r in qs:
        a, sa = G0.bc_exact(r)
        b, sb = G1.bc_exact(r)
        want, _ = oracle.bc_exact(g, r)
        print("gates r", r, sa["distinct_sources"], sb["distinct_sources"], a, b, flush=True)
        assert close(b, want) and close(b, a), (r, a, b, want)
        folded += sa["distinct_sources"] - sb["distinct_sources"]
    assert folded > 20
    assert close(G1.bc_set(qs)[0], oracle.bc_set(g, qs)[0])


def test_bcd_procedure_and_unpruned_sampling(B, oracle):
    g = gg.rmat(12, 8, seed=7)
    G = dev(B, g)
    r = gg.top_out_degree(g, 1)[0]
    k = len(oracle.rv(g, r))
    for tau, seed in [(k, 3), (k - 1, 3), (50, 11)]:
        got, st = G.bc_bcd(r, tau=tau, seed=seed)
        want, ex = oracle.bc_bcd(g, r, tau, seed)
        assert close(got, want) and bool(st["ran_exact"]) == ex, (tau, got, want)
    got, st = G.bc_sampled(r, T=64, seed=5, flags=B.BCD_SAMPLE_ALL_VERTICES)
    assert close(got, oracle.bc_sampled_all(g, r, 64, 5)) and st["rv_size"] == g.n - 1


# ------------------------------------ full-size workloads, sampled sources

def _sampled_parity(B, oracle, g, r, nsrc, seed, **cfg):
    G = dev(B, g, **cfg)
    rv = G.rv(r)
    assert np.array_equal(rv, oracle.rv(g, r))
    pick = rv[np.sort(np.unique(gg.below(gg.stream(seed, 0, nsrc), rv.size).astype(np.int64)))]
    dep, cnt = G.dependencies(r, pick, counters=True)
    odep, ocnt = oracle.dependencies(g, r, pick)
    assert close(dep, odep)
    assert np.array_equal(cnt, ocnt)
    return G, rv


def _full_width(B, g, r, rv, tracked, seed, width):
    """Dependencies of the tracked sources computed inside one batch of the
    full width: the list is padded with further seeded sources of RV(r)
    (positions disjoint from the tracked ones) up to `width`, then the
    tracked sources' results are picked out."""
    pad = rv[gg.seeded_subset(rv.size, max(0, width - tracked.size), seed, skip=tracked.size)]
    allsrc = np.concatenate([tracked, pad]).astype(np.int32)
    assert allsrc.size == min(width, rv.size) and np.unique(allsrc).size == allsrc.size
    return allsrc, tracked.size


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    src = np.array([int(x[0]) for x in rows], dtype=np.int32)
    dep = np.array([float.fromhex(x[1]) for x in rows])
    cnt = np.array([[int(x[2]), int(x[3]), int(x[4])] for x in rows], dtype=np.uint64)
    return src, dep, cnt


def test_rmat18_weighted_full_width(B, oracle):
    """R-MAT scale 18, edge factor 16, weights in [1,100], in the bench's
    width of 128 column groups: 1,024 seeded sources of RV(r) against the
    oracle inside one batch of 8,192 (the rest seeded padding from RV(r)),
    and again in a narrow batch."""
    g, q = gg.rmat18_weighted()
    r = q[0]
    G = dev(B, g, groups=128)
    rv = G.rv(r)
    assert np.array_equal(rv, oracle.rv(g, r))
    tracked = rv[gg.seeded_subset(rv.size, 1024, 18)]
    allsrc, k = _full_width(B, g, r, rv, tracked, 18, 128 * 64)
    print("rmat18w full width", g.m, allsrc.size, flush=True)
    dep, cnt = G.dependencies(r, allsrc, counters=True)
    odep, ocnt = oracle.dependencies(g, r, tracked)
    assert close(dep[:k], odep) and np.array_equal(cnt[:k], ocnt)
    assert np.array_equal(dev(B, g, groups=4).dependencies(r, tracked[:256]), dep[:256])


def test_rmat20_full_width(B):
    """R-MAT scale 20, edge factor 16, a giant-class vertex, in the bench's
    batch (64 column groups, 8 XCD partitions, bottom-up levels on): 1,024
    seeded sources of RV(r) padded to 4,096 with further RV sources, against
    the oracle's dependencies and pass counters stored by
    tests/golden/make_fullwidth_deps.py."""
    g = gg.rmat20()
    r = gg.top_out_degree(g, 1)[0]
    src, odep, ocnt = _golden("rmat20_fullwidth_deps.txt")
    G = dev(B, g)
    cfg = G.config()
    assert cfg.groups == 64 and cfg.bottom_up == 4
    rv = G.rv(r)
    assert np.array_equal(src, rv[gg.seeded_subset(rv.size, 1024, 2020)])
    allsrc, k = _full_width(B, g, r, rv, src, 2020, 64 * 64)
    print("rmat20 full width", g.m, allsrc.size, flush=True)
    dep, cnt = G.dependencies(r, allsrc, counters=True)
    assert close(dep[:k], odep)
    assert np.array_equal(cnt[:k], ocnt)
    # top-down levels only, and pushed path counts: the same bits
    assert np.array_equal(dev(B, g, bottom_up=0).dependencies(r, allsrc)[:k], dep[:k])
    assert np.array_equal(dev(B, g, push=1).dependencies(r, allsrc)[:k], dep[:k])


def test_rmat20_dag_set_uneven(B, oracle):
    """The acyclic R-MAT 20 set of 64 vertices with |RV(r)| spread from 15 to
    1e5 (the bench's set, listed with the oracle's |RV| sizes): the GPU's RV
    sizes equal the stored ones, the set call's values equal the oracle's
    set values on every member with |RV| <= 100, and the largest member's
    dependencies on sampled sources equal the oracle's."""
    import os
    g = gg.rmat20_dag()
    path = os.path.join(os.path.dirname(__file__), "golden", "rmat20_dag_set64.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    qs = [int(x[0]) for x in rows]
    sizes = [int(x[1]) for x in rows]
    print("rmat20 dag", g.m, "set of", len(qs), flush=True)
    G = dev(B, g)
    assert [len(G.rv(r)) for r in qs] == sizes
    bcs, st = G.bc_set(qs)
    small = [i for i, sz in enumerate(sizes) if sz <= 100]
    want, _ = oracle.bc_set(g, [qs[i] for i in small])
    assert close(bcs[small], want)
    assert np.all(np.isfinite(bcs)) and np.all(bcs >= 0)
    _sampled_parity(B, oracle, g, qs[int(np.argmax(sizes))], 16, 2020)


def test_rmat22_full_width_and_draws(B, oracle):
    """R-MAT scale 22, edge factor 16: 1,024 seeded sources of RV(r) (one
    full batch of the default 16 column groups, 8 partitions, bottom-up
    levels on) against the oracle's stored dependencies and counters, the
    same sources in the serving width (3 groups per batch), and an A-BCD
    call whose draws the oracle recomputes."""
    g = gg.rmat22()
    r = gg.top_out_degree(g, 1)[0]
    src, odep, ocnt = _golden("rmat22_fullwidth_deps.txt")
    print("rmat22", g.m, flush=True)
    G = dev(B, g)
    cfg = G.config()
    assert cfg.groups == 16 and cfg.bottom_up == 4
    rv = G.rv(r)
    assert np.array_equal(rv, oracle.rv(g, r))
    assert np.array_equal(src, rv[gg.seeded_subset(rv.size, 1024, 2022)])
    dep, cnt = G.dependencies(r, src, counters=True)
    assert close(dep, odep)
    assert np.array_equal(cnt, ocnt)
    G3 = dev(B, g, groups=3)
    assert np.array_equal(G3.dependencies(r, src[:384]), dep[:384])
    G3.set_config(push=1)
    assert np.array_equal(G3.dependencies(r, src[:384]), dep[:384])
    got, st = G.bc_sampled(r, T=12, seed=7, flags=B.BCD_NO_EXACT_FALLBACK)
    want, ost = oracle.bc_sampled(g, r, 12, 7)
    assert close(got, want) and st["distinct_sources"] == ost["distinct_sources"]
