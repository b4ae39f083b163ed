"""Serving loop on the GPU: every result equals the standalone call bit for
bit, whether the query runs alone or mixed with others arriving while
batches run; set and sampled queries; budget admission; errors."""
import time

import numpy as np
import pytest

from paper_1708_08739_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1708_08739_amd import bcd
    bcd.load()
    return bcd


def drain(S, n, timeout=120.0):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in S.poll(timeout_s=1.0):
            got[r["ticket"]] = r
        assert time.time() - t0 < timeout, "server did not finish"
    return got


@pytest.mark.parametrize("weighted", [False, True])
def test_server_mixed_equals_alone(B, oracle, weighted):
    g = gg.rmat(12, 8, seed=8, weighted=weighted, max_weight=50)
    G = B.Graph.from_digraph(g)
    G.set_config(groups=2)
    qs = gg.queries_top_and_random(g, seed=4, top=4, rnd=6)
    alone = {r: G.bc_exact(r)[0] for r in qs}
    samp = {r: G.bc_sampled(r, T=40, seed=r, flags=B.BCD_NO_EXACT_FALLBACK)[0] for r in qs[:3]}
    sets = G.bc_set(qs[:5])[0]
    # the unpruned baseline (draws over V minus r) through the server too
    allv = {r: G.bc_sampled(r, T=30, seed=r + 1, flags=B.BCD_SAMPLE_ALL_VERTICES)[0] for r in qs[:2]}
    S = B.Server(G, workers=2, groups=2)
    tickets = {}
    # staggered arrivals: some queries arrive while earlier batches are running
    for i, r in enumerate(qs):
        tickets[S.submit(B.BCD_QUERY_EXACT, r=r, tag=r)] = ("exact", r)
        if i < 3:
            tickets[S.submit(B.BCD_QUERY_SAMPLED, r=r, T=40, seed=r, flags=B.BCD_NO_EXACT_FALLBACK)] = ("samp", r)
        if i < 2:
            tickets[S.submit(B.BCD_QUERY_SAMPLED, r=r, T=30, seed=r + 1, flags=B.BCD_SAMPLE_ALL_VERTICES)] = ("allv", r)
        if i == 4:
            tickets[S.submit(B.BCD_QUERY_SET, rs=qs[:5])] = ("set", None)
        time.sleep(0.002)
    res = drain(S, len(tickets))
    S.close()
    for t, (kind, r) in tickets.items():
        out = res[t]
        assert out["status"] == B.BCD_OK, (kind, r, out)
        assert out["t_arrive_s"] <= out["t_admit_s"] <= out["t_done_s"]
        if kind == "exact":
            assert out["bc"] == alone[r], (r, out["bc"], alone[r])
            assert out["tag"] == r
        elif kind == "samp":
            assert out["bc"] == samp[r]
        elif kind == "allv":
            assert out["bc"] == allv[r] and out["stats"]["rv_size"] == g.n - 1, (r, out["bc"], allv[r])
        else:
            assert np.array_equal(out["bcs"], sets)
    for r in qs[:3]:
        want, _ = oracle.bc_exact(g, r)
        assert abs(alone[r] - want) <= 1e-10 * abs(want)
    for r in qs[:2]:
        want = oracle.bc_sampled_all(g, r, 30, r + 1)
        assert abs(allv[r] - want) <= 1e-10 * abs(want)


def test_server_budget_admission_and_errors(B):
    g = gg.rmat(11, 8, seed=2)
    G = B.Graph.from_digraph(g)
    G.set_config(groups=1)
    qs = gg.top_out_degree(g, 6)
    alone = {r: G.bc_exact(r)[0] for r in qs}
    # budget so tight that queries must wait for each other's buffers
    nrv = max(int(G.bc_exact(r)[1]["rv_size"]) for r in qs)
    ws = B.Server.workspace_bytes(G, groups=1, workers=1)
    S = B.Server(G, workers=1, groups=1, hbm_budget_bytes=ws + 8 * nrv + 64)
    ts = [S.submit(B.BCD_QUERY_EXACT, r=r) for r in qs]
    res = drain(S, len(ts))
    for t, r in zip(ts, qs):
        assert res[t]["status"] == B.BCD_OK and res[t]["bc"] == alone[r]
    with pytest.raises(B.BcdError) as e:
        S.submit(B.BCD_QUERY_EXACT, r=g.n + 5)
    assert e.value.code == B.BCD_ERR_INVALID_ARG
    S.close()
    with pytest.raises(B.BcdError) as e:
        B.Server(G, workers=1, groups=1, hbm_budget_bytes=1024)
    assert e.value.code == B.BCD_ERR_OUT_OF_MEMORY


def test_server_overflow_isolated(B):
    """A query whose sources overflow sigma fails alone; a query whose
    sources share its batch but not its overflow still gets its value."""
    gd, ids = gg.diamond_chain(64)
    s, d = gd.arcs()
    off = gd.n
    ps = np.arange(off, off + 5)
    g = gg.from_arcs(gd.n + 6, np.concatenate([s, ps]), np.concatenate([d, ps + 1]))
    G = B.Graph.from_digraph(g)
    ok_r = off + 2
    want = G.bc_exact(ok_r)[0]
    assert want == 2 * 3
    S = B.Server(G, workers=1, groups=1)
    t_bad = S.submit(B.BCD_QUERY_EXACT, r=ids["x"][40])
    t_ok = S.submit(B.BCD_QUERY_EXACT, r=ok_r)
    res = drain(S, 2)
    S.close()
    assert res[t_bad]["status"] == B.BCD_ERR_SIGMA_OVERFLOW
    assert res[t_ok]["status"] == B.BCD_OK and res[t_ok]["bc"] == want


def test_server_shutdown_cancels_queued(B):
    """bcd_server_shutdown: queries not yet admitted finish CANCELLED, those
    admitted finish with their standalone value, every result can still be
    polled, and later submissions are refused with CANCELLED."""
    g = gg.rmat(12, 8, seed=8)
    G = B.Graph.from_digraph(g)
    G.set_config(groups=1)
    qs = gg.top_out_degree(g, 40)
    alone = {r: G.bc_exact(r)[0] for r in qs[:4]}
    # one worker, one group: each query takes many batches, so most are still queued
    S = B.Server(G, workers=1, groups=1)
    ts = {S.submit(B.BCD_QUERY_EXACT, r=r): r for r in qs}
    S.shutdown()
    res = drain(S, len(ts))
    assert set(res) == set(ts)
    st = [res[t]["status"] for t in ts]
    assert all(x in (B.BCD_OK, B.BCD_ERR_CANCELLED) for x in st)
    assert st.count(B.BCD_ERR_CANCELLED) >= len(qs) // 2
    for t, r in ts.items():
        if res[t]["status"] == B.BCD_OK and r in alone:
            assert res[t]["bc"] == alone[r]
    with pytest.raises(B.BcdError) as e:
        S.submit(B.BCD_QUERY_EXACT, r=qs[0])
    assert e.value.code == B.BCD_ERR_CANCELLED
    S.close()


def test_server_rmat22_serving_config(B, oracle):
    """R-MAT scale 22, edge factor 16, in the serving benchmark's shape (3
    workers x 3 column groups, a 64 GB budget): sampled queries with Eq.(8)'s
    sample count and with 12 draws, all submitted at once, each equal bit for
    bit to the standalone call; the 12-draw values equal the oracle's A-BCD
    on the same draws."""
    g = gg.rmat22()
    G = B.Graph.from_digraph(g)
    ind, outd = g.in_degree(), g.out_degree()
    pool = [v for v in gg.uniform_vertices(g.n, 400, seed=105) if ind[v] > 0 and outd[v] > 0]
    big, small = pool[:3], pool[3:7]
    print("rmat22 serving", big, small, flush=True)
    alone = {("b", r): G.bc_sampled(r, eps=0.01, delta=0.1, seed=305 + i)[0] for i, r in enumerate(big)}
    alone.update({("s", r): G.bc_sampled(r, T=12, seed=7 + i, flags=B.BCD_NO_EXACT_FALLBACK)[0]
                  for i, r in enumerate(small)})
    S = B.Server(G, workers=3, groups=3, hbm_budget_bytes=64 * 10 ** 9)
    ts = {}
    for i, r in enumerate(big):
        ts[S.submit(B.BCD_QUERY_SAMPLED, r=r, eps=0.01, delta=0.1, seed=305 + i)] = ("b", r)
    for i, r in enumerate(small):
        ts[S.submit(B.BCD_QUERY_SAMPLED, r=r, T=12, seed=7 + i, flags=B.BCD_NO_EXACT_FALLBACK)] = ("s", r)
    res = drain(S, len(ts), timeout=300)
    S.close()
    for t, key in ts.items():
        assert res[t]["status"] == B.BCD_OK, (key, res[t])
        assert res[t]["bc"] == alone[key], (key, res[t]["bc"], alone[key])
    for i, r in enumerate(small[:2]):
        want, _ = oracle.bc_sampled(g, r, 12, 7 + i)
        got = alone[("s", r)]
        assert abs(got - want) <= 1e-10 * abs(want) and (got == 0) == (want == 0), (r, got, want)
