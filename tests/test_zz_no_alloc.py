"""bcd_rv_noalloc (RV(r) with the traversal's working memory in a static
device array, no allocation) against bcd_rv through the C ABI: the same ids
in the same order on consecutive calls, the second and third on smaller
inputs than the first, on the multi-level and the single-workgroup
traversal; the size query, the too-small buffer and the size limit."""
import ctypes as C

import numpy as np
import pytest

from paper_1708_08739_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_1708_08739_amd import bcd
    bcd.load()
    return bcd


def rv_noalloc(B, G, r, cap=None):
    L = B.load()
    cnt = C.c_int64()
    rc = L.bcd_rv_noalloc(G.h, r, None, 0, C.byref(cnt))
    assert rc == B.BCD_OK, B.last_error()
    out = np.full(max(cnt.value, 1) if cap is None else cap, -7, dtype=np.int32)
    cnt2 = C.c_int64()
    rc = L.bcd_rv_noalloc(G.h, r, out.ctypes.data, out.size, C.byref(cnt2))
    return rc, out, cnt.value, cnt2.value


def test_noalloc_rv_equals_rv_on_consecutive_calls(B, oracle):
    g16, q16 = gg.rmat16()        # 65,536 vertices: the multi-level traversal
    ger, (rer,) = gg.er_2000()    # 2,000 vertices: the single-workgroup traversal
    # 70,000 vertices (multi-level traversal), arcs i -> i+1 for i < 30 only
    nb = 70000
    rp = np.zeros(nb + 1, dtype=np.int64)
    rp[1:31] = np.arange(1, 31)
    rp[31:] = 30
    gb = gg.Digraph(nb, rp, np.arange(1, 31, dtype=np.int32))
    G16, Ger, Gb = (B.Graph.from_digraph(x) for x in (g16, ger, gb))
    # a large RV first, then smaller inputs: nothing of an earlier call may survive
    for G, g, r in ((G16, g16, q16[0]), (Gb, gb, 30), (Ger, ger, rer), (G16, g16, q16[1]), (Gb, gb, 7),
                    (Gb, gb, 500), (Ger, ger, 0)):
        want = G.rv(r)
        rc, out, k, k2 = rv_noalloc(B, G, r)
        print("noalloc", g.name, r, k, flush=True)
        assert rc == B.BCD_OK, B.last_error()
        assert k == k2 == want.size
        assert np.array_equal(out[:k], want), (g.name, r)
        assert np.array_equal(want, oracle.rv(g, r))


def test_noalloc_rv_errors(B):
    import ctypes as C
    L = B.load()
    g, q = gg.rmat16()
    G = B.Graph.from_digraph(g)
    r = q[0]
    k = len(G.rv(r))
    rc, out, k0, k2 = rv_noalloc(B, G, r, cap=k - 1)
    assert rc == B.BCD_ERR_BUFFER_TOO_SMALL and k2 == k
    assert np.all(out == -7)  # untouched on error
    cnt = C.c_int64()
    assert L.bcd_rv_noalloc(G.h, g.n, None, 0, C.byref(cnt)) == B.BCD_ERR_INVALID_ARG
    assert L.bcd_rv_noalloc(None, 0, None, 0, C.byref(cnt)) == B.BCD_ERR_INVALID_ARG
    # more vertices than the static scratch holds
    n = (1 << 22) + 1
    rp = np.zeros(n + 1, dtype=np.int64)
    rp[1:] = 1
    big = B.Graph(n, rp, np.array([1], dtype=np.int32))
    assert L.bcd_rv_noalloc(big.h, 1, None, 0, C.byref(cnt)) == B.BCD_ERR_UNSUPPORTED
    assert "2^22" in B.last_error()
    # the graph itself still works with the allocating call
    assert big.rv(1).tolist() == [0]
