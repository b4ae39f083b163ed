"""Brute-force betweenness straight from Eq.(1), with exact rationals.

TEST INFRASTRUCTURE ONLY.  For every ordered pair (s, t), s != t, all simple
s->t paths are enumerated; the shortest ones (fewest arcs, or least total
weight) are counted, and so are those that pass through each vertex.  Then
BC(v) = sum over s != v != t with sigma_st > 0 of sigma_st(v) / sigma_st
(Eq.(1)), as a ``fractions.Fraction``.  No shortest-path algorithm and no
dependency recursion is used, so this pins the oracle independently.
Exponential: for graphs of at most about a dozen sparse vertices.
"""
from __future__ import annotations

from fractions import Fraction


def _adj(g):
    rp = g.row_ptr
    out = []
    for v in range(g.n):
        arcs = []
        for e in range(int(rp[v]), int(rp[v + 1])):
            w = 1 if g.weight is None else int(g.weight[e])
            arcs.append((int(g.col[e]), w))
        out.append(arcs)
    return out


def all_pairs_paths(g):
    """{(s, t): (length, count, {v: count through v})} for every s != t with
    at least one path."""
    adj = _adj(g)
    res = {}
    for s in range(g.n):
        best: dict[int, list] = {}
        stack = [(s, 0, [s])]
        while stack:
            v, L, path = stack.pop()
            if v != s:
                b = best.get(v)
                if b is None or L < b[0]:
                    best[v] = [L, 1, {u: 1 for u in path}]
                elif L == b[0]:
                    b[1] += 1
                    for u in path:
                        b[2][u] = b[2].get(u, 0) + 1
            for w, lw in adj[v]:
                if w not in path:
                    stack.append((w, L + lw, path + [w]))
        for t, (L, cnt, through) in best.items():
            res[(s, t)] = (L, cnt, through)
    return res


def betweenness(g):
    """Exact BC(v) for every v, Eq.(1), ordered pairs, unnormalised."""
    paths = all_pairs_paths(g)
    bc = [Fraction(0)] * g.n
    for (s, t), (_, cnt, through) in paths.items():
        for v, c in through.items():
            if v != s and v != t:
                bc[v] += Fraction(c, cnt)
    return bc


def dependency(g, s, r, paths=None):
    """delta_s.(r) from Eq.(2)."""
    paths = paths if paths is not None else all_pairs_paths(g)
    tot = Fraction(0)
    if s == r:
        return tot
    for (a, t), (_, cnt, through) in paths.items():
        if a == s and t != r and r in through:
            tot += Fraction(through[r], cnt)
    return tot


def closure(g):
    """reach[u][v]: a directed u->v path of at least one arc exists
    (Warshall's transitive closure of the arc relation, no BFS)."""
    n = g.n
    reach = [[False] * n for _ in range(n)]
    for v in range(n):
        for e in range(int(g.row_ptr[v]), int(g.row_ptr[v + 1])):
            reach[v][int(g.col[e])] = True
    for k in range(n):
        for i in range(n):
            if reach[i][k]:
                ri, rk = reach[i], reach[k]
                for j in range(n):
                    if rk[j]:
                        ri[j] = True
    return reach


def reachers(g, r, reach=None):
    """RV(r) by Def.1: every v != r with a directed v->r path."""
    reach = reach if reach is not None else closure(g)
    return sorted(v for v in range(g.n) if v != r and reach[v][r])


def reached_from(g, r, reach=None):
    """Every t != r with a directed r->t path (the vertices r reaches)."""
    reach = reach if reach is not None else closure(g)
    return sorted(t for t in range(g.n) if t != r and reach[r][t])
