"""Pins of the oracle's maximum spanning forest and rooting (Section 3.1,
Section 3.2 Lemma nofill)."""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from workloads import sphere_cluster


def _graph_from_pairs(n, pairs, w):
    """Build an oracle Graph from explicit pairs (i < j) and weights."""
    pairs = sorted(zip([min(a, b) for a, b in pairs], [max(a, b) for a, b in pairs], w))
    ei = np.array([p[0] for p in pairs], np.int32)
    ej = np.array([p[1] for p in pairs], np.int32)
    ww = np.array([p[2] for p in pairs], np.float64)
    m = len(pairs)
    u = np.tile([1.0, 0.0, 0.0], (m, 1))
    rowptr = np.zeros(n + 1, np.int32)
    nb = [[] for _ in range(n)]
    for a, b in zip(ei, ej):
        nb[a].append(b); nb[b].append(a)
    col = []
    for i in range(n):
        col += sorted(nb[i]); rowptr[i + 1] = len(col)
    return O.Graph(n, rowptr, np.array(col, np.int32), ei, ej, ww, u)


def _brute_msf(g):
    """Enumerate every spanning forest (edge subsets of size n - #components
    without a cycle) and return the one the strict order (w desc, id asc)
    prefers: the lexicographically smallest sorted rank sequence.  For a
    matroid this greedy-optimal basis is unique."""
    n, m = g.n, g.m
    rank = {e: r for r, e in enumerate(sorted(range(m), key=lambda e: (-g.w[e], e)))}

    def comps(edges):
        par = list(range(n))

        def f(x):
            while par[x] != x:
                x = par[x]
            return x
        for e in edges:
            a, b = f(g.ei[e]), f(g.ej[e])
            if a == b:
                return None
            par[a] = b
        return len({f(x) for x in range(n)})
    c_all = n - _rank_of(g)
    best = None
    for sub in itertools.combinations(range(m), n - c_all):
        if comps(sub) != c_all:
            continue
        key = sorted(rank[e] for e in sub)
        if best is None or key < best[0]:
            best = (key, sorted(sub))
    return np.array(best[1] if best else [], np.int32)


def _rank_of(g):
    par = list(range(g.n))

    def f(x):
        while par[x] != x:
            x = par[x]
        return x
    r = 0
    for a, b in zip(g.ei, g.ej):
        a, b = f(a), f(b)
        if a != b:
            par[a] = b; r += 1
    return r


@pytest.mark.parametrize("seed", range(40))
def test_prim_equals_kruskal_equals_enumeration_tiny(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 8))
    allp = [(a, b) for a in range(n) for b in range(a + 1, n)]
    m = int(rng.integers(0, min(len(allp), 11) + 1))
    pick = rng.choice(len(allp), size=m, replace=False) if m else []
    pairs = [allp[k] for k in pick]
    # few distinct weights so that ties are common
    w = rng.choice([0.05, 0.1, 0.1, 0.2], size=m).tolist()
    g = _graph_from_pairs(n, pairs, w)
    te_p = np.sort(O.prim(g)[0])
    te_k = np.sort(O.kruskal(g))
    te_b = _brute_msf(g)
    assert np.array_equal(te_p, te_k)
    assert np.array_equal(te_p, te_b)


def test_all_ties_picks_smallest_ids():
    """All weights equal: the forest is the greedy one over ascending edge id."""
    c = sphere_cluster(600, 2)
    g = O.collide(c["pos"], c["radius"])
    g.w[:] = 0.1
    te = np.sort(O.prim(g)[0])
    assert np.array_equal(te, np.sort(O.kruskal(g)))
    # greedy over ascending id with union-find, written out here
    par = list(range(g.n))

    def f(x):
        while par[x] != x:
            x = par[x]
        return x
    want = []
    for e in range(g.m):
        a, b = f(g.ei[e]), f(g.ej[e])
        if a != b:
            par[a] = b; want.append(e)
    assert np.array_equal(te, want)


@pytest.mark.parametrize("n,seed", [(1000, 0), (3000, 5)])
def test_prim_equals_kruskal_workload(n, seed):
    c = sphere_cluster(n, seed)
    g = O.collide(c["pos"], c["radius"])
    assert np.array_equal(np.sort(O.prim(g)[0]), np.sort(O.kruskal(g)))


def test_max_weight_for_distinct_weights():
    """With distinct weights the maximum spanning tree maximises the total weight;
    a random spanning tree never beats it."""
    c = sphere_cluster(300, 4)
    g = O.collide(c["pos"], c["radius"])
    assert len(np.unique(g.w)) == g.m
    te = O.prim(g)[0]
    best = g.w[te].sum()
    rng = np.random.default_rng(0)
    for _ in range(20):
        g2 = O.Graph(g.n, g.rowptr, g.col, g.ei, g.ej, rng.random(g.m), g.u)
        other = O.prim(g2)[0]
        assert g.w[other].sum() <= best + 1e-15
        assert len(other) == len(te)


def test_forest_roots_and_depths():
    """Three separated clusters plus an isolated cell: a spanning forest, each
    tree rooted at its smallest vertex; parent is a tree neighbour one level up."""
    parts = []
    off = 0
    for k, n in enumerate([40, 25, 1, 60]):
        c = sphere_cluster(n, k)
        parts.append(c["pos"] + np.array([100.0 * k, 0, 0]))
    pos = np.concatenate(parts)
    # interleave ids so that roots are not simply the first vertex
    perm = np.random.default_rng(1).permutation(len(pos))
    pos = pos[perm]
    R = np.full(len(pos), 1.0)
    g = O.collide(pos, R)
    t = O.build_tree(g)
    comp_of = np.searchsorted(np.cumsum([40, 25, 1, 60]), perm, side="right")
    assert len(t.tree_edge) == len(pos) - 4
    roots = np.nonzero(t.parent < 0)[0]
    assert sorted(roots) == sorted(np.nonzero(comp_of == k)[0].min() for k in range(4))
    tree_pairs = {(int(g.ei[e]), int(g.ej[e])) for e in t.tree_edge}
    for v in range(len(pos)):
        p = t.parent[v]
        if p < 0:
            assert t.depth[v] == 0 and t.pedge[v] == -1
            continue
        assert (min(p, v), max(p, v)) in tree_pairs
        assert t.depth[v] == t.depth[p] + 1
        e = t.pedge[v]
        assert {int(g.ei[e]), int(g.ej[e])} == {int(p), v}
    # elimination order: children before parents (Lemma nofill)
    pos_in = np.empty(len(pos), int)
    pos_in[t.order] = np.arange(len(pos))
    for v in range(len(pos)):
        if t.parent[v] >= 0:
            assert pos_in[v] < pos_in[t.parent[v]]
    for v in range(len(pos)):
        ch = t.child[t.child_ptr[v]:t.child_ptr[v + 1]]
        assert np.all(np.diff(ch) > 0) and np.all(t.parent[ch] == v)


def test_workload_tree_depth_and_components():
    c = sphere_cluster(1000, 0)
    g = O.collide(c["pos"], c["radius"])
    t = O.build_tree(g)
    assert (t.parent < 0).sum() == 1 and t.parent[0] == -1
    assert len(t.tree_edge) == 999
    assert t.depth.max() == 83


def _elimination_game_fill(n, edges, order):
    """Fill edges made by eliminating vertices in `order` (Section 3.2's
    elimination game): each eliminated vertex's remaining neighbours become
    pairwise adjacent."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    fill = 0
    for v in order:
        nb = sorted(adj[v])
        for i in range(len(nb)):
            for j in range(i + 1, len(nb)):
                a, b = nb[i], nb[j]
                if b not in adj[a]:
                    adj[a].add(b)
                    adj[b].add(a)
                    fill += 1
        for a in nb:
            adj[a].discard(v)
        adj[v].clear()
    return fill


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_elimination_game_no_fill(seed):
    """Lemma nofill: the oracle's order (no vertex before its children) plays
    the elimination game on its spanning tree without a single fill edge; the
    reversed order (roots first) on the same tree does make fill, so the
    game counts it."""
    c = sphere_cluster(80, seed)
    g = O.collide(c["pos"], c["radius"])
    t = O.build_tree(g)
    edges = [(int(g.ei[e]), int(g.ej[e])) for e in t.tree_edge]
    assert _elimination_game_fill(g.n, edges, list(t.order)) == 0
    assert _elimination_game_fill(g.n, edges, list(t.order)[::-1]) > 0
    # and on a hand-made path 0-1-2: eliminating the middle first makes one fill edge
    assert _elimination_game_fill(3, [(0, 1), (1, 2)], [1, 0, 2]) == 1
    assert _elimination_game_fill(3, [(0, 1), (1, 2)], [0, 1, 2]) == 0
