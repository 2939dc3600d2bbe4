"""Pins of the oracle's local-MST forest (Section 6, Discussion): the
Z-order partition against hand-worked Morton positions, cluster sizes,
the forest against Kruskal per cluster, the one-cluster and one-cell cases,
and the support bound of Section 4 (a subgraph of the collision graph:
lambda_min(P^{-1} Gamma) >= 1) from dense eigenvalues."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from workloads import sphere_cluster

G0 = 1e-3


def test_z_order_positions_hand_worked():
    """With K = 1 a cell's cluster id is its position in the Z-order.  Cells at
    the centres of the unit grid cubes of a 4 x 4 x 4 block (radius 0.5, so
    h = 1 and the block's corner cell sets the origin): the Morton position of
    (x, y, z) has bit b of x, y, z at bits 3b, 3b + 1, 3b + 2.  Worked by hand:
    (0,0,0) -> 0, (1,0,0) -> 1, (0,1,0) -> 2, (0,0,1) -> 4, (1,1,1) -> 7,
    (2,0,0) -> 8, (0,2,0) -> 16, (0,0,2) -> 32, (1,2,3) -> 53 (x = 01, y = 10,
    z = 11: low bits 1,0,1 -> 5, high bits 0,1,1 -> 6, 6 * 8 + 5), (3,3,3) -> 63."""
    cells = [(x, y, z) for z in range(4) for y in range(4) for x in range(4)]
    rng = np.random.default_rng(0)
    order = rng.permutation(len(cells))          # ids do not follow the grid
    pos = np.array([cells[k] for k in order], dtype=np.float64) + 0.5
    R = np.full(len(cells), 0.5)
    cl = O.forest_clusters(pos, R, 1)
    rank = {cells[k]: int(cl[i]) for i, k in enumerate(order)}
    want = {(0, 0, 0): 0, (1, 0, 0): 1, (0, 1, 0): 2, (0, 0, 1): 4, (1, 1, 1): 7, (2, 0, 0): 8, (0, 2, 0): 16,
            (0, 0, 2): 32, (1, 2, 3): 53, (3, 3, 3): 63}
    for c, r in want.items():
        assert rank[c] == r, (c, rank[c], r)
    assert sorted(rank.values()) == list(range(64))


def test_cluster_sizes_per_instance():
    c = sphere_cluster(1000, 0)
    off = np.array([0, 300, 300, 1000], np.int64)    # includes an empty instance
    cl = O.forest_clusters(c["pos"], c["radius"], 128, off)
    # instance 0: 3 clusters (128, 128, 44); instance 2: 6 clusters (5 x 128 + 60)
    counts = np.bincount(cl)
    assert list(counts) == [128, 128, 44, 128, 128, 128, 128, 128, 60]
    assert np.all(cl[:300] < 3) and np.all(cl[300:] >= 3)


def _kruskal_sub(g, idx):
    sub = O.Graph(g.n, g.rowptr, g.col, g.ei[idx], g.ej[idx], g.w[idx], g.u[idx])
    return np.sort(idx[O.kruskal(sub)])


@pytest.mark.parametrize("K", [1, 37, 128, 5000])
def test_forest_is_kruskal_of_each_cluster(K):
    c = sphere_cluster(1200, 3)
    g = O.collide(c["pos"], c["radius"])
    t, cl = O.build_forest(g, c["pos"], c["radius"], K)
    # every forest edge lies inside a cluster, and per cluster the forest is
    # the maximum spanning forest (Kruskal) of the cluster's own contacts
    assert np.all(cl[g.ei[t.tree_edge]] == cl[g.ej[t.tree_edge]])
    want = []
    for k in np.unique(cl):
        idx = np.nonzero((cl[g.ei] == k) & (cl[g.ej] == k))[0].astype(np.int32)
        if idx.size:
            want.append(_kruskal_sub(g, idx))
    want = np.sort(np.concatenate(want)) if want else np.zeros(0, np.int32)
    assert np.array_equal(t.tree_edge, want)
    if K == 1:
        assert t.tree_edge.size == 0 and np.all(t.parent == -1)
    if K >= g.n:   # one cluster: the global tree
        assert np.array_equal(t.tree_edge, O.build_tree(g).tree_edge)


def test_forest_with_one_cell_clusters_is_scaled_identity():
    c = sphere_cluster(200, 1)
    g = O.collide(c["pos"], c["radius"])
    t, _ = O.build_forest(g, c["pos"], c["radius"], 1)
    f = O.tree_factor(g, t)
    b = np.random.default_rng(2).normal(size=(200, 3))
    assert np.allclose(O.tree_solve(f, b), b / G0, rtol=1e-13, atol=0)


def test_forest_support_bound_and_dense_solve():
    """P of the forest is the block Laplacian of a subgraph plus g_med I, so
    lambda_min(Gamma, P) >= 1 (Section 4); the tree solve is the dense solve."""
    c = sphere_cluster(300, 5)
    g = O.collide(c["pos"], c["radius"])
    A = O.assemble(g)
    t, cl = O.build_forest(g, c["pos"], c["radius"], 64)
    assert len(np.unique(cl)) == 5
    f = O.tree_factor(g, t)
    G = A.dense()
    P = G0 * np.eye(3 * g.n)
    for e in t.tree_edge:
        i, j, w, u = g.ei[e], g.ej[e], g.w[e], g.u[e]
        W = w * (1.0 * np.outer(u, u) + 0.1 * (np.eye(3) - np.outer(u, u)))
        d = np.zeros(g.n); d[i] = 1; d[j] = -1
        P += np.kron(np.outer(d, d), W)
    lam = scipy.linalg.eigh(G, P, eigvals_only=True)
    assert lam.min() >= 1 - 1e-9
    b = np.random.default_rng(3).normal(size=(g.n, 3))
    x = O.tree_solve(f, b).ravel()
    xd = np.linalg.solve(P, b.ravel())
    assert np.linalg.norm(x - xd) <= 1e-10 * np.linalg.norm(xd)
    # PCG with the forest converges to the dense solution
    xs, info = O.pcg(A, b, "tree", f)
    assert info.relres_true <= 1.0001e-8
