"""Pins of the oracle's augmented MST (Section 3.1, Vaidya's second
preconditioner) and of the flexible CG that solves with it through an inner
tree-PCG (Sections 3 and 5): the pieces and the added contacts by brute
force, the subgraph bounds of Section 4 from dense eigenvalues, the
reduction to plain PCG when the preconditioner is fixed, and convergence."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from workloads import sphere_cluster


def _setup(n, seed):
    c = sphere_cluster(n, seed)
    g = O.collide(c["pos"], c["radius"])
    t = O.build_tree(g)
    return c, g, t


def test_assemble_edges_of_all_contacts_is_gamma():
    c, g, t = _setup(400, 1)
    A = O.assemble(g)
    B = O.assemble_edges(g, np.arange(g.m))
    assert np.array_equal(A.rowptr, B.rowptr) and np.array_equal(A.bcol, B.bcol) and np.array_equal(A.val, B.val)


@pytest.mark.parametrize("parts", [1, 3, 8, 40])
def test_pieces_and_added_contacts_brute_force(parts):
    c, g, t = _setup(1500, 2)
    aug, piece, added = O.augment(g, t, parts)
    s = -(-g.n // parts)
    # pieces: connected parts of the MST headed by a root or a cut vertex;
    # weights recomputed here by a recursive walk of the rooted tree
    children = [[] for _ in range(g.n)]
    for v in range(g.n):
        if t.parent[v] >= 0:
            children[t.parent[v]].append(v)
    weight = np.zeros(g.n, np.int64)

    def walk(v):
        stack = [(v, False)]
        while stack:
            u, done = stack.pop()
            if done:
                weight[u] = 1 + sum(weight[c] for c in children[u] if weight[c] < s)
            else:
                stack.append((u, True))
                stack.extend((c, False) for c in children[u])

    for r in np.nonzero(t.parent < 0)[0]:
        walk(r)
    heads = set(np.nonzero((t.parent < 0) | (weight >= s))[0].tolist())
    assert set(np.unique(piece).tolist()) == heads
    for h in heads:
        members = np.nonzero(piece == h)[0]
        te = t.tree_edge
        inside = (piece[g.ei[te]] == h) & (piece[g.ej[te]] == h)
        assert inside.sum() == members.size - 1            # a connected subtree
        if t.parent[h] >= 0:
            assert members.size >= s                       # a cut piece holds at least s cells
    assert len(heads) <= g.n // s + int((t.parent < 0).sum())
    # added: for every pair of pieces with a contact, its heaviest (then smallest id)
    best = {}
    for e in range(g.m):
        a, b = piece[g.ei[e]], piece[g.ej[e]]
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        if key not in best or g.w[e] > g.w[best[key]] or (g.w[e] == g.w[best[key]] and e < best[key]):
            best[key] = e
    te = t.tree_edge
    want = np.array(sorted(set(best.values()) - set(te.tolist())), dtype=np.int32)
    assert np.array_equal(added, want)
    assert np.array_equal(aug, np.union1d(te, want))
    if parts == 1:
        assert added.size == 0 and np.array_equal(aug, te)


def test_augmented_support_bounds_dense():
    """P <= P' <= Gamma in the Loewner order (nested subgraphs plus g_med I):
    lambda_min(Gamma, P') >= 1 (Section 4) and P'^{-1} Gamma has a smaller
    largest eigenvalue than P^{-1} Gamma."""
    c, g, t = _setup(300, 3)
    aug, piece, added = O.augment(g, t, 6)
    assert added.size > 0
    G = O.assemble(g).dense()
    Pa = O.assemble_edges(g, aug).dense()
    P = O.assemble_edges(g, t.tree_edge).dense()
    la = scipy.linalg.eigh(G, Pa, eigvals_only=True)
    lt = scipy.linalg.eigh(G, P, eigvals_only=True)
    assert la.min() >= 1 - 1e-9 and lt.min() >= 1 - 1e-9
    assert la.max() <= lt.max() * (1 + 1e-9)
    assert scipy.linalg.eigh(Pa - P, eigvals_only=True).min() >= -1e-12 * np.abs(Pa).max()


def test_fcg_with_a_fixed_preconditioner_is_pcg():
    """With no added contacts (one part) P' = P, and an inner solve to 1e-13
    applies P^{-1} to rounding: flexible CG then takes plain PCG's iterations
    and reaches its solution."""
    c, g, t = _setup(1000, 0)
    A = O.assemble(g)
    f = O.tree_factor(g, t)
    aug, _, added = O.augment(g, t, 1)
    assert added.size == 0
    Pa = O.assemble_edges(g, aug)
    x, info = O.fcg(A, Pa, f, c["force"], tol=1e-8, inner_tol=1e-13)
    xp, ip = O.pcg(A, c["force"], "tree", f)
    assert info.iters == ip.iters
    assert np.linalg.norm(x - xp) <= 1e-9 * np.linalg.norm(xp)
    assert info.outer >= info.iters   # at least one inner iteration per application


def test_fcg_converges_with_inexact_inner_solves():
    c, g, t = _setup(1200, 4)
    A = O.assemble(g)
    f = O.tree_factor(g, t)
    aug, _, added = O.augment(g, t)
    Pa = O.assemble_edges(g, aug)
    x, info = O.fcg(A, Pa, f, c["force"], tol=1e-8, inner_tol=0.1)
    assert info.status == O.OK and info.relres_true <= 1.0001e-8
    xd = np.linalg.solve(A.dense(), c["force"].ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 2e3 * 1e-8 * np.linalg.norm(xd)
    # zero force: zero velocity, no iterations
    x0, i0 = O.fcg(A, Pa, f, np.zeros_like(c["force"]))
    assert i0.iters == 0 and not np.any(x0)
