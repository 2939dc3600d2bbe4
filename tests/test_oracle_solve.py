"""Pins of the oracle's TreeLDLT (Alg. 2), tree solves (Appendix B.1) and
PCG (Section 1.1), against dense linear algebra, closed forms and the
support-graph theorems of Section 4."""
import json
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

from oracle import oracle as O
from workloads import sphere_cluster

GOLD = os.path.join(os.path.dirname(__file__), "golden")
GP, GQ, G0 = 1.0, 0.1, 1e-3


def _setup(n, seed=0):
    c = sphere_cluster(n, seed)
    g = O.collide(c["pos"], c["radius"])
    A = O.assemble(g)
    t = O.build_tree(g)
    f = O.tree_factor(g, t)
    return c, g, A, t, f


def _dense_laplacian(n, pairs_w_u, g_med):
    """Block Laplacian sum_e (e_i - e_j)(e_i - e_j)^T (x) W_e + g_med I, built
    with Kronecker products (independent of the oracle's assembly loop)."""
    P = g_med * np.eye(3 * n)
    for i, j, w, u in pairs_w_u:
        W = w * (GP * np.outer(u, u) + GQ * (np.eye(3) - np.outer(u, u)))
        d = np.zeros(n); d[i] = 1; d[j] = -1
        P += np.kron(np.outer(d, d), W)
    return P


def _dense_P(g, t):
    return _dense_laplacian(g.n, [(g.ei[e], g.ej[e], g.w[e], g.u[e]) for e in t.tree_edge], G0)


def test_gamma_equals_kronecker_laplacian():
    _, g, A, _, _ = _setup(150, 3)
    want = _dense_laplacian(g.n, [(g.ei[e], g.ej[e], g.w[e], g.u[e]) for e in range(g.m)], G0)
    assert np.allclose(A.dense(), want, rtol=1e-13, atol=1e-16)


def test_ldlt_reconstructs_P():
    _, g, _, t, f = _setup(300, 1)
    n = g.n
    Lfull = np.eye(3 * n)
    Dfull = np.zeros((3 * n, 3 * n))
    for i in range(n):
        Dfull[3 * i:3 * i + 3, 3 * i:3 * i + 3] = f.D[i]
        p = t.parent[i]
        if p >= 0:
            Lfull[3 * p:3 * p + 3, 3 * i:3 * i + 3] = f.L[i]
    P = _dense_P(g, t)
    R = Lfull @ Dfull @ Lfull.T
    assert np.abs(R - P).max() <= 1e-13 * np.abs(P).max()
    # L is P's sparsity pattern (Thm. following Alg. 2): nonzero blocks only at tree edges
    for i in range(n):
        if t.parent[i] >= 0:
            assert np.abs(f.L[i]).max() > 0


def test_tree_solve_matches_dense_solve():
    c, g, _, t, f = _setup(400, 2)
    P = _dense_P(g, t)
    b = c["force"]
    x = O.tree_solve(f, b)
    xd = np.linalg.solve(P, b.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-10 * np.linalg.norm(xd)
    # forward/diag/backward written out with dense triangular solves
    n = g.n
    Lfull = np.eye(3 * n); Dfull = np.zeros((3 * n, 3 * n))
    for i in range(n):
        Dfull[3 * i:3 * i + 3, 3 * i:3 * i + 3] = f.D[i]
        if t.parent[i] >= 0:
            Lfull[3 * t.parent[i]:3 * t.parent[i] + 3, 3 * i:3 * i + 3] = f.L[i]
    perm = np.concatenate([[3 * v, 3 * v + 1, 3 * v + 2] for v in t.order])
    Lp = Lfull[np.ix_(perm, perm)]
    assert np.allclose(Lp, np.tril(Lp))  # lower triangular in elimination order
    z = scipy.linalg.solve_triangular(Lp, b.ravel()[perm], lower=True)
    y = np.linalg.solve(Dfull[np.ix_(perm, perm)], z)
    xx = scipy.linalg.solve_triangular(Lp.T, y, lower=False)
    xo = np.empty_like(xx); xo[perm] = xx
    assert np.linalg.norm(x.ravel() - xo) <= 1e-12 * np.linalg.norm(xo)


def test_rigid_translation_through_tree_solve():
    _, g, _, t, f = _setup(2000, 4)
    tvec = np.array([0.5, -1.0, 2.0])
    x = O.tree_solve(f, np.tile(tvec, (g.n, 1)))
    assert np.allclose(x, np.tile(tvec / G0, (g.n, 1)), rtol=1e-9)


def test_support_bounds_dense():
    """Thm (subgraph): lambda_min(Gamma, P) >= 1; attained by rigid translations.
    Thm (MST): lambda_max(Gamma, P) <= kappa m (n-1)."""
    _, g, A, t, _ = _setup(200, 6)
    G = A.dense(); P = _dense_P(g, t)
    lam = scipy.linalg.eigh(G, P, eigvals_only=True)
    assert lam[0] >= 1 - 1e-10
    assert abs(lam[0] - 1) < 1e-8
    kappa = g.w.max() * GP / GQ
    assert lam[-1] <= kappa * g.m * (g.n - 1)
    # P is a worse approximation of Gamma than Gamma itself: lambda_max > 1
    assert lam[-1] > 1


@pytest.mark.parametrize("prec", ["none", "jacobi", "tree"])
def test_pcg_matches_dense_cholesky(prec):
    c, g, A, t, f = _setup(500, 7)
    G = A.dense()
    xd = scipy.linalg.cho_solve(scipy.linalg.cho_factor(G), c["force"].ravel())
    x, info = O.pcg(A, c["force"], prec, f, tol=1e-8)
    assert info.relres_rec <= 1e-8 and info.relres_true <= 1.01e-8
    kappa = np.linalg.cond(G)
    err = np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd)
    assert err <= kappa * info.relres_true
    x13, info13 = O.pcg(A, c["force"], prec, f, tol=1e-13)
    assert np.linalg.norm(x13.ravel() - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("prec", ["none", "jacobi", "tree"])
def test_iteration_count_matches_scipy_cg(prec):
    c, g, A, t, f = _setup(1000, 0)
    rows = np.repeat(np.arange(g.n), np.diff(A.rowptr))
    S = scipy.sparse.bsr_matrix((A.val, A.bcol, A.rowptr), shape=(3 * g.n, 3 * g.n))
    if prec == "none":
        M = None
    elif prec == "jacobi":
        blocks = [A.val[A.rowptr[i] + np.searchsorted(A.bcol[A.rowptr[i]:A.rowptr[i + 1]], i)] for i in range(g.n)]
        Minv = scipy.sparse.block_diag([np.linalg.inv(B) for B in blocks]).tocsr()
        M = scipy.sparse.linalg.aslinearoperator(Minv)
    else:
        M = scipy.sparse.linalg.LinearOperator(S.shape, matvec=lambda r: O.tree_solve(f, r).ravel())
    count = [0]

    def cb(_):
        count[0] += 1
    xs, flag = scipy.sparse.linalg.cg(S, c["force"].ravel(), rtol=1e-8, atol=0.0, M=M, maxiter=10000, callback=cb)
    assert flag == 0
    _, info = O.pcg(A, c["force"], prec, f, tol=1e-8)
    assert abs(info.iters - count[0]) <= 1
    assert {"none": 164, "jacobi": 164, "tree": 133}[prec] == info.iters


def _chain_or_comb(kind):
    if kind == "chain":
        n = 30
        pos = np.array([[1.9 * k, 0.1 * np.sin(k), 0.0] for k in range(n)])
    else:  # comb: spine along x, a tooth above every 2nd spine cell
        sp = [[1.9 * k, 0.0, 0.0] for k in range(20)]
        teeth = [[1.9 * k, 1.9, 0.01 * k] for k in range(0, 20, 2)]
        pos = np.array(sp + teeth)
    R = np.full(len(pos), 1.0)
    return pos, R


@pytest.mark.parametrize("kind", ["chain", "comb"])
def test_tree_graph_converges_in_one_iteration(kind):
    """If the collision graph is itself a tree, P = Gamma and PCG takes one step."""
    pos, R = _chain_or_comb(kind)
    g = O.collide(pos, R)
    assert g.m == g.n - 1
    A = O.assemble(g)
    t = O.build_tree(g)
    f = O.tree_factor(g, t)
    F = np.random.default_rng(0).normal(size=(g.n, 3))
    x, info = O.pcg(A, F, "tree", f, tol=1e-12)
    assert info.iters == 1
    xd = np.linalg.solve(A.dense(), F.ravel())
    assert np.linalg.norm(x.ravel() - xd) <= 1e-12 * np.linalg.norm(xd)


def test_golden_two_cell_solution():
    gold = json.load(open(os.path.join(GOLD, "two_cell.json")))
    out = O.solve_pipeline(np.array(gold["pos"]), np.array(gold["radius"]), np.array(gold["force"]),
                           tol=1e-14, g_par=gold["g_par"], g_perp=gold["g_perp"], g_med=gold["g_med"])
    ex = gold["expected"]
    assert out["info"].iters == ex["tree_pcg_iterations"]
    assert np.allclose(out["x"][0], ex["v1"], rtol=1e-12)
    assert np.allclose(out["x"][1], ex["v2"], rtol=1e-12)


def test_fixed_iterations_mode():
    c, g, A, t, f = _setup(500, 1)
    x5, i5 = O.pcg(A, c["force"], "tree", f, fixed_iters=5)
    assert i5.iters == 5
    x, info = O.pcg(A, c["force"], "tree", f)
    xk, ik = O.pcg(A, c["force"], "tree", f, fixed_iters=info.iters)
    assert np.array_equal(x, xk)


def test_warm_start_and_edge_cases():
    c, g, A, t, f = _setup(300, 2)
    x, info = O.pcg(A, c["force"], "tree", f)
    # warm start at the answer: no iteration needed
    x2, info2 = O.pcg(A, c["force"], "tree", f, x0=x)
    assert info2.iters == 0 and np.array_equal(x2, x)
    # zero force: zero velocity
    x0, info0 = O.pcg(A, np.zeros((g.n, 3)), "tree", f)
    assert info0.iters == 0 and not x0.any()
    # iteration cap
    _, infoc = O.pcg(A, c["force"], "tree", f, max_iter=1, check=False)
    assert infoc.status == O.ENOCONV and infoc.iters == 1
    # non-finite input
    Fb = c["force"].copy(); Fb[3, 1] = np.nan
    _, infon = O.pcg(A, Fb, "tree", f, check=False)
    assert infon.status == O.ENONFINITE


def test_singular_pivot_detected():
    """g_med = 0 with an isolated cell: its pivot block is zero (not SPD)."""
    pos = np.array([[0.0, 0, 0], [1.9, 0, 0], [50.0, 0, 0]])
    g = O.collide(pos, np.ones(3))
    t = O.build_tree(g)
    with pytest.raises(O.OracleError) as e:
        O.tree_factor(g, t, g_med=0.0)
    assert e.value.status == O.ENOTSPD


def test_mixed_precision_refinement():
    c, g, A, t, f = _setup(1000, 0)
    x, info = O.ir_solve(A, c["force"], f, tol=1e-8, inner_tol=1e-5)
    assert info.status == O.OK and info.relres_rec <= 1e-8 and info.outer >= 2
    G = A.dense()
    xd = np.linalg.solve(G, c["force"].ravel())
    err = np.linalg.norm(x.ravel() - xd) / np.linalg.norm(xd)
    assert err <= np.linalg.cond(G) * 1e-8
    # the FP32 inner solve alone stalls near FP32 accuracy: refinement is needed
    x1, info1 = O.ir_solve(A, c["force"], f, tol=1e-8, inner_tol=1e-12, max_outer=1, check=False)
    assert info1.status == O.ENOCONV


# ---------------------------------------------------------------- FP32 inner solve of the refinement

def test_fp32_tree_solve_against_fp64_and_dense():
    """The FP32 sweeps solve P x = b to FP32 accuracy: against the FP64 tree
    solve and against a dense solve of P (a transposed or misplaced coupling
    would leave an O(1) error).  Bound: the forward error of a solve with
    FP32 data and arithmetic, kappa(P) * n_depth * 2^-24, loosely 1e-3 here."""
    _, g, _, t, f = _setup(400, 2)
    b = np.random.default_rng(5).normal(size=(g.n, 3))
    x32 = O.tree_solve_f32(f, b)
    x64 = O.tree_solve(f, b)
    xd = np.linalg.solve(_dense_P(g, t), b.ravel()).reshape(-1, 3)
    e64 = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    ed = np.linalg.norm(x32 - xd) / np.linalg.norm(xd)
    assert e64 <= 1e-3 and ed <= 1e-3, (e64, ed)
    # not FP64: the FP32 path really rounds
    assert e64 > 1e-12
    # the residual of the FP32 result in P is small relative to b
    r = b.ravel() - _dense_P(g, t) @ x32.ravel()
    assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(b)


def test_fp32_tree_solve_rigid_translation():
    """P (1 (x) t) = g_med (1 (x) t) (tree Laplacian rows sum to zero), so the
    FP32 tree solve maps 1 (x) t to (1 (x) t)/g_med to FP32 accuracy."""
    _, g, _, t, f = _setup(300, 4)
    tv = np.array([0.3, -1.2, 0.7])
    b = np.tile(tv, (g.n, 1))
    x = O.tree_solve_f32(f, b)
    assert np.allclose(x, b / G0, rtol=1e-3, atol=0.0)


@pytest.mark.parametrize("kind", ["chain", "comb"])
def test_fp32_inner_solve_one_iteration_on_tree_graphs(kind):
    """A tree-shaped collision graph has P = Gamma, so the inner FP32 CG stops
    after one iteration with FP32 accuracy; its result is the dense solution
    to FP32 accuracy (this pins the FP32 sweeps' couplings: a transposed one
    makes P != Gamma)."""
    pos, R = _chain_or_comb(kind)
    g = O.collide(pos, R)
    A = O.assemble(g)
    t = O.build_tree(g)
    f = O.tree_factor(g, t)
    rhs = np.random.default_rng(1).normal(size=(g.n, 3))
    d, it, st = O.ir_inner(A, f, rhs, inner_tol=1e-4)
    assert st == O.OK and it == 1
    xd = np.linalg.solve(A.dense(), rhs.ravel())
    assert np.linalg.norm(d.ravel() - xd) <= 1e-4 * np.linalg.norm(xd)


def test_fp32_inner_iterations_match_fp64_pcg():
    """At an inner tolerance FP32 can reach (1e-4), the FP32 inner CG takes the
    FP64 tree-PCG's iteration count to within rounding (+-2), and its result
    has the FP64 solve's accuracy at that tolerance."""
    c, g, A, t, f = _setup(1000, 0)
    rhs = c["force"]
    for tol in (1e-3, 1e-4):
        d, it, st = O.ir_inner(A, f, rhs, inner_tol=tol)
        x64, info = O.pcg(A, rhs, "tree", f, tol=tol)
        assert st == O.OK and abs(it - info.iters) <= 2, (tol, it, info.iters)
        r = rhs.ravel() - O.spmv(A, d).ravel()
        assert np.linalg.norm(r) <= 1.5 * tol * np.linalg.norm(rhs)
