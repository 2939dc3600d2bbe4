"""Pins of the oracle's friction matrix (eq. cell_cell_friction, Def. Block
Laplacian, Lemmas SymPosDefBuildingBlocks and blapposdef)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import sphere_cluster

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _graph(n, seed=0):
    c = sphere_cluster(n, seed)
    return c, O.collide(c["pos"], c["radius"])


def test_block_eigenstructure():
    """Lemma SymPosDefBuildingBlocks: W = w(g_par uu^T + g_perp(I - uu^T)) has
    eigenvalue w g_par on span(u) and w g_perp (twice) on its complement."""
    _, g = _graph(300, 5)
    for e in range(0, g.m, 7):
        W = O.friction_block(g.w[e], g.u[e], 1.0, 0.1)
        assert np.array_equal(W, W.T)
        lam, vec = np.linalg.eigh(W)
        assert np.allclose(lam, g.w[e] * np.array([0.1, 0.1, 1.0]), rtol=1e-13, atol=0)
        assert abs(abs(vec[:, 2] @ g.u[e]) - 1.0) < 1e-12
        assert np.allclose(W @ g.u[e], g.w[e] * g.u[e], rtol=0, atol=1e-15)


def test_rigid_translation_gives_g_med():
    """Block row sums of Gamma equal the self-loop g_med I, so Gamma(1 (x) t) = g_med (1 (x) t)."""
    _, g = _graph(2000, 1)
    A = O.assemble(g)
    for t in (np.array([1.0, 0, 0]), np.array([0.3, -2.0, 0.7])):
        x = np.tile(t, (g.n, 1))
        y = O.spmv(A, x)
        assert np.allclose(y, 1e-3 * x, rtol=0, atol=1e-14 * np.abs(A.val).max())


def test_structure_and_bitwise_symmetry():
    _, g = _graph(800, 3)
    A = O.assemble(g)
    assert A.rowptr[-1] == g.n + 2 * g.m
    D = A.dense()
    assert np.array_equal(D, D.T)
    for i in range(g.n):
        cols = A.bcol[A.rowptr[i]:A.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    # off-diagonal blocks are negative definite, diagonal blocks positive definite
    for k in range(0, A.bcol.size, 5):
        lam = np.linalg.eigvalsh(A.val[k])
        i = np.searchsorted(A.rowptr, k, side="right") - 1
        assert (lam > 0).all() if A.bcol[k] == i else (lam < 0).all()


def test_diagonal_is_g_med_plus_incident_blocks():
    _, g = _graph(500, 4)
    A = O.assemble(g, 1.0, 0.1, 1e-3)
    for i in range(0, g.n, 13):
        k = A.rowptr[i] + np.searchsorted(A.bcol[A.rowptr[i]:A.rowptr[i + 1]], i)
        want = 1e-3 * np.eye(3)
        for e in np.nonzero((g.ei == i) | (g.ej == i))[0]:
            u = g.u[e]
            want = want + g.w[e] * (1.0 * np.outer(u, u) + 0.1 * (np.eye(3) - np.outer(u, u)))
        assert np.allclose(A.val[k], want, rtol=1e-14, atol=1e-17)


def test_lambda_min_is_g_med_three_fold():
    """Lemma blapposdef: PSD block Laplacian + g_med I; the rigid translations attain g_med."""
    _, g = _graph(200, 9)
    comps = _components(g)
    assert comps == 1
    lam = np.linalg.eigvalsh(O.assemble(g).dense())
    assert np.allclose(lam[:3], 1e-3, rtol=1e-9)
    assert lam[3] > 1e-3 * (1 + 1e-6)


def _components(g):
    par = list(range(g.n))

    def f(x):
        while par[x] != x:
            par[x] = par[par[x]]
            x = par[x]
        return x
    for a, b in zip(g.ei, g.ej):
        par[f(a)] = f(b)
    return len({f(x) for x in range(g.n)})


def test_golden_two_cell_matrix():
    gold = json.load(open(os.path.join(GOLD, "two_cell.json")))
    g = O.collide(np.array(gold["pos"]), np.array(gold["radius"]))
    A = O.assemble(g, gold["g_par"], gold["g_perp"], gold["g_med"]).dense()
    W = np.diag(gold["expected"]["W_diag"])
    I = np.eye(3)
    want = np.block([[gold["g_med"] * I + W, -W], [-W, gold["g_med"] * I + W]])
    assert np.allclose(A, want, rtol=1e-14, atol=1e-17)
