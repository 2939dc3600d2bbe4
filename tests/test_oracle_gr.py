"""Oracle pins: PCG stopped on the Gauss-Radau bound of the energy-norm error
(Section 5 monitors CG with Gauss-Radau error estimates; Section 4's bound
lambda_min(P^-1 Gamma) >= 1 for a subgraph preconditioner gives the node
mu = 1).  The bound is checked against the true error from a dense solve at
every iteration, the running sum S_k against ||x||_Gamma^2 - eps_k, the
one-step exactness on tree-shaped graphs (P = Gamma, one eigenvalue), the
monotonicity in mu, and the final error against the tolerance."""
import numpy as np
import pytest
import scipy.linalg

from oracle import oracle as O
from workloads import sphere_cluster

G0 = 1e-3   # the oracle's default g_med: lambda_min(Gamma) >= g_med (Lemma blapposdef)


def _setup(n, seed):
    c = sphere_cluster(n, seed)
    g = O.collide(c["pos"], c["radius"])
    A = O.assemble(g)
    t = O.build_tree(g)
    return c, g, A, O.tree_factor(g, t)


def _true_errors(A, F, prec, f, kmax):
    """eps_k = ||x - x_k||_Gamma^2 for k = 0..kmax from the plain PCG's iterates
    (the same recurrence from x0 = 0) and a dense solve."""
    G = A.dense()
    xs = scipy.linalg.cho_solve(scipy.linalg.cho_factor(G), F.ravel())
    eps = []
    for k in range(kmax + 1):
        if k == 0:
            xk = np.zeros_like(xs)
        else:
            xk = O.pcg(A, F, prec, f, fixed_iters=k)[0].ravel()
        e = xs - xk
        eps.append(float(e @ G @ e))
    return np.array(eps), float(xs @ G @ xs)


@pytest.mark.parametrize("prec,mu", [("tree", 1.0), ("tree", 0.5), ("none", G0)])
def test_bound_dominates_the_true_error(prec, mu):
    c, g, A, f = _setup(300, 4)
    F = c["force"]
    x, info, hist = O.pcg_gr(A, F, prec, f, tol=1e-6, mu=mu)
    assert info.status == 0
    k = info.iters
    eps, xnorm2 = _true_errors(A, F, prec, f, k)
    S, bound = hist[:, 0], hist[:, 1]
    # eps_k drops by alpha_k rho_k per step: S_k + eps_k = ||x||^2 (x0 = 0)
    assert np.allclose(S + eps, xnorm2, rtol=1e-9, atol=0)
    # the Gauss-Radau bound holds at every iteration (up to rounding)
    assert np.all(eps <= bound * (1 + 1e-9) + 1e-12 * xnorm2), np.max(eps / bound)
    # and the solve stops where the bound of the relative error meets tol
    rel = np.sqrt(bound / (S + bound))
    assert rel[-1] <= 1e-6 < rel[-2]
    assert np.sqrt(eps[-1] / xnorm2) <= 1e-6


def test_one_step_exact_on_tree_graphs():
    """A tree-shaped collision graph: P = Gamma, so P^-1 Gamma = I, mu = 1 is
    its only eigenvalue, and the Gauss-Radau bound is exact: at k = 0 it is
    F' Gamma^-1 F = ||x||^2, after one step it is zero."""
    n = 30
    pos = np.array([[1.9 * k, 0.1 * np.sin(k), 0.0] for k in range(n)])
    g = O.collide(pos, np.full(n, 1.0))
    assert g.m == n - 1
    A = O.assemble(g)
    f = O.tree_factor(g, O.build_tree(g))
    F = np.random.default_rng(1).normal(size=(n, 3))
    x, info, hist = O.pcg_gr(A, F, "tree", f, tol=1e-10, mu=1.0)
    G = A.dense()
    xd = np.linalg.solve(G, F.ravel())
    assert info.iters == 1
    assert abs(hist[0, 1] - xd @ F.ravel()) <= 1e-12 * (xd @ F.ravel())
    assert abs(hist[1, 1]) <= 1e-12 * (xd @ F.ravel()) and info.relres_rec <= 1e-6
    assert np.linalg.norm(x.ravel() - xd) <= 1e-12 * np.linalg.norm(xd)


def test_smaller_mu_is_a_looser_bound():
    c, g, A, f = _setup(300, 5)
    runs = {mu: O.pcg_gr(A, c["force"], "tree", f, tol=1e-6, mu=mu) for mu in (1.0, 0.5, 0.1)}
    k = min(r[1].iters for r in runs.values())
    b1, b05, b01 = (runs[mu][2][:k + 1, 1] for mu in (1.0, 0.5, 0.1))
    assert np.all(b05 >= b1 * (1 - 1e-12)) and np.all(b01 >= b05 * (1 - 1e-12))
    assert runs[1.0][1].iters <= runs[0.5][1].iters <= runs[0.1][1].iters


def test_edge_cases():
    c, g, A, f = _setup(100, 6)
    # zero force: x = 0 at once
    x, info, hist = O.pcg_gr(A, np.zeros((g.n, 3)), "tree", f, tol=1e-8)
    assert info.iters == 0 and not np.any(x)
    # mu must be positive; non-finite forces are refused
    _, info, _ = O.pcg_gr(A, c["force"], "tree", f, mu=0.0, check=False)
    assert info.status == O.EINVAL
    Fb = c["force"].copy()
    Fb[3, 1] = np.nan
    _, info, _ = O.pcg_gr(A, Fb, "tree", f, check=False)
    assert info.status == O.ENONFINITE
    # the iteration cap
    _, info, _ = O.pcg_gr(A, c["force"], "tree", f, tol=1e-12, max_iter=3, check=False)
    assert info.status == O.ENOCONV and info.iters == 3
