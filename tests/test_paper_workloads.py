"""The paper's benchmark geometries (Section 5.1) as generated here, and the
oracle's solves on them: hexagonal close packing (12 neighbours before the
noise), random packings that respect their hard-core distance and domain,
the dumbbell's bridge, and the known-solution protocol F = Gamma x_true."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import oracle as O
from workloads import paper as W


def test_hcp_unjittered_has_twelve_neighbours_inside():
    sites = W.hcp_sites(3000)
    g = O.collide(sites, np.full(3000, W.RADIUS))
    deg = np.diff(g.rowptr)
    r = np.linalg.norm(sites, axis=1)
    inner = r < r.max() - 2.0
    assert inner.sum() > 500 and np.all(deg[inner] == 12)
    # nearest-neighbour distance is the spacing
    d = cKDTree(sites).query(sites, k=2)[0][:, 1]
    assert np.allclose(d, W.HEX_SPACING, rtol=1e-12)


@pytest.mark.parametrize("kind", ["random", "dumbbell"])
def test_random_packings_respect_hard_core_and_domain(kind):
    c = W.paper_cells(kind, 4000, 3)
    pos = c["pos"]
    assert pos.shape == (4000, 3)
    d = cKDTree(pos).query(pos, k=2)[0][:, 1]
    assert d.min() >= W.MIN_DIST
    if kind == "random":
        ax = W._spheroid_semi_axes(4000)
        assert np.all(((pos / np.array(ax)) ** 2).sum(1) <= 1.0)
    else:
        # two balls and a bridge: cells near x = 0 lie in the thin cylinder
        mid = np.abs(pos[:, 0]) < 0.5
        assert mid.sum() > 0 and np.all(pos[mid, 1] ** 2 + pos[mid, 2] ** 2 <= W.BRIDGE_RADIUS ** 2)
    # seeded: the same seed gives the same cells
    assert np.array_equal(W.paper_cells(kind, 4000, 3)["pos"], pos)


@pytest.mark.parametrize("kind", ["hex", "hex_ill", "random", "dumbbell"])
def test_oracle_solves_the_known_solution_problem(kind):
    """F = Gamma x_true; every preconditioner reaches relres 1e-8, its true
    error stays small, and a preconditioner needs fewer iterations than
    none."""
    c = W.paper_cells(kind, 2000, 1)
    g = O.collide(c["pos"], c["radius"], area="hertz")
    A = O.assemble(g, c["g_par"], c["g_perp"], c["g_med"])
    F = O.spmv(A, c["x_true"])
    f = O.tree_factor(g, O.build_tree(g), c["g_par"], c["g_perp"], c["g_med"])
    it = {}
    for prec in ("none", "jacobi", "tree"):
        x, info = O.pcg(A, F, prec, f if prec == "tree" else None)
        it[prec] = info.iters
        assert info.relres_true <= 1.0001e-8
        err = np.linalg.norm(x - c["x_true"]) / np.linalg.norm(c["x_true"])
        assert err <= 1e-3, (prec, err)
    assert it["tree"] < it["none"] and it["jacobi"] < it["none"], it
