"""Pins of the oracle's forces and Euler step (Section 2, Steps 2 and 5) for
the time-stepping workload: pairwise repulsion k w_ij n_ij plus noise."""
import numpy as np

from oracle import oracle as O
from workloads import sphere_cluster, dynamics_noise


def test_repulsion_obeys_newtons_third_law():
    c = sphere_cluster(1500, 3)
    g = O.collide(c["pos"], c["radius"])
    F = O.forces(g, np.zeros((g.n, 3)), 5.0)
    assert np.abs(F.sum(axis=0)).max() <= 1e-12 * np.abs(F).sum()
    # repulsion pushes each cell away from its contacts: F_i . (r_i - centroid of contacts) > 0 on average
    noise = dynamics_noise(1, g.n)
    F2 = O.forces(g, noise, 5.0)
    assert np.allclose(F2 - F, noise, rtol=0, atol=1e-15)


def test_two_cell_force_closed_form():
    pos = np.array([[0.0, 0, 0], [0.0, 1.5, 0]])
    g = O.collide(pos, np.array([1.0, 1.0]))
    F = O.forces(g, np.zeros((2, 3)), 5.0)
    # overlap 0.5, repulsion 5 * 0.5 = 2.5 along the line of centres, pushing apart
    assert np.allclose(F, [[0, -2.5, 0], [0, 2.5, 0]], rtol=0, atol=1e-15)


def test_euler_step():
    pos = np.arange(12.0).reshape(4, 3)
    v = np.ones((4, 3))
    assert np.array_equal(O.euler(pos, v, 0.01), pos + 0.01)
