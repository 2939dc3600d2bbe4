"""Pins of the oracle's collision detection (Section 2, Steps 1-2)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from workloads import sphere_cluster
from workloads.spheres import unjittered_cluster

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n,seed", [(0, 0), (1, 0), (2, 3), (57, 1), (1000, 0), (2500, 7)])
def test_cell_list_equals_all_pairs(n, seed):
    c = sphere_cluster(n, seed)
    a = O.collide(c["pos"], c["radius"], "brute")
    b = O.collide(c["pos"], c["radius"], "cells")
    for f in ("rowptr", "col", "ei", "ej", "w", "u"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f


def test_brute_force_matches_numpy_pair_scan():
    """Independent all-pairs scan in numpy (vectorised, same rounding order)."""
    c = sphere_cluster(400, 11)
    g = O.collide(c["pos"], c["radius"], "cells")
    p, R = c["pos"], c["radius"]
    i, j = np.triu_indices(len(R), 1)
    d = p[j] - p[i]
    dist = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
    s = R[i] + R[j]
    hit = dist < s
    assert np.array_equal(g.ei, i[hit]) and np.array_equal(g.ej, j[hit])
    assert np.array_equal(g.w, (s - dist)[hit])
    assert np.array_equal(g.u, (d / dist[:, None])[hit])


def test_rows_sorted_and_symmetric():
    c = sphere_cluster(3000, 2)
    g = O.collide(c["pos"], c["radius"])
    n = g.n
    assert g.rowptr[-1] == 2 * g.m
    for i in range(n):
        row = g.col[g.rowptr[i]:g.rowptr[i + 1]]
        assert np.all(np.diff(row) > 0)
        assert i not in row
    pairs = set(zip(g.ei.tolist(), g.ej.tolist()))
    assert len(pairs) == g.m
    assert np.all(g.ei < g.ej)
    order = np.lexsort((g.ej, g.ei))
    assert np.array_equal(order, np.arange(g.m))
    assert np.allclose(np.linalg.norm(g.u, axis=1), 1.0, atol=1e-15)
    assert np.all(g.w > 0)


def test_unjittered_fcc_closed_form_degree_12():
    """FCC with nearest-neighbour spacing 1.9 and unit radii: every site whose 12
    lattice neighbours are all present has exactly 12 contacts, overlap 0.1."""
    n = 2000
    c = unjittered_cluster(n)
    g = O.collide(c["pos"], c["radius"])
    deg = np.diff(g.rowptr)
    assert deg.max() == 12
    sites = np.rint(c["pos"] / (1.9 / np.sqrt(2))).astype(int)
    index = {tuple(s): k for k, s in enumerate(sites)}
    nbr = [(a, b, 0) for a in (-1, 1) for b in (-1, 1)]
    nbr += [(a, 0, b) for a in (-1, 1) for b in (-1, 1)]
    nbr += [(0, a, b) for a in (-1, 1) for b in (-1, 1)]
    interior = [k for k, s in enumerate(sites) if all(tuple(s + np.array(o)) in index for o in nbr)]
    assert len(interior) > 500
    assert np.all(deg[interior] == 12)
    for k in interior[:50]:
        expect = sorted(index[tuple(sites[k] + np.array(o))] for o in nbr)
        assert g.col[g.rowptr[k]:g.rowptr[k + 1]].tolist() == expect
    assert np.allclose(g.w, 0.1, rtol=0, atol=1e-12)


def test_strict_contact_and_golden_two_cells():
    gold = json.load(open(os.path.join(GOLD, "two_cell.json")))
    g = O.collide(np.array(gold["pos"]), np.array(gold["radius"]))
    assert g.m == gold["expected"]["m"]
    assert g.w[0] == gold["expected"]["w"]
    assert np.array_equal(g.u[0], gold["expected"]["u"])
    # exactly touching spheres (d == R_i + R_j) are not in contact
    g2 = O.collide(np.array([[0.0, 0, 0], [2.0, 0, 0]]), np.array([1.0, 1.0]))
    assert g2.m == 0
    g3 = O.collide(np.array([[0.0, 0, 0], [0.0, 0, 1.5]]), np.array([1.0, 0.75]))
    assert g3.m == 1 and np.array_equal(g3.u[0], [0.0, 0.0, 1.0]) and g3.w[0] == 0.25


def test_coincident_centres_rejected():
    with pytest.raises(O.OracleError) as e:
        O.collide(np.zeros((2, 3)), np.ones(2), "brute")
    assert e.value.status == O.EINVAL
    with pytest.raises(O.OracleError):
        O.collide(np.zeros((2, 3)), np.ones(2), "cells")


def test_hertz_contact_area_closed_form():
    """Two spheres pressed together by an overlap delta touch in a disc of
    radius sqrt(R* delta), R* = R1 R2 / (R1 + R2) (Hertz), so the area is
    pi R* delta; equal spheres of radius r give pi r delta / 2."""
    r1, r2, d = 0.5, 0.75, 1.1
    pos = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    R = np.array([r1, r2])
    g0 = O.collide(pos, R)
    g1 = O.collide(pos, R, area="hertz")
    delta = (r1 + r2) - d
    assert g0.w[0] == delta
    want = np.pi * (r1 * r2 / (r1 + r2)) * delta
    assert abs(g1.w[0] - want) <= 1e-15 * want
    # the area grows linearly with the overlap and with the reduced radius
    pos2 = np.array([[0.0, 0.0, 0.0], [0.9, 0.0, 0.0]])
    g2 = O.collide(pos2, np.array([0.5, 0.5]), area="hertz")
    assert abs(g2.w[0] - np.pi * 0.25 * 0.1) <= 1e-15
    # same contacts, same u, same numbering as the overlap model
    assert np.array_equal(g0.ei, g1.ei) and np.array_equal(g0.u, g1.u)
