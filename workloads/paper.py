"""The paper's own benchmark geometries (Section 5.1, "Experimental Setup").

Spherical cells of radius r = 0.5 in four scenarios:

* ``hex``: hexagonal close packing (every cell has 12 nearest neighbours),
  each centre moved by N(0, (0.3 r)^2) per coordinate;
* ``random``: centres placed one by one at uniform random points of a
  spheroid, a point rejected when it lies closer than a minimum distance to
  a centre already placed;
* ``dumbbell``: two such random packings (balls) joined by a thin cylinder
  of randomly placed cells.

The paper does not give the lattice spacing, the minimum distance, the
domain sizes or the bridge's shape; the values below are this project's
readings (each named where it is set).  Cells touch when their centres are
closer than 2r (the collision rule of the library and of the oracle); the
contact area of the Hertz model, pi R_i R_j / (R_i + R_j) times the overlap,
is computed by the library and the oracle, not here.

Known-solution protocol (Section 5.1): the velocity x_true ~ N(0, 1) per
component is drawn here; the force is F = Gamma x_true, formed by whichever
implementation is being run.

Random draws: numpy PCG64 ``default_rng(seed)``; no method arithmetic here.
"""
from __future__ import annotations

import math

import numpy as np

RADIUS = 0.5
# HCP nearest-neighbour spacing: 0.9 (centres 10 % of a diameter closer than
# touching, so the unjittered lattice has 12 contacts per inner cell)
HEX_SPACING = 0.9
NOISE_SD = 0.3 * RADIUS
# random packings: hard-core distance 0.7 between centres and a number density
# of 1.6 centres per unit volume (a hard-core volume fraction of 0.29, well
# below the 0.38 at which random sequential addition jams, so the sampler
# never stalls; about 5.8 contacts per cell)
MIN_DIST = 0.7
DENSITY = 1.6
SPHEROID_AXES = (1.0, 1.0, 1.5)   # prolate spheroid, long axis z (relative)
# dumbbell: two equal balls whose surfaces are this many ball radii apart,
# joined by a cylinder of this radius filled at the same density (it reaches
# BRIDGE_OVERLAP into each ball so that its cells touch the balls' cells)
BRIDGE_GAP = 0.6
BRIDGE_RADIUS = 1.5
BRIDGE_OVERLAP = 0.5

# the paper's friction coefficients (Section 5.1) and substrate frictions
G_PAR, G_PERP = 2.0e6, 8.0e7
G_MED = {"hex": 3.0e4, "hex_ill": 3.0e3, "random": 3.0e4, "dumbbell": 3.0e4}


def hcp_sites(n: int, a: float = HEX_SPACING) -> np.ndarray:
    """The n sites of an ABAB-stacked hexagonal close packing (nearest-
    neighbour distance a) closest to the origin, ties by (x, y, z)."""
    n = int(n)
    if n <= 0:
        return np.zeros((0, 3))
    # sites per unit volume: sqrt(2) / a^3
    rho = (3.0 * n * a ** 3 / (4.0 * math.pi * math.sqrt(2.0))) ** (1.0 / 3.0)
    k = int(math.ceil(rho / a)) + 3
    while True:
        i, j, l = np.meshgrid(np.arange(-2 * k, 2 * k + 1), np.arange(-2 * k, 2 * k + 1), np.arange(-k, k + 1),
                              indexing="ij")
        i, j, l = i.ravel(), j.ravel(), l.ravel()
        odd = (l & 1).astype(np.float64)
        x = a * (i + 0.5 * j) + odd * (a / 2.0)
        y = a * (math.sqrt(3.0) / 2.0) * j + odd * (a / (2.0 * math.sqrt(3.0)))
        z = a * math.sqrt(2.0 / 3.0) * l
        r2 = x * x + y * y + z * z
        inside = r2 <= (k * a) ** 2
        if int(inside.sum()) >= n:
            x, y, z, r2 = x[inside], y[inside], z[inside], r2[inside]
            break
        k += 2
    order = np.lexsort((z, y, x, r2))[:n]
    return np.stack([x[order], y[order], z[order]], axis=1)


def _rsa(rng, n, inside, lo, hi, min_dist, placed=None):
    """Random sequential addition: uniform proposals in the box [lo, hi],
    taken in order; a proposal is kept when `inside` accepts it and no kept
    centre (from `placed` or kept before it) is closer than min_dist.
    Proposals are drawn 4096 at a time and resolved in their order."""
    from scipy.spatial import cKDTree
    lo, hi = np.asarray(lo, dtype=np.float64), np.asarray(hi, dtype=np.float64)
    old = np.zeros((0, 3)) if placed is None else np.asarray(placed, dtype=np.float64)
    kept = []
    count, tries = 0, 0
    while count < n:
        batch = rng.uniform(lo, hi, (4096, 3))
        tries += batch.shape[0]
        if tries > 400 * max(n, 1000):
            raise RuntimeError("random packing: too many rejections")
        cand = batch[inside(batch)]
        if cand.shape[0] == 0:
            continue
        prev = np.concatenate([old] + kept) if (old.shape[0] or kept) else np.zeros((0, 3))
        if prev.shape[0]:
            d, _ = cKDTree(prev).query(cand, k=1)
            cand = cand[d >= min_dist]
        if cand.shape[0] == 0:
            continue
        # within the batch: the first of every close pair wins, in order
        close = [[] for _ in range(cand.shape[0])]
        for a, b in cKDTree(cand).query_pairs(min_dist):
            if np.sum((cand[a] - cand[b]) ** 2) < min_dist * min_dist:
                lo_i, hi_i = (a, b) if a < b else (b, a)
                close[hi_i].append(lo_i)
        take = np.zeros(cand.shape[0], dtype=bool)
        for k in range(cand.shape[0]):
            if count >= n:
                break
            if not any(take[j] for j in close[k]):
                take[k] = True
                count += 1
        kept.append(cand[take])
    return np.concatenate(kept) if kept else np.zeros((0, 3))


def _spheroid_semi_axes(n):
    vol = n / DENSITY
    s = (3.0 * vol / (4.0 * math.pi * SPHEROID_AXES[0] * SPHEROID_AXES[1] * SPHEROID_AXES[2])) ** (1.0 / 3.0)
    return tuple(s * c for c in SPHEROID_AXES)


def _ball_radius(n):
    return (3.0 * n / (4.0 * math.pi * DENSITY)) ** (1.0 / 3.0)


def paper_cells(kind: str, n: int, seed: int = 0):
    """One of the paper's geometries with n cells: dict of pos [n,3], radius
    [n], x_true [n,3] (the known solution), g_par, g_perp, g_med."""
    rng = np.random.default_rng(seed)
    n = int(n)
    if kind in ("hex", "hex_ill"):
        pos = hcp_sites(n) + rng.normal(0.0, NOISE_SD, (n, 3))
    elif kind == "random":
        ax = _spheroid_semi_axes(n)

        def inside(p):
            return (p[:, 0] / ax[0]) ** 2 + (p[:, 1] / ax[1]) ** 2 + (p[:, 2] / ax[2]) ** 2 <= 1.0

        pos = _rsa(rng, n, inside, [-ax[0], -ax[1], -ax[2]], [ax[0], ax[1], ax[2]], MIN_DIST)
    elif kind == "dumbbell":
        rb = _ball_radius(n / 2.0)
        gap = BRIDGE_GAP * rb
        cx = rb + gap / 2.0   # ball centres at (+-cx, 0, 0)
        half = gap / 2.0 + BRIDGE_OVERLAP   # the bridge spans |x| <= half
        n_bridge = max(1, int(round(DENSITY * math.pi * BRIDGE_RADIUS ** 2 * gap)))
        na = (n - n_bridge) // 2
        nb = n - n_bridge - na

        def ball(c):
            return lambda p: (p[:, 0] - c) ** 2 + p[:, 1] ** 2 + p[:, 2] ** 2 <= rb * rb

        a = _rsa(rng, na, ball(-cx), [-cx - rb, -rb, -rb], [-cx + rb, rb, rb], MIN_DIST)
        b = _rsa(rng, nb, ball(cx), [cx - rb, -rb, -rb], [cx + rb, rb, rb], MIN_DIST)

        def bridge(p):
            return (np.abs(p[:, 0]) <= half) & (p[:, 1] ** 2 + p[:, 2] ** 2 <= BRIDGE_RADIUS ** 2)

        c = _rsa(rng, n_bridge, bridge, [-half, -BRIDGE_RADIUS, -BRIDGE_RADIUS], [half, BRIDGE_RADIUS, BRIDGE_RADIUS],
                 MIN_DIST, placed=np.concatenate([a, b]))
        pos = np.concatenate([a, c, b])
    else:
        raise ValueError(f"unknown geometry {kind!r}")
    x_true = rng.normal(0.0, 1.0, (n, 3))
    return {"pos": np.ascontiguousarray(pos), "radius": np.full(n, RADIUS), "x_true": np.ascontiguousarray(x_true),
            "g_par": G_PAR, "g_perp": G_PERP, "g_med": G_MED[kind]}
