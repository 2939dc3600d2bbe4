"""Sphere packings used as synthetic workloads.

The paper benchmarks on jittered lattices and random packings of spherical
cells (Section 5, "Experimental Setup").  The workloads here follow the same
pattern at the sizes we measure:

* centres on a face-centred cubic (FCC) lattice whose nearest-neighbour
  spacing is 1.9, filling a ball around the origin, jittered by N(0, 0.05^2);
* radii uniform in [0.95, 1.05], so nearest neighbours overlap by ~0.1 and a
  cell has up to 12 contacts;
* forces F ~ N(0, 1) per component.

Site selection: the FCC sites are the integer triples (x, y, z) with x+y+z
even, scaled by a = 1.9/sqrt(2).  The N sites with the smallest integer
x^2+y^2+z^2 are taken, ties broken by (x, y, z) lexicographically ascending;
the vertex id is the rank in that order, so vertex 0 is the origin.

Random draws use numpy's PCG64 `default_rng(seed)` in the order
jitter -> radii -> forces.
"""
from __future__ import annotations

import math

import numpy as np

A_FCC = 1.9 / math.sqrt(2.0)
JITTER_SD = 0.05
R_LO, R_HI = 0.95, 1.05


def fcc_ball_sites(n: int) -> np.ndarray:
    """Integer FCC sites (x+y+z even) of the n smallest |site|^2, ties by (x,y,z)."""
    n = int(n)
    if n <= 0:
        return np.zeros((0, 3), dtype=np.int64)
    # FCC sites are half of the integer points: count(|s| <= rho) ~ (2 pi / 3) rho^3
    rho = (3.0 * n / (2.0 * math.pi)) ** (1.0 / 3.0)
    k = int(math.ceil(rho * 1.05)) + 2
    while True:
        ax = np.arange(-k, k + 1, dtype=np.int64)
        x, y, z = np.meshgrid(ax, ax, ax, indexing="ij")
        x = x.ravel(); y = y.ravel(); z = z.ravel()
        keep = ((x + y + z) & 1) == 0
        x = x[keep]; y = y[keep]; z = z[keep]
        r2 = x * x + y * y + z * z
        inside = r2 <= k * k
        # every site with |s|^2 <= k^2 lies in the cube; need n of them
        if int(inside.sum()) >= n:
            x = x[inside]; y = y[inside]; z = z[inside]; r2 = r2[inside]
            break
        k += 2
    order = np.lexsort((z, y, x, r2))[:n]
    return np.stack([x[order], y[order], z[order]], axis=1)


def sphere_cluster(n: int, seed: int = 0, rng: np.random.Generator | None = None):
    """Jittered FCC ball of n spheres.

    Returns a dict with float64 arrays: pos [n,3], radius [n], force [n,3].
    """
    if rng is None:
        rng = np.random.default_rng(seed)
    sites = fcc_ball_sites(n)
    jitter = rng.normal(0.0, JITTER_SD, (n, 3))
    radius = rng.uniform(R_LO, R_HI, n)
    force = rng.normal(0.0, 1.0, 3 * n).reshape(n, 3)
    pos = sites.astype(np.float64) * A_FCC + jitter
    return {
        "pos": np.ascontiguousarray(pos),
        "radius": np.ascontiguousarray(radius),
        "force": np.ascontiguousarray(force),
    }


def unjittered_cluster(n: int):
    """FCC ball with no jitter and unit radii (closed-form degree 12 inside)."""
    sites = fcc_ball_sites(n)
    return {
        "pos": np.ascontiguousarray(sites.astype(np.float64) * A_FCC),
        "radius": np.ones(n),
        "force": np.zeros((n, 3)),
    }


BATCH_NMIN, BATCH_NMAX = 1_000, 200_000


def batched_sizes(n_inst: int = 256, first_seed: int = 1):
    """Instance sizes of the batched workload: log-uniform in [1e3, 2e5].

    Instance k uses `default_rng(first_seed + k)`; its first draw is the size.
    """
    out = []
    for k in range(n_inst):
        rng = np.random.default_rng(first_seed + k)
        out.append(int(math.floor(math.exp(rng.uniform(math.log(BATCH_NMIN), math.log(BATCH_NMAX))))))
    return out


def batched_instance(seed: int, n_override: int | None = None):
    """One instance of the batched workload (size drawn first, then the cluster)."""
    rng = np.random.default_rng(seed)
    n = int(math.floor(math.exp(rng.uniform(math.log(BATCH_NMIN), math.log(BATCH_NMAX)))))
    if n_override is not None:
        n = int(n_override)
    return sphere_cluster(n, rng=rng)


def dynamics_noise(step: int, n: int, sd: float = 0.1) -> np.ndarray:
    """Active-force noise of time step `step`: N(0, sd^2) per component, own stream."""
    rng = np.random.default_rng(10_000 + int(step))
    return np.ascontiguousarray(rng.normal(0.0, sd, (n, 3)))
