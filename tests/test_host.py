"""Host-side logic that needs no GPU: the benchmark's contract checks, its
byte count for the product's roofline, and the seeded workload generators
that feed both the oracle and the library."""
import json
import math
import os
import subprocess
import sys

import numpy as np

from workloads import batched_instance, batched_sizes, dynamics_noise, fcc_ball_sites, sphere_cluster

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    # a single solve is not sharded: any N other than 1 is an error, before
    # anything touches a device
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60, cwd=ROOT)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_product_bytes_at_one_million_cells():
    # 1M-cell workload: n = 1,000,000 rows, m = 5,226,135 contacts, so
    # 10,452,270 off-diagonal entries and nnzb = n + 2m blocks.  Edge form:
    # per entry v = sqrt(w) u 24 B + column 4 B; per row a 6-entry diagonal block
    # (48 B), a row pointer, x and y (24 B each), plus the final row pointer.
    sys.path.insert(0, ROOT)
    import bench
    n, m = 1_000_000, 5_226_135
    nnzb = n + 2 * m
    assert bench.spmv_bytes(n, nnzb, form=1) == 392_663_564
    # block form: every block's 6 distinct FP64 entries and its column
    assert bench.spmv_bytes(n, nnzb, form=0) == 647_518_044
    # FP32 values halve the block bytes only
    assert bench.spmv_bytes(n, nnzb, form=0, val_bytes=24) == 647_518_044 - 24 * nnzb


def test_fcc_sites_are_a_closed_ball():
    s = fcc_ball_sites(1000)
    assert s.shape == (1000, 3)
    assert np.all(s.sum(axis=1) % 2 == 0)                      # FCC: x + y + z even
    assert len({tuple(r) for r in s.tolist()}) == 1000         # distinct sites
    r2 = (s * s).sum(axis=1)
    # the n smallest |site|^2: no site outside the set is closer than the farthest inside
    lim = int(math.isqrt(int(r2.max()))) + 2
    g = np.mgrid[-lim:lim + 1, -lim:lim + 1, -lim:lim + 1].reshape(3, -1).T
    g = g[g.sum(axis=1) % 2 == 0]
    gr2 = (g * g).sum(axis=1)
    assert np.count_nonzero(gr2 < r2.max()) <= 1000 <= np.count_nonzero(gr2 <= r2.max())
    assert fcc_ball_sites(0).shape == (0, 3)


def test_sphere_cluster_is_seeded():
    a, b, c = sphere_cluster(500, 0), sphere_cluster(500, 0), sphere_cluster(500, 1)
    for k in ("pos", "radius", "force"):
        assert a[k].dtype == np.float64 and np.all(np.isfinite(a[k]))
        assert np.array_equal(a[k], b[k])
        assert not np.array_equal(a[k], c[k])
    assert a["pos"].shape == (500, 3) and a["radius"].shape == (500,) and a["force"].shape == (500, 3)
    assert np.all(a["radius"] > 0)


def test_batched_sizes_are_log_uniform_in_range():
    s = np.asarray(batched_sizes(256, 1))
    assert s.shape == (256,)
    assert s.min() >= 1000 and s.max() <= 200_000
    assert np.array_equal(s, batched_sizes(256, 1))
    # the size is the instance's first draw: batched_instance agrees with it
    assert batched_instance(1)["pos"].shape[0] == s[0]
    # log-uniform: the median of log n sits near the middle of [log 1e3, log 2e5]
    mid = 0.5 * (math.log(1e3) + math.log(2e5))
    assert abs(float(np.median(np.log(s))) - mid) < 0.5


def test_dynamics_noise_streams():
    a, b = dynamics_noise(3, 2000), dynamics_noise(3, 2000)
    assert np.array_equal(a, b) and not np.array_equal(a, dynamics_noise(4, 2000))
    assert abs(a.std() - 0.1) < 0.01 and abs(a.mean()) < 0.01
