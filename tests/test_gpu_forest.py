"""GPU parity of the local-MST forest (Section 6, Discussion) against the
oracle: the Z-order clusters and the forest (edges, parent, depth) bit for
bit, the forest's preconditioner apply to FP64 rounding, and the PCG
velocity (gpu_util.check_velocity_spread: these preconditioners converge
more slowly than the global tree, and the recurrence residual can creep
along the tolerance for a few iterations), for single and batched graphs and
at the 1M-cell workload."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import batched_instance, sphere_cluster

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import check_velocity_spread, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    yield c
    c.close()


def _forest_equal(ctx, T, n, ot, ocl):
    cl, nc = ctx.tree_clusters(T, n)
    assert np.array_equal(host(cl), ocl)
    assert nc == int(ocl.max()) + 1 if n else nc == 0
    e = {k: host(v) for k, v in ctx.tree_export(T, n).items()}
    assert np.array_equal(e["tree_edge"], ot.tree_edge)
    assert np.array_equal(e["parent"], ot.parent)
    assert np.array_equal(e["depth"], ot.depth)


@pytest.mark.parametrize("n,seed,K", [(1000, 0, 1), (1000, 1, 37), (1000, 2, 5000), (20000, 3, 512),
                                      (30000, 4, 1024)])
def test_forest_bit_exact_and_solve(ctx, n, seed, K):
    c = sphere_cluster(n, seed)
    print(f"forest: n={n} K={K}", flush=True)
    pos, R, F = to_dev(c["pos"]), to_dev(c["radius"]), to_dev(c["force"])
    g = ctx.collide(pos, R)
    T = ctx.build_forest(g, pos, R, K)
    og = O.collide(c["pos"], c["radius"])
    ot, ocl = O.build_forest(og, c["pos"], c["radius"], K)
    _forest_equal(ctx, T, n, ot, ocl)
    M = ctx.factor_tree(g, T)
    info = M.info()
    if info["steps"] >= 2:
        assert info["tail_step"] == info["steps"]   # grouped by component, no single-workgroup tail
    fo = O.tree_factor(og, ot)
    b = np.random.default_rng(seed).normal(size=(n, 3))
    z = host(ctx.prec_apply(M, to_dev(b)))
    zo = O.tree_solve(fo, b)
    assert np.linalg.norm(z - zo) <= 1e-11 * np.linalg.norm(zo)
    A = ctx.assemble_gamma(g)
    v, vi = ctx.pcg_solve(A, M, F)
    assert vi["status"] == 0
    err, spread = check_velocity_spread(host(v), vi["iters"], O.assemble(og), c["force"], fo)
    print(f"forest: n={n} K={K}: {vi['iters']} iterations, velocity error vs the oracle {err:.2e} "
          f"(spread {spread})", flush=True)


def test_forest_batched(ctx):
    sizes = [1000, 300, 2000, 57, 1500, 1, 2]
    parts = [batched_instance(k + 1, n_override=s) for k, s in enumerate(sizes)]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pos = np.concatenate([p["pos"] for p in parts])
    R = np.concatenate([p["radius"] for p in parts])
    F = np.concatenate([p["force"] for p in parts])
    dpos, dR = to_dev(pos), to_dev(R)
    g = ctx.collide_batched(off, dpos, dR)
    T = ctx.build_forest(g, dpos, dR, 256)
    n = int(off[-1])
    # the oracle on the batch as one graph (its collide on the concatenation
    # would join instances; the graph is the union of the instances' graphs)
    e = {k: host(t) for k, t in ctx.graph_export(g).items()}
    og = O.Graph(n, e["rowptr"], e["col"], e["ei"], e["ej"], e["w"], e["u"])
    for k, p in enumerate(parts):   # the union really is the instances' graphs
        ok = O.collide(p["pos"], p["radius"])
        sel = (e["ei"] >= off[k]) & (e["ei"] < off[k + 1])
        assert np.array_equal(e["ei"][sel] - off[k], ok.ei) and np.array_equal(e["w"][sel], ok.w)
    ot, ocl = O.build_forest(og, pos, R, 256, off)
    _forest_equal(ctx, T, n, ot, ocl)
    M = ctx.factor_tree(g, T)
    A = ctx.assemble_gamma(g)
    v, infos = ctx.pcg_solve_batched(A, M, off, to_dev(F))
    vh = host(v)
    eoff = 0
    for k, p in enumerate(parts):
        sub = slice(int(off[k]), int(off[k + 1]))
        ok = O.collide(p["pos"], p["radius"])
        # the instance's share of the batch's forest (the grid is the batch's)
        mine = ot.tree_edge[(ot.tree_edge >= eoff) & (ot.tree_edge < eoff + ok.m)] - eoff
        eoff += ok.m
        assert infos[k]["status"] == 0
        check_velocity_spread(vh[sub], infos[k]["iters"], O.assemble(ok), p["force"],
                              O.tree_factor(ok, O.tree_from_edges(ok, mine)))


def test_forest_1M_bench_configuration(ctx):
    """The 1M-cell workload with 512-cell clusters: clusters and forest bit for
    bit, the apply against the oracle's tree solve, and the PCG velocity
    against the oracle's own PCG with the same forest."""
    n, K = 1_000_000, 512
    c = sphere_cluster(n, 0)
    print("forest 1M: GPU chain", flush=True)
    pos, R, F = to_dev(c["pos"]), to_dev(c["radius"]), to_dev(c["force"])
    g = ctx.collide(pos, R)
    T = ctx.build_forest(g, pos, R, K)
    M = ctx.factor_tree(g, T)
    A = ctx.assemble_gamma(g)
    v, vi = ctx.pcg_solve(A, M, F)
    assert vi["status"] == 0
    print("forest 1M: oracle", flush=True)
    og = O.collide(c["pos"], c["radius"])
    ot, ocl = O.build_forest(og, c["pos"], c["radius"], K)
    _forest_equal(ctx, T, n, ot, ocl)
    fo = O.tree_factor(og, ot)
    b = np.random.default_rng(0).normal(size=(n, 3))
    z = host(ctx.prec_apply(M, to_dev(b)))
    zo = O.tree_solve(fo, b)
    assert np.linalg.norm(z - zo) <= 1e-10 * np.linalg.norm(zo)
    print("forest 1M: oracle PCG", flush=True)
    err, spread = check_velocity_spread(host(v), vi["iters"], O.assemble(og), c["force"], fo)
    print(f"forest 1M: {vi['iters']} iterations, velocity error vs the oracle {err:.2e} (spread {spread})",
          flush=True)
