"""The one-workgroup PCG for small single systems (knob small_solve, on by
default): every iteration of Section 1.1's PCG with the tree preconditioner
inside one launch.  Checked against the oracle's tree-PCG (same x0, stopping
rule and preconditioner), against the launch-per-kernel path, and on the
edge cases of the solve (one cell, no contacts, zero and non-finite forces,
the iteration cap, fixed iteration counts, a warm start)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import sphere_cluster

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import check_velocity, host, to_dev  # noqa: E402


@pytest.fixture()
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    yield c
    c.close()


def _setup(ctx, c):
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    T = ctx.build_tree(g)
    M = ctx.factor_tree(g, T)
    return g, A, M


def _oracle(c):
    og = O.collide(c["pos"], c["radius"])
    return O.assemble(og), O.tree_factor(og, O.build_tree(og))


def _both(ctx, A, M, F, **kw):
    assert ctx.tune_get("small_solve") == 1
    vs, js = ctx.pcg_solve(A, M, F, **kw)
    ctx.tune("small_solve", 0)
    try:
        vm, jm = ctx.pcg_solve(A, M, F, **kw)
    finally:
        ctx.tune("small_solve", 1)
    return (vs, js), (vm, jm)


@pytest.mark.parametrize("n,seed", [(1000, 31), (1024, 32), (700, 33), (77, 34), (2, 35)])
def test_small_solve_matches_oracle(ctx, n, seed):
    c = sphere_cluster(n, seed)
    g, A, M = _setup(ctx, c)
    assert M.info()["tail_step"] == 0   # the whole elimination in one workgroup
    F = to_dev(c["force"])
    (vs, js), (vm, jm) = _both(ctx, A, M, F)
    print(f"small n={n}: {js['iters']} iterations (launch path {jm['iters']}), relres {js['relres_true']:.2e}",
          flush=True)
    assert js["status"] == 0 and js["relres_true"] <= 1.0001e-8
    assert abs(js["iters"] - jm["iters"]) <= 1
    oa, of = _oracle(c)
    check_velocity(host(vs), js["iters"], oa, c["force"], of)
    if n == 1000:
        # a different launch structure really ran (the dot products' sums differ)
        assert not torch.equal(vs, vm)
    # bitwise reproducible
    v2, j2 = ctx.pcg_solve(A, M, F)
    assert j2["iters"] == js["iters"] and torch.equal(v2, vs)


def test_small_solve_warm_start_and_fixed_iterations(ctx):
    c = sphere_cluster(1000, 36)
    g, A, M = _setup(ctx, c)
    F = to_dev(c["force"])
    oa, of = _oracle(c)
    rng = np.random.default_rng(5)
    x0 = rng.normal(0.0, 1e-3, c["force"].shape)
    vs, js = ctx.pcg_solve(A, M, F, to_dev(x0), use_x0=True)
    assert js["status"] == 0
    check_velocity(host(vs), js["iters"], oa, c["force"], of, x0=x0)
    # fixed iteration counts: early iterates agree with the oracle's closely
    for k in (1, 3, 7):
        v, j = ctx.pcg_solve(A, M, F, fixed_iters=k)
        xo, io = O.pcg(oa, c["force"], "tree", of, fixed_iters=k)
        assert j["iters"] == k == io.iters
        assert np.linalg.norm(host(v) - xo) <= 1e-12 * np.linalg.norm(xo), k


def test_small_solve_edge_cases(ctx):
    # one cell, and cells without any contact: the solve is P^{-1} F = F / g_med
    for pos in (np.zeros((1, 3)), np.arange(30, dtype=np.float64).reshape(10, 3) * 10.0):
        n = pos.shape[0]
        c = {"pos": pos, "radius": np.full(n, 1.0), "force": np.random.default_rng(n).normal(size=(n, 3))}
        g, A, M = _setup(ctx, c)
        v, j = ctx.pcg_solve(A, M, to_dev(c["force"]))
        assert j["status"] == 0 and j["iters"] <= 1
        oa, of = _oracle(c)
        xo, _ = O.pcg(oa, c["force"], "tree", of)
        assert np.allclose(host(v), xo, rtol=1e-13, atol=0)
    c = sphere_cluster(500, 37)
    g, A, M = _setup(ctx, c)
    F = to_dev(c["force"])
    # zero force: v = 0 without iterations
    v, j = ctx.pcg_solve(A, M, torch.zeros_like(F), torch.ones_like(F), use_x0=True)
    assert j["status"] == 0 and j["iters"] == 0 and not torch.any(v)
    # non-finite force
    Fb = F.clone()
    Fb[7, 1] = float("nan")
    _, j = ctx.pcg_solve(A, M, Fb, check=False)
    assert j["status"] == P.ENONFINITE
    # the iteration cap
    _, j = ctx.pcg_solve(A, M, F, max_iter=3, check=False)
    assert j["status"] == P.ENOCONV and j["iters"] == 3


def test_small_solve_falls_back_outside_its_range(ctx):
    # more cells than one workgroup holds, and a tail that does not reach the
    # first step: the launch-per-kernel path, same results as with the knob off
    for n, tail in ((1500, None), (1000, 300)):
        c = sphere_cluster(n, 38)
        if tail is not None:
            ctx.tune("tail_max", tail)
        try:
            g, A, M = _setup(ctx, c)
        finally:
            ctx.tune("tail_max", 2200)
        F = to_dev(c["force"])
        (vs, js), (vm, jm) = _both(ctx, A, M, F)
        assert js["iters"] == jm["iters"] and torch.equal(vs, vm), n
