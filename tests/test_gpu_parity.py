"""GPU parity: the HIP library, called through the C ABI, against the FP64
oracle on the same seeded inputs.

Bars: graph (neighbour lists, edge list, w, u), Gamma, tree edges, parent and
depth bit-exact; preconditioner apply and velocities to relative error 1e-8
or better (see each test for the tolerance and its reason)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from workloads import sphere_cluster
from workloads.spheres import unjittered_cluster

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2410_04512_amd")
from tests.gpu_util import gpu_chain, host, to_dev  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = P.Context()
    yield c
    c.close()


def _graph_equal(ctx, g, og):
    e = {k: host(v) for k, v in ctx.graph_export(g).items()}
    assert e["ei"].shape[0] == og.m
    for f in ("rowptr", "col", "ei", "ej", "w", "u"):
        assert np.array_equal(e[f], getattr(og, f)), f


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (1000, 0), (4097, 3), (20000, 5)])
def test_collide_bit_exact(ctx, n, seed):
    c = sphere_cluster(n, seed)
    print(f"collide n={n} seed={seed}", flush=True)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    _graph_equal(ctx, g, O.collide(c["pos"], c["radius"]))


def test_collide_unjittered_ties(ctx):
    c = unjittered_cluster(3000)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    _graph_equal(ctx, g, O.collide(c["pos"], c["radius"]))


@pytest.mark.parametrize("n,seed", [(1000, 0), (20000, 5)])
def test_assemble_bit_exact(ctx, n, seed):
    c = sphere_cluster(n, seed)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    b = {k: host(v) for k, v in ctx.bsr_export(A).items()}
    oa = O.assemble(O.collide(c["pos"], c["radius"]))
    assert np.array_equal(b["rowptr"], oa.rowptr)
    assert np.array_equal(b["bcol"], oa.bcol)
    assert np.array_equal(b["val"], oa.val)


def test_spmv_matches_oracle(ctx):
    c = sphere_cluster(5000, 2)
    og = O.collide(c["pos"], c["radius"])
    oa = O.assemble(og)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    A = ctx.assemble_gamma(g)
    x = np.random.default_rng(0).normal(size=(5000, 3))
    y = host(ctx.spmv(A, to_dev(x)))
    yo = O.spmv(oa, x)
    assert np.abs(y - yo).max() <= 1e-14 * np.abs(yo).max()


def _tree_equal(ctx, T, n, ot):
    e = {k: host(v) for k, v in ctx.tree_export(T, n).items()}
    assert np.array_equal(e["tree_edge"], ot.tree_edge)
    assert np.array_equal(e["parent"], ot.parent)
    assert np.array_equal(e["depth"], ot.depth)


@pytest.mark.parametrize("n,seed", [(2, 0), (1000, 0), (20000, 7)])
def test_tree_bit_exact(ctx, n, seed):
    c = sphere_cluster(n, seed)
    print(f"tree n={n}", flush=True)
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    T = ctx.build_tree(g)
    _tree_equal(ctx, T, n, O.build_tree(O.collide(c["pos"], c["radius"])))


def test_tree_all_ties_and_forest(ctx):
    # unjittered lattice: many exactly equal overlaps; plus separated clusters
    parts = [unjittered_cluster(500)["pos"], sphere_cluster(300, 1)["pos"] + 80.0,
             np.array([[300.0, 0, 0]]), sphere_cluster(40, 2)["pos"] - 90.0]
    pos = np.concatenate(parts)
    perm = np.random.default_rng(3).permutation(len(pos))
    pos = pos[perm]
    R = np.ones(len(pos))
    g = ctx.collide(to_dev(pos), to_dev(R))
    T = ctx.build_tree(g)
    og = O.collide(pos, R)
    _graph_equal(ctx, g, og)
    ot = O.build_tree(og)
    assert (ot.parent < 0).sum() == 4
    _tree_equal(ctx, T, len(pos), ot)


@pytest.mark.parametrize("schedule", ["level", "contract"])
@pytest.mark.parametrize("n,seed", [(1000, 0), (6000, 4)])
def test_tree_apply_matches_oracle(ctx, schedule, n, seed):
    """P^{-1} b is unique; the GPU's elimination order differs from Alg. 2's
    (contract) or only its rounding differs (level).  Tolerance: kappa(P) eps
    with kappa(P) <~ 1e4 here -> 1e-11 relative."""
    c = sphere_cluster(n, seed)
    og = O.collide(c["pos"], c["radius"])
    of = O.tree_factor(og, O.build_tree(og))
    g = ctx.collide(to_dev(c["pos"]), to_dev(c["radius"]))
    T = ctx.build_tree(g)
    M = ctx.factor_tree(g, T, schedule=schedule)
    b = np.random.default_rng(1).normal(size=(n, 3))
    z = host(ctx.prec_apply(M, to_dev(b)))
    zo = O.tree_solve(of, b)
    assert np.linalg.norm(z - zo) <= 1e-11 * np.linalg.norm(zo)
    # rigid translation: P (1 x t) = g_med (1 x t)
    t = np.tile([1.0, -2.0, 0.5], (n, 1))
    zt = host(ctx.prec_apply(M, to_dev(t)))
    assert np.allclose(zt, t / 1e-3, rtol=1e-9)
    if schedule == "contract":
        assert M.steps() < 60


@pytest.mark.parametrize("prec", ["tree", "jacobi", "none"])
def test_pcg_velocity_parity_n1000(ctx, prec):
    """Same x0, stopping rule and preconditioner: identical iteration counts,
    velocities within 1e-8 relative of the oracle."""
    c = sphere_cluster(1000, 0)
    out = gpu_chain(ctx, c, prec=prec)
    oo = O.solve_pipeline(c["pos"], c["radius"], c["force"], prec=prec)
    info = out["info"]
    assert info["status"] == 0
    assert info["iters"] == oo["info"].iters, (info, oo["info"])
    v, vo = host(out["v"]), oo["x"]
    assert np.linalg.norm(v - vo) <= 1e-8 * np.linalg.norm(vo)
    assert info["relres_true"] <= 1.01e-8


def _numpy_pcg(A, f, F, k):
    """Second CPU implementation of the same CG (numpy dots, scipy product):
    differs from the oracle only in rounding."""
    import scipy.sparse as sp
    S = sp.bsr_matrix((A.val, A.bcol, A.rowptr), shape=(3 * A.n, 3 * A.n)).tocsr()
    b = F.ravel()
    x = np.zeros_like(b); r = b.copy(); z = O.tree_solve(f, r).ravel(); p = z.copy(); rho = r @ z
    for _ in range(k):
        q = S @ p; a = rho / (p @ q); x += a * p; r -= a * q
        z = O.tree_solve(f, r).ravel(); rn = r @ z; p = z + (rn / rho) * p; rho = rn
    return x.reshape(-1, 3)


def test_pcg_fixed_iterations_parity(ctx):
    """The k-th iterate is a well-defined function of the inputs, but CG's
    intermediate iterates amplify rounding: two correct CPU implementations
    that differ only in summation order already differ by ~3e-8 (relative) at
    k = 40 on this system.  Early iterates must agree to 1e-12; later ones to
    within 10x the spread of the two CPU implementations."""
    c = sphere_cluster(3000, 2)
    for k in (1, 7, 40):
        out = gpu_chain(ctx, c, fixed_iters=k)
        oo = O.solve_pipeline(c["pos"], c["radius"], c["force"], fixed_iters=k)
        assert out["info"]["iters"] == k
        v, vo = host(out["v"]), oo["x"]
        err = np.linalg.norm(v - vo) / np.linalg.norm(vo)
        if k <= 7:
            assert err <= 1e-12, (k, err)
        else:
            x2 = _numpy_pcg(oo["A"], oo["factor"], c["force"], k)
            spread = np.linalg.norm(x2 - vo) / np.linalg.norm(vo)
            assert err <= 10 * max(spread, 1e-12), (k, err, spread)


def test_level_schedule_solve(ctx):
    c = sphere_cluster(2000, 6)
    out = gpu_chain(ctx, c, schedule="level")
    oo = O.solve_pipeline(c["pos"], c["radius"], c["force"])
    assert out["info"]["iters"] == oo["info"].iters
    assert np.linalg.norm(host(out["v"]) - oo["x"]) <= 1e-8 * np.linalg.norm(oo["x"])


def test_determinism(ctx):
    c = sphere_cluster(20000, 9)
    a = gpu_chain(ctx, c)
    b = gpu_chain(ctx, c)
    assert a["info"] == b["info"]
    assert torch.equal(a["v"], b["v"])


def test_warm_start_and_zero_force(ctx):
    c = sphere_cluster(1000, 1)
    out = gpu_chain(ctx, c)
    v2, info2 = ctx.pcg_solve(out["A"], out["M"], out["F"], v=out["v"].clone(), use_x0=True)
    assert info2["iters"] == 0
    zero = torch.zeros_like(out["F"])
    v0, info0 = ctx.pcg_solve(out["A"], out["M"], zero, v=torch.ones_like(zero), use_x0=True)
    assert info0["iters"] == 0 and not v0.any()


def test_error_paths(ctx):
    c = sphere_cluster(1000, 1)
    out = gpu_chain(ctx, c)
    _, info = ctx.pcg_solve(out["A"], out["M"], out["F"], max_iter=1, check=False)
    assert info["status"] == P.ENOCONV and info["iters"] == 1
    Fb = out["F"].clone()
    Fb[5, 1] = float("nan")
    _, info = ctx.pcg_solve(out["A"], out["M"], Fb, check=False)
    assert info["status"] == P.ENONFINITE
    with pytest.raises(P.SgpError) as e:
        ctx.collide(out["pos"], out["R"], max_deg=4)
    assert e.value.status == P.ECAPACITY
    pos = to_dev(np.array([[0.0, 0, 0], [0.0, 0, 0], [5.0, 0, 0]]))
    with pytest.raises(P.SgpError) as e:
        ctx.collide(pos, to_dev(np.ones(3)))
    assert e.value.status == P.EINVAL
    # singular pivot: no medium friction and an isolated cell
    pos = to_dev(np.array([[0.0, 0, 0], [1.9, 0, 0], [50.0, 0, 0]]))
    g = ctx.collide(pos, to_dev(np.ones(3)))
    T = ctx.build_tree(g)
    with pytest.raises(P.SgpError) as e:
        ctx.factor_tree(g, T, g_med=0.0)
    assert e.value.status == P.ENOTSPD


def test_empty_input(ctx):
    g = ctx.collide(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                    torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert g.size() == (0, 0)
    A = ctx.assemble_gamma(g)
    T = ctx.build_tree(g)
    M = ctx.factor_tree(g, T)
    v, info = ctx.pcg_solve(A, M, torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    assert info["iters"] == 0


@pytest.mark.parametrize("waves", [2, 4, 8])
def test_no_contacts(ctx, waves):
    """Cells that touch nothing: Gamma = g_med I (a product without
    off-diagonal entries), every cell is a tree of its own, and the tree
    preconditioner is Gamma itself, so CG stops after one iteration at
    v = F / g_med."""
    n = 300
    pos = np.stack([np.arange(n) * 5.0, np.zeros(n), np.zeros(n)], axis=1)
    c = {"pos": pos, "radius": np.ones(n), "force": np.random.default_rng(3).normal(size=(n, 3))}
    ctx.tune("spmv_waves", waves)
    try:
        out = gpu_chain(ctx, c)
        assert out["g"].size() == (n, 0)
        x = np.random.default_rng(4).normal(size=(n, 3))
        y = host(ctx.spmv(out["A"], to_dev(x)))
        assert np.array_equal(y, x * O.G_MED)
        oo = O.solve_pipeline(c["pos"], c["radius"], c["force"])
        assert out["info"]["status"] == 0 and out["info"]["iters"] == oo["info"].iters == 1
        v = host(out["v"])
        assert np.abs(v - oo["x"]).max() <= 1e-12 * np.abs(oo["x"]).max()
    finally:
        ctx.tune("spmv_waves", 4)


def test_tree_graph_one_iteration(ctx):
    pos = np.array([[1.9 * k, 0.1 * np.sin(k), 0.0] for k in range(40)])
    c = {"pos": pos, "radius": np.ones(40), "force": np.random.default_rng(0).normal(size=(40, 3))}
    out = gpu_chain(ctx, c, rtol=1e-12)
    assert out["info"]["iters"] == 1
